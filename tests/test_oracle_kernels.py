"""Pins for the covariance kernels of the oracle (Sec. 4.2 eq. ``equation_Q``;
Sec. 3.3 list of kernels).

K(r) = theta exp(-(r / ell)^gamma) is fixed at three distances for every
exponent: K(0) = theta, K(ell) = theta / e, and K(2 ell) = theta exp(-2^gamma).
A mistake in the scale (r^gamma / ell instead of (r / ell)^gamma), in the sign
or in theta moves at least one of these values.  The dense Q built from K is
symmetric with K(0) on its diagonal.
"""

import math

import numpy as np
import pytest

import synth
from oracle import kernels


@pytest.mark.parametrize("gamma", [0.5, 1.0, 1.5, 2.0])
@pytest.mark.parametrize("theta,ell", [(1.0, 0.3), (2.5, 0.05), (0.7, 1.7)])
def test_powexp_closed_form_values(theta, ell, gamma):
    K = kernels.kernel("powexp", theta, ell, gamma)
    assert K(0.0) == theta
    assert abs(K(ell) - theta / math.e) <= 1e-15 * theta
    assert abs(K(2.0 * ell) - theta * math.exp(-(2.0 ** gamma))) <= 1e-15 * theta
    # a half-length: exp(-2^-gamma), distinguishes the exponent's argument
    assert abs(K(0.5 * ell) - theta * math.exp(-(0.5 ** gamma))) <= 1e-15 * theta
    assert kernels.diag_value("powexp", theta, ell, gamma) == theta


def test_powexp_is_monotone_and_positive():
    r = np.linspace(0.0, 3.0, 301)
    for gamma in (0.5, 1.0, 2.0):
        k = kernels.powexp(r, 1.3, 0.4, gamma)
        assert np.all(k > 0.0) and np.all(np.diff(k) < 0.0)


def test_r2_kernel_values():
    assert kernels.r2(0.0, 2.0) == 0.0
    assert kernels.r2(3.0, 2.0) == 18.0
    assert kernels.diag_value("r2", 2.0) == 0.0


def test_dense_q_symmetric_with_kernel_diagonal():
    pts = synth.cell_centres(2, 8)
    Q = kernels.dense_q(pts, "powexp", 1.5, 0.2, 1.0)
    np.testing.assert_array_equal(Q, Q.T)
    np.testing.assert_array_equal(np.diag(Q), np.full(64, 1.5))
    # cells (0, 0) and (1, 0) are one cell width h = 1/8 apart
    assert abs(Q[0, 1] - 1.5 * math.exp(-(1.0 / 8) / 0.2)) < 1e-15
    # cells (0, 0) and (1, 1): h sqrt(2)
    assert abs(Q[0, 9] - 1.5 * math.exp(-(math.sqrt(2.0) / 8) / 0.2)) < 1e-15
