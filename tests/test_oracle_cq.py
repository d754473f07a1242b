"""Pins for oracle tier C (exact Q H^T, Sec. 3.2) and the ray operator.

The three routes to Q H^T (dense, FFT circulant embedding, direct sums over
the nonzeros of H) are written independently and must agree; a nearly
constant kernel reduces Q H^T to a rank-one closed form; the rows of H sum to
the ray lengths (Sec. 4.1, eq. ``equation_traveltimeintegral``).
"""

import numpy as np
import pytest

import synth
from oracle import cq_exact


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dim,n,p", [(2, 32, 16), (2, 64, 16), (3, 8, 16)])
def test_ray_rows_sum_to_lengths(dim, n, p):
    rp, col, val = synth.crosswell_h(dim, n, p, planes=2 if dim == 3 else 8)
    sums = np.add.reduceat(val, rp[:-1])
    lens = synth.ray_lengths(dim, p, planes=2 if dim == 3 else 8)
    np.testing.assert_allclose(sums, lens, rtol=1e-13)
    assert np.all(val > 0)
    assert np.all(val <= np.sqrt(dim) / n * (1 + 1e-12))
    for a in range(p):
        c = col[rp[a]:rp[a + 1]]
        assert np.all(np.diff(c) > 0)
        assert c.min() >= 0 and c.max() < n ** dim


def test_generators_are_deterministic():
    a = synth.crosswell_h(2, 64, 16)
    b = synth.crosswell_h(2, 64, 16)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    np.testing.assert_array_equal(synth.normal_draws(5, 3, 4), synth.normal_draws(5, 3, 4))


@pytest.mark.parametrize("family,ell,gamma", [("powexp", 0.3, 1.0),
                                              ("powexp", 0.05, 2.0),
                                              ("r2", 1.0, 1.0)])
def test_three_routes_agree(family, ell, gamma):
    n, p = 32, 16
    rp, col, val = synth.crosswell_h(2, n, p)
    pts = synth.cell_centres(2, n)
    Ht = cq_exact.h_dense(rp, col, val, n * n).T
    dense = cq_exact.cq_dense(pts, Ht, family, 1.0, ell, gamma)
    fft = cq_exact.cq_fft(2, n, Ht, family, 1.0, ell, gamma)
    rows = cq_exact.cq_rows(2, n, rp, col, val, np.arange(n * n), family, 1.0, ell, gamma)
    assert _rel(fft, dense) < 1e-13
    assert _rel(rows, dense) < 1e-13


def test_three_routes_agree_3d():
    n, p = 8, 16
    rp, col, val = synth.crosswell_h(3, n, p, planes=2)
    pts = synth.cell_centres(3, n)
    Ht = cq_exact.h_dense(rp, col, val, n ** 3).T
    dense = cq_exact.cq_dense(pts, Ht, "powexp", 1.0, 0.2, 1.0)
    fft = cq_exact.cq_fft(3, n, Ht, "powexp", 1.0, 0.2, 1.0)
    rows = cq_exact.cq_rows(3, n, rp, col, val, np.arange(0, n ** 3, 7), "powexp", 1.0, 0.2, 1.0)
    assert _rel(fft, dense) < 1e-13
    assert _rel(rows, dense[::7]) < 1e-13


def test_sampled_rows_match_fft_large():
    n, p = 256, 64
    rp, col, val = synth.crosswell_h(2, n, p)
    Ht = np.zeros((n * n, p))
    for a in range(p):
        Ht[col[rp[a]:rp[a + 1]], a] = val[rp[a]:rp[a + 1]]
    fft = cq_exact.cq_fft(2, n, Ht, "powexp", 1.0, 0.1, 1.0)
    rows = np.random.default_rng(1).choice(n * n, 64, replace=False)
    direct = cq_exact.cq_rows(2, n, rp, col, val, rows, "powexp", 1.0, 0.1, 1.0)
    assert _rel(direct, fft[rows]) < 1e-12


def test_constant_kernel_closed_form():
    # K = theta * exp(-r / ell) with ell -> infinity is theta everywhere, so
    # Q H^T = theta * 1 (H 1)^T.
    n, p, theta = 16, 16, 2.5
    rp, col, val = synth.crosswell_h(2, n, p)
    Ht = cq_exact.h_dense(rp, col, val, n * n).T
    fft = cq_exact.cq_fft(2, n, Ht, "powexp", theta, 1e12, 1.0)
    closed = theta * np.ones((n * n, 1)) @ Ht.sum(axis=0)[None, :]
    assert _rel(fft, closed) < 1e-11
