"""The sensitivity ceilings behind the GPU step tolerances.

The GPU step tests hold C_Q to CQ_TOL against the oracle and the filter
outputs to KAPPA * CQ_TOL.  KAPPA is the gain's amplification of a C_Q error
into x_hat and diag P (Sec. 3.1: C_Q enters G = H C_prior and the gain
K = C_prior (H C_prior + R)^{-1}, whose condition grows like |H Q H^T| / R).
Here the oracle measures that amplification on the reference C_Q of every
GPU case, with no GPU involved, and the ceilings must exceed it by 1.5x.
"""

import pytest

from helpers import KAPPA, Case, output_sensitivity


def _case(key):
    if key[0] == "direct":
        _, n, p = key
        return Case(2, n, p, ell=0.3, gamma=1.0, steps=6), None
    _, n, p, n_c = key
    ell, gamma = {32: (0.3, 1.0), 64: (0.1, 2.0), 59: (0.2, 1.0)}[n]
    return Case(2, n, p, ell=ell, gamma=gamma, steps=4), n_c


@pytest.mark.parametrize("key", sorted(KAPPA, key=str))
def test_kappa_ceilings_hold(key):
    case, n_c = _case(key)
    ref = case.cq_exact() if n_c is None else case.cq_bbfmm(n_c)
    kx, kv = output_sensitivity(case, ref)
    cx, cv = KAPPA[key]
    print(f"{key}: measured kappa x {kx:.2f} var {kv:.2f}; ceilings {cx}, {cv}")
    assert 1.5 * kx <= cx and 1.5 * kv <= cv
    # the amplification is real: a C_Q error is not damped below itself in x_hat
    assert kx > 0.5
