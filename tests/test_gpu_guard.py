"""The PSD guard and checkpoints through the C ABI.

A smooth Gaussian kernel (ell = 0.2 on a 64 x 64 grid, p = 64, n_c = 6):
the H^2 approximation makes H Q H^T indefinite, and the literal filter's S
fails its Cholesky within tens of steps (the oracle shows the same, see
tests/test_oracle_kf.py).  With hikf_options.psd_guard the filter keeps
going and follows the oracle's guarded filter (oracle/kf_crosscov.py,
crosscov_kf_guarded) on the oracle's own FP64 bbFMM C_Q.  The GPU forms the
PSD part with a fixed number of Newton-Schulz sign iterations instead of an
eigendecomposition; eigenvalues below 1.5^-64 of ||G_Q||_F keep a partly
converged sign, which moves S by less than 1e-10 in those directions.
"""

import numpy as np
import pytest

from helpers import Case, max_step_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_3816_amd import hikf  # noqa: F401  (fails loudly without libhikf.so)


def _gauss_case(steps=40):
    case = Case(2, 64, 64, ell=0.2, gamma=2.0, steps=steps)
    case.ys = np.random.default_rng(4).standard_normal((steps, 64)) * 1e-2
    return case


def test_unguarded_filter_loses_definiteness_and_guard_keeps_it():
    case = _gauss_case()
    _, _, _, st = case.gpu_run(n_c=6, precision="f64")
    assert st.last_status == 4 and st.steps_applied < case.steps
    _, xs, vs, sg = case.gpu_run(n_c=6, precision="f64", psd_guard=True)
    assert sg.last_status == 0 and sg.steps_applied == case.steps
    assert np.all(np.isfinite(xs)) and np.all(vs > 0)


@pytest.mark.parametrize("graph", [False, True])
def test_guard_matches_oracle_guarded_filter(graph):
    from oracle import kf_crosscov
    case = _gauss_case()
    cq_ref = case.cq_bbfmm(6)
    H = case.h_dense()
    G0 = 2.0 * kf_crosscov.psd_part(H @ cq_ref)
    xo, vo = kf_crosscov.crosscov_kf_guarded(cq_ref, H, np.diag(case.r_diag), np.zeros(case.m),
                                             cq_ref, np.ones(case.m), 1.0, case.ys, G0=G0)
    cq, xs, vs, st = case.gpu_run(n_c=6, precision="f64", psd_guard=True, graph=graph)
    ex, ev = max_step_rel(xs, xo), max_step_rel(vs, vo)
    print(f"guarded GPU vs oracle guarded filter: x {ex:.3e} var {ev:.3e}")
    assert st.last_status == 0 and st.steps_applied == case.steps
    assert ev < 1e-8 and ex < 1e-4


@pytest.mark.parametrize("mode", ["gather", "riccati", "guard"])
def test_checkpoint_roundtrip_is_bitwise(mode):
    import torch
    case = Case(2, 64, 32, ell=0.1, steps=6)
    opts = {"gather": {}, "riccati": {"riccati": 3}, "guard": {"psd_guard": True}}[mode]
    y = torch.as_tensor(case.ys, device="cuda")
    fa = case.gpu_filter(n_c=4, precision="f32", **opts)
    for k in range(4):
        fa.step(y[k])
    x, v, c, ps, info = fa.export_checkpoint()
    assert info.steps_applied == 4 and info.steps_issued == 4 and info.p == case.p
    fb = case.gpu_filter(n_c=4, precision="f32", **opts)
    fb.import_checkpoint(x, v, c, ps, info)
    assert fb.query().steps_applied == 4
    for k in (4, 5):
        fa.step(y[k])
        fb.step(y[k])
    sa, sb = fa.export_state(), fb.export_state()
    assert all(torch.equal(a, b) for a, b in zip(sa, sb))
    assert fa.query().steps_applied == fb.query().steps_applied == 6
    fa.close()
    fb.close()


def test_checkpoint_of_another_problem_is_refused():
    from paper_1404_3816_amd import hikf as H
    case = Case(2, 64, 32, ell=0.1, steps=2)
    fa = case.gpu_filter(n_c=4, precision="f32")
    x, v, c, ps, info = fa.export_checkpoint()
    other = Case(2, 64, 32, ell=0.1, steps=2, r_var=2e-4)       # a different R
    fb = other.gpu_filter(n_c=4, precision="f32")
    with pytest.raises(H.HikfError) as err:
        fb.import_checkpoint(x, v, c, ps, info)
    assert err.value.status == H.HIKF_E_INVALID
    fc = case.gpu_filter(n_c=5, precision="f32")                  # another n_c
    with pytest.raises(H.HikfError):
        fc.import_checkpoint(x, v, c, ps, info)
    for f in (fa, fb, fc):
        f.close()
