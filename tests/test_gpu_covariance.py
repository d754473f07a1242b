"""Posterior covariance queries (P_t v) through the C ABI against the FP64
oracle: the dense Kalman filter's full P_t in the all-pairs mode (no H^2
error), and the cross-covariance filter's Z history with the oracle's
bbFMM for the tree mode (P_t v = P_0 v + t Q v - sum_s Z_s Z_s^T v)."""

import numpy as np
import pytest

from helpers import Case, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_3816_amd import hikf  # noqa: F401  (fails loudly without libhikf.so)


def _filter(case, n_c=4, precision="f64", direct=True, history=8):
    from paper_1404_3816_amd import filter as F
    pr, keep = F.problem_from_csr(case.dim, case.n, case.rowptr, case.col, case.val,
                                  case.r_diag, prior=case.prior, alpha=case.alpha,
                                  **case.kparams())
    return F.HikfFilter(pr, F.make_options(n_c, precision, direct, history=history), keep)


@pytest.mark.parametrize("prior,alpha", [("kernel", 0.0), ("scaled_i", 0.5), ("zero", 0.0)])
def test_cov_apply_matches_dense_kf(prior, alpha):
    import torch
    from oracle import kernels, kf_dense
    import synth
    case = Case(2, 32, 16, ell=0.3, steps=4, prior=prior, alpha=alpha)
    Q = kernels.dense_q(synth.cell_centres(2, 32), **case.kparams())
    P0 = {"kernel": Q, "scaled_i": alpha * np.eye(case.m), "zero": np.zeros((case.m, case.m))}[prior]
    _, _, Ps = kf_dense.dense_kf(Q, case.h_dense(), np.diag(case.r_diag), np.zeros(case.m), P0,
                                 case.ys)
    v = np.random.default_rng(11).standard_normal(case.m)
    vd = torch.as_tensor(v, device="cuda")
    f = _filter(case)
    y = torch.as_tensor(case.ys, device="cuda")
    got0 = f.cov_apply(vd).cpu().numpy()           # before any step: P_0 v
    if prior == "zero":
        assert np.all(got0 == 0.0)
    else:
        assert rel(got0, P0 @ v) < 1e-12
    for k in range(case.steps):
        f.step(y[k])
        got = f.cov_apply(vd).cpu().numpy()
        assert rel(got, Ps[k] @ v) < 1e-10, k
    f.close()


@pytest.mark.parametrize("precision,tol", [("f64", 1e-11), ("f32", 1e-4)])
def test_cov_apply_tree_matches_oracle_history(precision, tol):
    import torch
    from oracle import bbfmm, kf_crosscov
    case = Case(2, 64, 32, ell=0.1, steps=3)
    v = np.random.default_rng(12).standard_normal(case.m)
    cq = case.cq_bbfmm(4)
    qv = bbfmm.bbfmm_apply(2, 64, v[:, None], 4, None, **case.kparams())[:, 0]
    _, _, zs = kf_crosscov.crosscov_kf(cq, case.h_dense(), np.diag(case.r_diag),
                                       np.zeros(case.m), cq, np.ones(case.m), 1.0, case.ys,
                                       return_Z=True)
    f = _filter(case, precision=precision, direct=False)
    y = torch.as_tensor(case.ys, device="cuda")
    vd = torch.as_tensor(v, device="cuda")
    for k in range(case.steps):
        f.step(y[k])
        ref = (k + 2) * qv - sum(z @ (z.T @ v) for z in zs[:k + 1])
        assert rel(f.cov_apply(vd).cpu().numpy(), ref) < tol, k
    f.close()


def test_cov_apply_needs_history():
    import torch
    from paper_1404_3816_amd import hikf as H
    case = Case(2, 32, 16, ell=0.3, steps=3)
    y = torch.as_tensor(case.ys, device="cuda")
    vd = torch.zeros(case.m, dtype=torch.float64, device="cuda")
    f0 = _filter(case, history=0)
    with pytest.raises(H.HikfError):
        f0.cov_apply(vd)
    f0.close()
    f2 = _filter(case, history=2)
    for k in range(3):
        f2.step(y[k])
    with pytest.raises(H.HikfError):
        f2.cov_apply(vd)                 # three steps applied, two kept
    f2.close()
