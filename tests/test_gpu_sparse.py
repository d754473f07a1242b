"""GPU parity of the sparse-W mode (hikf_options.sparse = 1).

P2M and the near field read only the nonzeros of W = H^T, bucketed by leaf;
the product is the same H^2 approximation as the dense mode, so the oracle
bbFMM and its tolerances apply unchanged (FP64: rounding only, 1e-12; FP32:
2e-6 normwise; BF16x3 with the FP32 near field: 1e-4), and against the dense
mode in FP64 the difference is the order of rounding only.
"""

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


def _cq(case, **kw):
    f = case.gpu_filter(**kw)
    cq = f.export_cq().cpu().numpy()
    f.close()
    return cq


@pytest.mark.parametrize("dim,n,p,n_c,ell,gamma", [
    (2, 32, 16, 4, 0.3, 1.0),      # depth 2
    (2, 64, 32, 4, 0.1, 1.0),      # depth 3
    (2, 128, 48, 5, 0.05, 2.0),    # depth 4, Gaussian, ragged column tile
    (2, 100, 32, 5, 0.1, 2.0),     # padded tree (100 -> 128)
    (3, 16, 16, 3, 0.2, 1.0),      # octree depth 2
    (3, 20, 32, 4, 0.2, 1.0),      # padded octree (20 -> 32), r = 64
])
@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x3"])
def test_sparse_cq_matches_oracle_bbfmm(dim, n, p, n_c, ell, gamma, precision):
    case = Case(dim, n, p, ell=ell, gamma=gamma, steps=1, planes=2)
    cq = _cq(case, n_c=n_c, precision=precision, sparse=True)
    ref = case.cq_bbfmm(n_c)
    tol = {"f64": 1e-12, "f32": 2e-6, "bf16x3": 1e-4}[precision]
    assert rel(cq, ref) < tol
    if precision == "f32":
        assert np.all(np.abs(cq - ref) <= 1e-5 * np.abs(ref) + 2e-6 * np.abs(ref).max())


@pytest.mark.parametrize("dim,n,p", [(2, 64, 64), (2, 72, 512), (3, 16, 64)])
def test_sparse_equals_dense_f64(dim, n, p):
    # same sums in another order: FP64 rounding only
    case = Case(dim, n, p, ell=0.2, steps=1, planes=2)
    dense = _cq(case, n_c=4, precision="f64")
    sparse = _cq(case, n_c=4, precision="f64", sparse=True)
    assert rel(sparse, dense) < 1e-13


@pytest.mark.parametrize("dim,n,n_c", [(2, 64, 3), (2, 40, 4), (3, 16, 3)])
def test_sparse_polynomial_kernel_exact(dim, n, n_c):
    # K = r^2 is reproduced exactly by the interpolation: every bucket, list
    # and near-field table slot must be right for the dense product to come out
    case = Case(dim, n, 16, family="r2", steps=1)
    cq = _cq(case, n_c=n_c, precision="f64", sparse=True)
    assert rel(cq, case.cq_exact()) < 1e-12


@pytest.mark.parametrize("dim,n", [(2, 8), (2, 16), (3, 4), (3, 8), (2, 5)])
def test_sparse_shallow_trees_exact(dim, n):
    # depth 0 / 1: near field only, which is then the exact product
    case = Case(dim, n, 16, ell=0.3, steps=1)
    cq = _cq(case, n_c=4, precision="f64", sparse=True)
    assert rel(cq, case.cq_exact()) < 1e-13


def test_sparse_steps_match_dense_steps():
    # the filter run on the sparse-mode C_Q: FP64 throughout, so the two runs
    # differ by rounding only
    case = Case(2, 64, 32, ell=0.1, steps=4)
    cq_d, xs_d, vs_d, st_d = case.gpu_run(n_c=4, precision="f64")
    cq_s, xs_s, vs_s, st_s = case.gpu_run(n_c=4, precision="f64", sparse=True)
    assert st_d.last_status == 0 and st_s.last_status == 0
    assert rel(cq_s, cq_d) < 1e-13
    assert rel(xs_s, xs_d) < 1e-10
    assert rel(vs_s, vs_d) < 1e-12


def test_sparse_empty_h():
    import torch
    from paper_1404_3816_amd import filter as F
    p, n = 32, 64
    rowptr = np.zeros(p + 1, np.int64)
    pr, keep = F.problem_from_csr(2, n, rowptr, np.zeros(0, np.int32), np.zeros(0),
                                  np.full(p, 1e-4), ell=0.2)
    f = F.HikfFilter(pr, F.make_options(4, "f32", False, sparse=True), keep)
    y = torch.as_tensor(np.random.default_rng(3).standard_normal(p), device="cuda")
    f.step(y)
    cq = f.export_cq().cpu().numpy()
    st = f.query()
    f.close()
    assert st.last_status == 0 and np.all(cq == 0.0)


def test_sparse_with_history_riccati_and_queries():
    # the sparse mode under the other options: a step graph, the p-space
    # recursion and the covariance history; in FP64 every output agrees
    # with the dense-mode filter up to rounding
    import torch
    case = Case(2, 64, 32, ell=0.1, steps=4)
    v = torch.as_tensor(np.random.default_rng(5).standard_normal(case.m), device="cuda")
    y = torch.as_tensor(case.ys, device="cuda")
    out = {}
    for sparse in (False, True):
        f = case.gpu_filter(n_c=4, precision="f64", sparse=sparse, history=4, riccati=2, graph=True)
        x = torch.empty(case.m, dtype=torch.float64, device="cuda")
        var = torch.empty(case.m, dtype=torch.float64, device="cuda")
        for k in range(case.steps):
            f.step(y[k], x, var)
        pv = f.cov_apply(v).cpu().numpy()
        st = f.query()
        out[sparse] = (x.cpu().numpy(), var.cpu().numpy(), pv)
        f.close()
        assert st.last_status == 0 and st.steps_applied == case.steps
    for a, b in zip(out[True], out[False]):
        assert rel(a, b) < 1e-10
