"""GPU parity at the benchmark sizes, over every step of each workload, in
the launch configurations bench.py times (sparse source side; the step as a
captured HIP graph, and eagerly with phase timing):

* 256 x 256, p = 64, exponential ell = 0.1, n_c = 4, FP32 FMM, 100 steps;
* 1024 x 1024, p = 256, Gaussian ell = 0.05, n_c = 5, FP32 FMM, 50 steps;
* 128^3, p = 512, exponential ell = 0.2, n_c = 4, BF16x3 FMM, 20 steps.

At these sizes the oracle cannot run the whole filter live, so two kinds of
reference are used.
* tests/golden/fullsize_<workload>.npz, written by make_fullsize_refs.py (a
  script that runs only the oracle): x_hat_k and diag P_k on 255 report rows
  for every step, from the cross-covariance filter on the ray cells plus the
  report rows, once with the exact C_Q and once with the oracle's FP64
  black-box FMM C_Q of the same n_c; C_Q on the report rows both ways; and
  the filter's measured sensitivity kappa to a C_Q error at that size.
* Live: the oracle's FP64 black-box FMM on 16 whole columns of W = H^T.

The error of the GPU against the exact filter (eps_total) splits into the H^2
error of n_c (eps_H2, oracle FMM vs exact; fixed by the workload) and the
arithmetic error (eps_arith, GPU vs oracle FMM).  The bounds are
* C_Q vs the oracle FMM: CQ_TOL of the precision (2e-6 FP32, 1e-4 BF16x3);
* outputs vs the oracle-FMM filter: 1.5 kappa CQ_TOL;
* outputs vs the exact filter: eps_H2 + 1.5 kappa CQ_TOL.
No bound is computed from GPU output.
"""

import os

import numpy as np
import pytest

import synth
from helpers import CQ_TOL, max_step_rel, rel

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CASES = [
    ("crosswell-256x256-p64", "f32", True),
    ("crosswell-1024x1024-p256", "f32", True),
    ("crosswell-1024x1024-p256", "f32", False),
    ("crosswell-128cube-p512", "bf16x3", True),
]


def _refs(name):
    path = os.path.join(GOLDEN, f"fullsize_{name}.npz")
    assert os.path.exists(path), f"{path} missing: run tests/golden/make_fullsize_refs.py"
    return dict(np.load(path, allow_pickle=False))


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-{c[1]}-{'graph' if c[2] else 'eager'}")
def run(request):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_3816_amd import filter as F
    name, precision, graph = request.param
    w = synth.workload(name)
    dim, n, p, m, K = w["dim"], w["n"], w["p"], w["m"], w["steps"]
    print(f"\n[fullsize] {name} precision={precision} graph={graph}", flush=True)
    rowptr, col, val = synth.crosswell_h(dim, n, p, planes=8)
    ys = synth.plume_observations(dim, n, rowptr, col, val, K, w["r_var"], w["seed"] + 1)
    ref = _refs(name)
    rows = ref["rows"]
    pr, keep = F.problem_from_csr(dim, n, rowptr, col, val, np.full(p, w["r_var"]),
                                  theta=w["theta"], ell=w["ell"], gamma=w["gamma"],
                                  prior=w["prior"])
    f = F.HikfFilter(pr, F.make_options(w["n_c"], precision, False, timing=not graph,
                                        graph=graph, sparse=True), keep)
    rd = torch.as_tensor(rows, device="cuda")
    cols16 = torch.as_tensor(np.arange(0, p, p // 16), device="cuda")
    cq_full = f.export_cq()
    cq_rows = cq_full[rd].cpu().numpy()
    cq_cols = cq_full[:, cols16].cpu().numpy()
    del cq_full
    yd = torch.as_tensor(ys, device="cuda")
    x = torch.empty(m, dtype=torch.float64, device="cuda")
    v = torch.empty_like(x)
    xs = torch.empty(K, len(rows), dtype=torch.float64, device="cuda")
    vs = torch.empty_like(xs)
    for k in range(K):
        f.step(yd[k], x, v)
        xs[k] = x[rd]
        vs[k] = v[rd]
    st = f.query()
    f.close()
    return dict(name=name, w=w, precision=precision, rowptr=rowptr, col=col, val=val, ref=ref,
                cq_rows=cq_rows, cq_cols=cq_cols, cols=np.arange(0, p, p // 16),
                x=xs.cpu().numpy(), v=vs.cpu().numpy(), stats=st)


def test_fullsize_all_steps_applied(run):
    st = run["stats"]
    assert st.last_status == 0 and st.steps_applied == run["w"]["steps"]
    assert np.all(np.isfinite(run["x"])) and np.all(np.isfinite(run["v"]))


def test_fullsize_cq_rows(run):
    ref, tol = run["ref"], CQ_TOL[run["precision"]]
    e_arith = rel(run["cq_rows"], ref["cq_bbfmm"])
    e_total = rel(run["cq_rows"], ref["cq_exact"])
    e_h2 = rel(ref["cq_bbfmm"], ref["cq_exact"])
    print(f"{run['name']}: C_Q on {len(ref['rows'])} rows: eps_total {e_total:.3e} "
          f"eps_H2 {e_h2:.3e} eps_arith {e_arith:.3e}")
    assert e_arith < tol
    assert e_total < e_h2 + tol


def test_fullsize_cq_columns_match_oracle_bbfmm(run):
    # 16 whole columns of C_Q (every row) against the oracle's FP64 bbFMM
    from oracle import bbfmm
    w, cols = run["w"], run["cols"]
    m = w["m"]
    W = np.zeros((m, len(cols)))
    rp, col, val = run["rowptr"], run["col"], run["val"]
    for j, a in enumerate(cols):
        W[col[rp[a]:rp[a + 1]], j] = val[rp[a]:rp[a + 1]]
    ref = bbfmm.bbfmm_apply(w["dim"], w["n"], W, w["n_c"], None, "powexp", w["theta"],
                            w["ell"], w["gamma"])
    err = rel(run["cq_cols"], ref)
    print(f"{run['name']}: C_Q on 16 whole columns vs oracle bbFMM: {err:.3e}")
    assert err < CQ_TOL[run["precision"]]


def test_fullsize_trajectory(run):
    ref, tol = run["ref"], CQ_TOL[run["precision"]]
    kx, kv = ref["kappa"]
    bx, bv = 1.5 * kx * tol, 1.5 * kv * tol
    ax, av = max_step_rel(run["x"], ref["x_bbfmm"]), max_step_rel(run["v"], ref["var_bbfmm"])
    tx, tv = max_step_rel(run["x"], ref["x_exact"]), max_step_rel(run["v"], ref["var_exact"])
    hx, hv = (max_step_rel(ref["x_bbfmm"], ref["x_exact"]),
              max_step_rel(ref["var_bbfmm"], ref["var_exact"]))
    print(f"{run['name']} ({run['precision']}, {run['w']['steps']} steps): "
          f"x_hat eps_total {tx:.3e} eps_H2 {hx:.3e} eps_arith {ax:.3e} (bound {bx:.1e}); "
          f"var eps_total {tv:.3e} eps_H2 {hv:.3e} eps_arith {av:.3e} (bound {bv:.1e})")
    assert ax < bx and av < bv
    assert tx < hx + bx and tv < hv + bv
