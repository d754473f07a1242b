"""The ensemble Kalman filter (include/hikf_enkf.h) against the oracle's EnKF.

Same seeded inputs on both sides: the initial ensemble and the model-error
draws are L xi with L the Cholesky factor of the kernel matrix Q of an
exponential kernel on the grid (draws xi from synth.normal_draws), the
observation perturbations sqrt(R) xi', the data H x_true + noise.  The GPU
applies the analysis as X <- (X + E) W; the oracle applies the gain
K~ = A (H A)^T S^{-1} to every member's innovation.  Both are FP64: the
difference is rounding, amplified by the conditioning of S = (HA)(HA)^T + R
(R = 1e-4 I against (HA)(HA)^T of order 1: cond(S) <~ 1e4), so the bound on
the ensemble, its mean and its variance is 1e-10 relative (FP64 unit
roundoff 1.1e-16 times 1e4, with a margin of ~100 for the sums over nnz(H)
and N).  The variance of a row is a sum of squared anomalies: an error
delta in the members moves it by at most 2 sqrt(2) delta max|X| sqrt(var)
per row, so its bound is TOL times that factor over var, taken from the
oracle's ensemble (it matters for tiny ensembles, whose analysis spread
is small against the state: N = 2).  Grids of 37 x 37 and 45 x 45 cells
span several row tiles of the transform with a ragged last tile; N covers
both tile forms (ld <= 256 and ld > 256) and sizes that need padding.
"""

import numpy as np
import pytest

import synth
from oracle import enkf as oracle_enkf
from oracle import kernels

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_3816_amd import hikf  # noqa: F401  (fails loudly without libhikf.so)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _var_tol(X, var):
    """TOL scaled by the cancellation in the variance of the oracle's ensemble."""
    amp = (2.0 * np.sqrt(2.0) * np.max(np.abs(X)) * np.linalg.norm(np.sqrt(var))
           / np.linalg.norm(var))
    return TOL * max(1.0, amp)


class EnCase:
    def __init__(self, n, p, N, steps=3, ell=0.2, r_var=1e-4, seed=0, noise=True):
        self.n, self.p, self.N, self.steps = n, p, N, steps
        self.m = n * n
        self.rowptr, self.col, self.val = synth.crosswell_h(2, n, p)
        self.r = np.full(p, r_var)
        pts = synth.cell_centres(2, n)
        Q = kernels.dense_q(pts, "powexp", 1.0, ell, 1.0)
        L = np.linalg.cholesky(Q + 1e-10 * np.eye(self.m))
        m = self.m
        self.X0 = L @ synth.normal_draws(seed + 1, m, N)
        self.Es = [L @ synth.normal_draws(seed + 10 + k, m, N) for k in range(steps)] \
            if noise else None
        self.Vs = [np.sqrt(r_var) * synth.normal_draws(seed + 20 + k, p, N) for k in range(steps)]
        truth = L @ synth.normal_draws(seed + 2, m)
        import scipy.sparse as sp
        self.H = sp.csr_matrix((self.val, self.col, self.rowptr), shape=(p, m))
        self.ys = [self.H @ truth + np.sqrt(r_var) * synth.normal_draws(seed + 30 + k, p)
                   for k in range(steps)]

    def oracle(self):
        return oracle_enkf.enkf_run(self.X0, self.H, self.r, self.ys, self.Es, self.Vs)

    def gpu(self, timing=False, tile_rows=0):
        import torch
        from paper_1404_3816_amd import enkf as EN
        pr, keep = EN.enkf_problem(self.rowptr, self.col, self.val, self.r, self.m, self.N,
                                   timing=timing, tile_rows=tile_rows)
        f = EN.EnkfFilter(pr, torch.as_tensor(self.X0, device="cuda"), keep)
        means, vars_ = [], []
        for k in range(self.steps):
            e = None
            if self.Es is not None:
                e = torch.zeros(self.m, f.ld, dtype=torch.float64, device="cuda")
                e[:, :self.N] = torch.as_tensor(self.Es[k], device="cuda")
                # the columns beyond N are not members: whatever they hold is ignored
                e[:, self.N:] = float("nan")
            mo = torch.empty(self.m, dtype=torch.float64, device="cuda")
            vo = torch.empty(self.m, dtype=torch.float64, device="cuda")
            f.step(e, torch.as_tensor(self.ys[k], device="cuda"),
                   torch.as_tensor(self.Vs[k], device="cuda"), mo, vo)
            means.append(mo.cpu().numpy())
            vars_.append(vo.cpu().numpy())
        X = f.export().cpu().numpy()
        st = f.query()
        f.close()
        return X, np.array(means), np.array(vars_), st


@pytest.mark.parametrize("n,p,N", [(37, 16, 16), (37, 32, 40), (45, 48, 100), (37, 64, 300),
                                   (37, 32, 400), (45, 16, 2)])
def test_enkf_matches_oracle(n, p, N):
    case = EnCase(n, p, N)
    Xo, mo, vo = case.oracle()
    Xg, mg, vg, st = case.gpu()
    assert st.last_status == 0 and st.init_status == 0 and st.steps_applied == case.steps
    em = max(_rel(mg[k], mo[k]) for k in range(case.steps))
    ev = max(_rel(vg[k], vo[k]) for k in range(case.steps))
    ex = _rel(Xg, Xo)
    print(f"[enkf parity] n={n} p={p} N={N}: mean {em:.2e} var {ev:.2e} ensemble {ex:.2e}")
    vtol = max(_var_tol(Xo, vo[k]) for k in range(case.steps))
    assert em < TOL and ex < TOL and ev < vtol
    # elementwise on the ensemble, relative to its scale
    assert np.max(np.abs(Xg - Xo)) < TOL * np.max(np.abs(Xo))


@pytest.mark.parametrize("N,tile_rows", [(100, 32), (400, 32), (100, 64), (256, 64),
                                        (100, 128), (256, 128)])
def test_enkf_tile_forms_match_oracle(N, tile_rows):
    # every transform tile form against the oracle: 32-row tiles (four
    # column quarters per row group), 64-row tiles (two halves; the default
    # above N = 256) and 128-row tiles (every wave on all columns; the
    # default up to N = 256)
    case = EnCase(37, 32, N, steps=2)
    Xo, mo, vo = case.oracle()
    Xg, mg, vg, st = case.gpu(tile_rows=tile_rows)
    assert st.steps_applied == case.steps
    assert _rel(Xg, Xo) < TOL and _rel(mg[-1], mo[-1]) < TOL
    assert _rel(vg[-1], vo[-1]) < _var_tol(Xo, vo[-1])


def test_enkf_without_model_error():
    case = EnCase(37, 32, 48, noise=False)
    Xo, mo, vo = case.oracle()
    Xg, mg, vg, st = case.gpu()
    assert st.steps_applied == case.steps
    assert _rel(Xg, Xo) < TOL and _rel(mg[-1], mo[-1]) < TOL and _rel(vg[-1], vo[-1]) < TOL


def test_enkf_bad_perturbations_leave_the_ensemble_unchanged():
    import torch
    from paper_1404_3816_amd import enkf as EN
    case = EnCase(37, 16, 32, steps=2)
    pr, keep = EN.enkf_problem(case.rowptr, case.col, case.val, case.r, case.m, case.N)
    f = EN.EnkfFilter(pr, torch.as_tensor(case.X0, device="cuda"), keep)
    y = torch.as_tensor(case.ys[0], device="cuda")
    v = torch.as_tensor(case.Vs[0], device="cuda").clone()
    v[3, 5] = float("nan")
    e = torch.zeros(case.m, f.ld, dtype=torch.float64, device="cuda")
    e[:, :case.N] = torch.as_tensor(case.Es[0], device="cuda")
    before = f.export()
    f.step(e, y, v)
    st = f.query()
    assert st.last_status == 1 and st.steps_applied == 0
    assert torch.equal(f.export(), before)
    # a good step afterwards is the oracle's first step
    f.step(e, y, torch.as_tensor(case.Vs[0], device="cuda"))
    st = f.query()
    assert st.last_status == 0 and st.steps_applied == 1
    Xo, _, _ = oracle_enkf.enkf_step(case.X0, case.Es[0], case.H, case.ys[0], case.Vs[0], case.r)
    assert _rel(f.export().cpu().numpy(), Xo) < TOL
    f.close()


def test_enkf_export_import_round_trip():
    import torch
    from paper_1404_3816_amd import enkf as EN
    case = EnCase(37, 16, 24, steps=2)
    pr, keep = EN.enkf_problem(case.rowptr, case.col, case.val, case.r, case.m, case.N)
    f = EN.EnkfFilter(pr, torch.zeros(case.m, case.N, dtype=torch.float64, device="cuda"), keep)
    f.import_(torch.as_tensor(case.X0, device="cuda"))
    assert torch.equal(f.export().cpu(), torch.as_tensor(case.X0))
    e = torch.zeros(case.m, f.ld, dtype=torch.float64, device="cuda")
    e[:, :case.N] = torch.as_tensor(case.Es[0], device="cuda")
    f.step(e, torch.as_tensor(case.ys[0], device="cuda"), torch.as_tensor(case.Vs[0], device="cuda"))
    Xo, _, _ = oracle_enkf.enkf_step(case.X0, case.Es[0], case.H, case.ys[0], case.Vs[0], case.r)
    assert _rel(f.export().cpu().numpy(), Xo) < TOL
    f.close()


def test_enkf_bad_h_poisons_the_filter():
    import torch
    from paper_1404_3816_amd import enkf as EN
    case = EnCase(37, 16, 16, steps=1)
    col = case.col.copy()
    col[7] = case.m + 5                      # a column outside the grid
    pr, keep = EN.enkf_problem(case.rowptr, col, case.val, case.r, case.m, case.N)
    f = EN.EnkfFilter(pr, torch.as_tensor(case.X0, device="cuda"), keep)
    before = f.export()
    f.step(None, torch.as_tensor(case.ys[0], device="cuda"),
           torch.as_tensor(case.Vs[0], device="cuda"))
    st = f.query()
    assert st.init_status == 1 and st.last_status == 1 and st.steps_applied == 0
    assert torch.equal(f.export(), before)
    f.close()


def test_enkf_fullsize_matches_oracle_on_sampled_rows():
    """1024 x 1024 grid, p = 256 crosswell rays, N = 400 members, two steps,
    in the bench's launch configuration (64-row transform tiles).  The
    analysis couples rows only through H X, i.e. through the ray cells, so
    the oracle run on the ray cells plus 256 report rows is exact for those
    rows.  Inputs: white-noise initial ensemble and model-error draws."""
    import scipy.sparse as sp
    import torch
    from paper_1404_3816_amd import enkf as EN
    w = synth.workload("crosswell-1024x1024-p256")
    n, p, m, N, K = w["n"], w["p"], w["m"], 400, 2
    rowptr, col, val = synth.crosswell_h(2, n, p, planes=8)
    r = np.full(p, w["r_var"])
    ys = synth.plume_observations(2, n, rowptr, col, val, K, w["r_var"], w["seed"] + 1)
    X0 = synth.normal_draws(w["seed"] + 101, m, N)
    Es = [synth.normal_draws(w["seed"] + 102 + k, m, N) for k in range(K)]
    Vs = [np.sqrt(w["r_var"]) * synth.normal_draws(w["seed"] + 200 + k, p, N) for k in range(K)]
    report = np.random.default_rng(7).choice(m, 256, replace=False)
    rows = np.union1d(np.unique(col), report)
    pos = np.searchsorted(rows, report)
    Hs = sp.csr_matrix((val, col, rowptr), shape=(p, m))[:, rows].tocsr()
    Xo, mo, vo = oracle_enkf.enkf_run(X0[rows], Hs, r, ys, [E[rows] for E in Es], Vs)

    pr, keep = EN.enkf_problem(rowptr, col, val, r, m, N)
    f = EN.EnkfFilter(pr, torch.as_tensor(X0, device="cuda"), keep)
    assert f.ld == N
    rd = torch.as_tensor(report, device="cuda")
    mg, vg = [], []
    mout = torch.empty(m, dtype=torch.float64, device="cuda")
    vout = torch.empty(m, dtype=torch.float64, device="cuda")
    for k in range(K):
        f.step(torch.as_tensor(Es[k], device="cuda"), torch.as_tensor(ys[k], device="cuda"),
               torch.as_tensor(Vs[k], device="cuda"), mout, vout)
        mg.append(mout[rd].cpu().numpy())
        vg.append(vout[rd].cpu().numpy())
    Xg = f.export()[rd].cpu().numpy()
    st = f.query()
    f.close()
    assert st.last_status == 0 and st.steps_applied == K
    em = max(_rel(mg[k], mo[k][pos]) for k in range(K))
    ev = max(_rel(vg[k], vo[k][pos]) for k in range(K))
    ex = _rel(Xg, Xo[pos])
    print(f"[enkf fullsize] mean {em:.2e} var {ev:.2e} ensemble rows {ex:.2e}")
    assert em < TOL and ex < TOL and ev < _var_tol(Xo[pos], vo[-1][pos])
