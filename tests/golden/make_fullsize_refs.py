"""Write the full-size oracle references used by tests/test_gpu_fullsize.py
and by the accuracy report of bench.py.

Runs only the oracle (``oracle/``) on the seeded inputs (``synth``); nothing
here touches the GPU path.  For each benchmark workload (the 256 x 256 / p 64
and 1024 x 1024 / p 256 grids, the 128^3 / p 512 octree) it

* takes the rows the rays cross plus seeded samples: the cross-covariance
  filter (Algorithm Algorithm_HiKF) is exact on any row set that holds every
  cell a ray crosses, because rows are independent given G = H C_prior;
* forms C_Q = Q H^T on those rows twice: exactly (FFT circulant embedding in
  2-D, direct sums over the nonzeros of H in 3-D) and by the FP64 black-box
  FMM with the workload's n_c (Sec. 3.2);
* runs the filter over all of the workload's steps with each C_Q and keeps
  x_hat_k and diag P_k on the report rows;
* measures the filter's sensitivity to a C_Q error at the FMM C_Q (the
  largest relative output change per unit normwise relative change of C_Q
  over two random directions of size 1e-6);
* stores everything in tests/golden/fullsize_<workload>.npz (no pickles).

Usage: python tests/golden/make_fullsize_refs.py [workload ...]
(about 1, 6 and 15 minutes on 8 cores for the three workloads).
"""

import os
import sys
import time

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import bbfmm, cq_exact, kernels, kf_crosscov  # noqa: E402

WORKLOADS = ("crosswell-256x256-p64", "crosswell-1024x1024-p256", "crosswell-128cube-p512")
REPORT_SEED = 7          # seeded report rows: half anywhere, half on ray cells
REPORT_ROWS = 256


def report_rows(m, col):
    """Sorted report rows: REPORT_ROWS / 2 seeded rows of the grid and as many
    seeded rows among the cells the rays cross (where x_hat moves most)."""
    rng = np.random.default_rng(REPORT_SEED)
    cells = np.unique(col)
    a = rng.choice(m, REPORT_ROWS // 2, replace=False)
    b = rng.choice(cells, REPORT_ROWS // 2, replace=False)
    return np.unique(np.concatenate([a, b]))


def inputs(name):
    """The workload's H (CSR arrays) and its y stream, as bench.py builds them."""
    w = synth.workload(name)
    rowptr, col, val = synth.crosswell_h(w["dim"], w["n"], w["p"], planes=8)
    ys = synth.plume_observations(w["dim"], w["n"], rowptr, col, val, w["steps"], w["r_var"],
                                  w["seed"] + 1)
    return w, rowptr, col, val, ys


def _dense_cols(rowptr, col, val, m, c0, c1):
    W = np.zeros((m, c1 - c0))
    for a in range(c0, c1):
        W[col[rowptr[a]:rowptr[a + 1]], a - c0] = val[rowptr[a]:rowptr[a + 1]]
    return W


def cq_on_rows(w, rowptr, col, val, sub, route, chunk):
    """C_Q[sub, :] by the exact route or by the oracle's FP64 bbFMM, computed
    a block of right-hand sides at a time (only the sub rows are kept)."""
    dim, n, p, m = w["dim"], w["n"], w["p"], w["m"]
    kp = ("powexp", w["theta"], w["ell"], w["gamma"])
    if route == "exact" and dim == 3:
        return cq_exact.cq_rows(dim, n, rowptr, col, val, sub, *kp, chunk=16)
    out = np.empty((len(sub), p))
    for c0 in range(0, p, chunk):
        c1 = min(p, c0 + chunk)
        W = _dense_cols(rowptr, col, val, m, c0, c1)
        if route == "exact":
            full = cq_exact.cq_fft(dim, n, W, *kp)
        else:
            full = bbfmm.bbfmm_apply(dim, n, W, w["n_c"], None, *kp)
        out[:, c0:c1] = full[sub]
        del W, full
    return out


def run_filter(w, H, CQ, ys):
    ns = CQ.shape[0]
    theta = kernels.diag_value("powexp", w["theta"], w["ell"], w["gamma"])
    return kf_crosscov.crosscov_kf(CQ, H, w["r_var"] * np.eye(w["p"]), np.zeros(ns), CQ,
                                   np.full(ns, theta), theta, ys)


def make(name):
    t0 = time.time()
    w, rowptr, col, val, ys = inputs(name)
    m, p = w["m"], w["p"]
    rows = report_rows(m, col)
    sub = np.union1d(np.unique(col), rows)
    pos = np.searchsorted(sub, rows)
    H = sp.csr_matrix((val, col, rowptr), shape=(p, m))[:, sub].tocsr()
    chunk = 64 if w["dim"] == 2 else 32
    cq_ex = cq_on_rows(w, rowptr, col, val, sub, "exact", chunk)
    print(f"[{name}] exact C_Q on {len(sub)} rows: {time.time() - t0:.0f} s", flush=True)
    cq_fmm = cq_on_rows(w, rowptr, col, val, sub, "bbfmm", chunk)
    print(f"[{name}] bbFMM C_Q: {time.time() - t0:.0f} s", flush=True)
    x_ex, v_ex = run_filter(w, H, cq_ex, ys)
    x_fmm, v_fmm = run_filter(w, H, cq_fmm, ys)
    print(f"[{name}] filters: {time.time() - t0:.0f} s", flush=True)
    # sensitivity of the outputs (on the sub rows) to a C_Q error at the FMM C_Q
    eps = 1e-6
    kx = kv = 0.0
    rng = np.random.default_rng(0)
    for t in range(2):
        E = rng.standard_normal(cq_fmm.shape)
        E *= np.abs(cq_fmm) if t == 0 else np.abs(cq_fmm).max()
        E *= eps * np.linalg.norm(cq_fmm) / np.linalg.norm(E)
        xp, vp = run_filter(w, H, cq_fmm + E, ys)
        kx = max(kx, max(np.linalg.norm(xp[k] - x_fmm[k]) / np.linalg.norm(x_fmm[k])
                         for k in range(len(ys))) / eps)
        kv = max(kv, max(np.linalg.norm(vp[k] - v_fmm[k]) / np.linalg.norm(v_fmm[k])
                         for k in range(len(ys))) / eps)
    print(f"[{name}] sensitivity x {kx:.2f} var {kv:.2f}: {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, f"fullsize_{name}.npz")
    np.savez_compressed(
        out, rows=rows, cq_exact=cq_ex[pos], cq_bbfmm=cq_fmm[pos],
        x_exact=x_ex[:, pos], var_exact=v_ex[:, pos], x_bbfmm=x_fmm[:, pos],
        var_bbfmm=v_fmm[:, pos], kappa=np.array([kx, kv]),
        # errors of the FMM filter over all rows it ran on (report rows are a sample)
        h2_sub=np.array([
            max(np.linalg.norm(x_fmm[k] - x_ex[k]) / np.linalg.norm(x_ex[k]) for k in range(len(ys))),
            max(np.linalg.norm(v_fmm[k] - v_ex[k]) / np.linalg.norm(v_ex[k]) for k in range(len(ys))),
            np.linalg.norm(cq_fmm - cq_ex) / np.linalg.norm(cq_ex)]),
        n_c=np.array(w["n_c"]), steps=np.array(len(ys)))
    print(f"[{name}] wrote {out} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or WORKLOADS:
        make(name)
