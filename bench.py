#!/usr/bin/env python3
"""HiKF hot-path benchmark on one MI355X.

One benchmark step is one whole assimilation job of the chosen workload:
hikf_init (W = H^T, the H^2 / FMM product C_Q = Q H^T, the initial state)
followed by the workload's assimilation steps (gather, p-space Cholesky and
inverse, fused row pass), all through the C ABI on one HIP stream.  Inputs
(H, R, the y stream) are resident in HBM before the timed region starts.

Prints one JSON line: whole-job assimilation steps/s, per-step latency
percentiles, the row-pass kernel against the FP64 MFMA roofline (kernel time
from HIP events the library records on the launch stream), the FMM passes
against their roofs, and the FP64 CPU oracle timed on a bounded sample of the
same workload.
"""

import argparse
import ctypes
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0   # dense BF16 MFMA


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed jobs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed jobs")
    ap.add_argument("--workload", default="crosswell-1024x1024-p256")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "bf16x3", "bf16"])
    ap.add_argument("--n-c", type=int, default=None)
    ap.add_argument("--assim-steps", type=int, default=None,
                    help="assimilation steps per job (default: the workload's)")
    ap.add_argument("--riccati", type=int, default=0,
                    help="gather G = H C_prior only every N steps and carry it between "
                         "(exact p-space recursion); 0 = every step")
    ap.add_argument("--w", default="sparse", choices=["dense", "sparse"],
                    help="FMM source side: dense W = H^T, or the nonzeros of H bucketed by leaf")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the accuracy job against the full-size oracle references")
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches with phase events instead of the step graph")
    ap.add_argument("--m2l-eps", type=float, default=0.0,
                    help="low-rank M2L: relative singular-value threshold of the bases (0: dense)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the row-pass autotuning (use --tune-cache as it is, or the default)")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning cache to read and update (default: a file in the temp dir)")
    ap.add_argument("--phase-jobs", type=int, default=2,
                    help="jobs of the separate phase-timed pass (eager launches, HIP events)")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="approximate seconds of CPU work for the oracle sample")
    ap.add_argument("--serving", action="store_true",
                    help="instead of the job benchmark: a serving mix of filters stepped "
                         "by hikf_step_batch under Poisson request arrivals")
    ap.add_argument("--enkf", action="store_true",
                    help="instead of the HiKF job: the ensemble Kalman filter (Sec. 2.3) on "
                         "the workload's grid and rays")
    ap.add_argument("--members", type=int, default=400, help="EnKF: ensemble size N")
    ap.add_argument("--enkf-tile-rows", type=int, default=0, choices=[0, 32, 64, 128],
                    help="EnKF: rows per workgroup of the transform (0 = automatic)")
    ap.add_argument("--streams", type=int, default=64, help="serving: filters")
    ap.add_argument("--requests", type=int, default=10000, help="serving: requests per run")
    ap.add_argument("--slots", type=int, default=8, help="serving: device streams")
    ap.add_argument("--serving-budget-gb", type=float, default=0.0,
                    help="serving: HBM budget of the filters (default 70%% of free memory)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the jobs, run one plain device copy of this many MiB "
                         "(reference kernel for hardware byte counters)")
    return ap.parse_args()


# the sources whose SHA-256 a traffic record carries, per kernel
KERNEL_SOURCES = {"k_rowpass": ("rowpass.h", "hikf_internal.h"),
                  "k_en_transform": ("enkf_transform.h", "enkf_internal.h", "hikf_internal.h")}


def kernel_source_digest(kernel="k_rowpass"):
    """SHA-256 over the sources of a dominant kernel (the row pass: rowpass.h
    and the shared header; the EnKF transform: its unit and headers)."""
    csrc = os.path.join(ROOT, "paper_1404_3816_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def calibration_copy(mib):
    """One plain device-to-device copy of `mib` MiB: the reference kernel
    whose FETCH_SIZE / WRITE_SIZE readings scale the counters of the others."""
    import torch
    nel = mib * 2**20 // 8
    src = torch.ones(nel, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy of {mib} MiB done")


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when there is no summary for this
    workload or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    digest = kernel_source_digest(kernel)
    for line in open(path):
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
            if rec.get("kernel") == kernel and rec.get("source_sha256") == digest:
                return int(rec["fetch_kib"] * 1024 * rec["fetch_scale"]
                           + rec["write_kib"] * 1024 * rec["write_scale"])
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, assim_steps, budget):
    """The FP64 oracle on a bounded sample of the workload, scaled to the
    whole job: exact C_Q by FFT (oracle tier C) on some of the p right-hand
    sides, and one cross-covariance step (tier B) on a subset of the rows,
    with the workload's own sparse H restricted to those rows."""
    import scipy.sparse as sp
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import cq_exact, kf_crosscov
    import synth

    dim, n, p, m = w["dim"], w["n"], w["p"], w["m"]
    rowptr, col, val = synth.crosswell_h(dim, n, p, planes=8)
    Hfull = sp.csr_matrix((val, col, rowptr), shape=(p, m))
    cells = np.unique(col)

    def fft_cols(cols):
        Ht = np.zeros((m, cols))
        for a in range(cols):
            Ht[col[rowptr[a]:rowptr[a + 1]], a] = val[rowptr[a]:rowptr[a + 1]]
        t0 = time.perf_counter()
        cq_exact.cq_fft(dim, n, Ht, "powexp", w["theta"], w["ell"], w["gamma"])
        return time.perf_counter() - t0

    def tier_b_rows(rows, steps):
        # the first `rows` ray cells: H restricted to them is the workload's
        # own operator on that sample; C_Q := H_s^T keeps S positive definite
        # (the cost of the dense FP64 work does not depend on the values)
        sub = cells[:rows] if rows <= len(cells) else np.arange(rows)
        Hs = Hfull[:, sub].tocsr()
        CQ = np.ascontiguousarray(Hs.T.toarray())
        ys = np.random.default_rng(0).standard_normal((steps, p)) * 1e-2
        t0 = time.perf_counter()
        kf_crosscov.crosscov_kf(CQ, Hs, w["r_var"] * np.eye(p), np.zeros(len(sub)), CQ,
                                np.ones(len(sub)), 1.0, ys)
        return time.perf_counter() - t0

    def measure(budget):
        # exact C_Q = Q H^T by FFT (tier C) on `cols` of the p rays: a
        # one-column probe sizes the sample to about half the budget
        t1 = fft_cols(1)
        cols = int(min(p, max(1, budget / 2 / max(t1, 1e-3))))
        t_fft = fft_cols(cols) if cols > 1 else t1
        t_cq_full = t_fft * p / cols
        # tier-B steps on `rows` of the m rows (cost is linear in the row count)
        probe = min(m, 8192)
        tp = tier_b_rows(probe, 1)
        rows = int(min(m, 262144, max(probe, probe * budget / 2 / max(tp, 1e-3))))
        t_b = tier_b_rows(rows, 1) if rows > probe else tp
        t_step_full = t_b * m / rows
        return t_cq_full, t_step_full, cols, t_fft, rows, t_b

    t_cq, t_step, cols, t_fft, rows, t_b = measure(budget)
    job = t_cq + assim_steps * t_step
    threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    # the same sample on one thread (the paper's timings are single-core)
    with threadpool_limits(limits=1):
        t_cq1, t_step1, _, _, _, _ = measure(budget / 2)
    job1 = t_cq1 + assim_steps * t_step1
    return {
        "value": assim_steps / job, "unit": "assim steps/s", "cores": int(threads),
        "kind": "oracle", "cpu": cpu_model(),
        "sample": (f"exact C_Q by FFT on {cols} of {p} rays ({t_fft:.1f} s, scaled x{p / cols:g}); "
                   f"1 cross-covariance step on {rows} of {m} rows with the workload's sparse H "
                   f"({t_b:.1f} s, scaled x{m / rows:g}); job = C_Q + {assim_steps} steps = "
                   f"{job:.0f} s"),
        "cq_fft_s": round(t_cq, 2), "step_s": round(t_step, 4),
        "single_thread": {"value": assim_steps / job1, "cq_fft_s": round(t_cq1, 2),
                          "step_s": round(t_step1, 4)},
    }


def accuracy_report(workload, K, n_c, x_rows, v_rows, cq_rows, stats):
    """Relative errors of the GPU's x_hat_k, diag P_k and C_Q on the report
    rows against the full-size oracle references (tests/golden): eps_total
    against the filter with the exact C_Q, eps_H2 of the oracle's own FP64
    black-box FMM (the Chebyshev order's error), eps_arith of the GPU against
    that oracle filter; max over the steps (Sec. 4.3 normwise metric)."""
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{workload}.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path, allow_pickle=False)
    if int(ref["steps"]) != K:
        return None

    def mrel(a, b):
        return float(max(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k]) for k in range(len(b))))

    # the bbFMM references hold the workload's own Chebyshev order; at any
    # other order only the error against the exact filter is defined
    same = int(ref["n_c"]) == int(n_c)

    def split(gpu, exact, fmm):
        if not same:
            return {"eps_total": mrel(gpu, exact), "eps_H2": None, "eps_arith": None}
        return {"eps_total": mrel(gpu, exact), "eps_H2": mrel(fmm, exact),
                "eps_arith": mrel(gpu, fmm)}

    def crel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    cq = {"eps_total": crel(cq_rows, ref["cq_exact"]), "eps_H2": None, "eps_arith": None}
    if same:
        cq.update(eps_H2=crel(ref["cq_bbfmm"], ref["cq_exact"]),
                  eps_arith=crel(cq_rows, ref["cq_bbfmm"]))

    return {
        "reference": "oracle cross-covariance filter (FP64) with exact C_Q and with the oracle's "
                     "FP64 bbFMM C_Q, on the ray cells plus report rows",
        "rows": int(len(ref["rows"])), "steps": K,
        "x_hat": split(x_rows, ref["x_exact"], ref["x_bbfmm"]),
        "var": split(v_rows, ref["var_exact"], ref["var_bbfmm"]),
        "n_c": int(n_c), "reference_n_c": int(ref["n_c"]),
        "C_Q": cq,
        "negative_variances": int(stats.negative_variances),
        "min_cholesky_pivot_last_step": float(stats.min_pivot),
    }


def enkf_bench(a):
    """The perturbed-observation EnKF (include/hikf_enkf.h) on the workload's
    grid, rays and R with N members.  Inputs (seeded, white-noise stand-ins
    for the model-error and initial-ensemble draws: the work of a step does
    not depend on their correlation): X_0 and two model-error matrices E of
    standard-normal draws (theta = K(0) = 1), the observation perturbations
    sqrt(R) xi, the plume data.  A job is a fresh filter (H, R and X_0
    copied in on the device) plus `assim_steps` steps, E alternating between
    the two matrices; the timed jobs run without events, a separate pass with
    HIP events around the phases gives the transform's kernel time for the
    roofline (2 m N^2 FP64 flops per launch).  The oracle's EnKF step on the
    ray cells plus 256 report rows, from the same inputs, gives the
    arithmetic error of the first step and the CPU baseline."""
    import scipy.sparse as sp
    import torch
    from threadpoolctl import threadpool_info

    import synth
    from oracle import enkf as oracle_enkf
    from paper_1404_3816_amd import enkf as EN

    w = synth.workload(a.workload)
    dim, n, p, m = w["dim"], w["n"], w["p"], w["m"]
    N = a.members
    K = a.assim_steps or 20
    torch.cuda.set_device(0)
    rowptr, col, val = synth.crosswell_h(dim, n, p, planes=8)
    r = np.full(p, w["r_var"])
    ys = synth.plume_observations(dim, n, rowptr, col, val, K, w["r_var"], w["seed"] + 1)
    t0 = time.perf_counter()
    X0 = synth.normal_draws(w["seed"] + 101, m, N)
    Es = [synth.normal_draws(w["seed"] + 102 + k, m, N) for k in range(2)]
    Vs = [np.sqrt(w["r_var"]) * synth.normal_draws(w["seed"] + 200 + k, p, N) for k in range(K)]
    log(f"[enkf] {a.workload}: m={m} p={p} N={N}, {K} steps per job; inputs drawn in "
        f"{time.perf_counter() - t0:.1f} s")
    pr, keep = EN.enkf_problem(rowptr, col, val, r, m, N, tile_rows=a.enkf_tile_rows)
    ld = int(EN.enkf_plan(pr).ld)
    X0d = torch.as_tensor(X0, device="cuda")
    Ed = []
    for E in Es:
        t = torch.zeros(m, ld, dtype=torch.float64, device="cuda")
        t[:, :N] = torch.as_tensor(E, device="cuda")
        Ed.append(t)
    Vd = [torch.as_tensor(v, device="cuda").contiguous() for v in Vs]
    yd = torch.as_tensor(ys, device="cuda").contiguous()
    mo = torch.empty(m, dtype=torch.float64, device="cuda")
    vo = torch.empty(m, dtype=torch.float64, device="cuda")
    if a.calibrate_copy_mib:
        calibration_copy(a.calibrate_copy_mib)

    def job(timing=False, steps=K):
        prb, kp = EN.enkf_problem(rowptr, col, val, r, m, N, timing=timing,
                                  tile_rows=a.enkf_tile_rows)
        f = EN.EnkfFilter(prb, X0d, kp)
        for k in range(steps):
            f.step(Ed[k % 2], yd[k], Vd[k], mo, vo)
        return f

    for _ in range(a.warmup):
        job().close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status = []
    for _ in range(a.steps):
        f = job()
        status.append(f.query())       # synchronises the job's stream
        f.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    failed = [s.last_status for s in status if s.last_status != 0 or s.steps_applied != K]
    # phase pass: HIP events around the gather, the N-space work and the transform
    f = job(timing=True, steps=min(K, 10))
    st = f.query()
    f.close()
    ph = {name: (st.time_ms[i] / st.time_count[i] if st.time_count[i] else None)
          for i, name in enumerate(("gather", "nspace", "transform"))}
    t_tf = ph["transform"]
    flops = 2.0 * m * N * N
    # first step against the oracle on the ray cells plus report rows
    cells = np.unique(col)
    report = np.random.default_rng(7).choice(m, 256, replace=False)
    rows = np.union1d(cells, report)
    Hs = sp.csr_matrix((val, col, rowptr), shape=(p, m))[:, rows].tocsr()
    t1 = time.perf_counter()
    _, om, ov = oracle_enkf.enkf_step(X0[rows], Es[0][rows], Hs, ys[0], Vs[0], r)
    t_oracle = time.perf_counter() - t1
    f = job(steps=1)
    gm, gv = mo.cpu().numpy(), vo.cpu().numpy()
    f.close()
    pos = np.searchsorted(rows, report)
    rel = lambda g, o: float(np.linalg.norm(g - o) / np.linalg.norm(o))  # noqa: E731
    acc = {"reference": "oracle EnKF step (FP64) on the ray cells plus 256 report rows, "
                        "same inputs", "steps": 1,
           "mean_eps_arith": rel(gm[report], om[pos]), "var_eps_arith": rel(gv[report], ov[pos])}
    threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    t_step_cpu = t_oracle * m / len(rows)
    print(json.dumps({
        "metric": "EnKF assim steps/s (perturbed observations, Sec. 2.3)",
        "value": round(a.steps * K / wall, 3), "unit": "assim steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(wall / a.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"enkf-{a.workload}-N{N}", "m": m, "p": p, "members": N,
                   "ld": ld, "tile_rows": a.enkf_tile_rows or (128 if ld <= 256 else 64),
                   "assim_steps_per_job": K,
                   "inputs": "white-noise X_0 and model-error draws (theta = 1)"},
        "phase_avg_ms": {k: (round(v, 4) if v is not None else None) for k, v in ph.items()},
        "roofline": {"bound": "mfma", "kernel": "k_en_transform (FP64 MFMA)",
                     "achieved": round(flops / (t_tf * 1e-3) / 1e12, 3), "peak": 78.6,
                     "unit": "TFLOP/s", "frac": round(flops / (t_tf * 1e-3) / 78.6e12, 4),
                     "traffic": measured_traffic(f"enkf-{a.workload}-N{N}", "k_en_transform"),
                     "traffic_unit": "bytes/launch", "algorithmic_bytes": int(24 * m * N),
                     "avg_ms": round(t_tf, 4)},
        "accuracy": acc, "failed_jobs": failed,
        "cpu_baseline": {"value": round(1.0 / t_step_cpu, 5), "unit": "assim steps/s",
                         "cores": int(threads), "kind": "oracle", "cpu": cpu_model(),
                         "sample": f"1 EnKF step on {len(rows)} of {m} rows "
                                   f"({t_oracle:.1f} s, scaled x{m / len(rows):.3g})"},
    }), flush=True)


def serving(a):
    """Serving mix (paper_1404_3816_amd/serve.py): `streams` filters of
    different sizes, kernels and ray counts; requests (one assimilation step
    each) arrive as a Poisson process with uniform stream ids.  The server
    dispatches continuously on `slots` device streams and admits filters by
    an HBM budget; the plain path steps one filter at a time on the same
    request sequence.  First closed loops (every request at time zero) give
    each path's saturation rate, then Poisson runs at 0.5x and 0.9x of the
    server's saturation measure the latency of both; a last server run with
    half the memory the filters need exercises eviction and re-admission."""
    import torch

    import synth
    from paper_1404_3816_amd import serve as SV

    torch.cuda.set_device(0)
    cfgs = synth.serving_streams(a.streams, seed=1)
    specs = []
    for i, c in enumerate(cfgs):
        rowptr, col, val = synth.crosswell_h(2, c["n"], c["p"])
        specs.append(SV.StreamSpec(2, c["n"], rowptr, col, val, np.full(c["p"], c["r_var"]),
                                   theta=c["theta"], ell=c["ell"], gamma=c["gamma"],
                                   n_c=c["n_c"], precision=c["precision"], prior=c["prior"],
                                   psd_guard=c["psd_guard"], name=f"s{i}"))
    # measurement streams: seeded draws (the work of a step does not depend
    # on them); every run takes the next requests of each stream's sequence
    per_stream = a.requests * 6 // len(cfgs) + 64
    ys = [torch.as_tensor(synth.normal_draws(c["seed"], per_stream, c["p"]) * 1e-2,
                          device="cuda") for c in cfgs]
    cursor = [0] * len(cfgs)
    sizes = [SV._Stream(sp, sp.plan().resident_bytes, 0).resident_bytes for sp in specs]
    resident = sum(sizes)
    free, total = torch.cuda.mem_get_info()
    budget = int(a.serving_budget_gb * 2**30) if a.serving_budget_gb else int(0.7 * free)
    log(f"[serving] {len(specs)} streams ({sum(c['gamma'] == 2.0 for c in cfgs)} Gaussian), "
        f"resident regions {resident / 2**30:.1f} GiB, budget {budget / 2**30:.1f} GiB")

    def requests(rate, seed, cursor):
        arr, sid = synth.poisson_requests(a.requests, len(cfgs), rate, seed)
        out = []
        for i in range(a.requests):
            s = int(sid[i])
            out.append(SV.Request(i, s, float(arr[i]), ys[s][cursor[s] % per_stream]))
            cursor[s] += 1
        return out

    def served(server, rate, seed):
        rq = requests(rate, seed, cursor)
        t0 = time.perf_counter()
        server.run(rq)
        return SV.latency_summary(rq, time.perf_counter() - t0)

    server = SV.Server(specs, budget, slots=a.slots)
    t0 = time.perf_counter()
    server.run(requests(None, 98, cursor))                       # admission + warm-up
    log(f"[serving] warm-up (admits every stream) {time.perf_counter() - t0:.1f} s")
    runs = {"server": {}, "sequential": {}}
    runs["server"]["saturation"] = served(server, None, 2)
    sat = runs["server"]["saturation"]["achieved_per_s"]
    log(f"[serving] server closed loop: {runs['server']['saturation']}")
    for frac, sd in ((0.5, 3), (0.9, 4)):
        runs["server"][f"poisson_{frac}x"] = served(server, frac * sat, sd)
        log(f"[serving] server at {frac} x saturation: {runs['server'][f'poisson_{frac}x']}")
    stats = server.query()
    failed = [i for i, st in enumerate(stats) if st is not None and st.last_status != 0]
    server_states = server.final_states()
    server_counts = [st.steps_done for st in server.streams]
    server.close()
    del server
    torch.cuda.synchronize()

    # the plain path: one filter at a time, the same request sequences
    cursor2 = [0] * len(cfgs)
    filters = SV.run_sequential(specs, requests(None, 98, cursor2))
    for name, rate, sd in (("saturation", None, 2), ("poisson_0.5x", 0.5 * sat, 3),
                           ("poisson_0.9x", 0.9 * sat, 4)):
        rq = requests(rate, sd, cursor2)
        t0 = time.perf_counter()
        filters = SV.run_sequential(specs, rq, filters=filters)
        runs["sequential"][name] = SV.latency_summary(rq, time.perf_counter() - t0)
        log(f"[serving] sequential {name}: {runs['sequential'][name]}")
    # each stream's state after the same requests, in the mix and alone
    same = 0
    for k, f in enumerate(filters):
        if f is None or server_states[k] is None:
            continue
        x, v, _ = f.export_state()
        same += int(torch.equal(x.cpu(), server_states[k][0]) and
                    torch.equal(v.cpu(), server_states[k][1]))
    active = sum(1 for k, f in enumerate(filters) if f is not None and server_states[k] is not None)
    for f in filters:
        if f is not None:
            f.close()
    torch.cuda.synchronize()

    # a budget of half the resident regions, Poisson arrivals at 0.5x the
    # full-memory saturation: streams that go idle are evicted when others
    # need the memory, and re-admitted (from their checkpoints) when their
    # next request arrives
    small = SV.Server(specs, max(resident // 2, max(sizes)), slots=a.slots)
    cursor3 = [0] * len(cfgs)
    t0 = time.perf_counter()
    rq = requests(0.5 * sat, 5, cursor3)[:max(1, a.requests // 5)]
    small.run(rq)
    evict_run = SV.latency_summary(rq, time.perf_counter() - t0)
    evict_run.update({k: int(v) for k, v in small.stats.items()})
    evict_run["offered_per_s"] = round(0.5 * sat, 1)
    small.close()
    log(f"[serving] half-memory, Poisson at 0.5 x saturation: {evict_run}")
    mean_flops = float(np.mean([2.0 * c["m"] * c["p"] ** 2 for c in cfgs]))
    print(json.dumps({
        "metric": "serving requests/s (assimilation steps over a mixed set of filters)",
        "value": runs["server"]["saturation"]["achieved_per_s"], "unit": "requests/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving-{len(cfgs)}-streams", "requests_per_run": a.requests,
                   "slots": a.slots, "budget_gib": round(budget / 2**30, 1),
                   "resident_gib": round(resident / 2**30, 2),
                   "streams": [{k: c[k] for k in ("n", "p", "gamma", "ell", "n_c", "precision",
                                                  "psd_guard")} for c in cfgs],
                   "mean_row_pass_flops": mean_flops},
        "runs": runs, "half_memory_run": evict_run,
        "mix_equals_solo": {"streams_compared": active, "bitwise_equal": same},
        "failed_streams": failed, "steps_per_stream": server_counts,
    }), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the hot path here is built and timed on a "
              "single MI355X; the multi-GPU sharding is a design note, not code.",
              file=sys.stderr)
        sys.exit(2)
    if a.serving:
        serving(a)
        return
    if a.enkf:
        enkf_bench(a)
        return
    import torch

    import synth
    from paper_1404_3816_amd import filter as F
    from paper_1404_3816_amd import hikf as H

    w = synth.workload(a.workload)
    dim, n, p, m = w["dim"], w["n"], w["p"], w["m"]
    n_c = a.n_c or w["n_c"]
    K = a.assim_steps or w["steps"]
    log(f"[bench] workload {a.workload}: m={m} p={p} n_c={n_c} precision={a.precision} "
        f"assim steps/job={K}")
    rowptr, col, val = synth.crosswell_h(dim, n, p, planes=8)
    ys = synth.plume_observations(dim, n, rowptr, col, val, K, w["r_var"], w["seed"] + 1)
    torch.cuda.set_device(0)
    pr, keep = F.problem_from_csr(dim, n, rowptr, col, val, np.full(p, w["r_var"]),
                                  theta=w["theta"], ell=w["ell"], gamma=w["gamma"],
                                  prior=w["prior"])
    # the timed jobs replay each step as the HIP graph captured at init (no
    # per-phase events); a separate pass with eager launches and HIP events
    # around every phase gives the kernel times and the roofline
    graph = not a.eager
    ydev = torch.as_tensor(ys, dtype=torch.float64, device="cuda").contiguous()
    # autotuning: every launch form of the row pass is timed on this problem
    # and the winner recorded in a tuning cache, which hikf_init then reads
    tuned = None
    cache = a.tune_cache or os.path.join(tempfile.gettempdir(), "hikf_tune_cache.json")
    if not a.no_tune:
        from paper_1404_3816_amd import tune as T
        best, ms = T.tune_problem(pr, keep, dict(n_c=n_c, precision=a.precision,
                                                 sparse=a.w == "sparse", riccati=a.riccati,
                                                 m2l_eps=a.m2l_eps),
                                  ydev, steps=6, repeats=2)
        T.merge_entry(cache, {"p": p, "cq": "f64" if a.precision == "f64" else "f32", "m": m,
                              "variant": int(best),
                              "ms": [round(ms[v], 4) if v in ms else None for v in T.VARIANTS],
                              "workload": a.workload})
        tuned = {"rowpass_candidates_ms": {str(v): round(t, 4) for v, t in ms.items()},
                 "cache": cache}
        log(f"[bench] row-pass launch forms (ms): {tuned['rowpass_candidates_ms']}, best {best}")
    tc = cache if os.path.exists(cache) else None
    op_run = F.make_options(n_c, a.precision, False, timing=not graph, graph=graph,
                            riccati=a.riccati, sparse=a.w == "sparse", tune_cache=tc,
                            m2l_eps=a.m2l_eps)
    op_phase = F.make_options(n_c, a.precision, False, timing=True, graph=False,
                              riccati=a.riccati, sparse=a.w == "sparse", tune_cache=tc,
                              m2l_eps=a.m2l_eps)
    info = F.plan(pr, op_run)
    resident = torch.empty(int(info.resident_bytes), dtype=torch.uint8, device="cuda")
    scratch = torch.empty(int(info.scratch_bytes), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sh = ctypes.c_void_p(stream.cuda_stream)
    if a.calibrate_copy_mib:
        calibration_copy(a.calibrate_copy_mib)
    log(f"[bench] resident {info.resident_bytes / 2**30:.2f} GiB, scratch "
        f"{info.scratch_bytes / 2**30:.2f} GiB, depth {info.depth}, near pairs "
        f"{info.near_pairs}, far pairs {info.far_pairs}")

    def job(op, latencies=None, probe=None, steps=K):
        handle = ctypes.c_void_p()
        H.check(H.hikf_init(ctypes.byref(pr), ctypes.byref(op),
                            ctypes.c_void_p(resident.data_ptr()), info.resident_bytes,
                            ctypes.c_void_p(scratch.data_ptr()), info.scratch_bytes, sh,
                            ctypes.byref(handle)), "hikf_init")
        if probe is not None:
            H.check(H.hikf_export_cq(handle, ctypes.c_void_p(probe["cq"].data_ptr()), sh),
                    "hikf_export_cq", handle)
            probe["cq_rows"] = probe["cq"][probe["rows"]].clone()
        for k in range(steps):
            if latencies is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            xo = ctypes.c_void_p(probe["x"].data_ptr()) if probe is not None else None
            vo = ctypes.c_void_p(probe["v"].data_ptr()) if probe is not None else None
            H.check(H.hikf_step(handle, ctypes.c_void_p(ydev[k].data_ptr()), xo, vo, sh),
                    "hikf_step", handle)
            if latencies is not None:
                e1.record(stream)
                latencies.append((e0, e1))
            if probe is not None:
                probe["xs"][k] = probe["x"][probe["rows"]]
                probe["vs"][k] = probe["v"][probe["rows"]]
        return handle

    def finish(handle):
        st = H.hikf_stats()
        H.check(H.hikf_query(handle, ctypes.byref(st)), "hikf_query", handle)
        H.hikf_destroy(handle)
        return st

    for i in range(a.warmup):
        st = finish(job(op_run))
        log(f"[bench] warmup job {i + 1}/{a.warmup} done (status {st.last_status}, "
            f"steps {st.steps_applied})")
    torch.cuda.synchronize()
    lat = []
    handles = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        handles.append(job(op_run, lat))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = [finish(h) for h in handles]
    last = stats[-1]
    if last.last_status != 0 or last.steps_applied != K:
        raise SystemExit(f"bench: filter reported status {last.last_status} after "
                         f"{last.steps_applied} of {K} steps")
    log(f"[bench] timed {a.steps} jobs in {t1 - t0:.3f} s ({'graph' if graph else 'eager'} steps, "
        f"row-pass variant {last.rowpass_variant})")
    lat_ms = np.array([e0.elapsed_time(e1) for e0, e1 in lat])

    # cold start: init (FMM, operators, graph capture) plus the first step of
    # a new filter, host clock, best of three jobs after the timed region
    cold = []
    for _ in range(3):
        torch.cuda.synchronize()
        tc0 = time.perf_counter()
        hc = job(op_run, steps=1)
        torch.cuda.synchronize()
        cold.append((time.perf_counter() - tc0) * 1e3)
        finish(hc)

    # phase pass: eager launches with HIP events on the launch stream
    pstats = [finish(job(op_phase)) for _ in range(a.phase_jobs)]
    torch.cuda.synchronize()
    log(f"[bench] phase-timed pass: {a.phase_jobs} jobs")
    tot = np.zeros(H.HIKF_NUM_PHASES)
    cnt = np.zeros(H.HIKF_NUM_PHASES)
    for s_ in pstats:
        tot += np.array(s_.time_ms[:])
        cnt += np.array(s_.time_count[:])
    avg = {name: (tot[i] / cnt[i] if cnt[i] else None) for i, name in enumerate(H.PHASES)}

    # roofline of the dominant kernel: the fused row pass, 2 m p^2 FP64 flops
    row_s = avg["rowpass"] / 1e3
    row_tflops = 2.0 * m * p * p / row_s / 1e12
    tqb = 8 if a.precision == "f64" else 4
    roof = {"bound": "mfma", "achieved": round(row_tflops, 3), "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(row_tflops / PEAK_FP64_TFLOPS, 4),
            "traffic": measured_traffic(a.workload, "k_rowpass"), "traffic_unit": "bytes/launch",
            "algorithmic_bytes": (8 + tqb + 8) * m * p, "kernel": "k_rowpass (FP64 MFMA)",
            "avg_ms": round(avg["rowpass"], 4), "launches": int(cnt[H.PHASES.index("rowpass")]),
            "timed_in": "phase pass (eager launches, HIP events on the launch stream)"}
    tq = tqb
    # M2L and P2P run on FP64 / FP32 MFMA, or on BF16 MFMA (three products per
    # FP32 product with the refinement terms): frac is issued work over peak
    issue = {"f64": 1, "f32": 1, "bf16x3": 3, "bf16": 1}[a.precision]
    peak_f = {"f64": PEAK_FP64_TFLOPS, "f32": PEAK_FP32_TFLOPS}.get(a.precision, PEAK_BF16_TFLOPS)
    leaves = m // 64
    fmm = {}
    nnz = len(col)
    if avg["p2p"] and a.w == "sparse":
        # one kernel evaluation and FMA per (target, nonzero of a neighbour
        # leaf) pair; HBM: read the bucketed nonzeros and L_leaf, write C_Q
        by = (nnz * (4 + tq) + leaves * info.r * p * tq + m * p * tq)
        fmm["p2p_l2p"] = {"ms": round(avg["p2p"], 4), "w": "sparse",
                          "GBps": round(by / avg["p2p"] / 1e6, 1),
                          "frac_hbm": round(by / avg["p2p"] / 1e6 / PEAK_HBM_GBS, 4)}
    elif avg["p2p"]:
        fl = 2.0 * info.near_pairs * 64 * 64 * p
        by = 2.0 * m * p * tq
        fmm["p2p_l2p"] = {"ms": round(avg["p2p"], 4),
                          "tflops": round(fl / avg["p2p"] / 1e9, 3),
                          "frac_fp_peak": round(issue * fl / avg["p2p"] / 1e9 / peak_f, 4),
                          "GBps": round(by / avg["p2p"] / 1e6, 1)}
    if avg["m2l"]:
        fl = 2.0 * info.far_pairs * info.r * info.r * p
        fmm["m2l"] = {"ms": round(avg["m2l"], 4), "tflops": round(fl / avg["m2l"] / 1e9, 3),
                      "frac_fp_peak": round(issue * fl / avg["m2l"] / 1e9 / peak_f, 4)}
    if avg["p2m"]:
        by = ((nnz * (4 + tq) if a.w == "sparse" else m * p * tq) + leaves * info.r * p * tq)
        fmm["p2m"] = {"ms": round(avg["p2m"], 4), "GBps": round(by / avg["p2m"] / 1e6, 1),
                      "frac_hbm": round(by / avg["p2m"] / 1e6 / PEAK_HBM_GBS, 4)}
    init_ms = sum(avg[k] or 0.0 for k in ("operators", "p2m", "m2m", "m2l", "l2l", "p2p", "init"))

    # accuracy: one more job in the timed configuration, x_hat / diag P on the
    # report rows of the full-size oracle references after every step
    acc = None
    if not a.no_accuracy:
        path = os.path.join(ROOT, "tests", "golden", f"fullsize_{a.workload}.npz")
        if os.path.exists(path):
            rows = np.load(path, allow_pickle=False)["rows"]
            rd = torch.as_tensor(rows, device="cuda")
            probe = {"rows": rd, "cq": torch.empty(m, p, dtype=torch.float64, device="cuda"),
                     "x": torch.empty(m, dtype=torch.float64, device="cuda"),
                     "v": torch.empty(m, dtype=torch.float64, device="cuda"),
                     "xs": torch.empty(K, len(rows), dtype=torch.float64, device="cuda"),
                     "vs": torch.empty(K, len(rows), dtype=torch.float64, device="cuda")}
            ast = finish(job(op_run, probe=probe))
            acc = accuracy_report(a.workload, K, n_c, probe["xs"].cpu().numpy(),
                                  probe["vs"].cpu().numpy(), probe["cq_rows"].cpu().numpy(), ast)
            del probe
            log(f"[bench] accuracy: {json.dumps(acc)}")

    wall = t1 - t0
    result = {
        "metric": "assim steps/s at m=1M,p=256; Q·H^T MFMA/HBM % of peak; p50/p99 step latency",
        "value": round(a.steps * K / wall, 3),
        "unit": "assim steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": a.workload, "m": m, "p": p, "dim": dim, "n_c": n_c,
                   "kernel": f"theta*exp(-(r/{w['ell']})^{w['gamma']:g})",
                   "fmm_dtype": a.precision, "step_dtype": "f64",
                   "assim_steps_per_job": K, "gather_every": a.riccati or 1, "fmm_w": a.w,
                   "m2l": (f"low-rank, threshold {a.m2l_eps:g}, ranks per level "
                           f"{[k for k in last.m2l_ranks if k]}" if a.m2l_eps > 0 else "dense"),
                   "step_launch": "hip graph per step" if graph else "eager, phase events",
                   "rowpass_variant": int(last.rowpass_variant),
                   "rowpass_form": ("persistent" if last.rowpass_variant & 1 else "one tile per "
                                    "workgroup") + (", 32-row tiles x 4 column parts"
                                                    if (last.rowpass_variant & 2 or p > 256)
                                                    else ", 64-row tiles x 2 column halves"),
                   "parallelism": "none (1 GPU)"},
        "warm_steps_per_s": round(1e3 / float(np.mean(lat_ms)), 2),
        "cold_ms": {"init_plus_first_step": round(min(cold), 3),
                    "timed_in": "host clock around hikf_init and one hikf_step (best of 3 jobs)"},
        "step_latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                            "p99": round(float(np.percentile(lat_ms, 99)), 4),
                            "mean": round(float(np.mean(lat_ms)), 4),
                            "timed_in": "timed jobs (host-stream events around each hikf_step)"},
        "init_ms_kernels": round(init_ms, 3),
        "phase_avg_ms": {k: (round(v, 4) if v is not None else None) for k, v in avg.items()},
        "phase_timed_in": "phase pass (eager launches, HIP events on the launch stream)",
        "roofline": roof,
        "fmm_roofline": fmm,
        "accuracy": acc,
        "autotune": tuned,
    }
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline(w, K, a.cpu_budget)
        log("[bench] CPU oracle done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
