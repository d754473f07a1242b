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
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="approximate seconds of CPU work for the oracle sample")
    ap.add_argument("--serving", action="store_true",
                    help="instead of the job benchmark: a serving mix of filters stepped "
                         "by hikf_step_batch under Poisson request arrivals")
    ap.add_argument("--streams", type=int, default=16, help="serving: filters")
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests per run")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the jobs, run one plain device copy of this many MiB "
                         "(reference kernel for hardware byte counters)")
    return ap.parse_args()


def kernel_source_digest():
    """SHA-256 over the source of the row-pass kernel (rowpass.h) and the
    shared header."""
    csrc = os.path.join(ROOT, "paper_1404_3816_amd", "csrc")
    h = hashlib.sha256()
    for name in ("rowpass.h", "hikf_internal.h"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when there is no summary for this
    workload or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    digest = kernel_source_digest()
    for line in open(path):
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
            if rec.get("kernel") == kernel and rec.get("source_sha256") == digest:
                return int(rec["fetch_kib"] * 1024 * rec["fetch_scale"]
                           + rec["write_kib"] * 1024 * rec["write_scale"])
    return None


def cpu_baseline(w, assim_steps, budget):
    """The FP64 oracle on a bounded sample of the workload, scaled to the
    whole job: exact C_Q by FFT (oracle tier C) on a few right-hand sides and
    cross-covariance steps (tier B) on a subset of rows."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import cq_exact, kf_crosscov
    import synth

    dim, n, p, m = w["dim"], w["n"], w["p"], w["m"]
    rowptr, col, val = synth.crosswell_h(dim, n, p, planes=8)
    def fft_cols(cols):
        Ht = np.zeros((m, cols))
        for a in range(cols):
            Ht[col[rowptr[a]:rowptr[a + 1]], a] = val[rowptr[a]:rowptr[a + 1]]
        t0 = time.perf_counter()
        cq_exact.cq_fft(dim, n, Ht, "powexp", w["theta"], w["ell"], w["gamma"])
        return time.perf_counter() - t0

    def tier_b_rows(rows, steps):
        rng = np.random.default_rng(0)
        Hs = np.zeros((p, rows))
        for a in range(p):
            Hs[a, rng.choice(rows, 8, replace=False)] = 1.0 / n
        # Q = I on the sample keeps H C_Q positive semidefinite; the cost of
        # the dense FP64 work does not depend on the values
        CQ = np.ascontiguousarray(Hs.T)
        ys = rng.standard_normal((steps, p)) * 1e-2
        t0 = time.perf_counter()
        kf_crosscov.crosscov_kf(CQ, Hs, w["r_var"] * np.eye(p), np.zeros(rows), CQ,
                                np.ones(rows), 1.0, ys)
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
        "kind": "oracle",
        "sample": (f"exact C_Q by FFT on {cols} of {p} rays ({t_fft:.1f} s, scaled x{p / cols:g}); "
                   f"1 cross-covariance step on {rows} of {m} rows ({t_b:.1f} s, scaled "
                   f"x{m / rows:g}); job = C_Q + {assim_steps} steps = {job:.0f} s"),
        "cq_fft_s": round(t_cq, 2), "step_s": round(t_step, 4),
        "single_thread": {"value": assim_steps / job1, "cq_fft_s": round(t_cq1, 2),
                          "step_s": round(t_step1, 4)},
    }


def serving(a):
    """Serving mix: `streams` filters of different sizes, requests arriving as a
    Poisson process with uniform stream ids.  The dispatcher takes, per round,
    the oldest pending request of every stream that has one (per-stream order
    is kept), steps them with one hikf_step_batch call on one stream, and
    waits for it; a request's latency runs from its arrival to the end of its
    round.  First a closed loop (all requests at time zero) gives the
    saturation rate, then Poisson runs at 0.5x, 0.9x and 1.2x of it (the last
    one overloaded: its queue, and so its latency, grows over the run)."""
    import collections

    import torch

    import synth
    from paper_1404_3816_amd import filter as F

    torch.cuda.set_device(0)
    cfgs = synth.serving_streams(a.streams, seed=1)
    filters, ys, xo, vo = [], [], [], []
    t0 = time.perf_counter()
    for c in cfgs:
        rowptr, col, val = synth.crosswell_h(2, c["n"], c["p"])
        pr, keep = F.problem_from_csr(2, c["n"], rowptr, col, val, np.full(c["p"], c["r_var"]),
                                      theta=c["theta"], ell=c["ell"], gamma=c["gamma"],
                                      prior=c["prior"])
        filters.append(F.HikfFilter(pr, F.make_options(c["n_c"], "f32", False, graph=True), keep))
        # measurement values do not change the work of a step
        ys.append(torch.as_tensor(synth.normal_draws(c["seed"], a.requests, c["p"]) * 1e-2,
                                  device="cuda"))
        xo.append(torch.empty(c["m"], dtype=torch.float64, device="cuda"))
        vo.append(torch.empty(c["m"], dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    log(f"[serving] {len(filters)} filters built in {time.perf_counter() - t0:.1f} s")
    step_of = [0] * len(filters)

    def run(rate, seed):
        arr, sid = synth.poisson_requests(a.requests, len(filters), rate, seed)
        queues = [collections.deque() for _ in filters]
        lat, done, i = [], 0, 0
        t_start = time.perf_counter()
        while done < a.requests:
            now = time.perf_counter() - t_start
            while i < a.requests and arr[i] <= now:
                queues[sid[i]].append(arr[i])
                i += 1
            batch = [s for s in range(len(filters)) if queues[s]]
            if not batch:
                time.sleep(max(0.0, min(1e-3, arr[i] - now)))
                continue
            yb = []
            for s in batch:
                yb.append(ys[s][step_of[s] % a.requests])
                step_of[s] += 1
            F.step_batch([filters[s] for s in batch], yb, [xo[s] for s in batch],
                         [vo[s] for s in batch])
            torch.cuda.synchronize()
            t_done = time.perf_counter() - t_start
            for s in batch:
                lat.append(t_done - queues[s].popleft())
            done += len(batch)
        wall = time.perf_counter() - t_start
        lat = np.array(lat) * 1e3
        return {"offered_per_s": rate, "achieved_per_s": round(a.requests / wall, 1),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3)}

    run(None, 99)                                       # warm-up
    sat = run(None, 2)
    log(f"[serving] closed loop: {sat}")
    runs = [sat]
    for frac, sd in ((0.5, 3), (0.9, 4), (1.2, 5)):
        r = run(frac * sat["achieved_per_s"], sd)
        log(f"[serving] {frac} x saturation: {r}")
        runs.append(r)
    stats = [f.query() for f in filters]
    failed = [{"stream": i, "status": st.last_status, "steps": st.steps_applied,
               "min_pivot": st.min_pivot, "n": cfgs[i]["n"], "p": cfgs[i]["p"]}
              for i, st in enumerate(stats) if st.last_status != 0]
    if failed:
        log(f"[serving] filters whose last step failed: {failed}")
    for f in filters:
        f.close()
    mean_flops = float(np.mean([2.0 * c["m"] * c["p"] ** 2 for c in cfgs]))
    print(json.dumps({
        "metric": "serving requests/s (assimilation steps over a mixed set of filters)",
        "value": sat["achieved_per_s"], "unit": "requests/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving-{len(filters)}-streams", "requests": a.requests,
                   "streams": [{k: c[k] for k in ("n", "p", "gamma", "ell", "n_c")} for c in cfgs],
                   "mean_row_pass_flops": mean_flops},
        "runs": runs, "failed_filters": failed,
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
    op = F.make_options(n_c, a.precision, False, timing=True, riccati=a.riccati,
                        sparse=a.w == "sparse")
    info = F.plan(pr, op)
    resident = torch.empty(int(info.resident_bytes), dtype=torch.uint8, device="cuda")
    scratch = torch.empty(int(info.scratch_bytes), dtype=torch.uint8, device="cuda")
    ydev = torch.as_tensor(ys, dtype=torch.float64, device="cuda").contiguous()
    stream = torch.cuda.current_stream()
    sh = ctypes.c_void_p(stream.cuda_stream)
    if a.calibrate_copy_mib:
        nel = a.calibrate_copy_mib * 2**20 // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {a.calibrate_copy_mib} MiB done")
        del src, dst
    log(f"[bench] resident {info.resident_bytes / 2**30:.2f} GiB, scratch "
        f"{info.scratch_bytes / 2**30:.2f} GiB, depth {info.depth}, near pairs "
        f"{info.near_pairs}, far pairs {info.far_pairs}")

    def job(latencies):
        handle = ctypes.c_void_p()
        H.check(H.hikf_init(ctypes.byref(pr), ctypes.byref(op),
                            ctypes.c_void_p(resident.data_ptr()), info.resident_bytes,
                            ctypes.c_void_p(scratch.data_ptr()), info.scratch_bytes, sh,
                            ctypes.byref(handle)), "hikf_init")
        for k in range(K):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            H.check(H.hikf_step(handle, ctypes.c_void_p(ydev[k].data_ptr()), None, None, sh),
                    "hikf_step", handle)
            e1.record(stream)
            latencies.append((e0, e1))
        return handle

    def finish(handle):
        st = H.hikf_stats()
        H.check(H.hikf_query(handle, ctypes.byref(st)), "hikf_query", handle)
        H.hikf_destroy(handle)
        return st

    for i in range(a.warmup):
        st = finish(job([]))
        log(f"[bench] warmup job {i + 1}/{a.warmup} done (status {st.last_status}, "
            f"steps {st.steps_applied})")
    torch.cuda.synchronize()
    lat = []
    handles = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        handles.append(job(lat))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = [finish(h) for h in handles]
    last = stats[-1]
    if last.last_status != 0 or last.steps_applied != K:
        raise SystemExit(f"bench: filter reported status {last.last_status} after "
                         f"{last.steps_applied} of {K} steps")
    log(f"[bench] timed {a.steps} jobs in {t1 - t0:.3f} s")
    lat_ms = np.array([e0.elapsed_time(e1) for e0, e1 in lat])
    tot = np.zeros(H.HIKF_NUM_PHASES)
    cnt = np.zeros(H.HIKF_NUM_PHASES)
    for s in stats:
        tot += np.array(s.time_ms[:])
        cnt += np.array(s.time_count[:])
    avg = {name: (tot[i] / cnt[i] if cnt[i] else None) for i, name in enumerate(H.PHASES)}

    # roofline of the dominant kernel: the fused row pass, 2 m p^2 FP64 flops
    row_s = avg["rowpass"] / 1e3
    row_tflops = 2.0 * m * p * p / row_s / 1e12
    roof = {"bound": "mfma", "achieved": round(row_tflops, 3), "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(row_tflops / PEAK_FP64_TFLOPS, 4),
            "traffic": measured_traffic(a.workload, "k_rowpass"), "traffic_unit": "bytes/launch",
            "algorithmic_bytes": (8 + 4 + 8) * m * p, "kernel": "k_rowpass (FP64 MFMA)",
            "avg_ms": round(avg["rowpass"], 4)}
    tq = 8 if a.precision == "f64" else 4
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
                   "parallelism": "none (1 GPU)"},
        "warm_steps_per_s": round(1e3 / float(np.mean(lat_ms)), 2),
        "step_latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                            "p99": round(float(np.percentile(lat_ms, 99)), 4),
                            "mean": round(float(np.mean(lat_ms)), 4)},
        "init_ms_kernels": round(init_ms, 3),
        "phase_avg_ms": {k: (round(v, 4) if v is not None else None) for k, v in avg.items()},
        "roofline": roof,
        "fmm_roofline": fmm,
    }
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline(w, K, a.cpu_budget)
        log("[bench] CPU oracle done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
