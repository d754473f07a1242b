"""Autotuner for the launch form of the fused row pass.

The row pass (one per assimilation step; the gain, state, variance and
cross-covariance rows of Algorithm Algorithm_HiKF) dominates the run time.
It has several launch forms (hikf_options.rowpass_variant): 8-wave
workgroups on 64- or 32-row tiles (columns in two halves or in four parts),
4-wave workgroups with one wave per SIMD and two row groups per wave (the
dual form), each with one workgroup per tile or persistent workgroups that
loop over tiles.  Which is fastest depends on p,
m and the device, so this module measures them on the problem at hand and
records the winner in a JSON cache that hikf_init reads (option tune_cache):

    {"device": "...", "rowpass": [{"p": 256, "cq": "f32", "m": 1048576,
      "variant": 1, "ms": [2.67, 2.31, 2.71, 2.40, 3.40, 3.50]}, ...]}

(ms: the row-pass time of each variant 0..5, null where a variant is the
same launch as another for this p).

Usage (on the GPU):
    python -m paper_1404_3816_amd.tune --out tune_cache.json \
        --workload crosswell-1024x1024-p256 [--workload ...]
or, from Python, ``tune_problem(problem, keepalive, options_kwargs, ...)``.
"""

import argparse
import json
import os

import numpy as np
import torch

from . import filter as F

VARIANTS = (0, 1, 2, 3, 4, 5)


def distinct_variants(p):
    """The variants that differ for p: persistence needs p / 16 even in the
    8-wave forms, p > 256 always uses the 32-row split, and the dual form
    (bit 2) is built for p = 64, 128 and 256 only."""
    out = []
    for v in VARIANTS:
        eff = v
        if v & 4:
            if p not in (64, 128, 256):
                continue
            eff = v & 5
        else:
            if (p // 16) % 2:
                eff &= ~1
            if p > 256:
                eff |= 2
        if eff not in out:
            out.append(eff)
    return out


def measure_variant(problem, keepalive, variant, steps, options_kwargs, ys):
    """Average row-pass time (ms, HIP events on the launch stream) over
    `steps` assimilation steps of a fresh filter forced to `variant`."""
    kw = dict(options_kwargs)
    kw.update(timing=True, graph=False, rowpass_variant=variant)
    f = F.HikfFilter(problem, F.make_options(**kw), keepalive)
    try:
        for k in range(steps):
            f.step(ys[k % len(ys)])
        st = f.query()
        if st.last_status != 0:
            raise RuntimeError(f"tuning step failed with status {st.last_status}")
        i = 10                                    # HIKF_PHASE_ROWPASS
        return (st.time_ms[i] / st.time_count[i]) if st.time_count[i] else float("nan")
    finally:
        f.close()


def tune_problem(problem, keepalive, options_kwargs, ys, steps=8, repeats=2):
    """Measure every distinct variant `repeats` times (interleaved) and
    return (best variant, {variant: best ms})."""
    p = int(problem.p)
    cands = distinct_variants(p)
    ms = {v: float("inf") for v in cands}
    for _ in range(repeats):
        for v in cands:
            ms[v] = min(ms[v], measure_variant(problem, keepalive, v, steps, options_kwargs, ys))
    best = min(cands, key=lambda v: ms[v])
    return best, ms


def merge_entry(path, entry):
    """Insert or replace the entry with the same (p, cq, m) in the cache."""
    data = {"device": "", "rowpass": []}
    if path and os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data.setdefault("rowpass", [])
    data["rowpass"] = [e for e in data["rowpass"]
                       if (e["p"], e["cq"], e["m"]) != (entry["p"], entry["cq"], entry["m"])]
    data["rowpass"].append(entry)
    data["rowpass"].sort(key=lambda e: (e["cq"], e["p"], e["m"]))
    data["device"] = torch.cuda.get_device_name(0) if torch.cuda.is_available() else ""
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1)
    return data


def tune_workload(name, out, precision=None, steps=8, repeats=2, n=None, p=None):
    """Tune the row pass on a crosswell workload of the input generators
    (or on its grid and ray count overridden by n and p) and record it."""
    import synth
    w = synth.workload(name)
    if n is not None:
        w["n"], w["m"] = n, n ** w["dim"]
    if p is not None:
        w["p"] = p
    prec = precision or ("bf16x3" if w["dim"] == 3 else "f32")
    rowptr, col, val = synth.crosswell_h(w["dim"], w["n"], w["p"], planes=8)
    ys = synth.plume_observations(w["dim"], w["n"], rowptr, col, val, steps, w["r_var"],
                                  w["seed"] + 1)
    pr, keep = F.problem_from_csr(w["dim"], w["n"], rowptr, col, val,
                                  np.full(w["p"], w["r_var"]), theta=w["theta"], ell=w["ell"],
                                  gamma=w["gamma"], prior=w["prior"])
    yd = torch.as_tensor(ys, device="cuda")
    okw = dict(n_c=w["n_c"], precision=prec, sparse=True)
    best, ms = tune_problem(pr, keep, okw, yd, steps, repeats)
    entry = {"p": int(w["p"]), "cq": "f64" if prec == "f64" else "f32", "m": int(w["m"]),
             "variant": int(best),
             "ms": [round(ms[v], 4) if v in ms else None for v in VARIANTS],
             "workload": name if n is None and p is None else
             f"crosswell-{w['n']}x{w['n']}-p{w['p']}"}
    if out:
        merge_entry(out, entry)
    return entry


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True, help="tuning cache (JSON) to create or update")
    ap.add_argument("--workload", action="append", default=[],
                    help="workload of the input generators (repeatable)")
    ap.add_argument("--p", type=int, action="append", default=[],
                    help="also tune these ray counts on the 2-D workload grid given by --n")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--steps", type=int, default=8)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    for name in args.workload:
        print(json.dumps(tune_workload(name, args.out, steps=args.steps)), flush=True)
    for p in args.p:
        print(json.dumps(tune_workload("crosswell-256x256-p64", args.out, steps=args.steps,
                                       n=args.n, p=p)), flush=True)


if __name__ == "__main__":
    main()
