"""Compile the HIP sources under csrc/ into libhikf.so for gfx950.

Run ``python -m paper_1404_3816_amd.build`` (or call ``build()``); the
library is written next to this file so that it travels with the source tree.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhikf.so")
SOURCES = ["api.hip", "fmm.hip", "step.hip", "pspace.hip", "enkf.hip"] + [
    f"enkf_transform_{k}.hip" for k in "abcde"] + [
    f"rowpass_{t}_{k}.hip" for t in ("f32", "f64") for k in (1, 2, 3, 4)]
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel, one object each) and link the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    cflags = [f for f in FLAGS if f != "-shared"]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc, *cflags, *inc, "-c", os.path.join(HERE, "csrc", src), "-o", obj]
        jobs.append((obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                           text=True)))
    failed = False
    for obj, proc in jobs:
        out, err = proc.communicate()
        if proc.returncode != 0:
            failed = True
            sys.stderr.write(out + err)
        elif verbose:
            sys.stderr.write(err)
    if failed:
        raise RuntimeError("hipcc failed building libhikf.so")
    tmp = LIB + ".tmp"
    res = subprocess.run([hipcc, *FLAGS, *[o for o, _ in jobs], "-o", tmp],
                         capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libhikf.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
