"""Build libspinsum.so (HIP, gfx950) in-tree.

    python paper_1705_06661_amd/build.py

Every HIP source is compiled with packed-FP32 instructions disabled
(``-target-feature -packed-fp32-ops``); the library is written for gfx950
only.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libspinsum.so")
ARCH = os.environ.get("SPINSUM_OFFLOAD_ARCH", "gfx950")

SOURCES = [f"spinsum_kern_{t}_d{d}.hip" for t in ("f64", "f32") for d in (4, 3, 2)] + [
    "spinsum_exec.hip", "spinsum_plan.cpp", "spinsum_tune.cpp"]
BUILD_DIR = os.path.join(HERE, "_build")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source to an object in parallel, then link the library."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + _flags() + list(extra or []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [src for src, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError(f"compilation failed: {failed}")
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
