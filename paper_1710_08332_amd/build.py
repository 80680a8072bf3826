"""Builds libdpia.so (gfx950) in-tree.

    python -m paper_1710_08332_amd.build

Host-only validation (plan.cpp) is compiled with g++; the kernels and the
C-ABI entry points with hipcc for gfx950.  Floating point: -ffp-contract=off
on both (no fused multiply-add anywhere: every product and sum of a strategy
is rounded on its own), no fast-math, denormals kept.  Packed FP32
instructions are disabled for the device code.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libdpia.so")

HIP_SOURCES = ["reduce.hip", "gemv.hip", "batch.hip", "map.hip", "module.hip", "stream.hip"]
CPP_SOURCES = ["plan.cpp"]

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-I" + INCLUDE, "-I" + CSRC]
HIP_FLAGS = COMMON + ["--offload-arch=gfx950", "-fno-gpu-rdc",
                      "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                      "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(["g++"] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr, file=sys.stderr)
    objs = [os.path.join(BUILD, s + ".o") for s in CPP_SOURCES + HIP_SOURCES]
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    from paper_1710_08332_amd.generator import catalog   # noqa: E402
    for p in catalog.build_all():
        print(p)
