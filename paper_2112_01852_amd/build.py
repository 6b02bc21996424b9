"""Builds libqdwf.so (the HIP kernels and the C ABI) in-tree for gfx950.

Usage: ``python -m paper_2112_01852_amd.build`` (or ``build()`` from Python).
Each source is compiled by hipcc in parallel into ``_build/``, then linked
into ``paper_2112_01852_amd/libqdwf.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libqdwf.so")
ARCH = os.environ.get("QDWF_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "hop.hip", "pack.hip", "local.hip", "solver.hip", "tune.cpp", "pool.cpp", "wilson.hip", "stream.hip", "halo.hip", "sweep.hip", "noalloc.hip", "group.hip"]

# Packed-FP32 instructions are switched off for all device code. The
# two-operand v_dot2c_f32_f16 and v_dot2c_f32_bf16 forms are switched off
# too: they accumulate into their destination, so every product chain that
# starts from zero cost a register clear; the three-operand v_dot2_f32_f16
# and v_dot2_f32_bf16 take the zero inline.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Xclang", "-target-feature", "-Xclang", "-dot5-insts",
                "-Xclang", "-target-feature", "-Xclang", "-dot13-insts"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
           "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC, *DEVICE_FLAGS,
           "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
