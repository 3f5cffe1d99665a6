"""Builds librfps.so (the HIP kernels and the C ABI of include/rfps.h) for gfx950.

Usage: python -m paper_2606_06255_amd.build   (or call build()).
Every translation unit is compiled with hipcc for gfx950 only, with FP
contraction off (the distance formula is fixed) and packed FP32 instructions
disabled; objects go to _build/ and are linked into the package directory.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librfps.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["rfps_api.hip", "index_build.hip", "sample_rfps.hip", "sample_rounds.hip", "sample_plain.hip", "sample_unfused.hip",
           "mlp.hip", "cpu_sampler.cpp"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link librfps.so.  Returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    # native driver of the C ABI (profiling without Python in the process)
    exe = os.path.join(PKG, "rfps_bench")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-o", exe + ".tmp",
           os.path.join(CSRC, "rfps_bench.cpp"), "-L" + PKG, "-lrfps", "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("rfps_bench failed to build:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(exe + ".tmp", exe)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
