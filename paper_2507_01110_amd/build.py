"""Builds liblodgs.so in-tree: HIP sources with hipcc for gfx950, the host
HSPT builder with g++ (OpenMP), linked into one shared library."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblodgs.so")

HIP_SOURCES = ["lodgs_api.hip", "lodgs_prims.hip", "lodgs_select.hip", "lodgs_render.hip", "lodgs_backward.hip", "lodgs_optim.hip", "lodgs_cache.hip", "lodgs_rows.hip", "lodgs_noalloc.hip", "lodgs_server.hip", "lodgs_pool.hip"]
CPP_SOURCES = ["lodgs_hspt.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # FP32 decisions must be reproducible: no contraction, IEEE / and sqrt, denormals kept.
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # atomics as written: no wave-level rewrite of LDS adds whose lanes are already reduced
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", INC, "-I", CSRC]
    jobs = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(OBJ, s + ".o")
        objs.append(o)
        jobs.append([HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, s), "-o", o])
    for s in CPP_SOURCES:
        o = os.path.join(OBJ, s + ".o")
        objs.append(o)
        jobs.append(["g++", "-O2", "-std=c++17", "-fPIC", "-fopenmp", "-ffp-contract=off", *inc,
                     "-I", "/opt/rocm/include", "-c", os.path.join(CSRC, s), "-o", o])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-lgomp", "-o", LIB + ".tmp"], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
