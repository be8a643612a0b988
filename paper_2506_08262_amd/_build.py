"""Builds librrs.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Each translation unit is compiled to an object file in parallel (no device
code crosses translation units, so no relocatable device code is needed),
then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librrs.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["rrs_kernels.hip", "rrs_select.hip", "rrs_select_rc.hip", "rrs_mfma.hip",
           "rrs_sign.hip", "rrs_maha.hip", "rrs_engine.hip", "rrs_api.hip", "rrs_noalloc.hip",
           "rrs_serve.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # every fused multiply-add is an explicit fma(); nothing else is contracted
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _jobs() -> int:
    n = os.cpu_count() or 4
    return max(1, min(n, 16, len(SOURCES)))


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def compile_one(s: str) -> str:
        obj = os.path.join(OBJ, os.path.splitext(s)[0] + ".o")
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
