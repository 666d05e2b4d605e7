"""Build ``libpsvt.so`` (hipcc, gfx950) in-tree.

Usage: ``python -m paper_2607_22484_amd.build``.  Every call compiles.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpsvt.so")
OBJ_DIR = os.path.join(HERE, "_build")
# the tile-kernel units first (one per operand type and tile configuration):
# they dominate the build
_TILE_UNITS = ["gemm_%s_%d.hip" % (t, bm) for t in ("f32", "bf16x3", "bf16", "fp8") for bm in (256, 192, 128, 64)]
SOURCES = _TILE_UNITS + ["gemm_f32.hip", "gemm_bf16x3.hip", "gemm_bf16.hip", "gemm_fp8.hip", "kernels.hip",
                         "api.hip", "trace.hip", "batch.hip", "server.hip", "noalloc.hip", "batched.hip", "persist.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled: the compiler must not form
# v_pk_{add,mul,fma}_f32 from scalar or float2 code on this hardware.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel: the per-operand-type tile units
    dominate) and link ``libpsvt.so``."""
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, src.replace(".hip", ".o")) for src in SOURCES]

    def one(pair):
        src, obj = pair
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(one, zip(SOURCES, objs)))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
