"""Build the gfx950 HIP library libnlrmm.so in-tree with hipcc.

Every source is compiled to its own object (in parallel), then the objects are linked into
the shared library.  The sources share no device symbols (the device helpers in the headers
are inline), so no relocatable device code is needed.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnlrmm.so")
SOURCES = ["api.cpp", "proj.hip", "krylov.hip", "solve_reg_a.hip", "solve_reg_b.hip",
           "solve_reg_c.hip", "solve_reg_d.hip", "solve_reg_e.hip", "solve_reg_f.hip",
           "gn.hip", "varpro.hip", "solver.cpp", "tune.cpp", "noalloc.hip", "fan.hip", "of.hip", "pat.hip"]
ARCH = os.environ.get("NLRMM_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # keep packed FP32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
]


def _jobs() -> int:
    n = os.cpu_count() or 1
    return max(1, min(len(SOURCES), n, 16))


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = list(SOURCES)

    def compile_one(src: str) -> str:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = ["hipcc", *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)
