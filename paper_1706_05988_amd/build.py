"""Build libpcg.so (the C-ABI library and its gfx950 kernels) in-tree with hipcc.

    python -m paper_1706_05988_amd.build

The shared library lands next to this file; ``paper_1706_05988_amd.pcg``
loads it from there.  Every call compiles (no staleness shortcut), so a
build after a source change is never skipped.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpcg.so")
ARCH = os.environ.get("PCG_OFFLOAD_ARCH", "gfx950")

SOURCES = ["pcg_solver.hip", "pcg_batch.hip", "pcg_server.hip", "pcg_tune.hip", "pcg_stream.hip", "pcg_shift.cpp"]

# -Xclang -target-feature -Xclang -packed-fp32-ops keeps the compiler from
# emitting packed FP32 VALU instructions on gfx950.
HIPCC_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile each source to an object in parallel, then link libpcg.so."""
    from concurrent.futures import ThreadPoolExecutor
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        if src.endswith(".cpp"):  # host-only sources
            cmd = ["g++"] + CXX_FLAGS + ["-I", INCLUDE, "-c", src, "-o", obj]
        else:
            cmd = [hipcc()] + compile_flags + ["-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(6, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
