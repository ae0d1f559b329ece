"""Build libmoe.so (gfx950) in-tree with hipcc.

Usage: python -m paper_2606_17065_amd.build   (or build() from Python).
Every call compiles from scratch; objects go to paper_2606_17065_amd/_build/.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmoe.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-fno-gpu-flush-denormals-to-zero",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]

# Sources and their extra flags.  The router / price loop is compiled
# without floating-point contraction: its operation sequence is part of the
# definition of the routing.
SOURCES = [
    ("route.hip", ["-ffp-contract=off"]),
    ("dispatch.hip", []),
    ("gemm.hip", []),
    ("bwd.hip", []),
    ("price.hip", []),
    ("mlp.hip", []),
    ("api.cpp", []),
    ("prof.cpp", []),
]


def _compile(src, extra):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src == "api.cpp":
        cmd = ["g++", "-O2", "-fPIC", "-std=c++17", "-c", os.path.join(CSRC, src), "-o", obj]
    elif src.endswith(".cpp"):  # host code that calls the HIP runtime
        cmd = [HIPCC, "-O2", "-fPIC", "-std=c++17", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(lambda a: _compile(*a), SOURCES))
    objs = []
    for src, obj, r in results:
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"compiling {src} failed")
        if verbose and r.stderr:
            sys.stderr.write(r.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking libmoe.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
