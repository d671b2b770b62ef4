"""Build libhpmg.so for gfx950 in-tree (hipcc, parallel object compilation).

Usage: python paper_2510_00998_amd/csrc/build.py
Run as a script (it must not import the package, which loads the library).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

CSRC = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(CSRC)
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhpmg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = [
    "basis.cpp",
    "hpmg.cpp",
    "cg_kernels.hip",
    "batch_kernels.hip",
    "batch_tile1.hip",
    "batch.cpp",
    "noalloc.hip",
    "adapt_kernels.hip",
    "dg_inst_2d_float.hip",
    "dg_inst_2d_double.hip",
    "dg_inst_2d_f16.hip",
    "dg_inst_2d_bf16.hip",
    "dg_inst_3d_float.hip",
    "dg_inst_3d_double.hip",
    "dg_inst_3d_f16.hip",
    "dg_inst_3d_bf16.hip",
]

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-std=c++17", "-O3", "-fPIC", "-I" + INCLUDE, "-I" + CSRC]


def _compile(src: str, build_dir: str, defines) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + [f"-D{d}" for d in defines] + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build_library(jobs: int | None = None, verbose: bool = False, out: str | None = None,
                  defines=(), build_dir: str | None = None) -> str:
    """Compile and link; `out`/`defines`/`build_dir` build tuning variants
    elsewhere without touching the in-tree library."""
    lib = out or LIB
    bdir = build_dir or BUILD
    os.makedirs(bdir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, bdir, defines), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build_library(verbose=True)
    sys.exit(0)
