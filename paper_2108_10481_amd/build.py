"""Build libpbm.so (HIP for gfx950) in-tree.

Each source is compiled to an object with hipcc in parallel, then linked into
``paper_2108_10481_amd/libpbm.so``.  Packed FP32 instructions are disabled
for all device code (``-packed-fp32-ops``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpbm.so")
# measurement library (roofline peaks), not part of the solver
PEAKS_SRC = "peaks.hip"
PEAKS_OUT = os.path.join(HERE, "libpbm_peaks.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("PBM_OFFLOAD_ARCH", "gfx950")
SOURCES = ["mesh_prep.cpp", "k_geometry.hip", "k_near.hip", "k_far.hip", "k_far_sym.hip", "k_tree.hip", "k_krylov.hip", "k_dense.hip",
           "k_batch.hip", "runtime.hip", "server.cpp", "autotune.cpp"]
FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fno-gpu-rdc", "-I", os.path.join(HERE, "..", "include")]
# roctx (phase ranges for marker traces) from the ROCm install
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
LIBS = ["-L" + ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + FLAGS + ["-c", os.path.join(SRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(SRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + LIBS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    tmp = PEAKS_OUT + ".tmp"
    cmd = [hipcc()] + FLAGS + ["-shared", os.path.join(SRC, PEAKS_SRC), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {PEAKS_SRC}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PEAKS_OUT)
    if verbose:
        print("built", OUT, "and", PEAKS_OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
