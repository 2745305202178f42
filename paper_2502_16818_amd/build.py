"""Compile the HIP/C++ sources of the CDBM library into libcdbm.so (gfx950).

Run as ``python -m paper_2502_16818_amd.build`` or call ``build()``.  Objects
go to ``_build/`` at the repository root; the library lands next to this
file.  Every call recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcdbm.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = [
    "model.cpp",
    "api.hip",
    "api_adjoint.hip",
    "api_batch.hip",
    "api_static.hip",
    "kernels_basic.hip",
    "kernels_step.hip",
    "kernels_adjoint.hip",
    "kernels_batch.hip",
]

ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-Wall",
    # packed FP32 (v_pk_*_f32) instructions stay off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the CDBM library needs ROCm's hipcc to build")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc()]
    if src.endswith(".hip"):
        cmd += ["-x", "hip", f"--offload-arch={ARCH}"]
    cmd += FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking libcdbm.so failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
