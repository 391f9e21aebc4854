"""Build the HIP library ``libdgamr.so`` in-tree for gfx950.

Host-only C++ (forest, reference operators) is compiled with g++; the kernels
and the C ABI with hipcc.  Always recompiles (the caller asked for a build).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libdgamr.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter"]

SOURCES = [
    ("refelem.cpp", "cxx"),
    ("forest.cpp", "cxx"),
    ("sphere.cpp", "cxx"),
    ("abi.cpp", "hip"),
    ("kernels.hip", "hip"),
    ("tracer.hip", "hip"),
    ("viscous.hip", "hip"),
    ("sphere.hip", "hip"),
]


def _compile(src: str, kind: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    inc = ["-I", INCLUDE, "-I", CSRC]
    if kind == "cxx":
        cmd = ["g++", *CXX_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
    else:
        cmd = [HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found")
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-lgomp", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
