"""Build the HIP library libpolydet.so in-tree for gfx950.

Usage: python -m paper_2010_12117_amd.build  (or build() from Python). Every call recompiles
all sources; objects go to paper_2010_12117_amd/_build/, the library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpolydet.so")
ARCH = "gfx950"
DET_PARTS = 8

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall"]
FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
    # no packed-fp32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the elimination kernels rely on full unrolling (static register indices); at n = 32
    # the unrolled body is larger than the default limit of the unroll pragma
    "-mllvm", "-pragma-unroll-threshold=200000",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-command-line-argument",
]


def _units():
    # every host source and every HIP source of csrc/ (det_part.hip once per slice)
    units = []
    for name in sorted(os.listdir(CSRC)):
        stem, ext = os.path.splitext(name)
        if ext in (".cpp", ".hip") and name != "det_part.hip":
            units.append((stem + ".o", os.path.join(CSRC, name), []))
    for part in range(DET_PARTS):
        units.append((f"det_part{part}.o", os.path.join(CSRC, "det_part.hip"),
                      [f"-DDET_PART={part}"]))
    return units


def _compile(unit):
    obj, src, extra = unit
    out = os.path.join(BUILD, obj)
    if src.endswith(".hip"):
        cmd = [HIPCC] + FLAGS + extra + ["-x", "hip", "-c", src, "-o", out]
    else:  # host-only C++ (plan, C-ABI): the HIP runtime API needs no device compiler
        cmd = [CXX] + HOST_FLAGS + extra + ["-c", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every source and link libpolydet.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), max(1, os.cpu_count() or 1), 16)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
