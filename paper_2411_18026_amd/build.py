"""Build the solver's shared library (libfds.so) for gfx950 with hipcc.

Usage: python -m paper_2411_18026_amd.build   (or call build()).
The library is written next to this file so that it travels with the tree.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfds.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["assembly.hip", "assembly_host.hip", "linalg.hip", "learned.hip", "fds.hip", "devmem.hip", "field.hip",
           "sweep.hip"]
ARCH = os.environ.get("FDS_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-pthread",
]


# The pair and field integrators read many FP64 constants (series and
# quadrature coefficients) inside their point loops.  Machine loop-invariant
# code motion hoists all of them out of the loops, where they exhaust the
# register file and spill to scratch (12 to 53 registers per lane); left at
# their uses they cost two scalar moves each and nothing spills (the
# 3-point series integrator 5 % faster, the coincident-pair one 25 %).  Code
# motion only: the arithmetic and its results are unchanged.
EXTRA = {
    "assembly.hip": ["-mllvm", "-disable-machine-licm"],
    "field.hip": ["-mllvm", "-disable-machine-licm"],
}


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
