"""Build the CPU oracle libraries (test infrastructure).

    python -m oracle.build

Compiles, next to this file, with g++ in strict IEEE mode (no -ffast-math,
no FMA contraction):

* ``liblskum_ref.so`` -- the parity oracle, single-threaded;
* ``liblskum_ref_omp.so`` -- the same source with OpenMP enabled: its forward
  point loops run on all host cores with identical results (used only for
  the benchmark's all-cores CPU figure).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblskum_ref.so")
LIB_OMP = os.path.join(HERE, "liblskum_ref_omp.so")
SOURCES = [os.path.join(HERE, "lskum_ref.cpp")]
FLAGS = ["-std=c++17", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
         "-Wall", "-Wextra"]


def _compile(out: str, extra, verbose: bool) -> str:
    tmp = out + ".tmp"
    cmd = ["g++", *FLAGS, *extra, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Both builds; returns the path of the parity (single-threaded) one."""
    _compile(LIB, ["-Wno-unknown-pragmas"], verbose)
    _compile(LIB_OMP, ["-fopenmp"], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
