"""Compile the HIP library in-tree for gfx950.

    python -m paper_2403_13287_amd._build

Produces ``paper_2403_13287_amd/liblskum.so`` from ``csrc/*.hip``.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblskum.so")
CALIB_LIB = os.path.join(HERE, "calib", "libelementary.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _hipcc(srcs, out, extra=(), verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, extra=()) -> str:
    """The sweep library, then the calibration kernels of the roofline report."""
    _hipcc(sources(), LIB, extra, verbose)
    _hipcc([os.path.join(HERE, "calib", "elementary.hip")], CALIB_LIB, extra, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
