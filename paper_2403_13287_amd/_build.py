"""Compile the HIP library in-tree for gfx950.

    python -m paper_2403_13287_amd._build

Produces ``paper_2403_13287_amd/liblskum.so`` from ``csrc/*.hip``.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblskum.so")
CALIB_LIB = os.path.join(HERE, "calib", "libelementary.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # No packed-FP32 instructions anywhere in the device code.  The device
    # (gfx950) compilation honours this feature switch; only the host pass,
    # which gets the same flags, prints that it does not know the feature.
    # tests/test_build_flags.py compiles a float2 kernel both ways and checks
    # that the switch removes its v_pk_* instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]

# Instruction scheduler of the AMDGPU back end per source file, chosen by
# timing the whole iteration on MI355X with every strategy: the derivative
# and time-step gathers run ~5 % faster with the ILP scheduler (the whole
# iteration ~2 %).  For the flux kernel no strategy gave a reproducible
# gain over the default, so it keeps the default with the other files.
SCHEDULER = {
    "lskum_deriv.hip": "iterative-ilp",
}


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _hipcc(srcs, out, extra=(), verbose=False):
    """Compile each source to an object with its own scheduler, then link the
    shared library (no relocatable device code: every kernel is launched
    from the file that defines it)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include")]
    tmp = out + ".tmp"
    with tempfile.TemporaryDirectory() as objdir:
        objs = []
        for src in srcs:
            name = os.path.basename(src)
            sched = SCHEDULER.get(name)
            flags = ["-mllvm", f"-amdgpu-sched-strategy={sched}"] if sched else []
            obj = os.path.join(objdir, name + ".o")
            _run([hipcc, *HIPCC_FLAGS, *flags, *extra, *inc, "-c", src, "-o", obj], verbose)
            objs.append(obj)
        _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
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
