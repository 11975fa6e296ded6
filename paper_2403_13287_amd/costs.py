"""Algorithmic work of the sweep kernels, for the roofline report.

Bytes: compulsory HBM traffic, each array read or written once per pass
(neighbour values reused from cache).  Connectivity C = 4*k_pad + 4 bytes
per point (padded column-major ids plus the count).

FP64 operations of the flux kernel: the operations of its formulation,
with each elementary function at its device cost (an FMA counts 2).  Every
FP64 operation the kernel executes belongs to that formulation (the only
wasted work is the n+ split flux evaluated with zero weight at wall points,
0.1 % of the edges of the 1M cloud), so the count is taken from the
hardware: SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes of one launch on the 1M cloud
divided by its edges, at the bench's developed input state (the free stream
advanced 500 iterations; from the free stream itself the kernel skips the
limiter divisions where the derivatives are still exactly zero and counts
fewer).  Per edge the formulation holds 4 erf, 6 exp, 3 Newton-refined
rsqrt, 8 Newton-refined divides and about 190 multiply/add/FMA operations;
the half-plane least-squares weights are computed once with the plan
(geometry only) and read per point.  The per-call costs of the elementary
functions measured by the calibration kernels on arguments in the sweep's
ranges are listed in ELEMENTARY_FLOPS (erf on wave-coherent arguments; on
scattered ones it costs 99; the kernel's own erf and exp cost the same FP64
operations as the library's with fewer other instructions).
"""
from __future__ import annotations

import hashlib
import os

# measured FP64 operations per call (FMA = 2), calibration kernels, gfx950
ELEMENTARY_FLOPS = {"exp": 27, "erf": 54.4, "log": 79, "sqrt": 17, "rsqrt": 9, "div": 14}

EDGE_FLOPS = 569.3  # flux kernel, FP64 operations per (point, neighbour) pair
# the SSP stage update and the q-variables of the new state (eq. (13)) run
# as the flux launch's epilogue: FP64 operations per point, the difference
# of the fused and the plain flux launch's SQ_INSTS_VALU_FLOPS_FP64 over the
# points of the 1M cloud (1.7286e10 - 569.3 x 29,967,646, averaged over the
# four stages).  The fused total is what the counters fix; the split moves
# with the state the plain launch is counted on (the RK4 run's) by a few
# operations per edge.
STAGE_FLOPS = 226.3


def flux_flops(n_points: int, n_edges: int, stage: bool = False) -> float:
    """FP64 operations of one flux launch; with `stage`, of the launch that
    also applies the SSP stage and writes the next q."""
    return float(n_edges) * EDGE_FLOPS + (float(n_points) * STAGE_FLOPS if stage else 0.0)


def conn_bytes(k_pad: int) -> int:
    return 4 * k_pad + 4


def flux_bytes(n_points: int, k_pad: int, stage: bool = False) -> float:
    """Flux pass: x, y, nx, ny, kind (33), q (32), dq (64), qlim (64),
    half-plane weights (64), connectivity; writes R (32).  With the SSP
    stage in its epilogue also U and dt in, U and the next q out, and U^n
    read at one stage in four and written at another (32 + 8 + 32 + 32 +
    32/4 + 32/4 = 120)."""
    return float(n_points) * (33 + 32 + 64 + 64 + 64 + 32 + conn_bytes(k_pad)
                              + (120 if stage else 0))


def stage_bytes(n_points: int, k_pad: int, n_inner: int, fused: bool = True) -> float:
    """One RK stage: first-order pass (16 + 32 + 64 + 64 + C), each inner
    sweep (16 + previous derivatives 64 + first-order derivatives 64 + new
    derivatives 64 + C), the flux pass with the SSP stage in its epilogue,
    plus the per-iteration time step amortised over 4 stages
    ((16 + 32 + 8 + C)/4; U^n is stored by the first stage, not copied).
    Unfused (classical RK4): the plain flux pass, a q-variables pass (64)
    and a stage update (Un, U, R, dt, kind in; U out; U^n out at one stage
    in four: 137 + 8) instead."""
    c = conn_bytes(k_pad)
    flux = flux_bytes(1, k_pad, stage=fused)
    per = (176 + c) + n_inner * (208 + c) + flux + (56 + c) / 4.0
    if not fused:
        per += 64 + 145
    return float(n_points) * per


# the sources the forward sweep kernels (k_flux among them) are compiled from
FORWARD_SOURCES = ("include/lskum.h", "paper_2403_13287_amd/csrc/lskum.hip",
                   "paper_2403_13287_amd/csrc/lskum_flux.hip",
                   "paper_2403_13287_amd/csrc/lskum_deriv.hip",
                   "paper_2403_13287_amd/csrc/lskum_impl.h",
                   "paper_2403_13287_amd/csrc/lskum_math.h",
                   "paper_2403_13287_amd/_build.py")  # the build recipe picks the schedulers


def kernel_source_hash(root: str | None = None) -> str:
    """sha256 of the forward kernels' sources (under the repository root, or
    `root`), to tie stored counter readings to the code they were taken on
    (the adjoint's source does not enter)."""
    if root is None:
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    h = hashlib.sha256()
    for rel in FORWARD_SOURCES:
        with open(os.path.join(root, rel), "rb") as f:
            h.update(rel.encode())
            h.update(f.read())
    return h.hexdigest()


def stored_flux_traffic(path: str):
    """HBM bytes per flux launch from a profile summary, or None when the
    summary was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["flux_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
