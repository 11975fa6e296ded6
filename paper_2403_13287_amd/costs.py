"""Algorithmic work of the sweep kernels, for the roofline report.

Bytes: compulsory HBM traffic, each array read or written once per pass
(neighbour values reused from cache).  Connectivity C = 4*k_pad + 4 bytes
per point (padded column-major ids plus the count).

FP64 operations: the operations of the method's formulas as written (one
per add, subtract, multiply, compare-free; a divide or square root counts
its FP64 instruction sequence), with each elementary function weighted by
the FP64 operations of the device math library's implementation on its
common path (an FMA counts 2).  EDGE_FLOPS is per (point, neighbour) pair of
the flux pass, POINT_FLOPS per point of that pass.
"""
from __future__ import annotations

# weights of the elementary functions in FP64 operations (FMA = 2)
W_DIV = 17
W_SQRT = 21
W_EXP = 32
W_LOG = 60
W_ERF = 70

# operation counts of one flux-pass edge (two reconstructions of 4
# components, two states, four split fluxes, two weighted accumulations)
EDGE_BASIC = 404
EDGE_DIV = 22
EDGE_SQRT = 5
EDGE_EXP = 6
EDGE_LOG = 2
EDGE_ERF = 4
EDGE_FLOPS = (EDGE_BASIC + EDGE_DIV * W_DIV + EDGE_SQRT * W_SQRT + EDGE_EXP * W_EXP
              + EDGE_LOG * W_LOG + EDGE_ERF * W_ERF)
POINT_FLOPS = 60  # split weights and the rotation back


def flux_flops(n_points: int, n_edges: int) -> float:
    return float(n_edges) * EDGE_FLOPS + float(n_points) * POINT_FLOPS


def conn_bytes(k_pad: int) -> int:
    return 4 * k_pad + 4


def flux_bytes(n_points: int, k_pad: int) -> float:
    """Flux pass: x, y, nx, ny, kind (33), q (32), dq (64), qlim (64),
    connectivity; writes R (32)."""
    return float(n_points) * (33 + 32 + 64 + 64 + 32 + conn_bytes(k_pad))


def stage_bytes(n_points: int, k_pad: int, n_inner: int) -> float:
    """One RK stage: q-variables (64), first-order pass (16 + 32 + 64 + 64
    + C), each inner sweep (16 + 32 + 64 + 64 + C), flux pass, stage update
    (Un, U, R, dt, kind in; U out: 137), plus the per-iteration time step
    and U^n copy amortised over 4 stages ((16 + 32 + 8 + C + 64)/4)."""
    c = conn_bytes(k_pad)
    per = 64 + (176 + c) + n_inner * (176 + c) + (225 + c) + 137 + (120 + c) / 4.0
    return float(n_points) * per
