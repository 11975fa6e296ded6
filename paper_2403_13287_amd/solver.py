"""Pseudo-time driver over the C ABI (the whole iteration runs in HIP).

The fixed-point loop of the paper's solver structure ("Regent based
Meshfree LSKUM Solver", Algorithm 1): a local time step, then four
Runge-Kutta stages of q-variables -> q-derivatives -> flux residual ->
state update, with the residual norm of each iteration kept on the device
(read back once, not every iteration).
"""
from __future__ import annotations

import torch

from . import lskum as L


class Solver:
    def __init__(self, cloud, params: L.Params, stream=None):
        self.plan = L.Plan(cloud, params, stream)
        self.n = self.plan.n
        self.U = self.plan.field(4)
        self.ws = L.workspace(self.plan)
        self.stream = stream
        L.lskum_init_state(self.plan, self.U, stream)
        self.iteration = 0
        self._hist = []

    def run(self, iters: int) -> torch.Tensor:
        """Advance `iters` iterations; returns the device residual history."""
        hist = torch.empty(max(int(iters), 1), dtype=torch.float64, device=self.U.device)
        L.lskum_iterate(self.plan, iters, self.U, hist, self.ws, self.stream)
        self.iteration += int(iters)
        self._hist.append(hist[:iters])
        return hist[:iters]

    def history(self) -> torch.Tensor:
        if not self._hist:
            return torch.empty(0, dtype=torch.float64)
        return torch.cat(self._hist)

    def status(self) -> int:
        return L.lskum_status(self.plan, self.stream)

    def force_coeffs(self, U=None) -> torch.Tensor:
        out = torch.empty(2, dtype=torch.float64, device=self.U.device)
        L.lskum_force_coeffs(self.plan, self.U if U is None else U, out, self.stream)
        return out

    def residual(self, U=None):
        """q, dq, qlim and R of the state U (default: the current state)."""
        U = self.U if U is None else U
        p = self.plan
        q, dq, qlim, work, R = p.field(4), p.field(8), p.field(8), p.field(8), p.field(4)
        L.lskum_q_vars(p, U, q, self.stream)
        L.lskum_q_derivs(p, q, dq, qlim, work, self.stream)
        L.lskum_flux_residual(p, q, dq, qlim, R, self.stream)
        return q, dq, qlim, R
