"""Pseudo-time driver over the C ABI (the whole iteration runs in HIP).

The fixed-point loop of the paper's solver structure ("Regent based
Meshfree LSKUM Solver", Algorithm 1): a local time step, then four
Runge-Kutta stages of q-variables -> q-derivatives -> flux residual ->
state update, with the residual norm of each iteration kept on the device
(read back once, not every iteration).

A Solver over a list of clouds is a batch: the clouds are concatenated
into one plan and advanced together (one launch per kernel for all of them,
or one graph launch per replay), each with its own Mach number and angle
of attack.
"""
from __future__ import annotations

import torch

from . import lskum as L


class Solver:
    def __init__(self, cloud, params, stream=None, tuning: L.Tuning | None = None):
        self.plan = L.Plan(cloud, params, stream, tuning)
        self.n = self.plan.n
        self.n_clouds = self.plan.n_clouds
        self.U = self.plan.field(4)
        self.ws = L.workspace(self.plan)
        self.stream = stream
        L.lskum_init_state(self.plan, self.U, stream)
        self.iteration = 0
        self._hist = []
        self._graph = None

    def _shape(self, hist):
        return hist[:, 0] if self.n_clouds == 1 else hist

    def run(self, iters: int) -> torch.Tensor:
        """Advance `iters` iterations; returns the device residual history
        (iters,) for one cloud, (iters, n_clouds) for a batch."""
        hist = torch.empty((max(int(iters), 1), self.n_clouds), dtype=torch.float64,
                           device=self.U.device)
        L.lskum_iterate(self.plan, iters, self.U, hist, self.ws, self.stream)
        self.iteration += int(iters)
        self._hist.append(hist[:iters])
        return self._shape(hist[:iters])

    def capture(self, iters: int, replays: int):
        """Capture `iters` iterations in a HIP graph with room for `replays`
        replays of history; returns (graph, hist) -- hist rows fill as the
        graph is launched."""
        hist = torch.full((iters * replays, self.n_clouds), float("nan"), dtype=torch.float64,
                          device=self.U.device)
        self._graph = L.Graph(self.plan, iters, self.U, hist, self.ws, self.stream)
        return self._graph, hist

    def history(self) -> torch.Tensor:
        if not self._hist:
            return torch.empty(0, dtype=torch.float64)
        return self._shape(torch.cat(self._hist))

    def status(self) -> int:
        return L.lskum_status(self.plan, self.stream)

    def force_coeffs(self, U=None) -> torch.Tensor:
        """(Cl, Cd) for one cloud, (n_clouds, 2) for a batch."""
        out = torch.empty(2 * self.n_clouds, dtype=torch.float64, device=self.U.device)
        L.lskum_force_coeffs(self.plan, self.U if U is None else U, out, self.stream)
        return out if self.n_clouds == 1 else out.view(self.n_clouds, 2)

    def cloud_state(self, c: int) -> torch.Tensor:
        return self.U[self.plan.cloud_slice(c)]

    def residual(self, U=None):
        """q, dq, qlim and R of the state U (default: the current state)."""
        U = self.U if U is None else U
        p = self.plan
        q, dq, qlim, work, R = p.field(4), p.field(8), p.field(8), p.field(16), p.field(4)
        L.lskum_q_vars(p, U, q, self.stream)
        L.lskum_q_derivs(p, q, dq, qlim, work, self.stream)
        L.lskum_flux_residual(p, q, dq, qlim, R, self.stream)
        return q, dq, qlim, R
