"""Differentiable residual and force coefficients over the library's adjoints.

``torch.autograd.Function`` wrappers whose forward and backward passes are the
HIP kernels of ``liblskum.so`` (``lskum_flux_residual`` and
``lskum_flux_residual_vjp``, ``lskum_force_coeffs`` and
``lskum_force_coeffs_vjp``); Python only marshals arguments.

theta is a (n_clouds, 2) float64 tensor of (Mach, angle of attack in
radians) per cloud.  The residual is a function of the interior and wall rows
of U and of theta: its forward pass first writes the free stream of theta
into the outer (Dirichlet) rows, so the outer rows of the U passed in do not
matter and get a zero gradient, and theta's gradient is the one that flows
through those rows.  The force coefficients depend on U at the wall points
and on theta through the dynamic pressure and the lift/drag axes.

The backward pass recomputes q and every least-squares iterate from U (the
forward keeps only U), differentiating the branch the forward took at each
limiter, stencil max/min and half-plane membership test.
"""
from __future__ import annotations

import dataclasses

import torch

from . import lskum as L


class Adjoint:
    """Differentiable residual R(U, theta) and coefficients C(U, theta) of a
    plan's clouds."""

    def __init__(self, cloud, params, stream=None, tuning: L.Tuning | None = None, plan=None):
        self.plan = plan if plan is not None else L.Plan(cloud, params, stream, tuning)
        self.stream = stream
        self._ws = None

    @property
    def n_clouds(self) -> int:
        return self.plan.n_clouds

    def theta(self) -> torch.Tensor:
        """The plan's current (Mach, alpha [rad]) per cloud, on the CPU."""
        return torch.tensor([[p.mach, p.alpha()] for p in self.plan.params], dtype=torch.float64)

    def set_theta(self, theta: torch.Tensor):
        th = theta.detach().to("cpu", torch.float64).reshape(self.n_clouds, 2).tolist()
        new = [dataclasses.replace(p, mach=float(m), aoa_rad=float(a))
               for p, (m, a) in zip(self.plan.params, th)]
        if any(p.mach != q.mach or p.alpha() != q.alpha() for p, q in zip(new, self.plan.params)):
            self.plan.set_params(new)

    def workspace(self) -> torch.Tensor:
        """Device workspace of the VJP and of the steady adjoint iteration."""
        if self._ws is None:
            self._ws = L.adjoint_workspace(self.plan)
        return self._ws

    def steady_gradient(self, U: torch.Tensor, Jbar, iters: int, Lam: torch.Tensor | None = None):
        """Total derivative of J = sum_c Jbar_c . (Cl, Cd)_c with respect to
        theta = (M, alpha [rad]) of each cloud, at a steady state U.

        The adjoint Lambda of the projected residual is found by `iters`
        pseudo-time steps of lskum_adjoint_iterate (from Lam, or zero); then
        lskum_adjoint_total forms dJ/dtheta = dJ/dtheta|_U - thetabar(Lambda)
        on the device.  Returns a dict with
        the total and partial derivatives ((n_clouds, 2) each), Lambda and
        the adjoint residual history ((iters, n_clouds))."""
        p, s = self.plan, self.stream
        dev = U.device
        Jb = torch.as_tensor(Jbar, dtype=torch.float64).reshape(p.n_clouds, 2).to(dev).contiguous()
        g = p.field(4)
        partial = torch.empty(2 * p.n_clouds, dtype=torch.float64, device=dev)
        L.lskum_force_coeffs_vjp(p, U, Jb.view(-1), g, partial, s)
        lam = p.field(4)
        if Lam is None:
            lam.zero_()
        else:
            lam.copy_(Lam)
        hist = torch.empty((max(int(iters), 1), p.n_clouds), dtype=torch.float64, device=dev)
        ws = self.workspace()
        L.lskum_adjoint_iterate(p, U, g, lam, iters, hist, ws, s)
        total = torch.empty(2 * p.n_clouds, dtype=torch.float64, device=dev)
        L.lskum_adjoint_total(p, U, lam, Jb.view(-1), total, partial, ws, s)
        return {"total": total.view(p.n_clouds, 2), "partial": partial.view(p.n_clouds, 2),
                "Lambda": lam, "history": hist[:iters]}

    def residual(self, U: torch.Tensor, theta: torch.Tensor) -> torch.Tensor:
        return _ResidualFn.apply(U, theta, self)

    def force_coeffs(self, U: torch.Tensor, theta: torch.Tensor) -> torch.Tensor:
        """(n_clouds, 2): (Cl, Cd) of each cloud."""
        return _ForceFn.apply(U, theta, self)

    # plain kernel sequences used by the Functions
    def _residual(self, Ue: torch.Tensor) -> torch.Tensor:
        p, s = self.plan, self.stream
        q, dq, qlim, work, R = p.field(4), p.field(8), p.field(8), p.field(16), p.field(4)
        L.lskum_q_vars(p, Ue, q, s)
        L.lskum_q_derivs(p, q, dq, qlim, work, s)
        L.lskum_flux_residual(p, q, dq, qlim, R, s)
        return R


class _ResidualFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, theta, op: Adjoint):
        op.set_theta(theta)
        Ue = U.detach().contiguous().clone()
        L.lskum_set_far_field(op.plan, Ue, op.stream)
        R = op._residual(Ue)
        ctx.save_for_backward(Ue, theta.detach())
        ctx.op = op
        return R

    @staticmethod
    def backward(ctx, Rb):
        Ue, theta = ctx.saved_tensors
        op = ctx.op
        op.set_theta(theta)
        p = op.plan
        Ub = p.field(4)
        tb = torch.empty(2 * p.n_clouds, dtype=torch.float64, device=Ub.device)
        L.lskum_flux_residual_vjp(p, Ue, Rb.contiguous(), Ub, tb, op.workspace(), op.stream)
        return Ub, tb.view(theta.shape).to(theta.device), None


class _ForceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, theta, op: Adjoint):
        op.set_theta(theta)
        Uc = U.detach().contiguous()
        out = torch.empty(2 * op.n_clouds, dtype=torch.float64, device=Uc.device)
        L.lskum_force_coeffs(op.plan, Uc, out, op.stream)
        ctx.save_for_backward(Uc, theta.detach())
        ctx.op = op
        return out.view(op.n_clouds, 2)

    @staticmethod
    def backward(ctx, Jb):
        Uc, theta = ctx.saved_tensors
        op = ctx.op
        op.set_theta(theta)
        p = op.plan
        Ub = p.field(4)
        tb = torch.empty(2 * p.n_clouds, dtype=torch.float64, device=Ub.device)
        L.lskum_force_coeffs_vjp(p, Uc, Jb.contiguous().view(-1), Ub, tb, op.stream)
        return Ub, tb.view(theta.shape).to(theta.device), None
