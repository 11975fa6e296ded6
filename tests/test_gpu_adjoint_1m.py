"""The residual VJP on the 1M-point cloud (the adjoint workload's cloud and
flow: 1000 x 1000 NACA 0012 O-cloud, k_max 30, M 0.63, AoA 2 deg, three
inner sweeps) in the launch configuration the benchmark times, checked
against the oracle's reverse sweep on a cut of that cloud, and against
central finite differences of the GPU forward on the whole cloud.

The cut: the cotangent Rbar is non-zero only at a set I of sampled points
(random interior and wall points, trailing-edge wall points and points next
to the outer boundary).  Then Ubar = sum over i in I of (dR_i/dU)^T Rbar_i,
and every R_i, i in I, is the same function of U on the sub-cloud of the
points within n_inner + 2 stencil hops of I (cloudgen.shapes.restrict) as on
the whole cloud, so the oracle's VJP on the sub-cloud is the exact
reference for the GPU's Ubar at every sub-cloud point (and Ubar is zero
elsewhere).  The state is the free stream advanced 1000 iterations.
"""
import sys

import numpy as np
import pytest
import torch

from cloudgen import named_cloud
from cloudgen.shapes import restrict
from oracle.ref import Oracle
from paper_2403_13287_amd import lskum as L
from paper_2403_13287_amd.adjoint import Adjoint
from paper_2403_13287_amd.solver import Solver

pytestmark = pytest.mark.gpu

TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(g, r):
    out = []
    for gc, rc in zip(np.atleast_2d(g), np.atleast_2d(r)):
        s = np.max(np.abs(rc))
        out.append(np.max(np.abs(gc - rc)) / s if s > 0 else np.max(np.abs(gc)))
    return max(out)


@pytest.fixture(scope="module")
def state1m():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    say("generating the 1M cloud")
    c = named_cloud("1m")
    params = L.Params(0.63, 2.0, 0.2, 5.0, 3)
    s = Solver(c, params)
    graph, _ = s.capture(100, 10)
    say("1000 GPU iterations at 1M, M 0.63")
    for _ in range(10):
        graph.launch()
    torch.cuda.synchronize()
    assert s.status() == L.OK
    rng = np.random.default_rng(63)
    interior = np.nonzero(c.kind == 0)[0]
    wall = np.nonzero(c.kind == 1)[0]
    outer = np.nonzero(c.kind == 2)[0]
    te = wall[np.argsort(-c.x[wall])[:4]]
    # interior points that list an outer point among their neighbours
    col = c.col.reshape(c.n, c.k_pad)
    near_outer = interior[np.isin(col[interior], outer).any(axis=1)]
    samples = np.unique(np.concatenate([rng.choice(interior, 24, replace=False),
                                        rng.choice(wall, 8, replace=False), te,
                                        rng.choice(near_outer, 4, replace=False)]))
    return c, params, s, samples


def test_1m_vjp_on_a_cut_against_oracle(state1m):
    c, params, s, samples = state1m
    rng = np.random.default_rng(7)
    Rb = np.zeros((c.n, 4))
    Rb[samples] = rng.standard_normal((samples.size, 4))
    ad = Adjoint(c, params, plan=s.plan)
    Ub = s.plan.field(4)
    tb = torch.empty(2, dtype=torch.float64, device="cuda")
    L.lskum_flux_residual_vjp(s.plan, s.U, torch.from_numpy(Rb).cuda(), Ub, tb, ad.workspace())
    torch.cuda.synchronize()
    assert s.status() == L.OK
    sub, ids = restrict(c, samples, params.n_inner + 2)
    say(f"oracle VJP on the {sub.n}-point cut of {samples.size} samples")
    o = Oracle(sub, params.mach, params.aoa_deg, cfl=params.cfl, venkat_k=params.venkat_k,
               n_inner=params.n_inner)
    U_sub = s.U[torch.from_numpy(ids).cuda()].cpu().numpy().T
    Ub_o, tb_o, flags = o.residual_vjp(U_sub, Rb[ids].T)
    # points on the cut's outermost rings lose the neighbours outside it, so
    # some of their half-plane stencils are singular (the degenerate bit);
    # their residuals carry a zero cotangent and do not enter Ubar.  No
    # state may be non-physical.
    assert flags & ~2 == 0, flags
    Ub_g = Ub.cpu().numpy()
    e = normwise(Ub_g[ids].T, Ub_o)
    say("1M cut Ubar normwise", e, "theta", tb.cpu().numpy(), tb_o)
    assert e <= TOL
    outside = np.ones(c.n, bool)
    outside[ids] = False
    assert np.all(Ub_g[outside] == 0.0)
    assert np.any(tb_o != 0.0)  # the cut reaches the outer boundary
    np.testing.assert_allclose(tb.cpu().numpy(), tb_o, rtol=TOL, atol=TOL * np.max(np.abs(tb_o)))


def test_1m_vjp_finite_difference_columns(state1m):
    """Columns of the VJP (random cotangents on the whole cloud) at sampled
    points against central differences of the GPU forward residual over the
    whole cloud; components whose difference quotient changes between h and
    h/4 (a limiter or max/min switch inside the difference) are skipped."""
    c, params, s, samples = state1m
    ad = Adjoint(c, params, plan=s.plan)
    theta = ad.theta()
    rng = np.random.default_rng(8)
    Rb = torch.from_numpy(rng.standard_normal((c.n, 4))).cuda()
    U = s.U.clone()
    Uv = U.clone().requires_grad_(True)
    (Ub,) = torch.autograd.grad(ad.residual(Uv, theta), Uv, Rb)
    Ub = Ub.cpu().numpy()
    scale = np.abs(Ub).max()
    Uh = U.cpu().numpy()

    def fd(j, m, h):
        Up, Um = U.clone(), U.clone()
        Up[j, m] += h
        Um[j, m] -= h
        d = ad.residual(Up, theta) - ad.residual(Um, theta)
        return float((Rb * d).sum()) / (2 * h)

    pts = samples[c.kind[samples] != 2][:16]
    checked = kinks = 0
    worst = worst_excess = 0.0
    for j in pts:
        for m in range(4):
            h = 1e-6 * np.abs(Uh[:, m]).max()
            f1, f2 = fd(int(j), m, h), fd(int(j), m, h / 4)
            if abs(f1 - f2) > 1e-7 * scale:
                kinks += 1
                continue
            checked += 1
            # error of the h/4 quotient: truncation c h^2/16 = |f1 - f2|/15
            # when truncation dominates, rounding r(h/4) = 4 r(h), i.e.
            # 4/3 |f1 - f2|, when rounding does; the VJP must agree within
            # 2 |f1 - f2| plus a floor of 1e-8 of its scale
            err = abs(Ub[j, m] - f2)
            worst = max(worst, err / scale)
            worst_excess = max(worst_excess, (err - 2.0 * abs(f1 - f2)) / scale)
    say("1M FD columns: checked", checked, "kinks", kinks, "worst", worst,
        "worst beyond the FD's own error", worst_excess)
    assert checked >= 48
    assert worst <= 2e-7
    assert worst_excess <= 1e-8
