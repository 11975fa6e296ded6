"""Adjoints on the GPU: the hand-written VJPs against the oracle's reverse
sweep and against central finite differences of the GPU forward.

Tolerances:
* GPU VJP vs oracle tape VJP at the same state and cotangent: normwise per
  component 1e-10 (FP64 both sides; the passes sum in different orders);
  theta cotangents relative 1e-10;
* finite differences (h = 1e-6 relative to each component's scale):
  per-component columns of the residual VJP to 5e-8 of the gradient's norm,
  skipping components whose difference quotient changes between h and h/4
  (the stencil of the difference crosses a limiter or max/min switch, where
  the residual is not differentiable); theta and the force coefficients
  (smooth in their arguments) relative 1e-7.
"""
import sys

import numpy as np
import pytest
import torch

from cloudgen import make_airfoil_cloud, named_cloud
from cloudgen.shapes import cylinder_cloud
from oracle.ref import Oracle
from paper_2403_13287_amd import lskum as L
from paper_2403_13287_amd.adjoint import Adjoint
from paper_2403_13287_amd.solver import Solver

pytestmark = pytest.mark.gpu

TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def up(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T, np.float64)).cuda()


def down(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().T


def normwise(g, r):
    out = []
    for gc, rc in zip(np.atleast_2d(g), np.atleast_2d(r)):
        s = np.max(np.abs(rc))
        out.append(np.max(np.abs(gc - rc)) / s if s > 0 else np.max(np.abs(gc)))
    return max(out)


CASES = {  # name: (cloud factory, mach, aoa_deg, n_inner, oracle iterations)
    "airfoil-40x16": (lambda: make_airfoil_cloud(40, 16, 25, 3), 0.6, 2.0, 2, 20),
    "airfoil-40x16-first-order": (lambda: make_airfoil_cloud(40, 16, 25, 3), 0.6, 2.0, 0, 20),
    "airfoil-64x40": (lambda: make_airfoil_cloud(64, 40, 25, 12), 0.7, 3.0, 3, 10),
    "cylinder-32x8": (lambda: cylinder_cloud(32, 8), 0.4, 3.0, 2, 10),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    make, mach, aoa, ni, iters = CASES[request.param]
    c = make()
    o = Oracle(c, mach, aoa, n_inner=ni)
    U, _, flags = o.iterate(o.init_state(), iters)
    assert flags == 0
    params = L.Params(mach, aoa, n_inner=ni)
    say("case", request.param, "n", c.n)
    return request.param, c, o, U, params


def test_residual_vjp_matches_oracle(case):
    name, c, o, U, params = case
    rng = np.random.default_rng(11)
    Rb = rng.standard_normal((4, c.n))
    Ub_o, tb_o, flags = o.residual_vjp(U, Rb)
    assert flags == 0
    plan = L.Plan(c, params)
    Ub = plan.field(4)
    tb = torch.empty(2, dtype=torch.float64, device="cuda")
    L.lskum_flux_residual_vjp(plan, up(U), up(Rb), Ub, tb, L.vjp_workspace(plan))
    assert L.lskum_status(plan) == L.OK
    Ub_g = down(Ub)
    assert np.all(np.isfinite(Ub_g))
    assert np.all(Ub_g[:, c.kind == 2] == 0.0)
    e = normwise(Ub_g, Ub_o)
    say(name, "Ubar normwise", e)
    assert e <= TOL
    np.testing.assert_allclose(tb.cpu().numpy(), tb_o, rtol=TOL, atol=0)


def test_force_vjp_matches_oracle(case):
    name, c, o, U, params = case
    if c.wall_loop.size == 0:
        pytest.skip("no wall")
    Jb = np.array([0.8, -1.7])
    Ub_o, tb_o = o.force_coeffs_vjp(U, Jb)
    plan = L.Plan(c, params)
    Ub = plan.field(4)
    tb = torch.empty(2, dtype=torch.float64, device="cuda")
    L.lskum_force_coeffs_vjp(plan, up(U), torch.tensor(Jb, device="cuda"), Ub, tb)
    assert normwise(down(Ub), Ub_o) <= 1e-12
    np.testing.assert_allclose(tb.cpu().numpy(), tb_o, rtol=1e-12)


@pytest.fixture(scope="module")
def cut10k():
    """The 10k-point cloud (100 wall points x 100 layers) at M 0.63, AoA 2,
    three inner sweeps, advanced 300 iterations on the GPU."""
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = named_cloud("10k")
    params = L.Params(0.63, 2.0, n_inner=3)
    s = Solver(c, params)
    s.run(300)
    assert s.status() == L.OK
    return c, params, s.U.clone()


def test_10k_vjp_matches_oracle(cut10k):
    c, params, U = cut10k
    o = Oracle(c, params.mach, params.aoa_deg, n_inner=params.n_inner)
    rng = np.random.default_rng(7)
    Rb = rng.standard_normal((4, c.n))
    Ub_o, tb_o, flags = o.residual_vjp(down(U), Rb)
    assert flags == 0
    ad = Adjoint(c, params)
    Ub = ad.plan.field(4)
    tb = torch.empty(2, dtype=torch.float64, device="cuda")
    L.lskum_flux_residual_vjp(ad.plan, U, up(Rb), Ub, tb, ad.workspace())
    e = normwise(down(Ub), Ub_o)
    say("10k Ubar normwise", e, "theta", tb.cpu().numpy(), tb_o)
    assert e <= TOL
    np.testing.assert_allclose(tb.cpu().numpy(), tb_o, rtol=TOL)


def test_adjoint_total_is_partial_minus_theta_cotangent(cut10k):
    """lskum_adjoint_total on an arbitrary adjoint field Lambda: the same
    values as the two VJP entry points it combines (bit for bit) and the
    oracle's partial minus its residual theta cotangent."""
    c, params, U = cut10k
    ad = Adjoint(c, params)
    rng = np.random.default_rng(21)
    Lam = torch.from_numpy(rng.standard_normal((c.n, 4))).cuda()
    Jb = torch.tensor([0.7, -1.9], dtype=torch.float64, device="cuda")
    ws = ad.workspace()
    total = torch.empty(2, dtype=torch.float64, device="cuda")
    partial = torch.empty(2, dtype=torch.float64, device="cuda")
    L.lskum_adjoint_total(ad.plan, U, Lam, Jb, total, partial, ws)
    Fb, fb = ad.plan.field(4), torch.empty(2, dtype=torch.float64, device="cuda")
    L.lskum_force_coeffs_vjp(ad.plan, U, Jb, Fb, fb)
    Ub, tb = ad.plan.field(4), torch.empty(2, dtype=torch.float64, device="cuda")
    L.lskum_flux_residual_vjp(ad.plan, U, Lam, Ub, tb, ws)
    torch.cuda.synchronize()
    assert torch.equal(partial, fb)
    assert torch.equal(total, fb - tb)
    o = Oracle(c, params.mach, params.aoa_deg, n_inner=params.n_inner)
    Uh = down(U)
    _, part_o = o.force_coeffs_vjp(Uh, Jb.cpu().numpy())
    _, tr_o, flags = o.residual_vjp(Uh, down(Lam))
    assert flags == 0
    np.testing.assert_allclose(total.cpu().numpy(), part_o - tr_o,
                               rtol=TOL, atol=TOL * np.max(np.abs(tr_o)))
    # outputs overlapping an input are rejected
    lib = ad.plan.lib
    assert lib.lskum_adjoint_total(ad.plan.handle, U.data_ptr(), Lam.data_ptr(), Jb.data_ptr(),
                                   Jb.data_ptr(), None, ws.data_ptr(), None) == L.ERR_INVALID_ARG
    assert lib.lskum_adjoint_total(ad.plan.handle, U.data_ptr(), Lam.data_ptr(), Jb.data_ptr(),
                                   total.data_ptr(), total.data_ptr(), ws.data_ptr(),
                                   None) == L.ERR_INVALID_ARG


def test_10k_vjp_finite_difference_columns(cut10k):
    c, params, U = cut10k
    ad = Adjoint(c, params)
    theta = ad.theta()
    rng = np.random.default_rng(8)
    Rb = torch.from_numpy(rng.standard_normal((c.n, 4))).cuda()
    Uv = U.clone().requires_grad_(True)
    R = ad.residual(Uv, theta)
    (Ub,) = torch.autograd.grad(R, Uv, Rb)
    Ub = Ub.cpu().numpy()
    scale = np.abs(Ub).max()
    Uh = U.cpu().numpy()

    def fd(j, m, h):
        Up, Um = U.clone(), U.clone()
        Up[j, m] += h
        Um[j, m] -= h
        d = ad.residual(Up, theta) - ad.residual(Um, theta)
        return float((Rb * d).sum()) / (2 * h)

    wall = np.nonzero(c.kind == 1)[0]
    interior = np.nonzero(c.kind == 0)[0]
    pts = np.concatenate([rng.choice(wall, 10, replace=False),
                          rng.choice(interior, 30, replace=False)])
    checked = kinks = 0
    worst = 0.0
    for j in pts:
        for m in range(4):
            h = 1e-6 * np.abs(Uh[:, m]).max()
            f1, f2 = fd(j, m, h), fd(j, m, h / 4)
            if abs(f1 - f2) > 1e-7 * scale:
                kinks += 1
                continue
            checked += 1
            worst = max(worst, abs(Ub[j, m] - f2) / scale)
    say("10k FD columns: checked", checked, "kinks", kinks, "worst", worst)
    assert checked >= 140 and kinks <= 20
    assert worst <= 5e-8


def test_10k_theta_and_force_finite_differences(cut10k):
    c, params, U = cut10k
    ad = Adjoint(c, params)
    theta0 = ad.theta()
    rng = np.random.default_rng(9)
    Rb = torch.from_numpy(rng.standard_normal((c.n, 4))).cuda()
    Jb = torch.tensor([[1.3, -0.4]], dtype=torch.float64, device="cuda")
    th = theta0.clone().requires_grad_(True)
    Uv = U.clone().requires_grad_(True)
    Lr = (ad.residual(Uv, th) * Rb).sum()
    g_th_r, = torch.autograd.grad(Lr, th)
    Lf = (ad.force_coeffs(Uv, th) * Jb).sum()
    g_u_f, g_th_f = torch.autograd.grad(Lf, (Uv, th))
    h = 1e-6
    for k in range(2):
        dth = torch.zeros_like(theta0)
        dth[0, k] = h
        fr = float(((ad.residual(U, theta0 + dth) - ad.residual(U, theta0 - dth)) * Rb).sum()) / (2 * h)
        ff = float(((ad.force_coeffs(U, theta0 + dth) - ad.force_coeffs(U, theta0 - dth)) * Jb).sum()) / (2 * h)
        say("theta", k, float(g_th_r[0, k]), fr, float(g_th_f[0, k]), ff)
        assert float(g_th_r[0, k]) == pytest.approx(fr, rel=1e-7)
        assert float(g_th_f[0, k]) == pytest.approx(ff, rel=1e-7)
    v = torch.from_numpy(rng.standard_normal((c.n, 4))).cuda() * U.abs().amax(dim=0)
    ff = float(((ad.force_coeffs(U + h * v, theta0) - ad.force_coeffs(U - h * v, theta0)) * Jb).sum()) / (2 * h)
    assert float((g_u_f * v).sum()) == pytest.approx(ff, rel=1e-7)


def test_residual_vjp_deterministic_and_tuning_invariant(cut10k):
    c, params, U = cut10k
    rng = np.random.default_rng(3)
    Rb = torch.from_numpy(rng.standard_normal((c.n, 4))).cuda()
    ref = None
    for t in L.TUNING_SPACE:
        ad = Adjoint(c, params, tuning=t)
        for _ in range(2):
            Ub = ad.plan.field(4)
            tb = torch.empty(2, dtype=torch.float64, device="cuda")
            L.lskum_flux_residual_vjp(ad.plan, U, Rb, Ub, tb, ad.workspace())
            torch.cuda.synchronize()
            if ref is None:
                ref = (Ub.clone(), tb.clone())
            else:
                assert torch.equal(Ub, ref[0]) and torch.equal(tb, ref[1]), t


def test_batch_vjp_equals_single_clouds():
    clouds = [make_airfoil_cloud(40, 16, 25, 3), make_airfoil_cloud(96, 24, 25, 14),
              make_airfoil_cloud(50, 30, 25, 13)]
    params = [L.Params(0.6, 2.0), L.Params(0.4, 3.0), L.Params(0.75, -1.0)]
    batch = Solver(clouds, params)
    batch.run(5)
    rng = np.random.default_rng(4)
    Rb = torch.from_numpy(rng.standard_normal((batch.n, 4))).cuda()
    Jb = torch.from_numpy(rng.standard_normal((len(clouds), 2))).cuda()
    Ub = batch.plan.field(4)
    tb = torch.empty(2 * len(clouds), dtype=torch.float64, device="cuda")
    L.lskum_flux_residual_vjp(batch.plan, batch.U, Rb, Ub, tb, L.vjp_workspace(batch.plan))
    Fb = batch.plan.field(4)
    fb = torch.empty(2 * len(clouds), dtype=torch.float64, device="cuda")
    L.lskum_force_coeffs_vjp(batch.plan, batch.U, Jb, Fb, fb)
    for k, (c, p) in enumerate(zip(clouds, params)):
        sl = batch.plan.cloud_slice(k)
        plan = L.Plan(c, p)
        U = batch.U[sl].contiguous()
        u1 = plan.field(4)
        t1 = torch.empty(2, dtype=torch.float64, device="cuda")
        L.lskum_flux_residual_vjp(plan, U, Rb[sl].contiguous(), u1, t1, L.vjp_workspace(plan))
        f1 = plan.field(4)
        g1 = torch.empty(2, dtype=torch.float64, device="cuda")
        L.lskum_force_coeffs_vjp(plan, U, Jb[k].contiguous(), f1, g1)
        torch.cuda.synchronize()
        assert torch.equal(Ub[sl], u1) and torch.equal(tb[2 * k:2 * k + 2], t1), k
        assert torch.equal(Fb[sl], f1) and torch.equal(fb[2 * k:2 * k + 2], g1), k


@pytest.mark.parametrize("block", [128, 256])
def test_residual_vjp_without_hilbert_order(block):
    """An airfoil cloud left in its O-grid (layer-by-layer) order: the tile
    tables of the in-edge rows fit the LDS budget with 128-point tiles (76 KB
    for the first-order reverse) but not with 256-point tiles (111 KB), where
    the transposed derivative gathers take their direct-gather path (as do
    the forward passes of the recompute).  Both must match the oracle."""
    c = make_airfoil_cloud(200, 40, 25, 21, reorder=False)
    o = Oracle(c, 0.6, 2.0, n_inner=3)
    U, _, flags = o.iterate(o.init_state(), 10)
    assert flags == 0
    rng = np.random.default_rng(17)
    Rb = rng.standard_normal((4, c.n))
    Ub_o, tb_o, flags = o.residual_vjp(U, Rb)
    assert flags == 0
    plan = L.Plan(c, L.Params(0.6, 2.0, n_inner=3), tuning=L.Tuning(block, 1))
    Ub = plan.field(4)
    tb = torch.empty(2, dtype=torch.float64, device="cuda")
    L.lskum_flux_residual_vjp(plan, up(U), up(Rb), Ub, tb, L.vjp_workspace(plan))
    assert L.lskum_status(plan) == L.OK
    e = normwise(down(Ub), Ub_o)
    say("unordered", block, "Ubar normwise", e)
    assert e <= TOL
    np.testing.assert_allclose(tb.cpu().numpy(), tb_o, rtol=TOL, atol=0)
