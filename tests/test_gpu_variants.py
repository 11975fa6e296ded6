"""Scheme options on the GPU against the oracle: the first-order flux, the
min-max limiter and classical RK4 time stepping, on the 9,600-point cloud at
the workload's flow and on the supersonic case (3 iterations; fields
normwise 1e-10, histories 1e-8).  The adjoint entry points refuse the two
residual options."""
import sys

import numpy as np
import pytest
import torch

from cloudgen import named_cloud
from oracle.ref import RK4, Oracle
from paper_2403_13287_amd import lskum as L
from paper_2403_13287_amd.solver import Solver

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(g, r):
    return max(np.max(np.abs(gc - rc)) / np.max(np.abs(rc)) for gc, rc in zip(g, r))


@pytest.fixture(scope="module")
def tiny():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return named_cloud("tiny")


@pytest.mark.parametrize("options", [L.FIRST_ORDER, L.MINMAX, L.FIRST_ORDER | L.MINMAX, L.RK4,
                                     L.RK4 | L.MINMAX])
@pytest.mark.parametrize("mach,aoa", [(0.63, 2.0), (1.2, 0.0)])
def test_variant_parity(tiny, options, mach, aoa):
    c = tiny
    o = Oracle(c, mach, aoa, n_inner=2, options=options)
    Uo, ho, flags = o.iterate(o.init_state(), 3)
    assert flags == 0
    s = Solver(c, L.Params(mach, aoa, n_inner=2, options=options))
    hg = s.run(3)
    torch.cuda.synchronize()
    assert s.status() == L.OK
    np.testing.assert_allclose(hg.cpu().numpy(), ho, rtol=1e-8)
    e = normwise(s.U.cpu().numpy().T, Uo)
    _, _, _, R = s.residual()
    Ro, _ = o.residual(Uo)
    eR = normwise(R.cpu().numpy().T, Ro)
    say("options", options, "M", mach, "U", e, "R", eR)
    assert e <= 1e-10 and eR <= 1e-10


@pytest.mark.parametrize("gamma", [1.3, 5.0 / 3.0])
def test_general_gamma_parity(tiny, gamma):
    """A ratio of specific heats other than 1.4 runs the flux kernel compiled
    for a general gamma (the end states' density through a log): 3
    iterations against the oracle at that gamma, SSP and RK4 stepping."""
    c = tiny
    for options in (0, L.RK4):
        o = Oracle(c, 0.63, 2.0, n_inner=2, gamma=gamma, options=options)
        Uo, ho, flags = o.iterate(o.init_state(), 3)
        assert flags == 0
        s = Solver(c, L.Params(0.63, 2.0, n_inner=2, gamma=gamma, options=options))
        hg = s.run(3)
        torch.cuda.synchronize()
        assert s.status() == L.OK
        np.testing.assert_allclose(hg.cpu().numpy(), ho, rtol=1e-8)
        e = normwise(s.U.cpu().numpy().T, Uo)
        _, _, _, R = s.residual()
        Ro, _ = o.residual(Uo)
        eR = normwise(R.cpu().numpy().T, Ro)
        say("gamma", gamma, "options", options, "U", e, "R", eR)
        assert e <= 1e-10 and eR <= 1e-10


def test_adjoint_refuses_variants(tiny):
    plan = L.Plan(tiny, L.Params(0.63, 2.0, options=L.MINMAX))
    U = plan.field(4)
    L.lskum_init_state(plan, U)
    tb = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LskumError):
        L.lskum_flux_residual_vjp(plan, U, U.clone(), plan.field(4), tb, L.vjp_workspace(plan))


def test_rk4_stage_entry_point(tiny):
    """lskum_rk4_stage called stage by stage with arbitrary residuals (the
    accumulator carried between calls) against the oracle's textbook
    stages, which keep every stage residual."""
    assert L.RK4 == RK4
    c = tiny
    o = Oracle(c, 0.63, 2.0, options=RK4)
    plan = L.Plan(c, L.Params(0.63, 2.0, options=L.RK4))
    rng = np.random.Generator(np.random.PCG64(21))
    Un = o.init_state() * (1 + 0.01 * rng.normal(size=(4, c.n)))
    Rs = [rng.normal(size=(4, c.n)) for _ in range(4)]
    dt = np.full(c.n, 1e-3) * (1 + rng.random(c.n))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a.T)).cuda()  # noqa: E731
    Ung, dtg = dev(Un), torch.from_numpy(dt).cuda()
    Ug, acc = Ung.clone(), plan.field(4)
    Uo = Un.copy()
    for s in range(4):
        L.lskum_rk4_stage(plan, s, Ung, dev(Rs[s]), dtg, acc, Ug)
        Uo = o.rk4_stage(s, Un, Rs, dt, Uo)
        torch.cuda.synchronize()
        e = normwise(Ug.cpu().numpy().T, Uo)
        say("rk4 stage", s, e)
        assert e <= 1e-14


def test_rk4_graph_replays(tiny):
    """Graph-captured RK4 iterations (two replays of two) against the oracle's
    four iterations."""
    c = tiny
    o = Oracle(c, 0.63, 2.0, n_inner=2, options=RK4)
    Uo, ho, flags = o.iterate(o.init_state(), 4)
    assert flags == 0
    s = Solver(c, L.Params(0.63, 2.0, n_inner=2, options=L.RK4))
    graph, hist = s.capture(2, 2)
    for _ in range(2):
        graph.launch()
        torch.cuda.synchronize()
    assert s.status() == L.OK
    np.testing.assert_allclose(hist[:, 0].cpu().numpy(), ho, rtol=1e-8)
    e = normwise(s.U.cpu().numpy().T, Uo)
    say("rk4 graph: U", e)
    assert e <= 1e-10


def test_rk4_adjoint_accepted(tiny):
    """RK4 changes the time stepping only: the residual VJP of an RK4 plan
    equals that of the default plan."""
    pa = L.Plan(tiny, L.Params(0.63, 2.0, options=L.RK4))
    pb = L.Plan(tiny, L.Params(0.63, 2.0))
    U = pa.field(4)
    L.lskum_init_state(pa, U)
    U = U * (1 + 0.01 * torch.randn(U.shape, dtype=torch.float64, device=U.device,
                                    generator=torch.Generator(device=U.device).manual_seed(5)))
    L.lskum_set_far_field(pa, U)
    Rb = torch.randn(U.shape, dtype=torch.float64, device=U.device,
                     generator=torch.Generator(device=U.device).manual_seed(6))
    out = []
    for p in (pa, pb):
        Ub, tb = p.field(4), torch.empty(2, dtype=torch.float64, device=U.device)
        L.lskum_flux_residual_vjp(p, U, Rb, Ub, tb, L.vjp_workspace(p))
        out.append((Ub, tb))
    torch.cuda.synchronize()
    eU = (out[0][0] - out[1][0]).abs().max() / out[1][0].abs().max()
    et = (out[0][1] - out[1][1]).abs().max() / out[1][1].abs().max()
    say("rk4 vjp vs default:", float(eU), float(et))
    assert eU <= 1e-14 and et <= 1e-14


def test_rk4_and_ssp_reach_the_same_steady_state():
    """The time integrator changes the path in pseudo-time, not the steady
    state R(U) = 0: SSPRK(4,3) and classical RK4 from the free stream on the
    10,000-point cloud (M 0.63, AoA 2 deg), 50,000 iterations each.  At
    CFL 0.2 the two stability polynomials differ only in their z^4 terms,
    so the transients agree closely but not bit for bit."""
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = named_cloud("10k")
    runs = {}
    for name, opt in (("ssp", 0), ("rk4", L.RK4)):
        s = Solver(c, L.Params(0.63, 2.0, n_inner=3, options=opt))
        graph, hist = s.capture(1000, 50)
        for _ in range(50):
            graph.launch()
        torch.cuda.synchronize()
        assert s.status() == L.OK
        h = hist[:, 0].cpu().numpy()
        runs[name] = (h, s.U.cpu().numpy(), s.force_coeffs().cpu().numpy())
        say(name, "residual", h[0], "->", h[-1], "Cl Cd", runs[name][2])
    (h0, U0, c0), (h1, U1, c1) = runs["ssp"], runs["rk4"]
    for h in (h0, h1):
        assert np.all(np.isfinite(h)) and h[-1] < 1e-4 * h[0]
    assert np.max(np.abs(h1 - h0) / h0) > 1e-12  # two different integrators
    e = normwise(U1.T, U0.T)
    say("steady U normwise", e, "Cl Cd", np.abs(c1 - c0) / np.abs(c0))
    assert e <= 1e-8
    np.testing.assert_allclose(c1, c0, rtol=1e-8)
