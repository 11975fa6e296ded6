"""GPU parity: the HIP library against the FP64 CPU oracle.

Tolerances (floating point, FP64 on both sides, different libm and FMA
contraction on the GPU):
* fields q, dq, qlim, R, U: normwise per component,
  max_i |gpu - oracle| / max_i |oracle| <= 1e-10, at every stage of the
  first two iterations and of the last one;
* residual-norm histories: relative 1e-8 while r_k / r_1 >= 1e-6;
* dt, rk stage, norms, force coefficients from identical inputs: 1e-12.
Split-stencil membership (an integer decision taken from floating point)
is computed with uncontracted products/sums on both sides, so it agrees
bit for bit.
"""
import math
import sys

import numpy as np
import pytest
import torch

from cloudgen.shapes import cylinder_cloud, from_lists
from cloudgen.workloads import WORKLOADS
from oracle.ref import Oracle
from paper_2403_13287_amd import lskum as L
from paper_2403_13287_amd.solver import Solver

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10
HIST_TOL = 1e-8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def up(a):
    """Oracle field (c, n) -> device field (n, c)."""
    return to_gpu(np.asarray(a).T)


def down(t):
    """Device field (n, c) -> oracle layout (c, n)."""
    return host(t).T


def normwise(gpu, ref_):
    gpu = np.atleast_2d(gpu)
    ref_ = np.atleast_2d(ref_)
    out = []
    for g, r in zip(gpu, ref_):
        scale = np.max(np.abs(r))
        err = np.max(np.abs(g - r))
        out.append(err / scale if scale > 0 else err)
    return max(out)


def assert_field(name, gpu, ref_, tol=FIELD_TOL):
    e = normwise(gpu, ref_)
    assert np.all(np.isfinite(gpu)), name
    assert e <= tol, f"{name}: normwise error {e:.3e} > {tol:.0e}"


def params_of(wl, **over):
    d = dict(mach=wl.mach, aoa_deg=wl.aoa_deg, cfl=wl.cfl, venkat_k=wl.venkat_k,
             n_inner=wl.n_inner, gamma=wl.gamma)
    d.update(over)
    return L.Params(**d)


def oracle_of(cloud, p: L.Params):
    return Oracle(cloud, p.mach, p.aoa_deg, cfl=p.cfl, venkat_k=p.venkat_k, n_inner=p.n_inner,
                  gamma=p.gamma)


@pytest.fixture(scope="module")
def tiny():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    wl = WORKLOADS["tiny"]
    return wl, wl.cloud()


def test_per_kernel_parity_tiny(tiny):
    wl, cloud = tiny
    for n_inner in (0, 1, 2, 3):
        say(f"per-kernel parity tiny n={cloud.n} n_inner={n_inner}")
        p = params_of(wl, n_inner=n_inner)
        o = oracle_of(cloud, p)
        U, _, _ = o.iterate(o.init_state(), 3)
        plan = L.Plan(cloud, p)
        Ug = up(U)
        q, dq, qlim, work, R = plan.field(4), plan.field(8), plan.field(8), plan.field(16), plan.field(4)
        L.lskum_q_vars(plan, Ug, q)
        qo, _ = o.q_vars(U)
        assert_field("q", down(q), qo)
        # derivatives from the oracle's own q: isolates the derivative kernels
        L.lskum_q_derivs(plan, up(qo), dq, qlim, work)
        dqo, qlimo = o.q_derivs(qo)
        assert_field("dq", down(dq), dqo)
        assert_field("qlim", down(qlim), qlimo, 1e-15)
        # flux kernel from the oracle's inputs
        L.lskum_flux_residual(plan, up(qo), up(dqo), up(qlimo), R)
        Ro, flags = o.flux_residual(qo, dqo, qlimo)
        assert flags == 0
        assert_field("R", down(R), Ro)
        assert L.lskum_status(plan) == L.OK
        plan.destroy()


def test_small_kernels_parity_tiny(tiny):
    wl, cloud = tiny
    p = params_of(wl)
    o = oracle_of(cloud, p)
    U, _, _ = o.iterate(o.init_state(), 3)
    plan = L.Plan(cloud, p)
    Ug = up(U)
    dt = plan.field(1)
    L.lskum_local_dt(plan, Ug, dt)
    dto = o.local_dt(U)
    np.testing.assert_allclose(host(dt), dto, rtol=1e-13)
    rng = np.random.Generator(np.random.PCG64(3))
    R = rng.normal(size=(4, cloud.n)) * 0.1
    Un = U * (1 + 1e-3 * rng.normal(size=U.shape))
    for s in range(4):
        Ug = up(U)
        L.lskum_rk_stage(plan, s, up(Un), up(R), to_gpu(dto), Ug)
        np.testing.assert_allclose(down(Ug), o.rk_stage(s, Un, R, dto, U), rtol=1e-13, atol=1e-15)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    L.lskum_residual_norm(plan, up(R), out)
    assert host(out)[0] == pytest.approx(o.residual_norm(R), rel=1e-12)
    L.lskum_force_coeffs(plan, up(U), out)
    np.testing.assert_allclose(host(out), o.force_coeffs(U), rtol=1e-11, atol=1e-14)
    Ui = plan.field(4)
    L.lskum_init_state(plan, Ui)
    np.testing.assert_allclose(down(Ui), o.init_state(), rtol=4e-16, atol=1e-16)


def _gpu_stages(plan, Ug, iters):
    """Stage-by-stage GPU driver through the individual entry points."""
    n = plan.n
    q, dq, qlim, work, R = plan.field(4), plan.field(8), plan.field(8), plan.field(16), plan.field(4)
    dt = plan.field(1)
    norm = torch.zeros(1, dtype=torch.float64, device="cuda")
    for it in range(iters):
        L.lskum_local_dt(plan, Ug, dt)
        Un = Ug.clone()
        for s in range(4):
            L.lskum_q_vars(plan, Ug, q)
            L.lskum_q_derivs(plan, q, dq, qlim, work)
            L.lskum_flux_residual(plan, q, dq, qlim, R)
            nv = None
            if s == 0:
                L.lskum_residual_norm(plan, R, norm)
                nv = float(host(norm)[0])
            L.lskum_rk_stage(plan, s, Un, R, dt, Ug)
            yield dict(it=it, stage=s, q=down(q), dq=down(dq), qlim=down(qlim), R=down(R),
                       dt=host(dt), U=down(Ug), norm=nv)


def _compare_stage(a, b, tag):
    for key in ("q", "dq", "R", "U"):
        assert_field(f"{tag} it{a['it']} stage{a['stage']} {key}", a[key], b[key])
    np.testing.assert_allclose(a["dt"], b["dt"], rtol=1e-12)
    if a["norm"] is not None:
        assert a["norm"] == pytest.approx(b["norm"], rel=HIST_TOL)


def test_stage_parity_first_two_and_last_iteration_tiny(tiny):
    wl, cloud = tiny
    p = params_of(wl)
    o = oracle_of(cloud, p)
    plan = L.Plan(cloud, p)
    U0 = o.init_state()
    say("stage parity: first two iterations")
    for a, b in zip(_gpu_stages(plan, up(U0), 2), o.stages(U0, 2)):
        _compare_stage(a, b, "first")
    # full run of wl.iters iterations: histories and the last iteration stage by stage
    say(f"full run: {wl.iters} iterations, oracle and lskum_iterate")
    last = wl.iters - 1
    Uo, hist_o, flags = o.iterate(U0, last)
    assert flags == 0
    Ug = up(U0)
    hist_g = torch.zeros(last, dtype=torch.float64, device="cuda")
    ws = L.workspace(plan)
    L.lskum_iterate(plan, last, Ug, hist_g, ws)
    hg = host(hist_g)
    ok = hist_o / hist_o[0] >= 1e-6
    np.testing.assert_allclose(hg[ok], hist_o[ok], rtol=HIST_TOL)
    assert np.all(np.abs(hg[~ok] - hist_o[~ok]) <= 1e-14 * hist_o[0])
    assert_field("U before last iteration", down(Ug), Uo)
    say("stage parity: last iteration")
    for a, b in zip(_gpu_stages(plan, Ug, 1), o.stages(Uo, 1)):
        _compare_stage(a, b, "last")
    assert L.lskum_status(plan) == L.OK


def test_solver_run_is_deterministic(tiny):
    wl, cloud = tiny
    p = params_of(wl)
    a, b = Solver(cloud, p), Solver(cloud, p)
    ha, hb = a.run(20), b.run(20)
    torch.cuda.synchronize()
    assert torch.equal(a.U, b.U) and torch.equal(ha, hb)
    assert a.status() == L.OK


def test_parity_1m_bench_configuration():
    """The 1M-point workload in the launch configuration the benchmark
    times (lskum_iterate), then every kernel on the state it produced, and
    one more whole iteration through lskum_iterate (local time step and the
    four fused flux + SSP stage launches) against the oracle's iteration
    from the same state."""
    wl = WORKLOADS["1m"]
    say("generating the 1M cloud")
    cloud = wl.cloud()
    p = params_of(wl)
    s = Solver(cloud, p)
    say("5 GPU iterations at 1M")
    s.run(5)
    U5 = down(s.U)
    q, dq, qlim, R = s.residual()
    o = oracle_of(cloud, p)
    say("oracle residual at 1M")
    qo, _ = o.q_vars(U5)
    dqo, qlimo = o.q_derivs(qo)
    Ro, flags = o.flux_residual(qo, dqo, qlimo)
    assert flags == 0
    assert_field("q 1M", down(q), qo)
    assert_field("dq 1M", down(dq), dqo)
    assert_field("R 1M", down(R), Ro)
    # the next iteration's history entry is the norm of R(U5)
    h = s.run(1)
    assert float(host(h)[0]) == pytest.approx(o.residual_norm(Ro), rel=HIST_TOL)
    say("oracle iteration at 1M")
    U6o, h6o, flags = o.iterate(U5, 1)
    assert flags == 0
    assert float(host(h)[0]) == pytest.approx(h6o[0], rel=HIST_TOL)
    U6 = down(s.U)
    assert_field("U after one lskum_iterate iteration at 1M", U6, U6o)
    assert normwise(U6 - U5, U6o - U5) <= 1e-8  # the increment itself, not only the state
    dt = s.plan.field(1)
    L.lskum_local_dt(s.plan, up(U5), dt)
    np.testing.assert_allclose(host(dt), o.local_dt(U5), rtol=1e-12)
    assert s.status() == L.OK


@pytest.mark.timeout(600)
def test_parity_1m_developed_state():
    """The 1M-point workload at the benchmark's input state (the free stream
    advanced 500 iterations through lskum_iterate, where every limiter is
    active): q, dq, qlim and R of that state, then one more lskum_iterate
    iteration, against the oracle on the whole cloud from the same state."""
    wl = WORKLOADS["1m"]
    say("generating the 1M cloud")
    cloud = wl.cloud()
    p = params_of(wl)
    s = Solver(cloud, p)
    say("500 GPU iterations at 1M")
    s.run(500)
    assert s.status() == L.OK
    U0 = down(s.U)
    q, dq, qlim, R = s.residual()
    o = oracle_of(cloud, p)
    say("oracle residual at the developed 1M state")
    qo, _ = o.q_vars(U0)
    dqo, qlimo = o.q_derivs(qo)
    Ro, flags = o.flux_residual(qo, dqo, qlimo)
    assert flags == 0
    assert_field("q 1M developed", down(q), qo)
    assert_field("dq 1M developed", down(dq), dqo)
    assert_field("qlim 1M developed", down(qlim), qlimo)
    assert_field("R 1M developed", down(R), Ro)
    say("oracle iteration from the developed 1M state")
    h = s.run(1)
    U1o, h1o, flags = o.iterate(U0, 1)
    assert flags == 0
    assert float(host(h)[0]) == pytest.approx(h1o[0], rel=HIST_TOL)
    U1 = down(s.U)
    assert_field("U after one iteration from the developed 1M state", U1, U1o)
    assert normwise(U1 - U0, U1o - U0) <= 1e-8
    assert s.status() == L.OK


@pytest.mark.timeout(600)
def test_parity_16m_sampled_points():
    """The 16M-point workload after 2 GPU iterations: q, dq, qlim and R at
    sampled points (random interior and wall points, and the wall points
    at the trailing edge, where the wall spacing is finest) against the
    oracle on the sub-cloud within n_inner + 2 hops of the samples, which
    reproduces their values exactly."""
    from cloudgen.shapes import restrict
    wl = WORKLOADS["16m"]
    say("generating the 16M cloud")
    cloud = wl.cloud()
    p = params_of(wl)
    s = Solver(cloud, p)
    say("2 GPU iterations at 16M")
    s.run(2)
    q, dq, qlim, R = s.residual()
    assert s.status() == L.OK
    rng = np.random.default_rng(16)
    wall = np.nonzero(cloud.kind == 1)[0]
    te = wall[np.argsort(-cloud.x[wall])[:6]]
    samples = np.unique(np.concatenate([
        rng.choice(np.nonzero(cloud.kind == 0)[0], 48, replace=False),
        rng.choice(wall, 16, replace=False), te]))
    sub, ids = restrict(cloud, samples, p.n_inner + 2)
    say(f"oracle on the {sub.n}-point sub-cloud of {samples.size} samples")
    pos = np.searchsorted(ids, samples)
    idx = torch.from_numpy(ids).cuda()
    U_sub = host(s.U[idx]).T
    o = oracle_of(sub, p)
    qo, _ = o.q_vars(U_sub)
    dqo, qlimo = o.q_derivs(qo)
    Ro, _ = o.flux_residual(qo, dqo, qlimo)
    sidx = torch.from_numpy(samples).cuda()
    assert_field("q 16M", host(q[sidx]).T, qo[:, pos])
    assert_field("dq 16M", host(dq[sidx]).T, dqo[:, pos])
    assert_field("qlim 16M", host(qlim[sidx]).T, qlimo[:, pos])
    assert_field("R 16M", host(R[sidx]).T, Ro[:, pos])
    # the fused flux + SSP stage launch the iteration driver uses: the
    # first stage from this state, with its local time step
    say("fused stage at 16M")
    dt = s.plan.field(1)
    L.lskum_local_dt(s.plan, s.U, dt)
    Un, U1, R1, qn = s.U.clone(), s.U.clone(), s.plan.field(4), s.plan.field(4)
    L.lskum_flux_residual_stage(s.plan, 0, q, dq, qlim, Un, dt, R1, U1, qn)
    assert s.status() == L.OK
    dto = o.local_dt(U_sub)
    np.testing.assert_allclose(host(dt[sidx]), dto[pos], rtol=1e-12)
    U1o = o.rk_stage(0, U_sub, Ro, dto, U_sub)
    q1o, _ = o.q_vars(U1o)
    assert_field("R fused 16M", host(R1[sidx]).T, Ro[:, pos])
    assert_field("U stage 16M", host(U1[sidx]).T, U1o[:, pos])
    assert_field("U stage increment 16M", host(U1[sidx] - Un[sidx]).T, (U1o - U_sub)[:, pos], 1e-8)
    assert_field("q next stage 16M", host(qn[sidx]).T, q1o[:, pos])


@pytest.mark.parametrize("block", [128, 256])
def test_parity_without_hilbert_order(block):
    """An airfoil cloud left in its O-grid (layer-by-layer) order: the halos
    of 256-point tiles span several layers and exceed the LDS tables, so the
    derivative passes gather directly; with 128-point tiles the first-order
    pass fits its table and the inner sweeps do not.  Both paths must give
    the oracle's fields."""
    from cloudgen import make_airfoil_cloud
    c = make_airfoil_cloud(200, 40, 25, 21, reorder=False)
    p = L.Params(0.6, 2.0, n_inner=3)
    o = oracle_of(c, p)
    Uo, ho, flags = o.iterate(o.init_state(), 3)
    assert flags == 0
    s = Solver(c, p, tuning=L.Tuning(block, 1))
    hg = s.run(3)
    np.testing.assert_allclose(host(hg), ho, rtol=HIST_TOL)
    assert_field("U unordered", down(s.U), Uo)
    q, dq, qlim, R = s.residual()
    qo, _ = o.q_vars(Uo)
    dqo, qlimo = o.q_derivs(qo)
    Ro, _ = o.flux_residual(qo, dqo, qlimo)
    assert_field("dq unordered", down(dq), dqo)
    assert_field("qlim unordered", down(qlim), qlimo)
    assert_field("R unordered", down(R), Ro)


@pytest.mark.parametrize("M,Lr", [(24, 8), (32, 8), (48, 12)])  # 192, 256, 576 points
def test_small_and_ragged_clouds_with_garbage_padding(M, Lr):
    c = cylinder_cloud(M=M, L=Lr)
    say(f"cylinder cloud n={c.n}")
    col = c.col.reshape(c.n, c.k_pad).copy()
    for i in range(c.n):
        col[i, c.nbr_count[i]:] = -7 - i  # pad entries are never read
    cg = from_lists(c.x, c.y, c.nx, c.ny, c.kind, [c.neighbours(i) for i in range(c.n)],
                    wall_loop=c.wall_loop, k_pad=c.k_pad)
    cg.col = col.reshape(-1)
    p = L.Params(0.4, 3.0, n_inner=2)
    o = oracle_of(c, p)
    Uo, ho, flags = o.iterate(o.init_state(), 4)
    assert flags == 0
    s = Solver(cg, p)
    hg = s.run(4)
    np.testing.assert_allclose(host(hg), ho, rtol=HIST_TOL)
    assert_field("U cylinder", down(s.U), Uo)
    _, _, _, R = s.residual()
    Ro, _ = o.residual(Uo)
    assert_field("R cylinder", down(R), Ro)


def test_nonphysical_state_sets_status(tiny):
    wl, cloud = tiny
    plan = L.Plan(cloud, params_of(wl))
    U = plan.field(4)
    L.lskum_init_state(plan, U)
    assert L.lskum_status(plan) == L.OK
    U[77, 3] = 0.0  # E = 0 -> p < 0
    q = plan.field(4)
    L.lskum_q_vars(plan, U, q)
    assert L.lskum_status(plan) == L.ERR_NONPHYSICAL
    L.lskum_clear_status(plan)
    assert L.lskum_status(plan) == L.OK


def test_degenerate_stencil_sets_status():
    x = [0.0, 1.0, 1.0, 2.0, 1.5, 1.2]
    y = [0.0, 1.0, -1.0, 0.3, -0.4, 0.1]
    nb = [[1, 2, 3, 4, 5]] + [[j for j in range(6) if j != k] for k in range(1, 6)]
    c = from_lists(x, y, [0] * 6, [1] * 6, [0, 2, 2, 2, 2, 2], nb)
    p = L.Params(0.5, 0.0)
    plan = L.Plan(c, p)
    o = oracle_of(c, p)
    U = o.init_state()
    U[0, 3] *= 1.1
    q, dq, qlim, work, R = plan.field(4), plan.field(8), plan.field(8), plan.field(16), plan.field(4)
    L.lskum_q_vars(plan, up(U), q)
    L.lskum_q_derivs(plan, q, dq, qlim, work)
    L.lskum_flux_residual(plan, q, dq, qlim, R)
    assert L.lskum_status(plan) == L.ERR_DEGENERATE
    Ro, flags = o.residual(U)
    assert_field("R degenerate", down(R), Ro)
