"""Batched plans, launch tuning and graph replays (GPU).

A batch concatenates clouds; every kernel computes each point from the
same inputs in the same order as a single-cloud plan, and the residual
norms use the same per-cloud chunking, so a cloud advanced inside a batch
must match the same cloud advanced alone bit for bit -- for every tuning
and through graph replays.  One batch member is also checked against the
oracle.
"""
import math
import sys

import numpy as np
import pytest
import torch

from cloudgen import make_airfoil_cloud
from oracle.ref import Oracle
from paper_2403_13287_amd import lskum as L
from paper_2403_13287_amd.solver import Solver

pytestmark = pytest.mark.gpu

CASES = [  # (W, L, seed, mach, aoa)
    (40, 30, 11, 0.4, -2.0),
    (64, 40, 12, 0.7, 3.0),
    (50, 50, 13, 0.55, 5.0),
    (96, 24, 14, 0.3, 0.5),
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    clouds = [make_airfoil_cloud(W, Lr, 25, seed) for W, Lr, seed, _, _ in CASES]
    params = [L.Params(m, a, n_inner=2) for _, _, _, m, a in CASES]
    return clouds, params


def test_batch_matches_single_clouds_bitwise(batch):
    clouds, params = batch
    say("batch of", [c.n for c in clouds])
    b = Solver(clouds, params)
    hb = b.run(6)
    torch.cuda.synchronize()
    assert hb.shape == (6, len(clouds))
    clb = b.force_coeffs()
    for c, (cloud, p) in enumerate(zip(clouds, params)):
        s = Solver(cloud, p)
        hs = s.run(6)
        torch.cuda.synchronize()
        assert torch.equal(b.cloud_state(c), s.U), c
        assert torch.equal(hb[:, c], hs), c
        assert torch.equal(clb[c], s.force_coeffs()), c
    assert b.status() == L.OK


def test_tuning_does_not_change_results(batch):
    clouds, params = batch
    ref = None
    for t in L.TUNING_SPACE + [L.Tuning(256, 1, 256)]:
        say("tuning", t)
        s = Solver(clouds, params, tuning=t)
        h = s.run(3)
        torch.cuda.synchronize()
        if ref is None:
            ref = (s.U.clone(), h.clone())
        else:
            assert torch.equal(s.U, ref[0]) and torch.equal(h, ref[1]), t


def test_graph_replays_match_eager(batch):
    clouds, params = batch
    eager = Solver(clouds, params)
    he = eager.run(6)
    g_s = Solver(clouds, params)
    graph, hist = g_s.capture(2, 3)
    for r in range(3):
        graph.launch()
        # eager work and a synchronisation between replays
        junk = torch.ones(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert float(junk) == 1000.0
        assert torch.equal(hist[: 2 * (r + 1)], he[: 2 * (r + 1)]), r
    assert torch.equal(g_s.U, eager.U)
    assert g_s.status() == L.OK


def test_autotune_keeps_results(batch):
    clouds, params = batch
    s = Solver(clouds, params)
    U0 = s.U.clone()
    best, times = L.autotune(s.plan, s.U, s.ws, iters=1, reps=1)
    assert torch.equal(s.U, U0)  # autotuning runs on a scratch copy
    assert len(times) == len(L.TUNING_SPACE)
    assert best in times
    assert len({(t.block, t.xcd_contiguous, t.flux_block) for t in times}) >= 12


def test_batch_member_against_oracle(batch):
    clouds, params = batch
    b = Solver(clouds, params)
    hb = b.run(3)
    c = 1
    p = params[c]
    o = Oracle(clouds[c], p.mach, p.aoa_deg, cfl=p.cfl, venkat_k=p.venkat_k, n_inner=p.n_inner)
    Uo, ho, flags = o.iterate(o.init_state(), 3)
    assert flags == 0
    Ug = b.cloud_state(c).cpu().numpy().T
    for m in range(4):
        assert np.max(np.abs(Ug[m] - Uo[m])) <= 1e-10 * np.max(np.abs(Uo[m]))
    np.testing.assert_allclose(hb[:, c].cpu().numpy(), ho, rtol=1e-8)


def test_set_params_per_cloud(batch):
    clouds, params = batch
    s = Solver(clouds, params)
    new = [L.Params(0.5, 1.0 * k, n_inner=2) for k in range(len(clouds))]
    s.plan.set_params(new)
    L.lskum_init_state(s.plan, s.U)
    torch.cuda.synchronize()
    for k in range(len(clouds)):
        outer = np.nonzero(clouds[k].kind == 2)[0][0]
        u = s.cloud_state(k)[outer].cpu().numpy()
        assert u[1] == pytest.approx(0.5 * math.cos(math.radians(k)), rel=1e-15)
    bad = [L.Params(0.5, 0.0, n_inner=2)] * (len(clouds) - 1) + [L.Params(0.5, 0.0, n_inner=3)]
    with pytest.raises(L.LskumError):
        s.plan.set_params(bad)


def test_batch_run_is_the_iteration_with_cloud_major_history(batch):
    clouds, params = batch
    plan = L.Plan(clouds, params)
    nc = len(clouds)
    Ua, Ub = plan.field(4), plan.field(4)
    L.lskum_init_state(plan, Ua)
    Ub.copy_(Ua)
    ws = L.workspace(plan)
    ha = torch.full((5, nc), float("nan"), dtype=torch.float64, device="cuda")
    hb = torch.full((nc, 5), float("nan"), dtype=torch.float64, device="cuda")
    L.lskum_iterate(plan, 5, Ua, ha, ws)
    L.lskum_batch_run(plan, 5, Ub, hb, ws)
    torch.cuda.synchronize()
    assert torch.equal(Ua, Ub)
    assert torch.equal(hb, ha.T.contiguous())
    assert L.lskum_status(plan) == L.OK
    # hist on the state or the workspace is rejected before any launch
    lib = plan.lib
    assert lib.lskum_batch_run(plan.handle, 5, Ub.data_ptr(), Ub.data_ptr(), ws.data_ptr(),
                               None) == L.ERR_INVALID_ARG
    assert lib.lskum_batch_run(plan.handle, 5, Ub.data_ptr(), ws.data_ptr() + 256, ws.data_ptr(),
                               None) == L.ERR_INVALID_ARG


@pytest.mark.timeout(900)
def test_64_cloud_batch_smallest_and_largest_members_against_oracle():
    """The 64-cloud batch workload (5k-250k points, log-uniform, each with
    its own Mach number and angle of attack) advanced 2 iterations in one
    plan; its smallest and largest members against the oracle."""
    from cloudgen import batch_sizes, make_airfoil_clouds
    draws = batch_sizes()
    say("generating the 64 batch clouds")
    clouds = make_airfoil_clouds([(d["W"], d["L"], 25, d["seed"]) for d in draws])
    params = [L.Params(d["mach"], d["aoa_deg"], 0.2, 5.0, 2) for d in draws]
    sizes = [c.n for c in clouds]
    say("batch of", sum(sizes), "points")
    b = Solver(clouds, params)
    hb = b.run(2)
    torch.cuda.synchronize()
    assert b.status() == L.OK
    for c in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        p = params[c]
        say(f"member {c}: {sizes[c]} points, M {p.mach:.3f}, AoA {p.aoa_deg:.2f}")
        o = Oracle(clouds[c], p.mach, p.aoa_deg, cfl=p.cfl, venkat_k=p.venkat_k,
                   n_inner=p.n_inner)
        Uo, ho, flags = o.iterate(o.init_state(), 2)
        assert flags == 0
        Ug = b.cloud_state(c).cpu().numpy().T
        for m in range(4):
            assert np.max(np.abs(Ug[m] - Uo[m])) <= 1e-10 * np.max(np.abs(Uo[m])), (c, m)
        np.testing.assert_allclose(hb[:, c].cpu().numpy(), ho, rtol=1e-8)
