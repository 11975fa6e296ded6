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
    for t in L.TUNING_SPACE:
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
    assert (best.block, best.xcd_contiguous) in times


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
