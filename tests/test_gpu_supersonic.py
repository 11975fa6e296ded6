"""The paper's supersonic case: NACA 0012 at Mach 1.2, zero incidence.

A bow shock stands ahead of the leading edge and the limiter is active
through it, so this case exercises the limiter branches and the positivity
of the reconstructed states far more than the subsonic workloads.

* Parity: the 9,600-point cloud, 3 iterations, GPU against the oracle at the
  usual tolerances (fields normwise 1e-10, histories relative 1e-8).
* Stability: the 10,000-point cloud, 5,000 iterations on the GPU: no
  non-physical state, the density residual falls, the lift of the
  symmetric section at zero incidence stays near zero and the (wave) drag is
  positive.
"""
import sys

import numpy as np
import pytest
import torch

from cloudgen import named_cloud
from oracle.ref import Oracle
from paper_2403_13287_amd import lskum as L
from paper_2403_13287_amd.solver import Solver

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(g, r):
    return max(np.max(np.abs(gc - rc)) / np.max(np.abs(rc)) for gc, rc in zip(g, r))


def test_supersonic_parity_tiny():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = named_cloud("tiny")
    p = L.Params(1.2, 0.0, n_inner=2)
    o = Oracle(c, 1.2, 0.0, n_inner=2)
    Uo, ho, flags = o.iterate(o.init_state(), 3)
    assert flags == 0
    s = Solver(c, p)
    hg = s.run(3)
    torch.cuda.synchronize()
    assert s.status() == L.OK
    np.testing.assert_allclose(hg.cpu().numpy(), ho, rtol=1e-8)
    Ug = s.U.cpu().numpy().T
    e = normwise(Ug, Uo)
    say("M 1.2 tiny: U normwise", e)
    assert e <= 1e-10
    _, _, _, R = s.residual()
    Ro, _ = o.residual(Uo)
    assert normwise(R.cpu().numpy().T, Ro) <= 1e-10


def test_supersonic_stability_10k():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = named_cloud("10k")
    s = Solver(c, L.Params(1.2, 0.0, n_inner=3))
    graph, hist = s.capture(500, 10)
    for _ in range(10):
        graph.launch()
    torch.cuda.synchronize()
    assert s.status() == L.OK
    h = hist[:, 0].cpu().numpy()
    cl, cd = s.force_coeffs().cpu().numpy()
    say("M 1.2 10k: residual", h[0], "->", h[-1], "Cl", cl, "Cd", cd)
    assert np.all(np.isfinite(h)) and h[-1] < 0.5 * h[0]
    assert abs(cl) < 0.01
    assert cd > 0.0
