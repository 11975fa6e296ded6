"""Scheme options on the GPU against the oracle: the first-order flux and
the min-max limiter, on the 9,600-point cloud at the workload's flow and on
the supersonic case (3 iterations; fields normwise 1e-10, histories 1e-8).
The adjoint entry points refuse them."""
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


@pytest.fixture(scope="module")
def tiny():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return named_cloud("tiny")


@pytest.mark.parametrize("options", [L.FIRST_ORDER, L.MINMAX, L.FIRST_ORDER | L.MINMAX])
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


def test_adjoint_refuses_variants(tiny):
    plan = L.Plan(tiny, L.Params(0.63, 2.0, options=L.MINMAX))
    U = plan.field(4)
    L.lskum_init_state(plan, U)
    tb = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LskumError):
        L.lskum_flux_residual_vjp(plan, U, U.clone(), plan.field(4), tb, L.vjp_workspace(plan))
