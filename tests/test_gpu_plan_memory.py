"""Device memory comes back when a plan is destroyed, including the tile
tables of the in-edge rows that the plan's first VJP call builds.

Each cycle creates a plan on a 200k-point airfoil cloud, runs one residual
VJP (which builds the in-edge tables: about 30 MB of slots at this size)
and destroys the plan; the device's free memory (hipMemGetInfo) after three
cycles must be within a few MB of what it was after the first."""
import sys

import pytest
import torch

from cloudgen import make_airfoil_cloud
from paper_2403_13287_amd import lskum as L

pytestmark = pytest.mark.gpu

LEAK_TOL = 8 << 20  # bytes; one cycle's in-edge slots alone are ~30 MB


def _cycle(cloud, params):
    plan = L.Plan(cloud, params)
    U = plan.field(4)
    L.lskum_init_state(plan, U)
    gen = torch.Generator(device="cuda").manual_seed(3)
    Rb = torch.randn(plan.n, 4, dtype=torch.float64, device="cuda", generator=gen)
    Ub = plan.field(4)
    tb = torch.empty(2, dtype=torch.float64, device="cuda")
    ws = L.vjp_workspace(plan)
    L.lskum_flux_residual_vjp(plan, U, Rb, Ub, tb, ws)
    torch.cuda.synchronize()
    assert L.lskum_status(plan) == L.OK
    plan.destroy()
    del U, Rb, Ub, tb, ws
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_plan_destroy_returns_device_memory():
    cloud = make_airfoil_cloud(500, 400, 30, 5)
    params = L.Params(0.63, 2.0, n_inner=3)
    print(f"[plan memory] n={cloud.n}", file=sys.stderr, flush=True)
    _cycle(cloud, params)  # one-time allocations of the runtime and the library
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        _cycle(cloud, params)
    free1 = torch.cuda.mem_get_info()[0]
    print(f"[plan memory] free before {free0} after {free1}", file=sys.stderr, flush=True)
    assert free0 - free1 <= LEAK_TOL
