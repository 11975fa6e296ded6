"""lskum_q_derivs_static, the entry point that allocates nothing (its inner
sweeps' scratch is a static device array of the library), against
lskum_q_derivs with a caller-allocated work buffer: dq and qlim equal bit
for bit, on two calls in a row, the second on a smaller cloud; and the
size limit of the static scratch."""
import numpy as np
import pytest
import torch

from cloudgen.airfoil import make_airfoil_cloud
from paper_2403_13287_amd import lskum as L

pytestmark = pytest.mark.gpu


def _state(plan, seed):
    """The free stream with a smooth seeded perturbation (positive rho, p),
    so that the derivatives are not zero."""
    U = plan.field(4)
    L.lskum_init_state(plan, U)
    rng = np.random.default_rng(seed)
    n = plan.n
    # per-point factors in [0.9, 1.1] for rho and E, momentum scaled by 0.8..1.2
    f = torch.from_numpy(rng.uniform(0.9, 1.1, size=(n, 2))).to(U.device)
    g = torch.from_numpy(rng.uniform(0.8, 1.2, size=(n, 2))).to(U.device)
    U[:, 0] *= f[:, 0]
    U[:, 1:3] *= g
    U[:, 3] *= f[:, 1]
    q = plan.field(4)
    L.lskum_q_vars(plan, U, q)
    return q


def _compare(cloud, n_inner, seed):
    p = L.Params(0.63, 2.0, n_inner=n_inner)
    plan = L.Plan(cloud, p)
    q = _state(plan, seed)
    dq_a, ql_a, work = plan.field(8), plan.field(8), plan.field(16)
    L.lskum_q_derivs(plan, q, dq_a, ql_a, work)
    dq_b, ql_b = plan.field(8), plan.field(8)
    dq_b.fill_(np.nan)
    ql_b.fill_(np.nan)
    L.lskum_q_derivs_static(plan, q, dq_b, ql_b)
    torch.cuda.synchronize()
    assert L.lskum_status(plan) == L.OK
    a, b = dq_a.cpu().numpy(), dq_b.cpu().numpy()
    assert np.all(np.isfinite(a)) and np.abs(a).max() > 0
    assert np.array_equal(a, b)
    assert np.array_equal(ql_a.cpu().numpy(), ql_b.cpu().numpy())
    return plan


def test_static_scratch_matches_q_derivs_on_two_calls_second_smaller():
    torch.cuda.set_device(0)
    big = make_airfoil_cloud(300, 200, 25, 11)     # 60k points, many tiles
    small = make_airfoil_cloud(160, 60, 25, 0)     # 9.6k points
    print(f"no-alloc q_derivs: n={big.n} then n={small.n}", flush=True)
    _compare(big, 3, 1)
    _compare(small, 2, 2)
    _compare(small, 0, 3)  # no inner sweeps: the scratch is not touched


def test_static_scratch_rejects_clouds_beyond_its_limit():
    torch.cuda.set_device(0)
    cloud = make_airfoil_cloud(1025, 1024, 12, 5)  # 1,049,600 points > 2^20
    print(f"no-alloc q_derivs limit: n={cloud.n}", flush=True)
    plan = L.Plan(cloud, L.Params(0.63, 2.0, n_inner=1))
    q, dq, ql = plan.field(4), plan.field(8), plan.field(8)
    q.fill_(1.0)  # any finite q: the derivatives of a uniform field are 0
    with pytest.raises(L.LskumError) as e:
        L.lskum_q_derivs_static(plan, q, dq, ql)
    assert e.value.code == L.ERR_SCRATCH_LIMIT
    # without inner sweeps the scratch is not needed and any size is accepted
    plan.set_params(L.Params(0.63, 2.0, n_inner=0))
    L.lskum_q_derivs_static(plan, q, dq, ql)
    torch.cuda.synchronize()
    assert np.all(dq.cpu().numpy() == 0.0)
