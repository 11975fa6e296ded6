"""Named workloads: cloud recipe plus flow and scheme settings.

Settings only (no solver arithmetic).  The limiter constant K = 5 is the
value used throughout: with K = 150 the Mach 0.85 case diverges near the
leading edge on the 9.6k-point cloud within 60 iterations.
"""
from __future__ import annotations

import dataclasses

from .airfoil import CONFIGS, make_airfoil_cloud

VENKAT_K = 5.0
CFL = 0.2
GAMMA = 1.4


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    W: int
    L: int
    k_max: int
    seed: int
    mach: float
    aoa_deg: float
    n_inner: int
    iters: int
    cfl: float = CFL
    venkat_k: float = VENKAT_K
    gamma: float = GAMMA

    @property
    def n_points(self) -> int:
        return self.W * self.L

    def cloud(self, workers: int | None = None):
        return make_airfoil_cloud(self.W, self.L, self.k_max, self.seed, workers=workers)


def _wl(name, mach, aoa, n_inner, iters):
    W, L, k, seed = CONFIGS[name]
    return Workload(name, W, L, k, seed, mach, aoa, n_inner, iters)


WORKLOADS = {
    # 160 x 60 airfoil cloud, M 0.63, AoA 2 deg, 2 inner iterations, 100 RK4 iterations
    "tiny": _wl("tiny", 0.63, 2.0, 2, 100),
    # 100 x 100 cloud for the adjoint checks
    "10k": _wl("10k", 0.63, 2.0, 3, 1000),
    # 1000 x 1000, M 0.85, AoA 1 deg, 3 inner iterations, 1000 RK4 iterations
    "1m": _wl("1m", 0.85, 1.0, 3, 1000),
    # 4000 x 4000, M 0.63, AoA 2 deg, 3 inner iterations, 50 timed iterations
    "16m": _wl("16m", 0.63, 2.0, 3, 50),
}
