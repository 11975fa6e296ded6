"""Small synthetic point sets for tests: generic point lists with kNN or
radius stencils, a mirror-symmetric cylinder cloud and a jittered square.

Geometry and connectivity only; none of the solver's arithmetic.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from .airfoil import KIND_INTERIOR, KIND_OUTER, KIND_WALL, Cloud


def from_lists(x, y, nx, ny, kind, nbrs, wall_loop=(), k_pad=None) -> Cloud:
    """Cloud from explicit neighbour lists (list of sequences, own id excluded)."""
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    k_max = max(1, max(len(r) for r in nbrs))
    if k_pad is None:
        k_pad = (k_max + 3) // 4 * 4
    if k_pad < k_max:
        raise ValueError("k_pad smaller than the longest row")
    col = np.repeat(np.arange(n, dtype=np.int32)[:, None], k_pad, axis=1)
    cnt = np.zeros(n, np.int32)
    for i, r in enumerate(nbrs):
        r = np.asarray(r, np.int64)
        if np.any(r == i) or np.any(r < 0) or np.any(r >= n):
            raise ValueError(f"bad neighbour list for point {i}")
        col[i, :len(r)] = r
        cnt[i] = len(r)
    return Cloud(x=np.ascontiguousarray(x), y=np.ascontiguousarray(np.asarray(y, np.float64)),
                 nx=np.ascontiguousarray(np.asarray(nx, np.float64)),
                 ny=np.ascontiguousarray(np.asarray(ny, np.float64)),
                 kind=np.ascontiguousarray(np.asarray(kind, np.int8)),
                 row_ptr=np.arange(n + 1, dtype=np.int64) * k_pad,
                 col=col.reshape(n * k_pad), nbr_count=cnt,
                 wall_loop=np.asarray(wall_loop, np.int32), k_max=k_max, k_pad=k_pad,
                 W=len(wall_loop), L=0, seed=-1, growth=0.0)


def _order_rows(pts, lists):
    out = []
    for i, r in enumerate(lists):
        r = np.array([j for j in r if j != i], dtype=np.int64)
        d2 = np.sum((pts[r] - pts[i]) ** 2, axis=1)
        o = np.lexsort((r, d2))
        out.append(r[o])
    return out


def from_points(x, y, nx, ny, kind, *, k=None, radius=None, wall_loop=(), k_pad=None) -> Cloud:
    """Cloud with stencils of the k nearest points or of all points within
    ``radius`` (scalar or per point), ordered by distance then id."""
    pts = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64)], axis=1)
    tree = cKDTree(pts)
    if radius is not None:
        lists = tree.query_ball_point(pts, r=radius)
    else:
        _, idx = tree.query(pts, k=k + 1)
        lists = [list(r) for r in idx]
    return from_lists(pts[:, 0], pts[:, 1], nx, ny, kind, _order_rows(pts, lists),
                      wall_loop=wall_loop, k_pad=k_pad)


def cylinder_cloud(M: int = 48, L: int = 12, r_body: float = 0.5, r_out: float = 4.0,
                   reach: float = 2.3) -> Cloud:
    """Rings of M points around a circular body, exactly mirror symmetric in y.

    Ring 0 is the wall (normal = radial outward, into the fluid), ring L-1 the
    outer boundary (radial normal); interior normals are (0, 1).  Stencils
    hold every point within ``reach`` times the local spacing, which keeps
    the connectivity mirror symmetric."""
    g = (r_out / r_body) ** (1.0 / (L - 1))
    radii = r_body * g ** np.arange(L)
    # angles 2 pi k / M, with point M-k set to the exact reflection of point k
    half = np.arange(M // 2 + 1)
    c = np.empty(M)
    s = np.empty(M)
    c[half] = np.cos(2.0 * np.pi * half / M)
    s[half] = np.sin(2.0 * np.pi * half / M)
    s[0] = 0.0
    if M % 2 == 0:
        s[M // 2] = 0.0
    up = np.arange(M // 2 + 1, M)
    c[up] = c[M - up]
    s[up] = -s[M - up]
    x = (radii[:, None] * c[None, :]).ravel()
    y = (radii[:, None] * s[None, :]).ravel()
    n = x.size
    kind = np.zeros((L, M), np.int8)
    kind[0] = KIND_WALL
    kind[-1] = KIND_OUTER
    nx = np.zeros((L, M))
    ny = np.ones((L, M))
    nx[0], ny[0] = c, s
    nx[-1], ny[-1] = c, s
    spacing = np.repeat(radii * (g - 1.0), M)
    cl = from_points(x, y, nx.ravel(), ny.ravel(), kind.ravel(), radius=reach * spacing,
                     wall_loop=np.arange(M))
    assert cl.n == n
    return cl


def square_cloud(nside: int, jitter: float = 0.25, seed: int = 0, k: int = 20,
                 random_frames: bool = False, margin_rings: int = 2) -> Cloud:
    """Jittered lattice on [0,1]^2.  The outer ``margin_rings`` rings are
    kind 2 (Dirichlet), the rest interior.  With ``random_frames`` every
    interior point gets a random unit normal instead of (0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / (nside - 1)
    i, j = np.meshgrid(np.arange(nside), np.arange(nside), indexing="ij")
    x = (i * h).ravel().astype(np.float64)
    y = (j * h).ravel().astype(np.float64)
    inner = ((i > 0) & (i < nside - 1) & (j > 0) & (j < nside - 1)).ravel()
    x[inner] += jitter * h * rng.uniform(-1, 1, inner.sum())
    y[inner] += jitter * h * rng.uniform(-1, 1, inner.sum())
    edge = np.minimum(np.minimum(i, nside - 1 - i), np.minimum(j, nside - 1 - j)).ravel()
    kind = np.where(edge < margin_rings, KIND_OUTER, KIND_INTERIOR).astype(np.int8)
    nx = np.zeros(x.size)
    ny = np.ones(x.size)
    if random_frames:
        a = rng.uniform(0, 2 * np.pi, x.size)
        nx, ny = np.cos(a), np.sin(a)
    return from_points(x, y, nx, ny, kind, k=k)


def restrict(cloud: Cloud, seeds, depth: int):
    """The sub-cloud of the points within `depth` stencil hops of `seeds`.

    Points keep their relative order and their rows keep the stored order of
    the neighbours that stay; rows of the outermost ring lose the neighbours
    outside.  A quantity of a seed point that reads rows up to depth - 1 and
    pointwise values up to `depth` (the residual with n inner sweeps reads
    derivative rows up to n + 1 hops, q up to n + 2) is the same on the
    sub-cloud as on the whole cloud.  Returns (sub-cloud, original ids)."""
    n, kp = cloud.n, cloud.k_pad
    col = cloud.col.reshape(n, kp)
    cnt = cloud.nbr_count
    mask = np.arange(kp)[None, :] < cnt[:, None]
    member = np.zeros(n, bool)
    frontier = np.unique(np.asarray(seeds, np.int64))
    member[frontier] = True
    for _ in range(depth):
        nb = col[frontier][mask[frontier]]
        nb = np.unique(nb[~member[nb]])
        member[nb] = True
        frontier = nb
    ids = np.nonzero(member)[0]
    new = np.full(n, -1, np.int64)
    new[ids] = np.arange(ids.size)
    rows = []
    for i in ids:
        r = col[i, :cnt[i]]
        rows.append(new[r[member[r]]])
    wall = [int(new[w]) for w in cloud.wall_loop if member[w]]
    sub = from_lists(cloud.x[ids], cloud.y[ids], cloud.nx[ids], cloud.ny[ids], cloud.kind[ids],
                     rows, wall_loop=wall, k_pad=kp)
    return sub, ids
