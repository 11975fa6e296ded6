"""Seeded synthetic point clouds around a symmetric NACA 4-digit section.

This module produces solver *inputs* only: coordinates, unit normals, point
kinds and the neighbour connectivity (padded CSR).  It holds none of the
flow solver's arithmetic, so both the CPU oracle and the GPU library may be
fed from it.

Layout of a cloud (all arrays numpy, structure-of-arrays):

* ``x, y``        float64 [n]   coordinates in chords
* ``nx, ny``      float64 [n]   unit normal; wall: into the fluid, outer:
                                radially outward, interior: (0, 1)
* ``kind``        int8    [n]   0 interior, 1 wall, 2 outer free stream
* ``row_ptr``     int64   [n+1] row i occupies col[row_ptr[i]:row_ptr[i+1]]
* ``col``         int32   [n*k_pad] neighbour ids, ascending distance, each
                                row padded to ``k_pad`` with the row's own id
* ``nbr_count``   int32   [n]   real neighbours in row i (<= k_max)
* ``wall_loop``   int32   [W]   wall point ids, counter-clockwise from the
                                trailing edge

Construction (an O-type point distribution, then Hilbert reordering):

1. Wall: theta_j = 2 pi j / W, x = (1 + cos theta)/2, y = +-y_t(x) with the
   closed-trailing-edge NACA 4-digit thickness law, upper surface for
   theta in (0, pi).
2. Layers: P_jl = W_j + s_l (C_j - W_j) with C_j on a circle of radius
   ``r_outer`` about (0.5, 0) and s_l = (g^l - 1)/(g^(L-1) - 1); g makes the
   first radial step equal to the mean wall spacing.
3. Jitter of every layer 1..L-2 by U(-1,1) * 0.2 of the local tangential and
   radial spacing (numpy PCG64 with the given seed).
4. Stencils: candidates from the (j, l) index window |dj|, |dl| <= w; keep
   the ``k_max`` nearest within 2.5x the distance to the 8th nearest
   candidate.  No wall-to-wall link joins the upper and lower surfaces aft
   of mid-chord (such a link would cross the body near the trailing edge).
   The window is widened (up to 8) for any point whose full stencil or whose
   used half-plane (split) stencils are too small or ill-conditioned; a
   point still failing takes the k_max nearest of the widest window without
   the radius cut (wall points at the trailing edge of the 16M cloud, where
   the wall spacing is far below the first layer's distance).
5. Points are reordered along a Hilbert curve on a 2^20 x 2^20 lattice over
   the bounding box (ties by original id); rows keep their order.
"""
from __future__ import annotations

import dataclasses
import math
import multiprocessing
import os

import numpy as np

KIND_INTERIOR = 0
KIND_WALL = 1
KIND_OUTER = 2

# Minimum number of points in every used half-plane stencil, and the minimum
# of det / (sum ds^2 * sum dn^2) accepted for a least-squares normal matrix.
MIN_SPLIT_POINTS = 2
MIN_REL_DET = 1e-3
# A neighbour only counts towards a half-plane stencil's sufficiency when it
# sits clearly off the splitting line (|ds| > SIDE_MARGIN * |d|).
SIDE_MARGIN = 1e-6


@dataclasses.dataclass
class Cloud:
    x: np.ndarray
    y: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    kind: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    nbr_count: np.ndarray
    wall_loop: np.ndarray
    k_max: int
    k_pad: int
    W: int
    L: int
    seed: int
    growth: float

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_wall(self) -> int:
        return int(self.wall_loop.shape[0])

    def neighbours(self, i: int) -> np.ndarray:
        s = int(self.row_ptr[i])
        return self.col[s:s + int(self.nbr_count[i])]


def naca4_thickness(x: np.ndarray, t: float = 0.12) -> np.ndarray:
    """Half-thickness of a symmetric NACA 4-digit section, closed trailing edge."""
    return 5.0 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2
                      + 0.2843 * x ** 3 - 0.1036 * x ** 4)


def _wall(W: int, t: float):
    j = np.arange(W)
    theta = 2.0 * np.pi * j / W
    x = 0.5 * (1.0 + np.cos(theta))
    side = np.zeros(W, dtype=np.int8)
    side[(j > 0) & (2 * j < W)] = 1
    side[2 * j > W] = -1
    y = side * naca4_thickness(x, t)
    return x, y, theta, side


def _solve_growth(L: int, first_step: float) -> float:
    """g > 1 with (g - 1)/(g^(L-1) - 1) == first_step (bisection)."""
    if first_step >= 1.0 / (L - 1):
        raise ValueError("wall spacing too coarse for the layer count")
    lo, hi = 1.0 + 1e-14, 2.0

    def f(g):
        if (L - 1) * math.log(g) > 700.0:  # g^(L-1) beyond double range: ratio ~ 0
            return -first_step
        return (g - 1.0) / (g ** (L - 1) - 1.0) - first_step
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _positions(W: int, L: int, seed: int, t: float, r_outer: float, jitter: float):
    xw, yw, theta, side = _wall(W, t)
    cx = 0.5 + r_outer * np.cos(theta)
    cy = r_outer * np.sin(theta)
    wall_xy = np.stack([xw, yw], axis=1)
    perim = float(np.sum(np.linalg.norm(np.roll(wall_xy, -1, axis=0) - wall_xy, axis=1)))
    h_w = perim / W
    reach = float(np.mean(np.hypot(cx - xw, cy - yw)))
    g = _solve_growth(L, h_w / reach)
    l = np.arange(L, dtype=np.float64)
    s = (g ** l - 1.0) / (g ** (L - 1) - 1.0)
    s[0], s[-1] = 0.0, 1.0
    # P[l, j]
    px = xw[None, :] + s[:, None] * (cx - xw)[None, :]
    py = yw[None, :] + s[:, None] * (cy - yw)[None, :]
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.uniform(-1.0, 1.0, size=(2, L - 2, W))
    if L > 2 and jitter > 0.0:
        tx = np.roll(px, -1, axis=1) - np.roll(px, 1, axis=1)
        ty = np.roll(py, -1, axis=1) - np.roll(py, 1, axis=1)
        rx = px[2:, :] - px[:-2, :]
        ry = py[2:, :] - py[:-2, :]
        tx, ty = tx[1:-1], ty[1:-1]
        tl = np.hypot(tx, ty)
        rl = np.hypot(rx, ry)
        # unit directions times half the local spacing == direction * |.|/2
        dx = jitter * (xi[0] * 0.5 * tx + xi[1] * 0.5 * rx)
        dy = jitter * (xi[0] * 0.5 * ty + xi[1] * 0.5 * ry)
        assert np.all(tl > 0) and np.all(rl > 0)
        px[1:-1] += dx
        py[1:-1] += dy
    return px, py, side, g


def _normals(px, py, W, L):
    n = W * L
    nx = np.zeros((L, W))
    ny = np.ones((L, W))
    Tx = np.roll(px[0], -1) - np.roll(px[0], 1)
    Ty = np.roll(py[0], -1) - np.roll(py[0], 1)
    Tl = np.hypot(Tx, Ty)
    nx[0] = Ty / Tl
    ny[0] = -Tx / Tl
    ox = px[-1] - 0.5
    oy = py[-1]
    ol = np.hypot(ox, oy)
    nx[-1] = ox / ol
    ny[-1] = oy / ol
    return nx.reshape(n), ny.reshape(n)


def _window_offsets(w: int):
    d = np.arange(-w, w + 1)
    dj, dl = np.meshgrid(d, d, indexing="xy")
    dj, dl = dj.ravel(), dl.ravel()
    keep = ~((dj == 0) & (dl == 0))
    return dj[keep], dl[keep]


def _select(ids, W, L, side, xflat, yflat, w, k_max, radius=2.5):
    """Neighbour selection for the points ``ids`` with index window ``w``:
    the k_max nearest candidates within ``radius`` times the distance to the
    8th nearest (no radius cut when ``radius`` is None).

    Returns (nbr [m, k_max] int64 padded with -1, count [m])."""
    j = ids % W
    l = ids // W
    dj, dl = _window_offsets(w)
    cj = (j[:, None] + dj[None, :]) % W
    cl = l[:, None] + dl[None, :]
    valid = (cl >= 0) & (cl < L)
    cl_c = np.clip(cl, 0, L - 1)
    cid = cl_c * W + cj
    # no wall-to-wall link across the aft body (upper <-> lower surface)
    ww = (l[:, None] == 0) & (cl == 0)
    aft = (xflat[j][:, None] > 0.5) & (xflat[cj] > 0.5)
    cross = ww & aft & (side[j][:, None] * side[cj] < 0)
    valid &= ~cross
    ddx = xflat[cid] - xflat[ids][:, None]
    ddy = yflat[cid] - yflat[ids][:, None]
    d2 = ddx * ddx + ddy * ddy
    d2 = np.where(valid, d2, np.inf)
    # sort by (distance, original id): order by id first, then stable by d2
    o1 = np.argsort(np.where(valid, cid, np.iinfo(np.int64).max), axis=1, kind="stable")
    d2_1 = np.take_along_axis(d2, o1, axis=1)
    cid_1 = np.take_along_axis(cid, o1, axis=1)
    o2 = np.argsort(d2_1, axis=1, kind="stable")
    d2s = np.take_along_axis(d2_1, o2, axis=1)
    cids = np.take_along_axis(cid_1, o2, axis=1)
    n_valid = np.sum(np.isfinite(d2s), axis=1)
    if np.any(n_valid < 8):
        raise RuntimeError("index window too small")
    r8 = np.sqrt(d2s[:, 7])
    if radius is None:
        inside = np.ones(d2s.shape, dtype=bool)
    else:
        inside = np.sqrt(d2s) <= radius * r8[:, None]
    rank = np.arange(d2s.shape[1])[None, :]
    take = inside & (rank < k_max) & np.isfinite(d2s)
    count = take.sum(axis=1)
    nbr = np.where(take, cids, -1)[:, :k_max]
    return nbr, count


def _stencil_ok(ids, nbr, count, kind, xflat, yflat, nxf, nyf):
    """Sufficiency of the full stencil and of every used half-plane stencil."""
    m, k = nbr.shape
    real = nbr >= 0
    safe = np.where(real, nbr, ids[:, None])
    dx = np.where(real, xflat[safe] - xflat[ids][:, None], 0.0)
    dy = np.where(real, yflat[safe] - yflat[ids][:, None], 0.0)
    sxx = np.sum(dx * dx, axis=1)
    syy = np.sum(dy * dy, axis=1)
    sxy = np.sum(dx * dy, axis=1)
    ok = (count >= 3) & (sxx * syy - sxy * sxy >= MIN_REL_DET * sxx * syy)
    nxp = nxf[ids][:, None]
    nyp = nyf[ids][:, None]
    ds = dx * nyp - dy * nxp
    dn = dx * nxp + dy * nyp
    dist = np.sqrt(dx * dx + dy * dy)
    kd = kind[ids]

    def split_ok(mask):
        c = np.sum(mask, axis=1)
        a = np.sum(np.where(mask, ds * ds, 0.0), axis=1)
        b = np.sum(np.where(mask, ds * dn, 0.0), axis=1)
        e = np.sum(np.where(mask, dn * dn, 0.0), axis=1)
        return (c >= MIN_SPLIT_POINTS) & (a * e - b * b >= MIN_REL_DET * a * e) & (a * e > 0)

    margin = SIDE_MARGIN * dist
    s_pos = split_ok(real & (ds < -margin))
    s_neg = split_ok(real & (ds > margin))
    n_pos = split_ok(real & (dn < -margin))
    n_neg = split_ok(real & (dn > margin))
    interior = kd == KIND_INTERIOR
    wall = kd == KIND_WALL
    ok &= np.where(interior, s_pos & s_neg & n_pos & n_neg, True)
    ok &= np.where(wall, s_pos & s_neg & n_neg, True)
    return ok


def _hilbert_key(xq: np.ndarray, yq: np.ndarray, order: int) -> np.ndarray:
    """Distance along a Hilbert curve of the lattice points (xq, yq) in [0, 2^order)."""
    x = xq.astype(np.int64).copy()
    y = yq.astype(np.int64).copy()
    key = np.zeros_like(x)
    s = 1 << (order - 1)
    while s > 0:
        rx = (x & s) > 0
        ry = (y & s) > 0
        key += np.int64(s) * np.int64(s) * ((3 * rx.astype(np.int64)) ^ ry.astype(np.int64))
        x &= s - 1
        y &= s - 1
        flip = (~ry) & rx
        x = np.where(flip, s - 1 - x, x)
        y = np.where(flip, s - 1 - y, y)
        swap = ~ry
        x, y = np.where(swap, y, x), np.where(swap, x, y)
        s >>= 1
    return key


def hilbert_order(x: np.ndarray, y: np.ndarray, order: int = 20) -> np.ndarray:
    """Permutation listing points in Hilbert-curve order (stable in original id)."""
    span = max(float(x.max() - x.min()), float(y.max() - y.min()))
    q = (1 << order) - 1
    xq = np.floor((x - x.min()) / span * q).astype(np.int64)
    yq = np.floor((y - y.min()) / span * q).astype(np.int64)
    return np.argsort(_hilbert_key(xq, yq, order), kind="stable")


# clouds above this many points build their stencils in worker processes
PARALLEL_POINTS = 1 << 22
_POOL_ARGS = None


def _chunk_stencils(start, W, L, side, xflat, yflat, kind, nxf, nyf, k_max, chunk, n):
    """Stencils of the points start .. start+chunk-1: the nearest-neighbour
    selection in the index window w = 3, widened for the points whose
    stencil fails the sufficiency test until it passes."""
    ids = np.arange(start, min(n, start + chunk), dtype=np.int64)
    nbr_out = np.full((ids.size, k_max), -1, dtype=np.int64)
    cnt_out = np.zeros(ids.size, dtype=np.int64)
    w = 3
    todo = ids
    while todo.size:
        if w > 9:
            raise RuntimeError(f"no valid stencil for {todo.size} points")
        # last resort (w = 9): the window of 8 without the radius cut, for
        # points whose 8 nearest candidates all lie on one side (wall points
        # at the trailing edge of very fine clouds, where the wall spacing is
        # far below the first layer's distance)
        nbr, cnt = _select(todo, W, L, side, xflat, yflat, min(w, 8), k_max,
                           radius=2.5 if w <= 8 else None)
        ok = _stencil_ok(todo, nbr, cnt, kind, xflat, yflat, nxf, nyf)
        nbr_out[todo[ok] - start] = nbr[ok]
        cnt_out[todo[ok] - start] = cnt[ok]
        todo = todo[~ok]
        w += 1
    return ids, nbr_out, cnt_out


def _chunk_stencils_pooled(start):
    return _chunk_stencils(start, *_POOL_ARGS)


def make_airfoil_cloud(W: int, L: int, k_max: int, seed: int, *, t: float = 0.12,
                       r_outer: float = 15.0, jitter: float = 0.2, reorder: bool = True,
                       chunk: int = 1 << 18, workers: int | None = None) -> Cloud:
    """Build the cloud described in the module docstring.  Stencils are built
    in forked worker processes for clouds above PARALLEL_POINTS points, or
    whenever `workers` > 1 is given (call it before the process initialises a
    GPU then); the result does not depend on it."""
    if W < 16 or L < 4 or k_max < 8:
        raise ValueError("cloud too small")
    k_pad = (k_max + 3) // 4 * 4
    px, py, side, g = _positions(W, L, seed, t, r_outer, jitter)
    n = W * L
    xflat = px.reshape(n)
    yflat = py.reshape(n)
    nxf, nyf = _normals(px, py, W, L)
    kind = np.zeros((L, W), dtype=np.int8)
    kind[0] = KIND_WALL
    kind[-1] = KIND_OUTER
    kind = kind.reshape(n)

    nbr_all = np.full((n, k_max), -1, dtype=np.int64)
    cnt_all = np.zeros(n, dtype=np.int64)
    starts = list(range(0, n, chunk))
    args = (W, L, side, xflat, yflat, kind, nxf, nyf, k_max, chunk, n)
    forced = workers is not None
    workers = min(len(starts), workers or os.cpu_count() or 1, 16)
    if (forced or n > PARALLEL_POINTS) and workers > 1:
        # chunks are independent (each point's stencil depends only on the
        # positions in its index window), so the result does not depend on
        # how they are distributed
        global _POOL_ARGS
        _POOL_ARGS = args
        try:
            with multiprocessing.get_context("fork").Pool(workers) as pool:
                parts = pool.map(_chunk_stencils_pooled, starts)
        finally:
            _POOL_ARGS = None
    else:
        parts = [_chunk_stencils(start, *args) for start in starts]
    for start, (ids, nbr, cnt) in zip(starts, parts):
        nbr_all[ids] = nbr
        cnt_all[ids] = cnt
    del parts

    wall_loop = np.arange(W, dtype=np.int64)  # ids l*W + j with l == 0
    if reorder:
        perm = hilbert_order(xflat, yflat)
    else:
        perm = np.arange(n, dtype=np.int64)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n, dtype=np.int64)

    nbr_new = nbr_all[perm]
    cnt_new = cnt_all[perm]
    real = nbr_new >= 0
    col = np.empty((n, k_pad), dtype=np.int32)
    self_id = np.arange(n, dtype=np.int64)[:, None]
    col[:, :k_max] = np.where(real, inv[np.where(real, nbr_new, 0)], self_id).astype(np.int32)
    col[:, k_max:] = self_id.astype(np.int32)
    return Cloud(
        x=np.ascontiguousarray(xflat[perm]),
        y=np.ascontiguousarray(yflat[perm]),
        nx=np.ascontiguousarray(nxf[perm]),
        ny=np.ascontiguousarray(nyf[perm]),
        kind=np.ascontiguousarray(kind[perm]),
        row_ptr=np.arange(n + 1, dtype=np.int64) * k_pad,
        col=col.reshape(n * k_pad),
        nbr_count=cnt_new.astype(np.int32),
        wall_loop=inv[wall_loop].astype(np.int32),
        k_max=k_max, k_pad=k_pad, W=W, L=L, seed=seed, growth=g,
    )


# Named workloads: (W, L, k_max, seed)
CONFIGS = {
    "tiny": (160, 60, 25, 0),
    "10k": (100, 100, 25, 1),
    "1m": (1000, 1000, 30, 2),
    "16m": (4000, 4000, 30, 3),
}


def _make_one(spec):
    return make_airfoil_cloud(*spec)


def make_airfoil_clouds(specs, workers: int | None = None):
    """make_airfoil_cloud(W, L, k_max, seed) for each (W, L, k_max, seed) in
    `specs`, in forked worker processes (the same clouds as one by one).
    Call it before the process initialises a GPU."""
    specs = [tuple(s) for s in specs]
    workers = min(len(specs), workers or os.cpu_count() or 1, 16)
    if workers <= 1:
        return [_make_one(s) for s in specs]
    # largest first, so that the big clouds do not end the map alone
    order = sorted(range(len(specs)), key=lambda k: -specs[k][0] * specs[k][1])
    with multiprocessing.get_context("fork").Pool(workers) as pool:
        made = pool.map(_make_one, [specs[k] for k in order], chunksize=1)
    out = [None] * len(specs)
    for k, c in zip(order, made):
        out[k] = c
    return out


def named_cloud(name: str, **kw) -> Cloud:
    W, L, k, seed = CONFIGS[name]
    return make_airfoil_cloud(W, L, k, seed, **kw)


def batch_sizes(n_clouds: int = 64, seed: int = 4242):
    """Uneven cloud sizes, log-uniform in [5k, 250k] points, and flow draws.

    Returns a list of dicts with W, L, seed, mach, aoa_deg."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_c = np.exp(rng.uniform(math.log(5e3), math.log(2.5e5), size=n_clouds))
    mach = rng.uniform(0.3, 0.9, size=n_clouds)
    aoa = rng.uniform(-4.0, 6.0, size=n_clouds)
    out = []
    for c in range(n_clouds):
        side = int(round(math.sqrt(n_c[c])))
        out.append(dict(W=side, L=side, seed=1000 + c, mach=float(mach[c]), aoa_deg=float(aoa[c])))
    return out
