"""Host-side checks of the synthetic cloud generator (no GPU)."""
import numpy as np
import pytest

from cloudgen import batch_sizes, make_airfoil_cloud, naca4_thickness
from cloudgen.airfoil import MIN_REL_DET, _hilbert_key, hilbert_order


def test_thickness_law_closed_trailing_edge():
    assert abs(naca4_thickness(np.array([1.0]))[0]) < 1e-15
    assert naca4_thickness(np.array([0.0]))[0] == 0.0
    # maximum thickness 12 % of chord near x = 0.3
    x = np.linspace(0, 1, 100001)
    yt = naca4_thickness(x)
    assert abs(2 * yt.max() - 0.12) < 2e-4
    assert 0.28 < x[np.argmax(yt)] < 0.32


def test_hilbert_key_is_a_bijection_on_small_lattice():
    order = 4
    xs, ys = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
    key = _hilbert_key(xs.ravel(), ys.ravel(), order)
    assert np.array_equal(np.sort(key), np.arange(256))
    # consecutive keys are lattice neighbours
    pos = np.empty((256, 2), np.int64)
    pos[key] = np.stack([xs.ravel(), ys.ravel()], axis=1)
    steps = np.abs(np.diff(pos, axis=0)).sum(axis=1)
    assert np.all(steps == 1)


@pytest.fixture(scope="module")
def cloud():
    return make_airfoil_cloud(160, 60, 25, 0)


def test_cloud_structure(cloud):
    c = cloud
    n = c.n
    assert n == 9600
    assert np.bincount(c.kind, minlength=3).tolist() == [9280, 160, 160]
    assert c.row_ptr.dtype == np.int64 and c.col.dtype == np.int32
    assert np.array_equal(c.row_ptr, np.arange(n + 1) * c.k_pad)
    assert c.k_pad % 4 == 0 and c.k_pad >= c.k_max
    col = c.col.reshape(n, c.k_pad)
    assert col.min() >= 0 and col.max() < n
    assert np.all(c.nbr_count <= c.k_max) and np.all(c.nbr_count >= 3)
    ids = np.arange(n)
    for i in range(0, n, 7):
        k = c.nbr_count[i]
        real = col[i, :k]
        assert np.all(col[i, k:] == i)  # padding is the row's own id
        assert np.all(real != i) and len(set(real.tolist())) == k
        d = np.hypot(c.x[real] - c.x[i], c.y[real] - c.y[i])
        assert np.all(np.diff(d) >= 0)  # ascending distance
    assert np.allclose(np.hypot(c.nx, c.ny), 1.0, atol=1e-14)
    assert np.all(c.nx[c.kind == 0] == 0) and np.all(c.ny[c.kind == 0] == 1)


def test_wall_loop_and_normals(cloud):
    c = cloud
    wl = c.wall_loop
    assert len(wl) == 160 and np.all(c.kind[wl] == 1)
    wx, wy = c.x[wl], c.y[wl]
    area = 0.5 * np.sum(wx * np.roll(wy, -1) - np.roll(wx, -1) * wy)
    assert 0.08 < area < 0.085  # NACA 0012 area ~ 0.0822 chord^2, counter-clockwise
    # wall normals point away from the body interior (into the fluid)
    cx, cy = 0.42, 0.0
    out = (c.nx[wl] * (wx - cx) + c.ny[wl] * (wy - cy))
    assert np.all(out > 0)
    # outer normals point radially out
    o = c.kind == 2
    assert np.all(c.nx[o] * (c.x[o] - 0.5) + c.ny[o] * c.y[o] > 0)


def test_used_split_stencils_are_sufficient(cloud):
    c = cloud
    col = c.col.reshape(c.n, c.k_pad)
    for i in range(c.n):
        if c.kind[i] == 2:
            continue
        real = col[i, :c.nbr_count[i]]
        dx, dy = c.x[real] - c.x[i], c.y[real] - c.y[i]
        ds = dx * c.ny[i] - dy * c.nx[i]
        dn = dx * c.nx[i] + dy * c.ny[i]
        masks = [ds < 0, ds > 0, dn > 0] + ([dn < 0] if c.kind[i] == 0 else [])
        for m in masks:
            assert m.sum() >= 2
            a, b, e = np.sum(ds[m] ** 2), np.sum(ds[m] * dn[m]), np.sum(dn[m] ** 2)
            assert a * e - b * b >= MIN_REL_DET * a * e * 0.999


def test_generator_is_deterministic_and_seeded():
    a = make_airfoil_cloud(100, 40, 25, 5)
    b = make_airfoil_cloud(100, 40, 25, 5)
    c = make_airfoil_cloud(100, 40, 25, 6)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.col, b.col)
    assert not np.array_equal(a.x, c.x)


def test_hilbert_order_improves_locality():
    a = make_airfoil_cloud(200, 200, 25, 0, reorder=False)
    b = make_airfoil_cloud(200, 200, 25, 0, reorder=True)
    def spread(c):
        col = c.col.reshape(c.n, c.k_pad)
        return np.median(np.abs(col - np.arange(c.n)[:, None]))
    assert spread(b) < spread(a)
    perm = hilbert_order(a.x, a.y)
    assert np.array_equal(np.sort(perm), np.arange(a.n))


def test_batch_draws():
    draws = batch_sizes()
    assert len(draws) == 64
    sizes = np.array([d["W"] * d["L"] for d in draws])
    assert sizes.min() >= 4000 and sizes.max() <= 260000
    assert all(0.3 <= d["mach"] <= 0.9 and -4 <= d["aoa_deg"] <= 6 for d in draws)


def test_restricted_cloud_reproduces_the_residual_at_its_seeds(tiny_cloud):
    """The residual at a seed reads derivative rows n_inner + 1 hops out and
    q n_inner + 2 hops out, so the sub-cloud of that depth gives the seeds'
    residual bit for bit (full-size parity tests compare sampled points this
    way)."""
    from cloudgen.shapes import restrict
    from oracle.ref import Oracle
    c = tiny_cloud
    o = Oracle(c, 0.63, 2.0, n_inner=2)
    U, _, _ = o.iterate(o.init_state(), 3)
    R, _ = o.residual(U)
    rng = np.random.default_rng(5)
    seeds = np.concatenate([rng.choice(np.nonzero(c.kind == 0)[0], 12, replace=False),
                            rng.choice(np.nonzero(c.kind == 1)[0], 6, replace=False)])
    sub, ids = restrict(c, seeds, 4)
    assert sub.n < c.n
    pos = np.searchsorted(ids, seeds)
    assert np.array_equal(ids[pos], seeds)
    os_ = Oracle(sub, 0.63, 2.0, n_inner=2)
    Rs, _ = os_.residual(U[:, ids])
    assert np.array_equal(Rs[:, pos], R[:, seeds])


def test_clouds_made_in_workers_equal_clouds_made_one_by_one():
    from cloudgen import make_airfoil_clouds
    specs = [(40, 16, 25, 3), (64, 24, 25, 12), (32, 20, 30, 5)]
    par = make_airfoil_clouds(specs, workers=3)
    for spec, c in zip(specs, par):
        s = make_airfoil_cloud(*spec)
        for f in ("x", "y", "nx", "ny", "kind", "row_ptr", "col", "nbr_count", "wall_loop"):
            np.testing.assert_array_equal(getattr(c, f), getattr(s, f))
