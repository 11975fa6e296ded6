"""Pins of the oracle's sweep routines (no GPU).

Each test checks the oracle against something other than itself: exactness
properties of least squares, the fixed point of the defect correction of
eq. (14)-(15), the consistency of the scheme of eq. (10) with the Euler
divergence of eq. (1) (second-order convergence), exact symmetries, a
brute-force assembly through numpy's least-squares solver, hand-computed
time steps, the stability polynomial of the Runge-Kutta scheme and the
divergence theorem for the force coefficients.
"""
import math

import numpy as np
import pytest

from cloudgen import make_airfoil_cloud, named_cloud
from cloudgen.airfoil import hilbert_order
from cloudgen.shapes import cylinder_cloud, from_lists, from_points, square_cloud
from oracle import ref
from oracle.ref import Oracle

GAMMA = 1.4


def prim_to_U(rho, u, v, p):
    return np.stack([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])


def smooth_prims(x, y):
    rho = 1.0 + 0.2 * np.sin(2.1 * x + 0.3) * np.cos(1.7 * y - 0.2)
    u = 0.55 + 0.15 * np.cos(1.3 * x) * np.sin(0.9 * y + 0.4)
    v = 0.25 + 0.1 * np.sin(1.1 * y - 0.5 * x)
    p = 1.0 / GAMMA + 0.12 * np.cos(0.8 * x + 1.9 * y)
    return rho, u, v, p


def euler_divergence(x, y, h=1e-3):
    """d Fx/dx + d Fy/dy of the Euler fluxes of eq. (1) for smooth_prims,
    by fourth-order central differences of the closed-form fluxes."""
    def fluxes(xx, yy):
        rho, u, v, p = smooth_prims(xx, yy)
        E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)
        Fx = np.stack([rho * u, rho * u * u + p, rho * u * v, (E + p) * u])
        Fy = np.stack([rho * v, rho * u * v, rho * v * v + p, (E + p) * v])
        return Fx, Fy

    def d4(f, a, b, da, db):
        return (-f(a + 2 * da, b + 2 * db) + 8 * f(a + da, b + db)
                - 8 * f(a - da, b - db) + f(a - 2 * da, b - 2 * db)) / (12 * h)

    dFx = d4(lambda a, b: fluxes(a, b)[0], x, y, h, 0.0)
    dFy = d4(lambda a, b: fluxes(a, b)[1], x, y, 0.0, h)
    return dFx + dFy


# ---------------------------------------------------------------------------
# least-squares derivatives (eq. (9), (14), (15))

def _linear_q(c, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.normal(size=4)
    b = rng.normal(size=4)
    d = rng.normal(size=4)
    q = a[:, None] + b[:, None] * c.x[None, :] + d[:, None] * c.y[None, :]
    return q, b, d


@pytest.mark.parametrize("name", ["tiny"])
def test_linear_field_gradients_exact(name, tiny_cloud):
    c = tiny_cloud
    o = Oracle(c, 0.63, 2.0)
    q, b, d = _linear_q(c)
    dq, qlim = o.q_derivs_first(q)
    scale = np.max(np.abs(np.concatenate([b, d])))
    for m in range(4):
        np.testing.assert_allclose(dq[m], b[m], atol=1e-10 * scale)
        np.testing.assert_allclose(dq[4 + m], d[m], atol=1e-10 * scale)
    for _ in range(3):
        dq = o.q_derivs_inner(q, dq)
        for m in range(4):
            np.testing.assert_allclose(dq[m], b[m], atol=1e-10 * scale)
            np.testing.assert_allclose(dq[4 + m], d[m], atol=1e-10 * scale)


def _quadratic(c, seed=1):
    rng = np.random.Generator(np.random.PCG64(seed))
    co = rng.normal(size=(4, 6))
    x, y = c.x[None, :], c.y[None, :]
    q = co[:, :1] + co[:, 1:2] * x + co[:, 2:3] * y + co[:, 3:4] * x * x \
        + co[:, 4:5] * x * y + co[:, 5:6] * y * y
    qx = co[:, 1:2] + 2 * co[:, 3:4] * x + co[:, 4:5] * y
    qy = co[:, 2:3] + co[:, 4:5] * x + 2 * co[:, 5:6] * y
    return q, np.concatenate([qx, qy])


def test_quadratic_exact_gradient_is_fixed_point_of_inner_iteration():
    """For a quadratic field, dq~_i = d.grad q_0 exactly when the previous
    iterate is the exact gradient, so one inner sweep returns it unchanged.
    A wrong sign in either modified q of eq. (14) breaks this."""
    c = square_cloud(15, seed=3)
    o = Oracle(c, 0.5, 0.0)
    q, g = _quadratic(c)
    g2 = o.q_derivs_inner(q, g)
    np.testing.assert_allclose(g2, g, rtol=0, atol=1e-10 * np.max(np.abs(g)))


def test_inner_iterations_converge_for_quadratic():
    c = square_cloud(21, seed=4)
    o = Oracle(c, 0.5, 0.0)
    q, g = _quadratic(c)
    dq, _ = o.q_derivs_first(q)
    errs = [np.max(np.abs(dq - g))]
    for _ in range(12):
        dq = o.q_derivs_inner(q, dq)
        errs.append(np.max(np.abs(dq - g)))
    # Jacobi sweeps contract (about 0.8 per sweep on this cloud)
    assert errs[0] > 1e-3
    assert errs[-1] < 0.05 * errs[0]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))


def test_first_order_derivatives_match_lstsq_and_bounds():
    c = square_cloud(9, seed=5, k=12)
    o = Oracle(c, 0.5, 0.0)
    rng = np.random.Generator(np.random.PCG64(6))
    q = rng.normal(size=(4, c.n))
    dq, qlim = o.q_derivs_first(q)
    for i in range(c.n):
        nb = c.neighbours(i)
        A = np.stack([c.x[nb] - c.x[i], c.y[nb] - c.y[i]], axis=1)
        for m in range(4):
            g, *_ = np.linalg.lstsq(A, q[m, nb] - q[m, i], rcond=None)
            np.testing.assert_allclose([dq[m, i], dq[4 + m, i]], g, rtol=1e-11, atol=1e-12)
            allv = np.concatenate([[q[m, i]], q[m, nb]])
            assert qlim[m, i] == allv.max() and qlim[4 + m, i] == allv.min()


def test_derivatives_invariant_to_stencil_order():
    c = square_cloud(11, seed=7, k=14)
    rng = np.random.Generator(np.random.PCG64(8))
    col = c.col.reshape(c.n, c.k_pad).copy()
    for i in range(c.n):
        k = c.nbr_count[i]
        col[i, :k] = rng.permutation(col[i, :k])
    c2 = from_lists(c.x, c.y, c.nx, c.ny, c.kind,
                    [col[i, :c.nbr_count[i]] for i in range(c.n)], k_pad=c.k_pad)
    q = rng.normal(size=(4, c.n))
    o1, o2 = Oracle(c, 0.5, 0.0), Oracle(c2, 0.5, 0.0)
    a, la = o1.q_derivs(q)
    b, lb = o2.q_derivs(q)
    np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-12)
    np.testing.assert_array_equal(la, lb)


# ---------------------------------------------------------------------------
# flux residual (eq. (10)-(12) with the modified q of eq. (14))

def test_free_stream_residual_is_exactly_zero(tiny_cloud):
    for mach, aoa in [(0.63, 2.0), (0.85, 1.0), (1.2, -3.0)]:
        o = Oracle(tiny_cloud, mach, aoa)
        U = np.repeat(o.free_stream()[:, None], tiny_cloud.n, axis=1)
        R, flags = o.residual(U)
        assert flags == 0
        assert np.all(R == 0.0)


def _mms_error(nside, n_inner, random_frames):
    c = square_cloud(nside, seed=11, k=20, random_frames=random_frames)
    o = Oracle(c, 0.5, 0.0, venkat_k=1e6, n_inner=n_inner)
    U = prim_to_U(*smooth_prims(c.x, c.y))
    R, flags = o.residual(U)
    assert flags == 0
    h = 1.0 / (nside - 1)
    inside = (np.minimum.reduce([c.x, 1 - c.x, c.y, 1 - c.y]) > 6 * h) & (c.kind == 0)
    exact = euler_divergence(c.x[inside], c.y[inside])
    return np.max(np.abs(R[:, inside] - exact))


@pytest.mark.parametrize("random_frames", [False, True])
def test_residual_converges_to_euler_divergence_second_order(random_frames):
    """R -> div(F_Euler) with error O(h^2) once the inner iterations of
    eq. (15) have converged (defect-corrected q~); with no inner iteration
    (first-order derivatives) the error is only O(h)."""
    e = [_mms_error(n, 40, random_frames) for n in (41, 81, 161)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert e[2] < 2e-4
    assert r1 > 3.2 and r2 > 3.2, e
    e0 = [_mms_error(n, 0, random_frames) for n in (81, 161)]
    assert e0[0] / e0[1] < 2.4, e0


def _nonuniform_state(c, o, iters=3):
    U = o.init_state()
    U, _, flags = o.iterate(U, iters)
    assert flags == 0
    return U


def test_rotation_by_quarter_turn_is_exact():
    c = cylinder_cloud()
    o = Oracle(c, 0.6, 10.0)
    U = _nonuniform_state(c, o)
    R, flags = o.residual(U)
    assert flags == 0
    # rotate everything by +90 degrees: (x, y) -> (-y, x)
    c2 = from_lists(-c.y, c.x, -c.ny, c.nx, c.kind,
                    [c.neighbours(i) for i in range(c.n)], wall_loop=c.wall_loop, k_pad=c.k_pad)
    o2 = Oracle(c2, 0.6, 100.0)
    U2 = np.stack([U[0], -U[2], U[1], U[3]])
    R2, flags2 = o2.residual(U2)
    assert flags2 == 0
    np.testing.assert_array_equal(R2, np.stack([R[0], -R[2], R[1], R[3]]))


def test_rotation_generic_angle_random_frames():
    """Covariance under a generic rotation, limiter switched off: the
    limiter bounds each q component in the global x/y basis, and the
    stencil bounds of (2 beta u, 2 beta v) only map onto each other under
    quarter turns and reflections."""
    c = square_cloud(17, seed=12, k=16, random_frames=True)
    o = Oracle(c, 0.6, 0.0, venkat_k=1e6)
    rng = np.random.Generator(np.random.PCG64(13))
    U = prim_to_U(*smooth_prims(c.x * 3, c.y * 3)) * (1 + 0.01 * rng.normal(size=(1, c.n)))
    R, flags = o.residual(U)
    assert flags == 0
    th = 0.37
    ct, st = math.cos(th), math.sin(th)
    c2 = from_lists(ct * c.x - st * c.y, st * c.x + ct * c.y, ct * c.nx - st * c.ny,
                    st * c.nx + ct * c.ny, c.kind, [c.neighbours(i) for i in range(c.n)],
                    k_pad=c.k_pad)
    o2 = Oracle(c2, 0.6, math.degrees(th), venkat_k=1e6)
    U2 = np.stack([U[0], ct * U[1] - st * U[2], st * U[1] + ct * U[2], U[3]])
    R2, _ = o2.residual(U2)
    Rrot = np.stack([R[0], ct * R[1] - st * R[2], st * R[1] + ct * R[2], R[3]])
    for m in range(4):
        assert np.max(np.abs(R2[m] - Rrot[m])) <= 1e-9 * np.max(np.abs(Rrot[m]))


def test_mirror_symmetry():
    c = cylinder_cloud()
    o = Oracle(c, 0.6, 0.0, venkat_k=5.0)
    # exactly mirror-symmetric state: rho, u, p even in y, v odd
    x, y = c.x, c.y
    y2 = y * y
    rho = 1.0 + 0.1 * np.exp(-(x * x + y2)) * np.cos(x)
    u = 0.6 + 0.1 * np.exp(-(x * x + y2))
    v = 0.2 * y * np.exp(-(x * x + y2))
    p = 1 / GAMMA + 0.05 * np.cos(x) * np.exp(-y2)
    U = prim_to_U(rho, u, v, p)
    R, flags = o.residual(U)
    assert flags == 0
    # mirror partner of every point
    key = {(float(a), float(b)): i for i, (a, b) in enumerate(zip(x, y))}
    mirror = np.array([key[(float(a), float(-b))] for a, b in zip(x, y)])
    Rm = R[:, mirror] * np.array([1, 1, -1, 1])[:, None]
    for m in range(4):
        assert np.max(np.abs(R[m] - Rm[m])) <= 1e-12 * np.max(np.abs(R[m]))


def _split_members(ds, dn, kind):
    sp = {"s+": ds < 0, "s-": ds > 0, "n-": dn > 0}
    if kind == 0:
        sp["n+"] = dn < 0
    return sp


def test_residual_brute_force_with_lstsq():
    """Assemble R at every point from numpy least squares on each half-plane
    stencil (no closed-form 2x2 inverse) and compare."""
    c = cylinder_cloud(M=24, L=6, reach=2.6)
    o = Oracle(c, 0.7, 3.0, venkat_k=5.0, n_inner=2)
    U = _nonuniform_state(c, o, iters=2)
    R, flags = o.residual(U)
    assert flags == 0
    n = c.n
    q, _ = o.q_vars(U)
    # derivatives: first-order then 2 Jacobi sweeps, all via lstsq
    def ls(i, rhs):
        nb = c.neighbours(i)
        A = np.stack([c.x[nb] - c.x[i], c.y[nb] - c.y[i]], axis=1)
        return np.linalg.lstsq(A, rhs, rcond=None)[0]
    dq = np.zeros((8, n))
    qmax = np.zeros((4, n))
    qmin = np.zeros((4, n))
    for i in range(n):
        nb = c.neighbours(i)
        for m in range(4):
            dq[[m, 4 + m], i] = ls(i, q[m, nb] - q[m, i])
            allv = np.concatenate([[q[m, i]], q[m, nb]])
            qmax[m, i], qmin[m, i] = allv.max(), allv.min()
    for _ in range(2):
        new = np.zeros_like(dq)
        for i in range(n):
            nb = c.neighbours(i)
            dx, dy = c.x[nb] - c.x[i], c.y[nb] - c.y[i]
            for m in range(4):
                qtj = q[m, nb] - 0.5 * (dx * dq[m, nb] + dy * dq[4 + m, nb])
                qt0 = q[m, i] - 0.5 * (dx * dq[m, i] + dy * dq[4 + m, i])
                new[[m, 4 + m], i] = ls(i, qtj - qt0)
        dq = new
    Rb = np.zeros((4, n))
    for i in range(n):
        if c.kind[i] == 2:
            continue
        nb = c.neighbours(i)
        t = np.array([c.ny[i], -c.nx[i]])
        nrm = np.array([c.nx[i], c.ny[i]])
        dx, dy = c.x[nb] - c.x[i], c.y[nb] - c.y[i]
        ds, dn = dx * t[0] + dy * t[1], dx * nrm[0] + dy * nrm[1]
        dist = np.sqrt(dx * dx + dy * dy)
        eps2 = (5.0 * dist) ** 3
        Rf = np.zeros(4)
        for name, mask in _split_members(ds, dn, c.kind[i]).items():
            dirn = 0 if name[0] == "s" else 1
            sign = 1 if name[1] == "+" else -1
            rows, dG = [], []
            for kk in np.nonzero(mask)[0]:
                j = nb[kk]
                qt = []
                for end in (j, i):
                    v = np.zeros(4)
                    for m in range(4):
                        delta = -0.5 * (dx[kk] * dq[m, end] + dy[kk] * dq[4 + m, end])
                        phi = ref.venkat_phi(delta, qmax[m, end] - q[m, end],
                                             qmin[m, end] - q[m, end], eps2[kk])
                        v[m] = q[m, end] + phi * delta
                    w = ref.prim_from_q(v)
                    qt.append(np.array([w[0], w[1:3] @ t, w[1:3] @ nrm, w[3]]))
                dG.append(ref.split_flux(qt[0], dirn, sign) - ref.split_flux(qt[1], dirn, sign))
                rows.append([ds[kk], dn[kk]])
            sol = np.linalg.lstsq(np.array(rows), np.array(dG), rcond=None)[0]
            Rf += sol[dirn]
        Rb[0, i] = Rf[0]
        Rb[1:3, i] = Rf[1] * t + Rf[2] * nrm
        Rb[3, i] = Rf[3]
    for m in range(4):
        assert np.max(np.abs(R[m] - Rb[m])) <= 1e-9 * np.max(np.abs(Rb[m])), m


def test_degenerate_split_stencil_is_flagged():
    # interior point 0 whose neighbours all lie at dx > 0: N_s^+ is empty
    x = [0.0, 1.0, 1.0, 2.0, 1.5, 1.2]
    y = [0.0, 1.0, -1.0, 0.3, -0.4, 0.1]
    kind = [0, 2, 2, 2, 2, 2]
    nb = [[1, 2, 3, 4, 5]] + [[0, 1, 2, 3, 4, 5][:k] + [0, 1, 2, 3, 4, 5][k + 1:] for k in range(1, 6)]
    c = from_lists(x, y, [0] * 6, [1] * 6, kind, nb)
    o = Oracle(c, 0.5, 0.0)
    U = o.init_state()
    U[0, 3] *= 1.1
    R, flags = o.residual(U)
    assert flags & ref.DEGENERATE


def test_nonphysical_state_is_flagged(tiny_cloud):
    o = Oracle(tiny_cloud, 0.63, 2.0)
    U = o.init_state()
    U[3, 123] = 0.5 * (U[1, 123] ** 2 + U[2, 123] ** 2) / U[0, 123] - 0.1  # p < 0
    _, flags = o.q_vars(U)
    assert flags & ref.NONPHYSICAL


# ---------------------------------------------------------------------------
# time step, Runge-Kutta stage, residual norm, force coefficients

def test_local_time_step_hand_computed():
    x = [0.0, 1.0, 0.0, -3.0]
    y = [0.0, 0.0, 2.0, 0.0]
    c = from_lists(x, y, [0] * 4, [1] * 4, [0, 2, 2, 2], [[1, 2, 3], [0], [0], [0]])
    o = Oracle(c, 0.5, 0.0, cfl=0.2)
    # neighbour 1: u = (3, 4), sqrt(p/rho) = 1 -> speed 8, d = 1 -> 1/8
    # neighbour 2: rho = 4, p = 1 -> sqrt = 0.5, speed 1.5, d = 2 -> 4/3
    # neighbour 3: rho = 1, p = 4 -> 3*2 = 6, d = 3 -> 1/2
    U = prim_to_U(np.array([1.0, 1.0, 4.0, 1.0]), np.array([0.0, 3.0, 0.0, 0.0]),
                  np.array([0.0, 4.0, 0.0, 0.0]), np.array([1.0, 1.0, 1.0, 4.0]))
    dt = o.local_dt(U)
    assert dt[0] == pytest.approx(0.2 / 8.0, rel=1e-15)
    assert dt[1] == pytest.approx(0.2 * 1.0 / 3.0, rel=1e-15)


def test_rk_stages_reproduce_ssp43_stability_polynomial():
    n = 5
    c = from_lists(np.arange(n, dtype=float), np.zeros(n), np.zeros(n), np.ones(n), [0] * n,
                   [[(i + 1) % n] for i in range(n)])
    o = Oracle(c, 0.5, 0.0)
    z = np.array([-0.3, -1.0, -2.0, -2.7, 0.1])
    U0 = np.ones((4, n)) * np.array([1.0, 0.5, -0.25, 3.0])[:, None]
    dt = np.ones(n)
    U = U0.copy()
    for s in range(4):
        R = -z[None, :] * U  # L(U) = z U  <=>  R = -z U
        U = o.rk_stage(s, U0, R, dt, U)
    P = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 48
    np.testing.assert_allclose(U, U0 * P[None, :], rtol=1e-14, atol=1e-15)


def test_rk_stage_boundary_conditions(tiny_cloud):
    c = tiny_cloud
    o = Oracle(c, 0.63, 2.0)
    rng = np.random.Generator(np.random.PCG64(14))
    U = o.init_state() * (1 + 0.01 * rng.normal(size=(4, c.n)))
    R = rng.normal(size=(4, c.n))
    dt = np.full(c.n, 1e-3)
    U1 = o.rk_stage(1, U, R, dt, U)
    wall, outer = c.kind == 1, c.kind == 2
    mn = U1[1] * c.nx + U1[2] * c.ny
    assert np.max(np.abs(mn[wall])) < 1e-15
    np.testing.assert_array_equal(U1[:, outer], np.repeat(o.free_stream()[:, None], outer.sum(), 1))


def test_residual_norm_definition(tiny_cloud):
    c = tiny_cloud
    o = Oracle(c, 0.63, 2.0)
    rng = np.random.Generator(np.random.PCG64(15))
    R = rng.normal(size=(4, c.n))
    keep = c.kind != 2
    assert o.residual_norm(R) == pytest.approx(math.sqrt(math.fsum(R[0, keep] ** 2)), rel=1e-14)


def test_force_coefficients_divergence_theorem(tiny_cloud):
    """Linear pressure p = p_inf + a x + b y on the closed wall polygon:
    -sum p nu = -(a, b) * area exactly (trapezoid rule exact per edge)."""
    c = tiny_cloud
    mach, aoa = 0.63, 2.0
    o = Oracle(c, mach, aoa)
    a, b = 0.3, -0.7
    p = 1 / GAMMA + a * c.x + b * c.y
    U = prim_to_U(np.ones(c.n), np.zeros(c.n), np.zeros(c.n), p)
    cl, cd = o.force_coeffs(U)
    wx, wy = c.x[c.wall_loop], c.y[c.wall_loop]
    area = 0.5 * np.sum(wx * np.roll(wy, -1) - np.roll(wx, -1) * wy)
    assert area > 0  # counter-clockwise
    Fx, Fy = -a * area / (0.5 * mach ** 2), -b * area / (0.5 * mach ** 2)
    al = math.radians(aoa)
    assert cl == pytest.approx(Fy * math.cos(al) - Fx * math.sin(al), rel=1e-12)
    assert cd == pytest.approx(Fx * math.cos(al) + Fy * math.sin(al), rel=1e-12)
    U0 = prim_to_U(np.ones(c.n), np.zeros(c.n), np.zeros(c.n), np.full(c.n, 0.9))
    assert np.max(np.abs(o.force_coeffs(U0))) < 1e-13


# ---------------------------------------------------------------------------
# relabelling

def test_hilbert_relabelling_is_bitwise_invariant():
    a = make_airfoil_cloud(160, 60, 25, 0, reorder=False)
    b = make_airfoil_cloud(160, 60, 25, 0, reorder=True)
    perm = hilbert_order(a.x, a.y)
    np.testing.assert_array_equal(b.x, a.x[perm])
    oa, ob = Oracle(a, 0.63, 2.0, venkat_k=5.0), Oracle(b, 0.63, 2.0, venkat_k=5.0)
    Ua, ha, _ = oa.iterate(oa.init_state(), 2)
    Ub, hb, _ = ob.iterate(ob.init_state(), 2)
    np.testing.assert_array_equal(Ub, Ua[:, perm])
    np.testing.assert_allclose(hb, ha, rtol=1e-13)
    Ra, _ = oa.residual(Ua)
    Rb, _ = ob.residual(Ub)
    np.testing.assert_array_equal(Rb, Ra[:, perm])
    np.testing.assert_array_equal(ob.force_coeffs(Ub), oa.force_coeffs(Ua))
