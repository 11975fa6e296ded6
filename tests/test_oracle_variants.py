"""Pins of the oracle's scheme options (CPU): the min-max limiter, the
first-order flux (split fluxes of q itself, the paper's first-order scheme
before the defect correction of eq. (14)) and classical RK4 time stepping."""
import numpy as np
import pytest

from cloudgen.shapes import cylinder_cloud, from_lists, square_cloud
from oracle import ref
from oracle.ref import FIRST_ORDER, MINMAX, RK4, Oracle

from test_oracle_sweep import euler_divergence, prim_to_U, smooth_prims


def test_minmax_keeps_the_reconstruction_within_the_bounds():
    """The limited increment phi*delta never leaves [dmin, dmax] (the
    reconstructed value stays inside the stencil's min/max), is left alone
    (phi = 1) when it is already inside, and reaches the bound exactly
    (to rounding) when it is not."""
    rng = np.random.default_rng(3)
    for _ in range(2000):
        dmax = abs(rng.normal()) * 10.0 ** rng.uniform(-6, 1)
        dmin = -abs(rng.normal()) * 10.0 ** rng.uniform(-6, 1)
        delta = rng.normal() * 10.0 ** rng.uniform(-6, 1)
        phi = ref.minmax_phi(delta, dmax, dmin)
        assert 0.0 <= phi <= 1.0
        assert dmin * (1 + 1e-15) <= phi * delta <= dmax * (1 + 1e-15)
        if dmin <= delta <= dmax:
            assert phi == 1.0
        else:
            bound = dmax if delta > 0 else dmin
            assert phi * delta == pytest.approx(bound, rel=1e-15)
    assert ref.minmax_phi(0.0, 1.0, -1.0) == 1.0
    assert ref.minmax_phi(0.5, 0.0, -1.0) == 0.0  # a local maximum: no increase


def test_first_order_flux_is_the_residual_of_zero_derivatives():
    """With q~ = q the residual must equal the default scheme's residual
    evaluated with every derivative set to zero (delta = 0, phi = 1), bit
    for bit, whatever the derivatives and bounds passed in."""
    c = square_cloud(15, seed=4, k=16, random_frames=True)
    o1 = Oracle(c, 0.5, 10.0, n_inner=2, options=FIRST_ORDER)
    o0 = Oracle(c, 0.5, 10.0, n_inner=2)
    U = prim_to_U(*smooth_prims(c.x, c.y))
    q, _ = o0.q_vars(U)
    rng = np.random.default_rng(1)
    dq = rng.standard_normal((8, c.n))
    qlim = np.concatenate([q + 1.0, q - 1.0])
    R1, f1 = o1.flux_residual(q, dq, qlim)
    R0, f0 = o0.flux_residual(q, np.zeros_like(dq), qlim)
    assert f1 == f0 == 0
    assert np.array_equal(R1, R0)


def _mms(nside, options, n_inner=40):
    c = square_cloud(nside, seed=11, k=20, random_frames=True)
    o = Oracle(c, 0.5, 0.0, venkat_k=1e6, n_inner=n_inner, options=options)
    U = prim_to_U(*smooth_prims(c.x, c.y))
    R, flags = o.residual(U)
    assert flags == 0
    h = 1.0 / (nside - 1)
    inside = (np.minimum.reduce([c.x, 1 - c.x, c.y, 1 - c.y]) > 6 * h) & (c.kind == 0)
    return np.max(np.abs(R[:, inside] - euler_divergence(c.x[inside], c.y[inside])))


def test_first_order_flux_converges_at_first_order():
    """The split-flux derivatives of q itself approximate div F with an O(h)
    error (the upwind splits do not cancel it): halving h halves the error,
    and the error is far above the defect-corrected scheme's."""
    e = [_mms(n, FIRST_ORDER) for n in (41, 81, 161)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 1.6 < r1 < 2.6 and 1.6 < r2 < 2.6, e
    assert e[2] > 10 * _mms(161, 0)


def test_minmax_limiter_error_lies_between_unlimited_and_first_order():
    """The min-max limiter clips the reconstruction at the smooth field's
    extrema (it does not tell an extremum from a discontinuity), so its
    error lies between the unlimited defect-corrected scheme's and the
    first-order scheme's."""
    e_mm = _mms(81, MINMAX)
    assert _mms(81, 0) < e_mm < _mms(81, FIRST_ORDER)


def _chain(n):
    """n interior points on a line, each linked to the next: the stage
    updates are pointwise, so the residuals can be set directly."""
    return from_lists(np.arange(n, dtype=float), np.zeros(n), np.zeros(n), np.ones(n), [0] * n,
                      [[(i + 1) % n] for i in range(n)])


def _rk4_step(o, U0, dt, rhs):
    """One classical RK4 step through the oracle's stage routine with
    R = rhs(U) re-evaluated at every stage input."""
    U, Rs = U0.copy(), []
    for s in range(4):
        Rs.append(rhs(U))
        U = o.rk4_stage(s, U0, Rs, dt, U)
    return U


def test_rk4_stages_reproduce_the_rk4_stability_polynomial():
    """On L(U) = z U the four stages give the degree-4 Taylor polynomial of
    exp(z) (classical RK4), not SSPRK(4,3)'s z^4/48 term."""
    n = 5
    o = Oracle(_chain(n), 0.5, 0.0, options=RK4)
    z = np.array([-0.3, -1.0, -2.0, -2.7, 0.1])
    U0 = np.ones((4, n)) * np.array([1.0, 0.5, -0.25, 3.0])[:, None]
    U = _rk4_step(o, U0, np.ones(n), lambda V: -z[None, :] * V)
    P = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    np.testing.assert_allclose(U, U0 * P[None, :], rtol=1e-14, atol=1e-15)


def test_rk4_is_fourth_order_on_a_nonlinear_ode():
    """U' = -U^2 (R = U^2) from U(0) = u0 has U(t) = u0/(1 + u0 t): the
    one-step error of RK4 falls 32-fold per halving of dt (local order 5),
    that of SSPRK(4,3) 16-fold (a wrong stage weight drops the order)."""
    n = 4
    o = Oracle(_chain(n), 0.5, 0.0, options=RK4)
    u0 = np.array([1.0, 0.7, 1.3, 0.4])
    U0 = np.repeat(u0[None, :], 4, axis=0)
    errs, errs_ssp = [], []
    for h in (0.04, 0.02, 0.01):
        dt = np.full(n, h)
        exact = u0 / (1 + u0 * h)
        errs.append(np.max(np.abs(_rk4_step(o, U0, dt, lambda V: V * V)[0] - exact)))
        U = U0.copy()
        for s in range(4):
            U = o.rk_stage(s, U0, U * U, dt, U)
        errs_ssp.append(np.max(np.abs(U[0] - exact)))
    for e in (errs, errs_ssp):
        assert e[0] > e[1] > e[2] > 0
    r = [errs[0] / errs[1], errs[1] / errs[2]]
    r_ssp = [errs_ssp[0] / errs_ssp[1], errs_ssp[1] / errs_ssp[2]]
    assert all(27 < x < 37 for x in r), r
    assert all(13.5 < x < 18 for x in r_ssp), r_ssp


def test_rk4_stage_boundary_conditions(tiny_cloud):
    c = tiny_cloud
    o = Oracle(c, 0.63, 2.0, options=RK4)
    rng = np.random.Generator(np.random.PCG64(16))
    U = o.init_state() * (1 + 0.01 * rng.normal(size=(4, c.n)))
    Rs = [rng.normal(size=(4, c.n)) for _ in range(4)]
    dt = np.full(c.n, 1e-3)
    wall, outer = c.kind == 1, c.kind == 2
    for s in range(4):
        U1 = o.rk4_stage(s, U, Rs, dt, U)
        mn = U1[1] * c.nx + U1[2] * c.ny
        assert np.max(np.abs(mn[wall])) < 1e-15
        np.testing.assert_array_equal(U1[:, outer],
                                      np.repeat(o.free_stream()[:, None], outer.sum(), 1))


def test_rk4_iterate_matches_the_stage_composition(tiny_cloud):
    """The oracle's whole-iteration routine with the RK4 bit is the stage
    routine applied to each stage's residual, and differs from SSPRK(4,3)."""
    o = Oracle(tiny_cloud, 0.63, 2.0, n_inner=1, options=RK4)
    U0 = o.init_state()
    U, h, flags = o.iterate(U0, 2)
    assert flags == 0
    st = list(o.stages(U0, 2))
    np.testing.assert_array_equal(U, st[-1]["U"])
    np.testing.assert_array_equal(h, [st[0]["norm"], st[4]["norm"]])
    Us, hs, _ = Oracle(tiny_cloud, 0.63, 2.0, n_inner=1).iterate(U0, 2)
    assert h[0] == hs[0]  # same first residual, different update
    assert np.max(np.abs(U - Us)) > 1e-8


def test_flux_operation_count_matches_the_formula_structure():
    """The counting scalar sees, per edge, the two states' densities (one
    exp and one log each) and, per used half-plane split, two split fluxes
    (one erf, one exp and two square roots each).  Which splits an edge uses
    follows from the geometry alone (s-split when ds != 0; n-split when
    dn > 0, or dn < 0 at interior points), so the totals are fixed exactly."""
    c = square_cloud(15, seed=4, k=16, random_frames=True)
    o = Oracle(c, 0.5, 10.0, n_inner=2)
    U = prim_to_U(*smooth_prims(c.x, c.y))
    q, _ = o.q_vars(U)
    dq, qlim = o.q_derivs(q)
    counts, flags = o.flux_op_counts(q, dq, qlim)
    assert flags == 0
    edges = splits = 0
    for i in range(c.n):
        if c.kind[i] == 2:
            continue
        tx, ty, nx, ny = c.ny[i], -c.nx[i], c.nx[i], c.ny[i]
        for k in range(c.nbr_count[i]):
            j = c.col[c.row_ptr[i] + k]
            dx, dy = c.x[j] - c.x[i], c.y[j] - c.y[i]
            ds, dn = dx * tx + dy * ty, dx * nx + dy * ny
            edges += 1
            splits += int(ds != 0.0) + int(dn > 0.0 or (dn < 0.0 and c.kind[i] == 0))
    assert counts["log"] == 2 * edges
    assert counts["exp"] == 2 * edges + 2 * splits
    assert counts["erf"] == 2 * splits
    assert counts["sqrt"] == 4 * splits
    # the fields agree with the plain evaluation of the same formulas
    R, _ = o.flux_residual(q, dq, qlim)
    assert np.all(np.isfinite(R))


def _structure(c):
    """Edges, used half-plane splits, interior and wall points of a cloud."""
    edges = splits = pi = pw = 0
    for i in range(c.n):
        if c.kind[i] == 2:
            continue
        pi += int(c.kind[i] == 0)
        pw += int(c.kind[i] == 1)
        tx, ty, nx, ny = c.ny[i], -c.nx[i], c.nx[i], c.ny[i]
        for k in range(c.nbr_count[i]):
            j = c.col[c.row_ptr[i] + k]
            dx, dy = c.x[j] - c.x[i], c.y[j] - c.y[i]
            ds, dn = dx * tx + dy * ty, dx * nx + dy * ny
            edges += 1
            splits += int(ds != 0.0) + int(dn > 0.0 or (dn < 0.0 and c.kind[i] == 0))
    return edges, splits, pi, pw


@pytest.mark.parametrize("which", ["square16", "square12", "square20", "cylinder"])
def test_flux_arithmetic_count_is_the_hand_count_of_the_formulas(which):
    """Additions (and subtractions), multiplications and divisions of the
    flux residual on state-dependent values, counted by hand from the
    formulas with every limiter increment non-zero (a smooth field):

    per edge, each of the 4 components at both ends: the increment
    -(dx q_x + dy q_y)/2 (3 mul, 1 add), the bound offsets (2 add), the
    Venkatakrishnan factor (7 mul, 5 add, 1 div), q~ = q + phi delta
    (1 mul, 1 add) -- 88 mul, 72 add, 8 div over the edge; the inverse
    of eq. (13) at both ends (7 mul, 3 add, 4 div each); the velocities
    in the point's frame (4 mul, 2 add each end):
        110 mul, 82 add, 16 div;
    per used split: two split fluxes (27 mul, 9 add, 3 div each) and the
    least-squares moment sums of the four flux differences (2 mul, 3 add
    each): 62 mul, 30 add, 6 div;
    per point and used split: the 2x2 solve per component (2 mul, 2 add,
    1 div); per point the momentum rotation (4 mul, 2 add).  Interior
    points use 4 splits (36 mul, 34 add, 16 div), wall points 3
    (28 mul, 26 add, 12 div).  A dropped or extra term anywhere in these
    formulas changes a total."""
    if which == "cylinder":
        c = cylinder_cloud(M=24, L=6)
    else:
        c = square_cloud(15, seed={"square16": 4, "square12": 5, "square20": 6}[which],
                         k=int(which[6:]), random_frames=True)
    o = Oracle(c, 0.5, 10.0, n_inner=2)
    U = prim_to_U(*smooth_prims(c.x, c.y))
    q, _ = o.q_vars(U)
    dq, qlim = o.q_derivs(q)
    counts, flags = o.flux_op_counts(q, dq, qlim)
    assert flags == 0
    E, S, PI, PW = _structure(c)
    assert PI > 0 and S > E
    assert counts["mul"] == 110 * E + 62 * S + 36 * PI + 28 * PW
    assert counts["add"] == 82 * E + 30 * S + 34 * PI + 26 * PW
    assert counts["div"] == 16 * E + 6 * S + 16 * PI + 12 * PW
    if which == "cylinder":
        assert PW > 0
