"""Pins of the oracle's reverse sweeps (CPU).

The adjoints are reverse mode through the same templated point formulas as
the forward sweeps, so they are pinned here against things that do not share
that machinery: central finite differences of the forward oracle, and the
closed-form Mach and angle-of-attack dependence of the force coefficients.

The residual is only piecewise smooth (limiter branch, stencil max/min), so a
finite difference whose stencil straddles a switch is not a derivative; such
components are recognised by the difference quotient changing between two
step sizes and skipped, as long as only a few are.
"""
import numpy as np
import pytest

from cloudgen import make_airfoil_cloud
from oracle.ref import Oracle


@pytest.fixture(scope="module")
def flow():
    c = make_airfoil_cloud(40, 16, 25, 3)
    o = Oracle(c, 0.6, 2.0, n_inner=2)
    U, _, flags = o.iterate(o.init_state(), 20)
    assert flags == 0
    return c, o, U


def _fd_column(res, U, Rb, j, m, h):
    Up = U.copy()
    Um = U.copy()
    Up[m, j] += h
    Um[m, j] -= h
    return float(np.sum(Rb * (res(Up) - res(Um)))) / (2 * h)


@pytest.mark.parametrize("n_inner", [0, 2])
def test_residual_vjp_matches_finite_difference_columns(flow, n_inner):
    c, o0, U = flow
    o = Oracle(c, 0.6, 2.0, n_inner=n_inner)
    rng = np.random.default_rng(17 + n_inner)
    Rb = rng.standard_normal((4, c.n))
    Ub, tb, flags = o.residual_vjp(U, Rb)
    assert flags == 0
    assert np.all(Ub[:, c.kind == 2] == 0.0)
    scale = np.abs(Ub).max()
    res = lambda X: o.residual(X)[0]  # noqa: E731
    wall = np.nonzero(c.kind == 1)[0]
    interior = np.nonzero(c.kind == 0)[0]
    pts = np.concatenate([rng.choice(wall, 10, replace=False),
                          rng.choice(interior, 30, replace=False)])
    checked = kinks = 0
    for j in pts:
        for m in range(4):
            h = 1e-6 * np.abs(U[m]).max()
            f1 = _fd_column(res, U, Rb, j, m, h)
            f2 = _fd_column(res, U, Rb, j, m, h / 4)
            if abs(f1 - f2) > 1e-7 * scale:
                kinks += 1
                continue
            checked += 1
            assert abs(Ub[m, j] - f2) <= 5e-8 * scale, (j, m, Ub[m, j], f2)
    assert checked >= 140 and kinks <= 20, (checked, kinks)


def test_residual_vjp_theta_matches_finite_difference(flow):
    c, o, U = flow
    rng = np.random.default_rng(5)
    Rb = rng.standard_normal((4, c.n))
    _, tb, _ = o.residual_vjp(U, Rb)
    outer = c.kind == 2
    a0 = o.params.aoa_rad

    def R(mach, aoa):
        o2 = o.with_flow(mach, aoa)
        U2 = U.copy()
        U2[:, outer] = o2.free_stream()[:, None]
        return o2.residual(U2)[0]

    h = 1e-6
    fd_m = np.sum(Rb * (R(0.6 + h, a0) - R(0.6 - h, a0))) / (2 * h)
    fd_a = np.sum(Rb * (R(0.6, a0 + h) - R(0.6, a0 - h))) / (2 * h)
    assert tb[0] == pytest.approx(fd_m, rel=1e-7)
    assert tb[1] == pytest.approx(fd_a, rel=1e-7)


def test_residual_vjp_is_linear_in_the_cotangent(flow):
    c, o, U = flow
    rng = np.random.default_rng(9)
    a, b = rng.standard_normal((2, 4, c.n))
    Ua, ta, _ = o.residual_vjp(U, a)
    Ub, tb, _ = o.residual_vjp(U, b)
    Uab, tab, _ = o.residual_vjp(U, 2.0 * a - 3.0 * b)
    np.testing.assert_allclose(Uab, 2.0 * Ua - 3.0 * Ub, rtol=0, atol=1e-12 * np.abs(Uab).max())
    np.testing.assert_allclose(tab, 2.0 * ta - 3.0 * tb, rtol=1e-12)


def test_force_coeffs_vjp_state_matches_finite_difference(flow):
    c, o, U = flow
    rng = np.random.default_rng(3)
    Jb = np.array([0.7, -1.3])
    Ub, _ = o.force_coeffs_vjp(U, Jb)
    nonwall = np.ones(c.n, bool)
    nonwall[c.wall_loop] = False
    assert np.all(Ub[:, nonwall] == 0.0)
    v = rng.standard_normal((4, c.n)) * np.abs(U).max(axis=1, keepdims=True)
    h = 1e-6
    fd = Jb @ (o.force_coeffs(U + h * v) - o.force_coeffs(U - h * v)) / (2 * h)
    assert np.sum(Ub * v) == pytest.approx(fd, rel=1e-8)


def test_force_coeffs_vjp_theta_closed_form(flow):
    """At fixed U, Cx and Cy scale as 1/M^2 (dynamic pressure M^2/2 with
    rho_inf = 1), and (Cl, Cd) is (Cx, Cy) rotated by -alpha, so
    dCl/dM = -2 Cl/M, dCd/dM = -2 Cd/M, dCl/dalpha = -Cd, dCd/dalpha = Cl."""
    c, o, U = flow
    Cl, Cd = o.force_coeffs(U)
    M = o.mach
    for Jb in (np.array([1.0, 0.0]), np.array([0.0, 1.0]), np.array([0.4, 2.5])):
        _, tb = o.force_coeffs_vjp(U, Jb)
        want = np.array([Jb[0] * (-2 * Cl / M) + Jb[1] * (-2 * Cd / M),
                         Jb[0] * (-Cd) + Jb[1] * Cl])
        np.testing.assert_allclose(tb, want, rtol=1e-12, atol=1e-15)
