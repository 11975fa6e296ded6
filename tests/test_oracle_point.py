"""Pins of the oracle's point-level formulas against kinetic theory,
textbook gas dynamics and numerical quadrature (no GPU).

* q-variables (eq. (13)): the Maxwellian whose logarithm is linear in
  (1, v1, v2, |v|^2/2) with coefficients q must have the moments
  (rho, u, v, p) the q-variables were built from.  The moments are taken by
  adaptive quadrature, so this pins every term of eq. (13), including the
  ln(beta)/(gamma-1) coefficient (gamma = 1.4 <=> 5 degrees of freedom).
* Kinetic split fluxes: half-range moments of the Maxwellian (eq. (2) with
  the CIR split of eq. (3)) by quadrature; G+ + G- equal to the Euler flux
  of eq. (1); limits and reflection symmetry.
* Venkatakrishnan factor: range, monotonicity and limits.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import ref

GAMMA = 1.4
DOF = 2.0 / (GAMMA - 1.0)  # 5: two translational + three internal
INTERNAL = DOF - 2.0


def random_prims(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = rng.uniform(0.2, 3.0, n)
    u = rng.uniform(-2.0, 2.0, n)
    v = rng.uniform(-2.0, 2.0, n)
    p = rng.uniform(0.2, 3.0, n)
    return np.stack([rho, u, v, p], axis=1)


def test_gamma_golden_matches_listing():
    # tests/golden/gamma.txt: 1/(gamma-1) printed as 2.5 in the q-variable listings
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "gamma.txt")
    vals = {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    assert vals["inv_gamma_minus_one"] == 2.5
    assert abs(1.0 / (GAMMA - 1.0) - vals["inv_gamma_minus_one"]) < 1e-15


@pytest.mark.parametrize("seed", [0, 1])
def test_prim_q_roundtrip(seed):
    for w in random_prims(50, seed):
        q = ref.q_from_prim(w)
        w2 = ref.prim_from_q(q)
        np.testing.assert_allclose(w2, w, rtol=1e-13, atol=1e-14)
        U = ref.cons_from_prim(w)
        np.testing.assert_allclose(ref.prim_from_cons(U), w, rtol=1e-13, atol=1e-14)


def _line_moment(a, b, k):
    """int v^k exp(a v + b v^2 / 2) dv over R (b < 0) by adaptive quadrature."""
    c = -a / b  # centre of the Gaussian, used only to place the breakpoints
    s = 1.0 / math.sqrt(-b)
    f = lambda t: t ** k * math.exp(a * t + 0.5 * b * t * t - (a * c + 0.5 * b * c * c))
    val = 0.0
    for lo, hi in [(-math.inf, c - 8 * s), (c - 8 * s, c), (c, c + 8 * s), (c + 8 * s, math.inf)]:
        val += integrate.quad(f, lo, hi, epsabs=0, epsrel=2e-14, limit=200)[0]
    return val * math.exp(a * c + 0.5 * b * c * c)


@pytest.mark.parametrize("seed", [3])
def test_q_is_log_maxwellian(seed):
    """ln F = q1 - (D/2) ln(pi) + q2 v1 + q3 v2 + q4 (|v|^2 + |I|^2)/2."""
    for w in random_prims(6, seed):
        q = ref.q_from_prim(w)
        # one-dimensional factors: translational v1, v2 and one internal dof
        m1 = [_line_moment(q[1], q[3], k) for k in range(3)]
        m2 = [_line_moment(q[2], q[3], k) for k in range(3)]
        mi = _line_moment(0.0, q[3], 0)
        scale = math.exp(q[0] - 0.5 * DOF * math.log(math.pi)) * mi ** INTERNAL
        rho = scale * m1[0] * m2[0]
        u = m1[1] / m1[0]
        v = m2[1] / m2[0]
        var = m1[2] / m1[0] - u * u  # <(v1 - u)^2> = p / rho
        np.testing.assert_allclose([rho, u, v, rho * var], w, rtol=1e-10, atol=1e-12)


def _half_moments(ud, beta, sign):
    """int_{sign v > 0} v^k f(v) dv, k = 0..3, f the 1D Maxwellian about ud."""
    norm = math.sqrt(beta / math.pi)
    out = []
    for k in range(4):
        f = lambda t: t ** k * norm * math.exp(-beta * (t - ud) ** 2)
        lo, hi = (0.0, math.inf) if sign > 0 else (-math.inf, 0.0)
        # split at the peak when it lies inside the half line
        pts = [lo, hi]
        if lo < ud < hi:
            pts = [lo, ud, hi]
        val = sum(integrate.quad(f, a, b, epsabs=0, epsrel=2e-14, limit=200)[0]
                  for a, b in zip(pts[:-1], pts[1:]))
        out.append(val)
    return out


def split_flux_by_quadrature(w, direction, sign):
    """Half-range moments of v_d * (1, v_s, v_n, |v|^2/2 + internal energy) * F."""
    rho, us, un, p = w
    beta = rho / (2.0 * p)
    ud, uo = (us, un) if direction == 0 else (un, us)
    M = _half_moments(ud, beta, sign)
    # moments of the other translational direction (full line): <1>, <v>, <v^2>
    o0, o1, o2 = 1.0, uo, uo * uo + 1.0 / (2.0 * beta)
    e_int = INTERNAL / (4.0 * beta)  # internal energy per unit mass
    mass = rho * M[1] * o0
    mom_d = rho * M[2] * o0
    mom_o = rho * M[1] * o1
    energy = rho * (0.5 * M[3] * o0 + 0.5 * M[1] * o2 + e_int * M[1] * o0)
    G = np.zeros(4)
    G[0] = mass
    G[1 if direction == 0 else 2] = mom_d
    G[2 if direction == 0 else 1] = mom_o
    G[3] = energy
    return G


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("sign", [1, -1])
def test_split_flux_matches_half_range_quadrature(direction, sign):
    for w in random_prims(8, 10 + direction * 2 + (sign > 0)):
        G = ref.split_flux(w, direction, sign)
        Gq = split_flux_by_quadrature(w, direction, sign)
        scale = np.max(np.abs(Gq)) + 1e-300
        np.testing.assert_allclose(G, Gq, rtol=0, atol=1e-11 * scale)


def euler_flux(w, direction):
    """Inviscid flux of eq. (1) in the local frame (mass, s-mom, n-mom, energy)."""
    rho, us, un, p = w
    E = p / (GAMMA - 1.0) + 0.5 * rho * (us * us + un * un)
    ud = us if direction == 0 else un
    F = np.array([rho * ud, rho * us * ud, rho * un * ud, (E + p) * ud])
    F[1 if direction == 0 else 2] += p
    return F


@pytest.mark.parametrize("direction", [0, 1])
def test_split_fluxes_sum_to_euler_flux(direction):
    for w in random_prims(200, 20 + direction):
        Gp = ref.split_flux(w, direction, 1)
        Gm = ref.split_flux(w, direction, -1)
        F = euler_flux(w, direction)
        np.testing.assert_allclose(Gp + Gm, F, rtol=1e-13, atol=1e-13 * np.max(np.abs(F)))


@pytest.mark.parametrize("direction", [0, 1])
def test_split_flux_supersonic_limits(direction):
    # S = u_d sqrt(beta) = 40: the whole distribution moves in +d
    w = np.array([1.2, 0.0, 0.0, 0.9])
    beta = w[0] / (2 * w[3])
    w[1 + direction] = 40.0 / math.sqrt(beta)
    w[2 - direction] = 0.3
    F = euler_flux(w, direction)
    np.testing.assert_array_equal(ref.split_flux(w, direction, -1), np.zeros(4))
    np.testing.assert_allclose(ref.split_flux(w, direction, 1), F, rtol=1e-15)


@pytest.mark.parametrize("direction", [0, 1])
def test_split_flux_reflection(direction):
    """G^-(u_d) = -Pi G^+(-u_d), Pi negating the d-momentum."""
    for w in random_prims(50, 30 + direction):
        wr = w.copy()
        wr[1 + direction] = -wr[1 + direction]
        Gm = ref.split_flux(w, direction, -1)
        Gp = ref.split_flux(wr, direction, 1)
        Pi = np.ones(4)
        Pi[1 + direction] = -1.0
        np.testing.assert_allclose(Gm, -Pi * Gp, rtol=1e-14, atol=1e-15)


def test_venkat_range_and_limits():
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(2000):
        delta = rng.normal() * 10 ** rng.uniform(-6, 1)
        dmax = abs(rng.normal()) * 10 ** rng.uniform(-6, 1)
        dmin = -abs(rng.normal()) * 10 ** rng.uniform(-6, 1)
        eps2 = 10 ** rng.uniform(-12, 0) if rng.uniform() < 0.8 else 0.0
        phi = ref.venkat_phi(delta, dmax, dmin, eps2)
        assert 0.0 <= phi <= 1.0
        # eps = 0: the limited value stays inside the stencil bounds
        phi0 = ref.venkat_phi(delta, dmax, dmin, 0.0)
        bound = dmax if delta > 0 else dmin
        assert abs(phi0 * delta) <= abs(bound) * (1 + 1e-14)
    assert ref.venkat_phi(0.0, 1.0, -1.0, 0.0) == 1.0
    # a large eps switches the limiter off
    assert ref.venkat_phi(0.3, 1e-8, -1e-8, 1e6) == pytest.approx(1.0, abs=1e-6)
    # small ratio r = D/delta: phi ~ r ; large ratio: phi -> 1
    assert ref.venkat_phi(1.0, 1e-6, -1.0, 0.0) == pytest.approx(1e-6, rel=1e-5)
    assert ref.venkat_phi(1.0, 1e6, -1.0, 0.0) == pytest.approx(1.0, abs=1e-5)
    # no bound room at all: fully limited
    assert ref.venkat_phi(0.5, 0.0, -1.0, 0.0) == 0.0
