"""Pins of the oracle's scheme options (CPU): the min-max limiter and the
first-order flux (split fluxes of q itself, the paper's first-order scheme
before the defect correction of eq. (14))."""
import numpy as np
import pytest

from cloudgen.shapes import square_cloud
from oracle import ref
from oracle.ref import FIRST_ORDER, MINMAX, Oracle

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
