"""Pins of the oracle's free stream, initial state and OpenMP build (no GPU).

The paper fixes a flow case only by its free-stream Mach number and angle of
attack (verification cases M 0.63, AoA 2 deg and M 1.2, AoA 0 deg).  The
oracle's non-dimensional free stream (reading: rho = 1, p = 1/gamma, so that
the sound speed is 1) is checked here against the definitions those two
numbers have, computed independently from the conserved state:

* Mach number = |u| / sqrt(gamma p / rho), with p recovered from the total
  energy E = p/(gamma-1) + rho |u|^2 / 2 of eq. (1);
* angle of attack = atan2(v, u);
* reference density and sound speed exactly 1.

The initial state (free stream, then flow tangency at the wall) is checked
for what the wall condition means: zero normal momentum, unchanged tangential
momentum, density and energy, and every other row equal to the free stream.

Mutant oracles, built from the oracle's own source with one planted mistake
each (p = 1 in place of 1/gamma, sine and cosine swapped, the wall
projection left out or taken along the tangent), must fail these checks.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from cloudgen.shapes import cylinder_cloud
from oracle import ref
from oracle.build import FLAGS, SOURCES
from oracle.ref import Oracle

GAMMA = 1.4
CASES = [(0.63, 2.0), (0.85, 1.0), (1.2, 0.0), (0.3, -4.0), (0.9, 6.0), (0.5, -30.0),
         (2.0, 135.0), (0.05, -170.0)]


def check_free_stream(Uinf, mach, aoa_deg, gamma=GAMMA):
    rho = Uinf[0]
    u, v = Uinf[1] / rho, Uinf[2] / rho
    p = (gamma - 1.0) * (Uinf[3] - 0.5 * rho * (u * u + v * v))
    a = math.sqrt(gamma * p / rho)
    assert rho == 1.0, f"reference density {rho}"
    assert abs(a - 1.0) <= 1e-15, f"reference sound speed {a}"
    assert abs(math.hypot(u, v) / a - mach) <= 1e-15 * max(1.0, mach), "Mach number"
    if mach > 0:
        d = math.remainder(math.atan2(v, u) - math.radians(aoa_deg), 2 * math.pi)
        assert abs(d) <= 2e-15 * max(1.0, abs(math.radians(aoa_deg))), "angle of attack"


def check_init_state(c, U, Uinf):
    wall = c.kind == 1
    other = ~wall
    np.testing.assert_array_equal(U[:, other], np.repeat(Uinf[:, None], other.sum(), 1))
    assert wall.any()
    nx, ny = c.nx[wall], c.ny[wall]
    tx, ty = ny, -nx
    mn = U[1, wall] * nx + U[2, wall] * ny
    mt = U[1, wall] * tx + U[2, wall] * ty
    mt_inf = Uinf[1] * tx + Uinf[2] * ty
    scale = math.hypot(Uinf[1], Uinf[2]) or 1.0
    assert np.max(np.abs(mn)) <= 1e-15 * max(1.0, scale), "normal momentum at the wall"
    assert np.max(np.abs(mt - mt_inf)) <= 4e-16 * max(1.0, scale), "tangential momentum"
    np.testing.assert_array_equal(U[0, wall], Uinf[0])
    np.testing.assert_array_equal(U[3, wall], Uinf[3])


def _all_checks(lib, c):
    for mach, aoa in CASES:
        o = Oracle(c, mach, aoa, lib=lib)
        Uinf = o.free_stream()
        check_free_stream(Uinf, mach, aoa)
        check_init_state(c, o.init_state(), Uinf)


@pytest.fixture(scope="module")
def cyl():
    # walls with normals in every direction (a full circle of wall points)
    return cylinder_cloud(M=24, L=6)


@pytest.mark.parametrize("mach,aoa", CASES)
def test_free_stream_matches_mach_and_angle_definitions(mach, aoa, cyl):
    o = Oracle(cyl, mach, aoa)
    check_free_stream(o.free_stream(), mach, aoa)


@pytest.mark.parametrize("mach,aoa", CASES)
def test_initial_state_is_free_stream_with_wall_tangency(mach, aoa, cyl, tiny_cloud):
    for c in (cyl, tiny_cloud):
        o = Oracle(c, mach, aoa)
        check_init_state(c, o.init_state(), o.free_stream())


def test_free_stream_residual_state_round_trip(cyl):
    """The primitive state the oracle converts from U_inf is the one the
    checks above recover by hand (same rho, u, v, p)."""
    o = Oracle(cyl, 0.63, 2.0)
    w = ref.prim_from_cons(o.free_stream())
    al = math.radians(2.0)
    np.testing.assert_allclose(w, [1.0, 0.63 * math.cos(al), 0.63 * math.sin(al), 1 / GAMMA],
                               rtol=1e-15, atol=1e-16)


# ---------------------------------------------------------------------------
# planted mistakes

def _function_start(src, name):
    k = src.index(name + "(")
    return src.index("{", k)


def _mutant(tmp_path, tag, edits):
    """Compile the oracle source with `edits` ((function or None, old, new):
    replace the first `old` inside that function's body) into tmp_path."""
    src = open(SOURCES[0]).read()
    for fn, old, new in edits:
        start = _function_start(src, fn) if fn else 0
        k = src.index(old, start)
        src = src[:k] + new + src[k + len(old):]
    path = os.path.join(str(tmp_path), f"mut_{tag}.cpp")
    with open(path, "w") as f:
        f.write(src)
    out = os.path.join(str(tmp_path), f"libmut_{tag}.so")
    inc = ["-I", os.path.dirname(SOURCES[0])]
    flags = [f for f in FLAGS if f != "-O2"] + ["-O0", "-Wno-unknown-pragmas"]
    subprocess.run(["g++", *flags, *inc, path, "-o", out], check=True)
    return ref.bind(out)


MUTANTS = {
    "p_one": [("free_stream_prim_t", "w[3] = T(1.0 / gamma);", "w[3] = T(1.0);")],
    "sin_cos": [("free_stream_prim_t", "w[1] = mach * cos(aoa);\n  w[2] = mach * sin(aoa);",
                 "w[1] = mach * sin(aoa);\n  w[2] = mach * cos(aoa);")],
    "no_projection": [("lskum_ref_init_state", "if (c->kind[i] == 1) {", "if (false) {")],
    "tangent_projection": [
        ("lskum_ref_init_state",
         "double mn = fld(U, 1, n, i) * c->nx[i] + fld(U, 2, n, i) * c->ny[i];\n"
         "      fld(U, 1, n, i) = fld(U, 1, n, i) - mn * c->nx[i];\n"
         "      fld(U, 2, n, i) = fld(U, 2, n, i) - mn * c->ny[i];",
         "double mn = fld(U, 1, n, i) * c->ny[i] - fld(U, 2, n, i) * c->nx[i];\n"
         "      fld(U, 1, n, i) = fld(U, 1, n, i) - mn * c->ny[i];\n"
         "      fld(U, 2, n, i) = fld(U, 2, n, i) + mn * c->nx[i];")],
    "energy_without_kinetic": [("cons_from_prim", "+ 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2])",
                                "+ 0.0 * w[0]")],
}


@pytest.mark.parametrize("tag", sorted(MUTANTS))
def test_planted_mistakes_fail_the_pins(tag, tmp_path, cyl):
    lib = _mutant(tmp_path, tag, MUTANTS[tag])
    with pytest.raises(AssertionError):
        _all_checks(lib, cyl)


def test_unmutated_source_passes_through_the_same_route(tmp_path, cyl):
    lib = _mutant(tmp_path, "none", [])
    _all_checks(lib, cyl)


# ---------------------------------------------------------------------------
# the OpenMP build of the same source

def test_openmp_build_equals_the_parity_build_bitwise(tiny_cloud):
    c = tiny_cloud
    a = Oracle(c, 0.85, 1.0, n_inner=3)
    b = Oracle(c, 0.85, 1.0, n_inner=3, lib=ref.load_omp())
    Ua, ha, fa = a.iterate(a.init_state(), 2)
    Ub, hb, fb = b.iterate(b.init_state(), 2)
    assert fa == fb == 0
    np.testing.assert_array_equal(Ua, Ub)
    np.testing.assert_array_equal(ha, hb)
    np.testing.assert_array_equal(a.local_dt(Ua), b.local_dt(Ub))
