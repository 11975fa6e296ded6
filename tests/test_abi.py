"""The C-ABI library loads, exports every declared entry point, and its
host-side validation rejects bad inputs before touching the GPU (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from cloudgen.shapes import cylinder_cloud
from paper_2403_13287_amd import lskum as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lskum.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(lskum_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_sweep_entry_points():
    names = declared_functions()
    for required in ["lskum_q_vars", "lskum_q_derivs", "lskum_flux_residual", "lskum_rk_stage",
                     "lskum_local_dt", "lskum_residual_norm", "lskum_force_coeffs",
                     "lskum_plan_create", "lskum_plan_destroy", "lskum_iterate"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.library_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(L._SIGS)


def test_strerror():
    assert L.strerror(0) == "ok"
    assert "static scratch" in L.strerror(L.ERR_SCRATCH_LIMIT)
    assert "validation" in L.strerror(L.ERR_BAD_CLOUD)
    assert L.strerror(12345) == "unknown status"


def _c_cloud(c, **over):
    arrs = dict(x=c.x, y=c.y, nx=c.nx, ny=c.ny, kind=c.kind, row_ptr=c.row_ptr, col=c.col,
                nbr_count=c.nbr_count, wall_loop=c.wall_loop)
    arrs.update(over)
    keep = {k: np.ascontiguousarray(v) for k, v in arrs.items()}
    k_pad = over.pop("k_pad", c.k_pad) if "k_pad" in over else c.k_pad
    s = L._Cloud(c.n, k_pad, *(keep[k].ctypes.data for k in
                               ("x", "y", "nx", "ny", "kind", "row_ptr", "col", "nbr_count",
                                "wall_loop")), int(keep["wall_loop"].size))
    return s, keep


def _create(c_struct, params=None):
    lib = L.load()
    h = ctypes.c_void_p()
    p = (params or L.Params(0.5, 0.0)).c()
    rc = lib.lskum_plan_create(ctypes.byref(h), ctypes.byref(c_struct), ctypes.byref(p), None)
    return rc, h


@pytest.fixture(scope="module")
def cyl():
    return cylinder_cloud(M=16, L=5)


def test_validation_rejects_bad_clouds(cyl):
    c = cyl
    col = c.col.copy()
    col[3] = c.n + 5  # out of range real neighbour of point 0
    s, keep = _c_cloud(c, col=col)
    assert _create(s)[0] == L.ERR_BAD_CLOUD
    col = c.col.copy()
    col[c.k_pad * 2] = 2  # self link among real entries
    s, keep = _c_cloud(c, col=col)
    assert _create(s)[0] == L.ERR_BAD_CLOUD
    cnt = c.nbr_count.copy()
    cnt[4] = c.k_pad + 1
    s, keep = _c_cloud(c, nbr_count=cnt)
    assert _create(s)[0] == L.ERR_BAD_CLOUD
    kind = c.kind.copy()
    kind[7] = 5
    s, keep = _c_cloud(c, kind=kind)
    assert _create(s)[0] == L.ERR_BAD_CLOUD
    wl = c.wall_loop.copy()
    wl[0] = int(np.nonzero(c.kind == 0)[0][0])  # not a wall point
    s, keep = _c_cloud(c, wall_loop=wl)
    assert _create(s)[0] == L.ERR_BAD_CLOUD
    x = c.x.copy()
    x[1] = np.nan
    s, keep = _c_cloud(c, x=x)
    assert _create(s)[0] == L.ERR_BAD_CLOUD
    rp = c.row_ptr.copy()
    rp[3] += 1  # row length differs from k_pad
    s, keep = _c_cloud(c, row_ptr=rp)
    assert _create(s)[0] == L.ERR_BAD_CLOUD
    wl = c.wall_loop.copy()
    wl[1] = wl[0]  # the wall loop visits a point twice
    s, keep = _c_cloud(c, wall_loop=wl)
    assert _create(s)[0] == L.ERR_BAD_CLOUD


def test_validation_rejects_bad_params(cyl):
    s, keep = _c_cloud(cyl)
    for bad in [L.Params(0.5, 0.0, cfl=0.0), L.Params(0.5, 0.0, n_inner=-1),
                L.Params(float("nan"), 0.0), L.Params(0.5, 0.0, gamma=1.0),
                L.Params(0.5, 0.0, options=8), L.Params(0.5, 0.0, options=-1)]:
        assert _create(s, bad)[0] == L.ERR_INVALID_ARG


def test_validation_rejects_bad_tunings(cyl):
    """Tile block, XCD mapping and flux block outside their sets are argument
    errors, found on the host before any device work."""
    s, keep = _c_cloud(cyl)
    lib = L.load()
    p = L.Params(0.5, 0.0).c()
    for bad in [L.Tuning(64, 1, 64), L.Tuning(256, 2, 64), L.Tuning(256, 1, 96),
                L.Tuning(256, 1, 512), L.Tuning(256, 1, -64)]:
        h = ctypes.c_void_p()
        t = bad.c()
        rc = lib.lskum_batch_plan_create(ctypes.byref(h), 1, ctypes.byref(s), ctypes.byref(p),
                                         ctypes.byref(t), None)
        assert rc == L.ERR_INVALID_ARG and not h.value, bad


def test_empty_cloud_is_rejected(cyl):
    """A cloud of no points is an argument error, found on the host before
    any device work."""
    s, keep = _c_cloud(cyl)
    s.n = 0
    rc, h = _create(s)
    assert rc == L.ERR_INVALID_ARG and not h.value


def test_null_arguments_are_rejected():
    lib = L.load()
    assert lib.lskum_plan_create(None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_q_vars(None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_q_derivs_static(None, None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_flux_residual(None, None, None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_rk_stage(None, 0, None, None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_rk4_stage(None, 0, None, None, None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_flux_residual_stage(None, 0, None, None, None, None, None, None, None, None,
                                         None) == L.ERR_INVALID_ARG
    assert lib.lskum_workspace_bytes(None) == 0
    assert lib.lskum_set_far_field(None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_flux_residual_vjp(None, None, None, None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_force_coeffs_vjp(None, None, None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_adjoint_iterate(None, None, None, None, 1, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lskum_vjp_workspace_bytes(None) == 0
    assert lib.lskum_adjoint_workspace_bytes(None) == 0
