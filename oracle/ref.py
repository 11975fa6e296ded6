"""ctypes binding of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
use this module.  Every array is a host numpy array in the component-major
layout of ``lskum_ref.h`` (shape (c, n)).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from .build import LIB, LIB_OMP, build

_c_dbl_p = ctypes.POINTER(ctypes.c_double)


class _Cloud(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("nx", ctypes.c_void_p), ("ny", ctypes.c_void_p), ("kind", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("nbr_count", ctypes.c_void_p), ("wall_loop", ctypes.c_void_p),
                ("n_wall", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("mach", ctypes.c_double),
                ("aoa_rad", ctypes.c_double), ("cfl", ctypes.c_double),
                ("venkat_k", ctypes.c_double), ("n_inner", ctypes.c_int32),
                ("options", ctypes.c_int32)]


FIRST_ORDER = 1  # options bits
MINMAX = 2
RK4 = 4

NONPHYSICAL = 1
DEGENERATE = 2

_lib = None


def load(rebuild: bool = False) -> ctypes.CDLL:
    """Load the oracle library, building it first if it is missing."""
    global _lib
    if _lib is not None and not rebuild:
        return _lib
    if rebuild or not os.path.exists(LIB):
        build()
    _lib = bind(LIB)
    return _lib


def load_omp() -> ctypes.CDLL:
    """The OpenMP build of the same source (all host cores, same results)."""
    if not os.path.exists(LIB_OMP):
        build()
    return bind(LIB_OMP)


def bind(path: str) -> ctypes.CDLL:
    """Load a build of lskum_ref.cpp at `path` and declare its signatures."""
    lib = ctypes.CDLL(os.path.abspath(path))
    vp = ctypes.c_void_p
    cp = ctypes.POINTER(_Cloud)
    pp = ctypes.POINTER(_Params)
    sig = {
        "lskum_ref_threads": (ctypes.c_int, []),
        "lskum_ref_free_stream": (None, [pp, vp]),
        "lskum_ref_q_from_prim": (None, [ctypes.c_double, vp, vp]),
        "lskum_ref_prim_from_q": (None, [ctypes.c_double, vp, vp]),
        "lskum_ref_cons_from_prim": (None, [ctypes.c_double, vp, vp]),
        "lskum_ref_prim_from_cons": (None, [ctypes.c_double, vp, vp]),
        "lskum_ref_split_flux": (None, [ctypes.c_double, ctypes.c_int, ctypes.c_int, vp, vp]),
        "lskum_ref_venkat_phi": (ctypes.c_double, [ctypes.c_double] * 4),
        "lskum_ref_minmax_phi": (ctypes.c_double, [ctypes.c_double] * 3),
        "lskum_ref_init_state": (None, [cp, pp, vp]),
        "lskum_ref_q_vars": (ctypes.c_uint, [cp, pp, vp, vp]),
        "lskum_ref_q_derivs_first": (None, [cp, vp, vp, vp]),
        "lskum_ref_q_derivs_inner": (None, [cp, vp, vp, vp]),
        "lskum_ref_q_derivs": (None, [cp, pp, vp, vp, vp]),
        "lskum_ref_flux_residual": (ctypes.c_uint, [cp, pp, vp, vp, vp, vp]),
        "lskum_ref_flux_op_counts": (ctypes.c_uint, [cp, pp, vp, vp, vp, vp]),
        "lskum_ref_local_dt": (None, [cp, pp, vp, vp]),
        "lskum_ref_rk_stage": (None, [cp, pp, ctypes.c_int, vp, vp, vp, vp]),
        "lskum_ref_rk4_stage": (None, [cp, pp, ctypes.c_int, vp, vp, vp, vp]),
        "lskum_ref_residual_norm": (ctypes.c_double, [cp, vp]),
        "lskum_ref_force_coeffs": (None, [cp, pp, vp, vp]),
        "lskum_ref_iterate": (ctypes.c_uint, [cp, pp, ctypes.c_int32, vp, vp]),
        "lskum_ref_residual_vjp": (ctypes.c_uint, [cp, pp, vp, vp, vp, vp]),
        "lskum_ref_force_coeffs_vjp": (None, [cp, pp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


# -- point-level formulas ----------------------------------------------------

def q_from_prim(prim, gamma=1.4):
    prim = _f64(prim, (4,))
    out = np.zeros(4)
    load().lskum_ref_q_from_prim(gamma, _ptr(prim), _ptr(out))
    return out


def prim_from_q(q, gamma=1.4):
    q = _f64(q, (4,))
    out = np.zeros(4)
    load().lskum_ref_prim_from_q(gamma, _ptr(q), _ptr(out))
    return out


def cons_from_prim(prim, gamma=1.4):
    prim = _f64(prim, (4,))
    out = np.zeros(4)
    load().lskum_ref_cons_from_prim(gamma, _ptr(prim), _ptr(out))
    return out


def prim_from_cons(U, gamma=1.4):
    U = _f64(U, (4,))
    out = np.zeros(4)
    load().lskum_ref_prim_from_cons(gamma, _ptr(U), _ptr(out))
    return out


def split_flux(local_prim, direction: int, sign: int, gamma=1.4):
    """G^{sign}_{dir} of the local state (rho, u_s, u_n, p); dir 0 = s, 1 = n."""
    w = _f64(local_prim, (4,))
    out = np.zeros(4)
    load().lskum_ref_split_flux(gamma, direction, sign, _ptr(w), _ptr(out))
    return out


def venkat_phi(delta, dmax, dmin, eps2):
    return load().lskum_ref_venkat_phi(float(delta), float(dmax), float(dmin), float(eps2))


def minmax_phi(delta, dmax, dmin):
    return load().lskum_ref_minmax_phi(float(delta), float(dmax), float(dmin))


# -- cloud-level sweeps ----------------------------------------------------------

class Oracle:
    """The oracle bound to one cloud and one flow condition."""

    def __init__(self, cloud, mach: float, aoa_deg: float, *, cfl: float = 0.2,
                 venkat_k: float = 5.0, n_inner: int = 2, gamma: float = 1.4,
                 options: int = 0, lib: ctypes.CDLL | None = None):
        self.lib = lib if lib is not None else load()
        self.cloud = cloud
        self.n = int(cloud.x.shape[0])
        # keep contiguous copies alive for the lifetime of the struct
        self._arrs = dict(
            x=np.ascontiguousarray(cloud.x, np.float64),
            y=np.ascontiguousarray(cloud.y, np.float64),
            nx=np.ascontiguousarray(cloud.nx, np.float64),
            ny=np.ascontiguousarray(cloud.ny, np.float64),
            kind=np.ascontiguousarray(cloud.kind, np.int8),
            row_ptr=np.ascontiguousarray(cloud.row_ptr, np.int64),
            col=np.ascontiguousarray(cloud.col, np.int32),
            nbr_count=np.ascontiguousarray(cloud.nbr_count, np.int32),
            wall_loop=np.ascontiguousarray(cloud.wall_loop, np.int32),
        )
        a = self._arrs
        self._c = _Cloud(self.n, _ptr(a["x"]), _ptr(a["y"]), _ptr(a["nx"]), _ptr(a["ny"]),
                         _ptr(a["kind"]), _ptr(a["row_ptr"]), _ptr(a["col"]),
                         _ptr(a["nbr_count"]), _ptr(a["wall_loop"]), int(a["wall_loop"].size))
        self._p = _Params(gamma, mach, math.radians(aoa_deg), cfl, venkat_k, n_inner, options)
        self.gamma, self.mach, self.aoa_deg = gamma, mach, aoa_deg
        self.cfl, self.venkat_k, self.n_inner = cfl, venkat_k, n_inner
        self.options = options

    @property
    def params(self):
        return self._p

    def _field(self, a, comps):
        return _f64(a, (comps, self.n))

    def free_stream(self):
        out = np.zeros(4)
        self.lib.lskum_ref_free_stream(ctypes.byref(self._p), _ptr(out))
        return out

    def init_state(self):
        U = np.zeros((4, self.n))
        self.lib.lskum_ref_init_state(ctypes.byref(self._c), ctypes.byref(self._p), _ptr(U))
        return U

    def q_vars(self, U):
        U = self._field(U, 4)
        q = np.zeros((4, self.n))
        flags = self.lib.lskum_ref_q_vars(ctypes.byref(self._c), ctypes.byref(self._p), _ptr(U),
                                          _ptr(q))
        return q, int(flags)

    def q_derivs_first(self, q):
        q = self._field(q, 4)
        dq = np.zeros((8, self.n))
        qlim = np.zeros((8, self.n))
        self.lib.lskum_ref_q_derivs_first(ctypes.byref(self._c), _ptr(q), _ptr(dq), _ptr(qlim))
        return dq, qlim

    def q_derivs_inner(self, q, dq_prev):
        q = self._field(q, 4)
        dq_prev = self._field(dq_prev, 8)
        out = np.zeros((8, self.n))
        self.lib.lskum_ref_q_derivs_inner(ctypes.byref(self._c), _ptr(q), _ptr(dq_prev), _ptr(out))
        return out

    def q_derivs(self, q):
        q = self._field(q, 4)
        dq = np.zeros((8, self.n))
        qlim = np.zeros((8, self.n))
        self.lib.lskum_ref_q_derivs(ctypes.byref(self._c), ctypes.byref(self._p), _ptr(q),
                                    _ptr(dq), _ptr(qlim))
        return dq, qlim

    def flux_residual(self, q, dq, qlim):
        q = self._field(q, 4)
        dq = self._field(dq, 8)
        qlim = self._field(qlim, 8)
        R = np.zeros((4, self.n))
        flags = self.lib.lskum_ref_flux_residual(ctypes.byref(self._c), ctypes.byref(self._p),
                                                 _ptr(q), _ptr(dq), _ptr(qlim), _ptr(R))
        return R, int(flags)

    def residual(self, U):
        """R(U): q-variables, derivatives and the flux residual."""
        q, f1 = self.q_vars(U)
        dq, qlim = self.q_derivs(q)
        R, f2 = self.flux_residual(q, dq, qlim)
        return R, f1 | f2

    OP_KINDS = ("add", "mul", "div", "sqrt", "exp", "log", "erf")

    def flux_op_counts(self, q, dq, qlim):
        """Floating-point operations of the flux residual on these fields,
        summed over the cloud, by kind (OP_KINDS), counted on state-dependent
        values by evaluating the same formulas with a counting scalar."""
        q = self._field(q, 4)
        dq = self._field(dq, 8)
        qlim = self._field(qlim, 8)
        out = np.zeros(7)
        flags = self.lib.lskum_ref_flux_op_counts(ctypes.byref(self._c), ctypes.byref(self._p),
                                                  _ptr(q), _ptr(dq), _ptr(qlim), _ptr(out))
        return dict(zip(self.OP_KINDS, out.tolist())), int(flags)

    def local_dt(self, U):
        U = self._field(U, 4)
        dt = np.zeros(self.n)
        self.lib.lskum_ref_local_dt(ctypes.byref(self._c), ctypes.byref(self._p), _ptr(U), _ptr(dt))
        return dt

    def rk_stage(self, stage: int, Un, R, dt, U):
        Un = self._field(Un, 4)
        R = self._field(R, 4)
        dt = _f64(dt, (self.n,))
        out = self._field(U, 4).copy()
        self.lib.lskum_ref_rk_stage(ctypes.byref(self._c), ctypes.byref(self._p), int(stage),
                                    _ptr(Un), _ptr(R), _ptr(dt), _ptr(out))
        return out

    def rk4_stage(self, stage: int, Un, Rs, dt, U):
        """Classical RK4 stage `stage`; Rs = [R of stage 0, ..., R of stage `stage`]."""
        Un = self._field(Un, 4)
        Rall = np.ascontiguousarray(np.stack([self._field(R, 4) for R in Rs[:stage + 1]]))
        dt = _f64(dt, (self.n,))
        out = self._field(U, 4).copy()
        self.lib.lskum_ref_rk4_stage(ctypes.byref(self._c), ctypes.byref(self._p), int(stage),
                                     _ptr(Un), _ptr(Rall), _ptr(dt), _ptr(out))
        return out

    def residual_norm(self, R):
        R = self._field(R, 4)
        return float(self.lib.lskum_ref_residual_norm(ctypes.byref(self._c), _ptr(R)))

    def force_coeffs(self, U):
        U = self._field(U, 4)
        out = np.zeros(2)
        self.lib.lskum_ref_force_coeffs(ctypes.byref(self._c), ctypes.byref(self._p), _ptr(U),
                                        _ptr(out))
        return out

    def residual_vjp(self, U, Rbar):
        """Cotangent of (interior and wall rows of U, theta) -> R(U), the
        outer rows being the free stream of theta = (M, alpha [rad]).
        Returns (Ubar (4, n) with zero outer rows, thetabar (2,), flags)."""
        U = self._field(U, 4)
        Rbar = self._field(Rbar, 4)
        Ubar = np.zeros((4, self.n))
        tb = np.zeros(2)
        flags = self.lib.lskum_ref_residual_vjp(ctypes.byref(self._c), ctypes.byref(self._p),
                                                _ptr(U), _ptr(Rbar), _ptr(Ubar), _ptr(tb))
        return Ubar, tb, int(flags)

    def force_coeffs_vjp(self, U, Jbar):
        """Cotangent of (U, theta) -> (Cl, Cd) with weights Jbar: (Ubar, thetabar)."""
        U = self._field(U, 4)
        Jbar = _f64(Jbar, (2,))
        Ubar = np.zeros((4, self.n))
        tb = np.zeros(2)
        self.lib.lskum_ref_force_coeffs_vjp(ctypes.byref(self._c), ctypes.byref(self._p), _ptr(U),
                                            _ptr(Jbar), _ptr(Ubar), _ptr(tb))
        return Ubar, tb

    def with_flow(self, mach: float, aoa_rad: float) -> "Oracle":
        """The same cloud and settings at another free stream (AoA in radians)."""
        o = Oracle(self.cloud, mach, math.degrees(aoa_rad), cfl=self.cfl,
                   venkat_k=self.venkat_k, n_inner=self.n_inner, gamma=self.gamma,
                   options=self.options, lib=self.lib)
        o._p.aoa_rad = aoa_rad  # exactly, not through degrees
        return o

    def iterate(self, U, iters: int):
        U = self._field(U, 4).copy()
        hist = np.zeros(max(int(iters), 1))
        flags = self.lib.lskum_ref_iterate(ctypes.byref(self._c), ctypes.byref(self._p),
                                           int(iters), _ptr(U), _ptr(hist))
        return U, hist[:iters], int(flags)

    def stages(self, U, iters: int):
        """Advance `iters` iterations stage by stage, yielding every stage's fields.

        Yields dicts with it, stage, q, dq, qlim, R, dt, U (the state after the
        stage) and norm (only on stage 0)."""
        U = self._field(U, 4).copy()
        for it in range(iters):
            dt = self.local_dt(U)
            Un = U.copy()
            Rs = []
            for s in range(4):
                q, f1 = self.q_vars(U)
                dq, qlim = self.q_derivs(q)
                R, f2 = self.flux_residual(q, dq, qlim)
                Rs.append(R)
                norm = self.residual_norm(R) if s == 0 else None
                if self.options & RK4:
                    U = self.rk4_stage(s, Un, Rs, dt, U)
                else:
                    U = self.rk_stage(s, Un, R, dt, U)
                yield dict(it=it, stage=s, q=q, dq=dq, qlim=qlim, R=R, dt=dt, U=U.copy(),
                           norm=norm, flags=f1 | f2)
