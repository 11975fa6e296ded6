"""Python binding of ``liblskum.so`` (argument marshalling only).

Every sweep function has the name of its C entry point in ``include/lskum.h``
and takes torch tensors: FP64, contiguous, on the plan's GPU, shaped (n, c)
for a c-component field (point-major, exactly the C layout).  The work
runs in the library's HIP kernels on the current torch stream (or the
stream passed in); nothing is computed in Python.  A missing library is an
error: there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _build

OK = 0
ERR_INVALID_ARG = -1
ERR_BAD_CLOUD = -2
ERR_HIP = -3
ERR_NONPHYSICAL = -4
ERR_NO_MEMORY = -5
ERR_DEGENERATE = -6
ERR_SCRATCH_LIMIT = -7

FIRST_ORDER = 1  # Params.options bits
MINMAX = 2
RK4 = 4


class LskumError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class _Cloud(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("k_pad", ctypes.c_int32),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("nx", ctypes.c_void_p), ("ny", ctypes.c_void_p),
                ("kind", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("nbr_count", ctypes.c_void_p),
                ("wall_loop", ctypes.c_void_p), ("n_wall", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("mach", ctypes.c_double),
                ("aoa_rad", ctypes.c_double), ("cfl", ctypes.c_double),
                ("venkat_k", ctypes.c_double), ("n_inner", ctypes.c_int32),
                ("options", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("xcd_contiguous", ctypes.c_int32),
                ("flux_block", ctypes.c_int32)]


# name -> (restype, argtypes); 'v' = void*, 'i' = int32, 'd' = double
_SIGS = {
    "lskum_plan_create": (ctypes.c_int, "vvvv"),
    "lskum_batch_plan_create": (ctypes.c_int, "vivvvv"),
    "lskum_plan_destroy": (ctypes.c_int, "v"),
    "lskum_plan_set_params": (ctypes.c_int, "vv"),
    "lskum_plan_set_tuning": (ctypes.c_int, "vv"),
    "lskum_plan_n": (ctypes.c_int32, "v"),
    "lskum_plan_clouds": (ctypes.c_int32, "v"),
    "lskum_plan_offset": (ctypes.c_int32, "vi"),
    "lskum_init_state": (ctypes.c_int, "vvv"),
    "lskum_q_vars": (ctypes.c_int, "vvvv"),
    "lskum_q_derivs": (ctypes.c_int, "vvvvvv"),
    "lskum_q_derivs_static": (ctypes.c_int, "vvvvv"),
    "lskum_flux_residual": (ctypes.c_int, "vvvvvv"),
    "lskum_local_dt": (ctypes.c_int, "vvvv"),
    "lskum_rk_stage": (ctypes.c_int, "vivvvvv"),
    "lskum_rk4_stage": (ctypes.c_int, "vivvvvvv"),
    "lskum_flux_residual_stage": (ctypes.c_int, "vivvvvvvvvv"),
    "lskum_residual_norm": (ctypes.c_int, "vvvv"),
    "lskum_force_coeffs": (ctypes.c_int, "vvvv"),
    "lskum_workspace_bytes": (ctypes.c_size_t, "v"),
    "lskum_iterate": (ctypes.c_int, "vivvvv"),
    "lskum_batch_run": (ctypes.c_int, "vivvvv"),
    "lskum_graph_create": (ctypes.c_int, "vvivvivv"),
    "lskum_graph_launch": (ctypes.c_int, "vv"),
    "lskum_graph_destroy": (ctypes.c_int, "v"),
    "lskum_status": (ctypes.c_int, "vv"),
    "lskum_clear_status": (ctypes.c_int, "vv"),
    "lskum_strerror": (ctypes.c_char_p, "i"),
    "lskum_set_far_field": (ctypes.c_int, "vvv"),
    "lskum_vjp_workspace_bytes": (ctypes.c_size_t, "v"),
    "lskum_flux_residual_vjp": (ctypes.c_int, "vvvvvvv"),
    "lskum_force_coeffs_vjp": (ctypes.c_int, "vvvvvv"),
    "lskum_adjoint_workspace_bytes": (ctypes.c_size_t, "v"),
    "lskum_adjoint_iterate": (ctypes.c_int, "vvvvivvv"),
    "lskum_adjoint_total": (ctypes.c_int, "vvvvvvvv"),
}
_CT = {"v": ctypes.c_void_p, "i": ctypes.c_int32, "d": ctypes.c_double}

_lib = None


def library_path() -> str:
    """The in-tree library, or LSKUM_LIBRARY if set (an alternative build)."""
    return os.environ.get("LSKUM_LIBRARY") or _build.LIB


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2403_13287_amd._build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = [_CT[a] for a in args]
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().lskum_strerror(int(code)).decode()


def _check(rc: int, where: str):
    if rc != OK:
        raise LskumError(rc, where)


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


@dataclass
class Params:
    mach: float
    aoa_deg: float
    cfl: float = 0.2
    venkat_k: float = 5.0
    n_inner: int = 2
    gamma: float = 1.4
    aoa_rad: float | None = None  # if set, the angle in radians (aoa_deg ignored)
    options: int = 0              # FIRST_ORDER | MINMAX | RK4 bits (0: the default scheme)

    def alpha(self) -> float:
        return float(self.aoa_rad) if self.aoa_rad is not None else math.radians(self.aoa_deg)

    def c(self) -> _Params:
        return _Params(self.gamma, self.mach, self.alpha(), self.cfl,
                       self.venkat_k, int(self.n_inner), int(self.options))


@dataclass(frozen=True)
class Tuning:
    """Block size of the gather kernels (points per LDS tile: 128, 256, 512),
    XCD-contiguous block mapping of the flux and per-point kernels (the
    derivative passes and the local time step always use it), and the flux
    kernel's block size (64, 128, 256); results do not depend on it."""
    block: int = 512
    xcd_contiguous: int = 0
    flux_block: int = 64

    def c(self) -> _Tuning:
        return _Tuning(int(self.block), int(self.xcd_contiguous), int(self.flux_block))

    def key(self) -> str:
        return f"{self.block}/{self.xcd_contiguous}/{self.flux_block}"


def _cloud_struct(cloud):
    n = int(cloud.x.shape[0])
    k_pad = int(getattr(cloud, "k_pad", 0)) or int(cloud.col.size // n)
    keep = dict(
        x=np.ascontiguousarray(cloud.x, np.float64), y=np.ascontiguousarray(cloud.y, np.float64),
        nx=np.ascontiguousarray(cloud.nx, np.float64), ny=np.ascontiguousarray(cloud.ny, np.float64),
        kind=np.ascontiguousarray(cloud.kind, np.int8),
        row_ptr=np.ascontiguousarray(cloud.row_ptr, np.int64),
        col=np.ascontiguousarray(cloud.col, np.int32),
        nbr_count=np.ascontiguousarray(cloud.nbr_count, np.int32),
        wall_loop=np.ascontiguousarray(cloud.wall_loop, np.int32))
    c = _Cloud(n, k_pad, *(keep[k].ctypes.data for k in
                           ("x", "y", "nx", "ny", "kind", "row_ptr", "col", "nbr_count",
                            "wall_loop")), int(keep["wall_loop"].size))
    return c, keep


class Plan:
    """Owner of an ``lskum_plan`` handle (device geometry + connectivity).

    ``cloud`` is one cloud or a list of clouds (a batched plan: the clouds are
    concatenated in order; ``params`` is then one Params per cloud or one
    shared by all)."""

    def __init__(self, cloud, params, stream=None, tuning: Tuning | None = None):
        self.lib = load()
        clouds = list(cloud) if isinstance(cloud, (list, tuple)) else [cloud]
        plist = list(params) if isinstance(params, (list, tuple)) else [params] * len(clouds)
        if len(plist) != len(clouds):
            raise ValueError("one Params per cloud")
        self.device = torch.cuda.current_device()
        structs, keeps = zip(*(_cloud_struct(c) for c in clouds))
        carr = (_Cloud * len(structs))(*structs)
        parr = (_Params * len(plist))(*(p.c() for p in plist))
        self._keep = keeps
        h = ctypes.c_void_p()
        tun = tuning.c() if tuning is not None else None
        rc = self.lib.lskum_batch_plan_create(ctypes.byref(h), len(structs), carr, parr,
                                              ctypes.byref(tun) if tun is not None else None,
                                              _stream(stream))
        _check(rc, "lskum_batch_plan_create")
        self.handle = h
        self.params = plist
        self.tuning = tuning or Tuning()
        self.n = int(self.lib.lskum_plan_n(h))
        self.n_clouds = int(self.lib.lskum_plan_clouds(h))
        self.offsets = [int(self.lib.lskum_plan_offset(h, c)) for c in range(self.n_clouds + 1)]

    def set_params(self, params):
        plist = list(params) if isinstance(params, (list, tuple)) else [params] * self.n_clouds
        arr = (_Params * len(plist))(*(p.c() for p in plist))
        if len(plist) != self.n_clouds:
            raise ValueError("one Params per cloud")
        _check(self.lib.lskum_plan_set_params(self.handle, arr), "lskum_plan_set_params")
        self.params = plist

    def set_tuning(self, tuning: Tuning):
        t = tuning.c()
        _check(self.lib.lskum_plan_set_tuning(self.handle, ctypes.byref(t)), "lskum_plan_set_tuning")
        self.tuning = tuning

    def destroy(self):
        if getattr(self, "handle", None):
            self.lib.lskum_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def cloud_slice(self, c: int) -> slice:
        return slice(self.offsets[c], self.offsets[c + 1])

    # tensor helpers (allocation is torch's; the library never allocates fields)
    def field(self, comps: int) -> torch.Tensor:
        shape = (self.n, comps) if comps > 1 else (self.n,)
        return torch.empty(shape, dtype=torch.float64, device=f"cuda:{self.device}")

    def _arg(self, t: torch.Tensor, comps: int, name: str) -> int:
        shape = (self.n, comps) if comps > 1 else (self.n,)
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda \
                or t.device.index != self.device or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"{name}: need a contiguous float64 cuda:{self.device} tensor of shape {shape}")
        return t.data_ptr()


def plan_create(cloud, params: Params, stream=None) -> Plan:
    return Plan(cloud, params, stream)


def lskum_init_state(plan: Plan, U, stream=None):
    _check(plan.lib.lskum_init_state(plan.handle, plan._arg(U, 4, "U"), _stream(stream)),
           "lskum_init_state")


def lskum_q_vars(plan: Plan, U, q, stream=None):
    _check(plan.lib.lskum_q_vars(plan.handle, plan._arg(U, 4, "U"), plan._arg(q, 4, "q"),
                                 _stream(stream)), "lskum_q_vars")


def lskum_q_derivs(plan: Plan, q, dq, qlim, work, stream=None):
    _check(plan.lib.lskum_q_derivs(plan.handle, plan._arg(q, 4, "q"), plan._arg(dq, 8, "dq"),
                                   plan._arg(qlim, 8, "qlim"), plan._arg(work, 16, "work"),
                                   _stream(stream)), "lskum_q_derivs")


def lskum_q_derivs_static(plan: Plan, q, dq, qlim, stream=None):
    """lskum_q_derivs with the library's static scratch in place of `work`
    (the call allocates nothing; plans up to 2^20 points when n_inner > 0)."""
    _check(plan.lib.lskum_q_derivs_static(plan.handle, plan._arg(q, 4, "q"),
                                          plan._arg(dq, 8, "dq"), plan._arg(qlim, 8, "qlim"),
                                          _stream(stream)), "lskum_q_derivs_static")


def lskum_flux_residual(plan: Plan, q, dq, qlim, R, stream=None):
    _check(plan.lib.lskum_flux_residual(plan.handle, plan._arg(q, 4, "q"), plan._arg(dq, 8, "dq"),
                                        plan._arg(qlim, 8, "qlim"), plan._arg(R, 4, "R"),
                                        _stream(stream)), "lskum_flux_residual")


def lskum_flux_residual_stage(plan: Plan, stage: int, q, dq, qlim, Un, dt, R, U, q_next,
                              stream=None):
    """Flux residual, SSP stage `stage` of U and the next stage's q in one launch."""
    _check(plan.lib.lskum_flux_residual_stage(
        plan.handle, int(stage), plan._arg(q, 4, "q"), plan._arg(dq, 8, "dq"),
        plan._arg(qlim, 8, "qlim"), plan._arg(Un, 4, "Un"), plan._arg(dt, 1, "dt"),
        plan._arg(R, 4, "R"), plan._arg(U, 4, "U"), plan._arg(q_next, 4, "q_next"),
        _stream(stream)), "lskum_flux_residual_stage")


def lskum_local_dt(plan: Plan, U, dt, stream=None):
    _check(plan.lib.lskum_local_dt(plan.handle, plan._arg(U, 4, "U"), plan._arg(dt, 1, "dt"),
                                   _stream(stream)), "lskum_local_dt")


def lskum_rk_stage(plan: Plan, stage: int, Un, R, dt, U, stream=None):
    _check(plan.lib.lskum_rk_stage(plan.handle, int(stage), plan._arg(Un, 4, "Un"),
                                   plan._arg(R, 4, "R"), plan._arg(dt, 1, "dt"),
                                   plan._arg(U, 4, "U"), _stream(stream)), "lskum_rk_stage")


def lskum_rk4_stage(plan: Plan, stage: int, Un, R, dt, acc, U, stream=None):
    _check(plan.lib.lskum_rk4_stage(plan.handle, int(stage), plan._arg(Un, 4, "Un"),
                                    plan._arg(R, 4, "R"), plan._arg(dt, 1, "dt"),
                                    plan._arg(acc, 4, "acc"), plan._arg(U, 4, "U"),
                                    _stream(stream)), "lskum_rk4_stage")


def _scalar_out(plan: Plan, t, count: int, name: str) -> int:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda \
            or t.device.index != plan.device or not t.is_contiguous() or t.numel() < count:
        raise ValueError(f"{name}: need a float64 cuda tensor with >= {count} elements")
    return t.data_ptr()


def lskum_residual_norm(plan: Plan, R, out, stream=None):
    """Per-cloud norms into out[0:n_clouds]."""
    _check(plan.lib.lskum_residual_norm(plan.handle, plan._arg(R, 4, "R"),
                                        _scalar_out(plan, out, plan.n_clouds, "out"),
                                        _stream(stream)), "lskum_residual_norm")


def lskum_force_coeffs(plan: Plan, U, clcd, stream=None):
    """Per-cloud (Cl, Cd) into clcd[2c], clcd[2c+1]."""
    _check(plan.lib.lskum_force_coeffs(plan.handle, plan._arg(U, 4, "U"),
                                       _scalar_out(plan, clcd, 2 * plan.n_clouds, "clcd"),
                                       _stream(stream)), "lskum_force_coeffs")


def lskum_workspace_bytes(plan: Plan) -> int:
    return int(plan.lib.lskum_workspace_bytes(plan.handle))


def workspace(plan: Plan) -> torch.Tensor:
    ws = torch.empty(lskum_workspace_bytes(plan), dtype=torch.uint8, device=f"cuda:{plan.device}")
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace not 256-byte aligned")
    return ws


def lskum_iterate(plan: Plan, iters: int, U, hist, ws, stream=None):
    """hist: iters x n_clouds residual norms (or None)."""
    hp = 0 if hist is None else _scalar_out(plan, hist, int(iters) * plan.n_clouds, "hist")
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or ws.numel() < lskum_workspace_bytes(plan):
        raise ValueError("ws: need a cuda tensor of lskum_workspace_bytes(plan) bytes")
    _check(plan.lib.lskum_iterate(plan.handle, int(iters), plan._arg(U, 4, "U"), hp, ws.data_ptr(),
                                  _stream(stream)), "lskum_iterate")


def lskum_batch_run(plan: Plan, iters: int, U, hist, ws, stream=None):
    """hist: n_clouds x iters residual norms, cloud-major (or None)."""
    hp = 0 if hist is None else _scalar_out(plan, hist, int(iters) * plan.n_clouds, "hist")
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or ws.numel() < lskum_workspace_bytes(plan):
        raise ValueError("ws: need a cuda tensor of lskum_workspace_bytes(plan) bytes")
    _check(plan.lib.lskum_batch_run(plan.handle, int(iters), plan._arg(U, 4, "U"), hp,
                                    ws.data_ptr(), _stream(stream)), "lskum_batch_run")


def lskum_set_far_field(plan: Plan, U, stream=None):
    _check(plan.lib.lskum_set_far_field(plan.handle, plan._arg(U, 4, "U"), _stream(stream)),
           "lskum_set_far_field")


def lskum_vjp_workspace_bytes(plan: Plan) -> int:
    return int(plan.lib.lskum_vjp_workspace_bytes(plan.handle))


def vjp_workspace(plan: Plan) -> torch.Tensor:
    ws = torch.empty(lskum_vjp_workspace_bytes(plan), dtype=torch.uint8,
                     device=f"cuda:{plan.device}")
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace not 256-byte aligned")
    return ws


def lskum_flux_residual_vjp(plan: Plan, U, Rbar, Ubar, thetabar, ws, stream=None):
    """Ubar (n, 4) and thetabar (n_clouds, 2) = (Mach, alpha [rad]) cotangents."""
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or \
            ws.numel() < lskum_vjp_workspace_bytes(plan):
        raise ValueError("ws: need a cuda tensor of lskum_vjp_workspace_bytes(plan) bytes")
    _check(plan.lib.lskum_flux_residual_vjp(plan.handle, plan._arg(U, 4, "U"),
                                            plan._arg(Rbar, 4, "Rbar"), plan._arg(Ubar, 4, "Ubar"),
                                            _scalar_out(plan, thetabar, 2 * plan.n_clouds,
                                                        "thetabar"),
                                            ws.data_ptr(), _stream(stream)),
           "lskum_flux_residual_vjp")


def lskum_force_coeffs_vjp(plan: Plan, U, Jbar, Ubar, thetabar, stream=None):
    """Jbar: (n_clouds, 2) weights of (Cl, Cd); Ubar (n, 4); thetabar (n_clouds, 2)."""
    _check(plan.lib.lskum_force_coeffs_vjp(plan.handle, plan._arg(U, 4, "U"),
                                           _scalar_out(plan, Jbar, 2 * plan.n_clouds, "Jbar"),
                                           plan._arg(Ubar, 4, "Ubar"),
                                           _scalar_out(plan, thetabar, 2 * plan.n_clouds,
                                                       "thetabar"),
                                           _stream(stream)), "lskum_force_coeffs_vjp")


def lskum_adjoint_workspace_bytes(plan: Plan) -> int:
    return int(plan.lib.lskum_adjoint_workspace_bytes(plan.handle))


def adjoint_workspace(plan: Plan) -> torch.Tensor:
    ws = torch.empty(lskum_adjoint_workspace_bytes(plan), dtype=torch.uint8,
                     device=f"cuda:{plan.device}")
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace not 256-byte aligned")
    return ws


def lskum_adjoint_iterate(plan: Plan, U, g, Lam, iters: int, hist, ws, stream=None):
    """hist: iters x n_clouds adjoint residual norms (or None)."""
    hp = 0 if hist is None else _scalar_out(plan, hist, int(iters) * plan.n_clouds, "hist")
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or \
            ws.numel() < lskum_adjoint_workspace_bytes(plan):
        raise ValueError("ws: need a cuda tensor of lskum_adjoint_workspace_bytes(plan) bytes")
    _check(plan.lib.lskum_adjoint_iterate(plan.handle, plan._arg(U, 4, "U"), plan._arg(g, 4, "g"),
                                          plan._arg(Lam, 4, "Lambda"), int(iters), hp,
                                          ws.data_ptr(), _stream(stream)), "lskum_adjoint_iterate")


def lskum_adjoint_total(plan: Plan, U, Lam, Jbar, total, partial, ws, stream=None):
    """total (and partial, or None): (n_clouds, 2) derivatives of Jbar . (Cl, Cd)."""
    pp = 0 if partial is None else _scalar_out(plan, partial, 2 * plan.n_clouds, "partial")
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or \
            ws.numel() < lskum_adjoint_workspace_bytes(plan):
        raise ValueError("ws: need a cuda tensor of lskum_adjoint_workspace_bytes(plan) bytes")
    _check(plan.lib.lskum_adjoint_total(plan.handle, plan._arg(U, 4, "U"),
                                        plan._arg(Lam, 4, "Lambda"),
                                        _scalar_out(plan, Jbar, 2 * plan.n_clouds, "Jbar"),
                                        _scalar_out(plan, total, 2 * plan.n_clouds, "total"), pp,
                                        ws.data_ptr(), _stream(stream)), "lskum_adjoint_total")


def lskum_status(plan: Plan, stream=None) -> int:
    """Synchronising status query; returns the status code (0, or
    ERR_NONPHYSICAL / ERR_DEGENERATE)."""
    return int(plan.lib.lskum_status(plan.handle, _stream(stream)))


def lskum_clear_status(plan: Plan, stream=None):
    _check(plan.lib.lskum_clear_status(plan.handle, _stream(stream)), "lskum_clear_status")


class Graph:
    """A captured run of `iters` iterations (lskum_graph_create); each
    launch() replays them and appends residual-norm rows to hist."""

    def __init__(self, plan: Plan, iters: int, U, hist, ws, stream=None):
        self.plan = plan
        rows = 0 if hist is None else hist.numel() // plan.n_clouds
        hp = 0 if hist is None else _scalar_out(plan, hist, plan.n_clouds, "hist")
        if not isinstance(ws, torch.Tensor) or not ws.is_cuda or ws.numel() < lskum_workspace_bytes(plan):
            raise ValueError("ws: need a cuda tensor of lskum_workspace_bytes(plan) bytes")
        g = ctypes.c_void_p()
        _check(plan.lib.lskum_graph_create(ctypes.byref(g), plan.handle, int(iters),
                                           plan._arg(U, 4, "U"), hp, int(rows), ws.data_ptr(),
                                           _stream(stream)), "lskum_graph_create")
        self.handle = g
        self._keep = (U, hist, ws)

    def launch(self, stream=None):
        _check(self.plan.lib.lskum_graph_launch(self.handle, _stream(stream)), "lskum_graph_launch")

    def destroy(self):
        if getattr(self, "handle", None):
            self.plan.lib.lskum_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


TUNING_SPACE = [Tuning(b, x, fb) for b in (128, 256, 512) for x in (1, 0) for fb in (64, 128)]


def autotune(plan: Plan, U, ws, iters: int = 2, reps: int = 3, space=None, stream=None):
    """Time `iters` iterations for every tuning in `space` (default: tile
    block 128/256/512 x XCD mapping on/off x flux block 64/128) on a scratch
    copy of U, keep the fastest on the plan and return (best, {tuning: ms})."""
    space = space or TUNING_SPACE
    scratch = U.clone()
    times = {}
    for t in space:
        plan.set_tuning(t)
        ms = []
        for _ in range(reps):
            scratch.copy_(U)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            lskum_iterate(plan, iters, scratch, None, ws, stream)
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        times[t] = min(ms)
    best = min(times, key=times.get)
    plan.set_tuning(best)
    lskum_clear_status(plan, stream)
    return best, times
