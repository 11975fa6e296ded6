#!/usr/bin/env python3
"""Throughput of the LSKUM residual sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 1m]

A step is one pseudo-time iteration of the whole hot path over the cloud:
the local time step, then four SSP Runge-Kutta stages, each of
q-variables -> least-squares q-derivatives (first-order + inner sweeps)
-> limited split-flux residual -> stage update, plus the device-side
residual norm.  Inputs are synthetic (seeded airfoil point cloud) and
resident in HBM before timing starts.  The value is point-stage updates per
second (points x 4 stages x steps / seconds).

Besides the throughput the JSON line carries:
* roofline: the flux kernel (the dominant one) -- algorithmic FP64
  operations per launch divided by its mean launch time, measured with HIP
  events around every flux launch in the timed region, against the MI355X
  FP64 vector peak;
* cpu_baseline: the FP64 oracle timed on this host on a bounded sample
  (whole RK stages over the cloud), single-threaded and, as `all_cores`,
  its OpenMP build on every host core, with the host's CPU model and count.
The default 1m line also carries (after the timed region):
* sustained: 1000 more iterations through the library's own loop;
* adjoint: the residual VJP against one forward residual (the metric's
  second figure);
* 16m: the 16M-point cloud, 2 warm-up + 10 timed iterations, with its flux
  roofline and compulsory HBM rate;
* batch: 64 uneven clouds in one plan (graph replays, autotuned) against
  the same clouds advanced one after the other, 500 iterations.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "point-RK-stage updates/s FP64 at 1M/16M pts; adjoint/forward time ratio"
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# worker processes for cloud generation (before the GPU is initialised;
# --gen-workers 1 builds in-process, e.g. under a profiler that has already
# initialised the GPU)
GEN_WORKERS = 16


def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "cpus_available": len(os.sched_getaffinity(0))}


def oracle_stages(cloud, wl, U_host, options: int, n_inner: int, min_seconds: float, lib=None):
    """Whole RK stages of the oracle from U_host, repeated until at least
    `min_seconds`; returns (stages, seconds)."""
    import numpy as np
    from oracle.ref import FIRST_ORDER, RK4, Oracle

    o = Oracle(cloud, wl.mach, wl.aoa_deg, cfl=wl.cfl, venkat_k=wl.venkat_k,
               n_inner=n_inner, gamma=wl.gamma, options=options, lib=lib)
    U = U_host.copy()
    Un = U_host.copy()
    dt = None
    Rs = []
    stages = 0
    t0 = time.perf_counter()
    while True:
        if stages % 4 == 0:
            dt = o.local_dt(U)
            Un = U.copy()
            Rs = []
        q, _ = o.q_vars(U)
        if options & FIRST_ORDER:
            dq, qlim = np.zeros((8, cloud.n)), np.zeros((8, cloud.n))
        else:
            dq, qlim = o.q_derivs(q)
        R, _ = o.flux_residual(q, dq, qlim)
        Rs.append(R)
        if options & RK4:
            U = o.rk4_stage(stages % 4, Un, Rs, dt, U)
        else:
            U = o.rk_stage(stages % 4, Un, R, dt, U)
        stages += 1
        sec = time.perf_counter() - t0
        if sec >= min_seconds:
            return stages, sec


def cpu_baseline(cloud, wl, U_host, options: int = 0, n_inner=None, min_seconds: float = 10.0,
                 all_cores: bool = True, state: str = "the initial state"):
    """The oracle, as it stands, on whole RK stages of the workload (same
    scheme options and inner sweeps as the GPU run), single-threaded (the
    parity build), repeated until at least `min_seconds` (one stage over the
    1M cloud takes about 4 s); with `all_cores` also the OpenMP build of the
    same source on every host core the process may use."""
    from oracle import ref

    n_inner = wl.n_inner if n_inner is None else n_inner
    what = (f"RK stages (local time step per 4 stages, q-variables, first-order + {n_inner} "
            f"inner LS sweeps, flux residual, stage update) over all {cloud.n} points of the "
            f"{wl.name} cloud from {state}" + (f", options {options}" if options else ""))
    stages, sec = oracle_stages(cloud, wl, U_host, options, n_inner, min_seconds)
    out = {"value": cloud.n * stages / sec, "unit": "point-stage updates/s", "cores": 1,
           "kind": "oracle", "sample": f"{stages} {what}, single thread, {sec:.1f} s",
           "host": host_info()}
    if all_cores:
        lib = ref.load_omp()
        threads = int(lib.lskum_ref_threads())
        stages, sec = oracle_stages(cloud, wl, U_host, options, n_inner, min_seconds, lib=lib)
        out["all_cores"] = {"value": cloud.n * stages / sec, "unit": "point-stage updates/s",
                            "cores": threads, "kind": "oracle (OpenMP build of the same source)",
                            "sample": f"{stages} {what}, {threads} threads, {sec:.1f} s"}
    return out


ELEMENTARY_RANGES = {
    # fn id: (name, low, high) -- argument ranges met in the flux kernel
    0: ("copy", 0.1, 3.0),
    1: ("exp", -6.0, 1.0),     # exp(-S^2), exp(q1 + beta |u|^2)
    2: ("erf", -2.5, 2.5),     # S = u_d sqrt(beta)
    3: ("log", 0.3, 3.0),
    4: ("sqrt", 1e-8, 1e-2),   # edge length squared
    5: ("rsqrt", 0.3, 3.0),    # beta
    6: ("divide", 0.1, 3.0),
    # the flux kernel's own versions (lskum_math.h)
    9: ("lk_div", 0.1, 3.0),
    10: ("lk_rsqrt", 0.3, 3.0),
    11: ("lk_erf", -2.5, 2.5),
    12: ("lk_exp", -6.0, 1.0),
}


def calibrate_elementary(n: int = 1 << 24) -> int:
    """One launch per elementary function over n seeded inputs."""
    import ctypes

    import numpy as np
    import torch

    from paper_2403_13287_amd import _build

    torch.cuda.set_device(0)
    lib = ctypes.CDLL(_build.CALIB_LIB)
    lib.lskum_calib_elementary.restype = ctypes.c_int
    lib.lskum_calib_elementary.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rng = np.random.Generator(np.random.PCG64(17))
    y = torch.from_numpy(rng.uniform(-2.0, 2.0, n)).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    # first pass: inputs in random order; second pass: sorted, so every
    # wavefront sees a narrow argument range (no divergence between the
    # branches of piecewise implementations)
    for order in ("random", "sorted"):
        for fn, (name, lo, hi) in ELEMENTARY_RANGES.items():
            xs = rng.uniform(lo, hi, n)
            if order == "sorted":
                xs = np.sort(xs)
            x = torch.from_numpy(xs).cuda()
            rc = lib.lskum_calib_elementary(fn, n, x.data_ptr(), y.data_ptr(), out.data_ptr(),
                                            stream)
            if rc != 0:
                raise RuntimeError(f"calibration kernel {name} failed ({rc})")
            torch.cuda.synchronize()
    print(json.dumps({"calibrate_elementary": {str(k): v[0] for k, v in ELEMENTARY_RANGES.items()},
                      "elements": n}), flush=True)
    return 0


def run_batch(clouds, draws, iters: int) -> dict:
    """The batch workload on clouds already generated: one plan over all the
    clouds (autotuned, one graph launch per replay of `per_graph`
    iterations) against the clouds advanced one after the other (each with
    its own graph of the same kernels); states must agree bit for bit."""
    import numpy as np
    import torch

    from paper_2403_13287_amd import lskum as L
    from paper_2403_13287_amd.solver import Solver

    per_graph = 25 if iters % 25 == 0 else 1
    replays = iters // per_graph
    params = [L.Params(d["mach"], d["aoa_deg"], 0.2, 5.0, 2) for d in draws]
    total = sum(c.n for c in clouds)
    log(f"[bench] batch: {total} points in {len(clouds)} clouds ({min(c.n for c in clouds)}-"
        f"{max(c.n for c in clouds)}), {iters} iterations")

    batch = Solver(clouds, params)
    best, tune_ms = L.autotune(batch.plan, batch.U, batch.ws, iters=2, reps=2)
    log(f"[bench] autotuned: {best} from {tune_ms}")
    graph, hist = batch.capture(per_graph, replays)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        graph.launch()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    status = batch.status()

    t_loop = 0.0
    loop_status = L.OK
    identical = True
    for c, (cloud, p) in enumerate(zip(clouds, params)):
        s = Solver(cloud, p)
        g, h = s.capture(per_graph, replays)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(replays):
            g.launch()
        torch.cuda.synchronize()
        t_loop += time.perf_counter() - t0
        loop_status = loop_status or s.status()
        if not torch.equal(s.U, batch.cloud_state(c)):
            log(f"[bench] cloud {c}: batched and single states differ")
            identical = False
        del g, s
    out = {
        "value": total * 4.0 * iters / t_batch,
        "unit": "point-stage updates/s",
        "iterations": iters,
        "points": total,
        "clouds": len(clouds),
        "iterations_per_graph": per_graph,
        "batch_seconds": t_batch,
        "loop_seconds": t_loop,
        "loop_value": total * 4.0 * iters / t_loop,
        "speedup_vs_loop": t_loop / t_batch,
        "tuning": {"block": best.block, "xcd_contiguous": best.xcd_contiguous,
                   "flux_block": best.flux_block},
        "autotune_ms_per_2_iterations (block/xcd_contiguous/flux_block)":
            {k.key(): v for k, v in tune_ms.items()},
        "batched_equals_looped": identical,
        "status": L.strerror(status),
        "loop_status": L.strerror(loop_status),
        "residual_last": float(np.nanmax(hist[-1].cpu().numpy())),
    }
    del graph, batch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


BATCH_CONFIG = ("batch: 64 NACA 0012 clouds, 5k-250k points log-uniform, M U[0.3, 0.9], "
                "AoA U[-4, 6] deg, k_max 25, n_inner 2, CFL 0.2")


def batch_clouds():
    from cloudgen import batch_sizes, make_airfoil_clouds

    draws = batch_sizes()
    log(f"[bench] generating the {len(draws)} batch clouds")
    clouds = make_airfoil_clouds([(d["W"], d["L"], 25, d["seed"]) for d in draws],
                                 workers=GEN_WORKERS)
    return clouds, draws


def bench_batch(args) -> int:
    """64 uneven airfoil clouds advanced together (one graph launch per
    replay, autotuned tile size and XCD mapping) against the same 64 clouds
    advanced one after the other (each with its own graph)."""
    import torch

    from paper_2403_13287_amd import lskum as L

    clouds, draws = batch_clouds()
    torch.cuda.set_device(0)
    iters = 500 if args.steps is None else args.steps
    r = run_batch(clouds, draws, iters)
    out = {
        "metric": "batched point-RK-stage updates/s FP64, 64 uneven airfoil clouds",
        "value": r["value"],
        "unit": "point-stage updates/s",
        "n_gpus": 1,
        "steps": iters,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": BATCH_CONFIG, "points": r["points"], "clouds": r["clouds"],
                   "iterations_per_graph": r["iterations_per_graph"]},
    }
    out.update({k: v for k, v in r.items() if k not in out and k != "unit"})
    print(json.dumps(out), flush=True)
    ok = r["status"] == L.strerror(L.OK) and r["loop_status"] == L.strerror(L.OK)
    return 0 if ok and r["batched_equals_looped"] else 1


def time_adjoint(plan, U, reps: int, warmup: int, force: bool = False) -> dict:
    """Mean times (ms, HIP events on the current stream) of one forward
    residual evaluation (q-variables, q-derivatives, flux residual) and of
    the residual VJP with respect to U and (M, AoA) (q and every derivative
    iterate recomputed) at the state U, with N(0, 1) cotangents (seed 7);
    with `force` also of the lift/drag VJP."""
    import numpy as np
    import torch

    from paper_2403_13287_amd import lskum as L

    n = plan.n
    gen = torch.Generator().manual_seed(7)
    Rb = torch.randn((n, 4), generator=gen, dtype=torch.float64).cuda()
    Jb = torch.tensor([1.0, 0.0], dtype=torch.float64, device="cuda")
    q, dq, qlim, work, R = (plan.field(c) for c in (4, 8, 8, 16, 4))
    Ub, Fb = plan.field(4), plan.field(4)
    tb = torch.empty(2, dtype=torch.float64, device="cuda")
    ws = L.vjp_workspace(plan)

    def forward():
        L.lskum_q_vars(plan, U, q)
        L.lskum_q_derivs(plan, q, dq, qlim, work)
        L.lskum_flux_residual(plan, q, dq, qlim, R)

    def vjp():
        L.lskum_flux_residual_vjp(plan, U, Rb, Ub, tb, ws)

    def force_vjp():
        L.lskum_force_coeffs_vjp(plan, U, Jb, Fb, tb)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    vjp()  # builds the plan's transposed connectivity once
    torch.cuda.synchronize()
    out = {"forward_ms": timed(forward), "vjp_ms": timed(vjp)}
    out["ratio"] = out["vjp_ms"] / out["forward_ms"]
    if force:
        out["force_vjp_ms"] = timed(force_vjp)
    out["vjp_workspace_bytes"] = L.lskum_vjp_workspace_bytes(plan)
    torch.cuda.synchronize()
    out["finite"] = bool(torch.isfinite(Ub).all()) and bool(torch.isfinite(tb).all())
    return out


def bench_adjoint(args) -> int:
    """Cost of the residual VJP (q and every derivative iterate recomputed)
    against one forward residual evaluation (q-variables, q-derivatives,
    flux residual) on the 1M-point cloud at M 0.63, AoA 2 deg, three inner
    sweeps; the state is the free stream advanced a few hundred iterations,
    the cotangents are N(0, 1) draws with seed 7."""
    import numpy as np
    import torch

    from cloudgen import named_cloud
    from paper_2403_13287_amd import lskum as L
    from paper_2403_13287_amd.solver import Solver

    log("[bench] generating the 1m cloud (1000 x 1000)")
    cloud = named_cloud("1m", workers=GEN_WORKERS)
    torch.cuda.set_device(0)
    reps = 20 if args.steps is None else args.steps
    state_iters = 300
    params = L.Params(0.63, 2.0, 0.2, 5.0, 3)
    s = Solver(cloud, params)
    s.run(state_iters)
    torch.cuda.synchronize()
    plan, U, n = s.plan, s.U, s.n
    t = time_adjoint(plan, U, reps, args.warmup, force=True)
    t_fwd, t_vjp, t_force, ratio = t["forward_ms"], t["vjp_ms"], t["force_vjp_ms"], t["ratio"]
    status = s.status()
    log(f"[bench] forward {t_fwd:.4f} ms, vjp {t_vjp:.4f} ms, ratio {ratio:.3f}, "
        f"force vjp {t_force:.4f} ms, status {status}")
    converged = None
    if args.converge:
        # the same flow advanced until the density residual has fallen 10
        # orders from the first iteration's or `converge` iterations have run
        chunk = 1000
        h = s.history().cpu().numpy()
        r1 = float(h[0])
        while s.iteration < args.converge:
            hc = s.run(min(chunk, args.converge - s.iteration)).cpu().numpy()
            rel = float(hc[-1]) / r1
            log(f"[bench] converging: iteration {s.iteration}, r/r1 {rel:.3e}, "
                f"status {s.status()}")
            if not np.isfinite(rel) or rel <= 1e-10 or s.status() != L.OK:
                break
        torch.cuda.synchronize()
        hist = s.history().cpu().numpy()
        tc = time_adjoint(plan, U, reps, args.warmup, force=True)
        cl_cd = s.force_coeffs().cpu().numpy()
        converged = {"iterations": s.iteration, "r_over_r1": float(hist[-1]) / r1,
                     "r_over_r1_min": float(np.min(hist)) / r1,
                     "cl": float(cl_cd[0]), "cd": float(cl_cd[1]),
                     "forward_ms": tc["forward_ms"], "vjp_ms": tc["vjp_ms"],
                     "force_vjp_ms": tc["force_vjp_ms"], "ratio": tc["ratio"],
                     "finite": tc["finite"], "status": L.strerror(s.status())}
        log(f"[bench] converged state: {converged}")
        if args.save_state:
            np.save(args.save_state, U.cpu().numpy())
        status = s.status() if status == L.OK else status
    out = {
        "metric": "adjoint/forward time ratio (residual VJP incl. recompute / forward residual)",
        "value": ratio,
        "unit": "x",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "ms_per_step": t_vjp,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "adjoint: NACA 0012 O-type airfoil cloud 1000 x 1000, k_max 30, "
                               f"M 0.63, AoA 2 deg, n_inner 3, state = free stream + {state_iters} "
                               "iterations, cotangents N(0,1) seed 7",
                   "points": n, "edges": int(cloud.nbr_count.astype(np.int64).sum())},
        "forward_ms": t_fwd,
        "vjp_ms": t_vjp,
        "force_vjp_ms": t_force,
        "vjp_workspace_bytes": t["vjp_workspace_bytes"],
        "status": L.strerror(status),
        "finite": t["finite"],
    }
    if converged is not None:
        out["converged_state"] = converged
    print(json.dumps(out), flush=True)
    return 0 if status == L.OK and out["finite"] else 1


def bench_ksweep(args) -> int:
    """Limiter sensitivity: the 9,600-point cloud at the 1M workload's flow
    (M 0.85, AoA 1 deg, n_inner 2) advanced 2,000 iterations with the
    Venkatakrishnan limiter at several K and with the min-max limiter;
    whether each stays physical, how far the residual falls, Cl and Cd."""
    import numpy as np
    import torch

    from cloudgen import named_cloud
    from paper_2403_13287_amd import lskum as L
    from paper_2403_13287_amd.solver import Solver

    cloud = named_cloud("tiny")
    torch.cuda.set_device(0)
    iters = 2000 if args.steps is None else args.steps
    per = 250 if iters % 250 == 0 else 1
    rows = []
    for label, K, opt in ([(f"venkat K={k:g}", k, 0) for k in (0.3, 1.0, 5.0, 15.0, 50.0, 150.0)]
                          + [("min-max", 5.0, L.MINMAX), ("first-order", 5.0, L.FIRST_ORDER)]):
        s = Solver(cloud, L.Params(0.85, 1.0, 0.2, K, 2, options=opt))
        graph, hist = s.capture(per, iters // per)
        t0 = time.perf_counter()
        for _ in range(iters // per):
            graph.launch()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        h = hist[:, 0].cpu().numpy()
        st = s.status()
        cl, cd = (float(v) for v in s.force_coeffs().cpu().numpy())
        finite = bool(np.all(np.isfinite(h)))
        row = {"limiter": label, "status": L.strerror(st), "residual_first": float(h[0]),
               "residual_last": float(h[-1]) if finite else None,
               "drop": float(h[-1] / h[0]) if finite else None,
               "Cl": cl if finite else None, "Cd": cd if finite else None, "seconds": sec}
        log(f"[bench] {label}: {row}")
        rows.append(row)
    print(json.dumps({"metric": "limiter sensitivity (stability and residual drop)",
                      "config": {"workload": "tiny cloud 160 x 60 at M 0.85, AoA 1 deg, n_inner 2, "
                                             f"CFL 0.2, {iters} iterations"},
                      "rows": rows}), flush=True)
    return 0


SUSTAINED_ITERS = 1000
# iterations that develop the flow before timing.  From the free stream the
# disturbance of the body crosses the 1M cloud's 1000 point layers in about
# 50 iterations (each stage reads n_inner + 2 = 5 stencil hops), the 16M
# cloud's 4000 in about 200; ahead of it the derivatives are exactly zero
# and the flux kernel skips its limiter divisions.  The 1M workload's input
# is the state half-way through its 1000 iterations (measured: 0.583 ms per
# flux launch from the free stream, 0.590 after 200 iterations, 0.614 after
# 1000); the 16M object's, the state well after the disturbance has crossed
# it.
PREPARE_ITERS = 500
PREPARE_ITERS_16M = 400
BATCH_ITERS = 500


def run_sweep(cloud, wl, steps: int, warm: int, options: int, n_inner: int,
              keep_initial: bool = True, tuning=None, prepare: int = 0,
              save_input: str | None = None, load_input: str | None = None) -> dict:
    """Time `steps` iterations (after `warm` untimed ones) of the whole
    iteration on `cloud`, issued from Python one entry point at a time, with
    HIP events around every flux launch.  The input state is the free stream
    advanced `prepare` iterations (untimed, through the library's own loop):
    from the free stream, the points the disturbance of the body has not yet
    reached have exactly zero derivatives, where the flux kernel skips its
    limiter divisions, so the first iterations are not representative of a
    run."""
    import numpy as np
    import torch

    from paper_2403_13287_amd import costs
    from paper_2403_13287_amd import lskum as L

    n = cloud.n
    edges = int(cloud.nbr_count.astype(np.int64).sum())
    p = L.Params(wl.mach, wl.aoa_deg, wl.cfl, wl.venkat_k, n_inner, wl.gamma, options=options)
    plan = L.Plan(cloud, p, tuning=tuning)
    U = plan.field(4)
    L.lskum_init_state(plan, U)
    if load_input:
        # a state saved by an earlier run with --save-input (e.g. prepared
        # outside a per-dispatch counter profiler)
        U_in = np.load(load_input)
        if U_in.shape != (n, 4) or U_in.dtype != np.float64:
            raise ValueError(f"{load_input}: need a float64 array of shape ({n}, 4)")
        U.copy_(torch.from_numpy(U_in))
        prepare = 0
    if prepare > 0:
        ws = L.workspace(plan)
        L.lskum_iterate(plan, prepare, U, None, ws)
        torch.cuda.synchronize()
        del ws
        if L.lskum_status(plan) != L.OK:
            raise RuntimeError("the prepared state is not physical")
    if save_input:
        np.save(save_input, U.cpu().numpy())
    # the input state in the oracle's layout (4, n), for the CPU baseline
    U0_host = U.cpu().numpy().T.copy() if keep_initial else None
    Un, q, dq, qlim, work, R = (plan.field(c) for c in (4, 4, 8, 8, 16, 4))
    dt, acc, q2 = plan.field(1), plan.field(4), plan.field(4)
    rk4 = bool(options & L.RK4)
    hist = torch.zeros(max(steps + warm, 1), dtype=torch.float64, device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(4 * steps)]
    qs = (q, q2)

    def step(k, timed):
        # SSP stages: the flux launch also applies the stage update and writes
        # the next stage's q into the other buffer (four stages bring q back
        # to qs[0]); q_vars runs only before the very first stage.  RK4 keeps
        # separate q_vars and stage launches.
        # the first stage's launch stores U, the step's U^n, in Un
        L.lskum_local_dt(plan, U, dt)
        for s in range(4):
            qc = q if rk4 else qs[s % 2]
            if rk4 or (k == 0 and s == 0):
                L.lskum_q_vars(plan, U, qc)
            if not options & L.FIRST_ORDER:  # the first-order flux reads no derivatives
                L.lskum_q_derivs(plan, qc, dq, qlim, work)
            if timed:
                ev[4 * (k - warm) + s][0].record()
            if rk4:
                L.lskum_flux_residual(plan, qc, dq, qlim, R)
            else:
                L.lskum_flux_residual_stage(plan, s, qc, dq, qlim, Un, dt, R, U, qs[(s + 1) % 2])
            if timed:
                ev[4 * (k - warm) + s][1].record()
            if s == 0:
                L.lskum_residual_norm(plan, R, hist[k:k + 1])
            if rk4:
                L.lskum_rk4_stage(plan, s, Un, R, dt, acc, U)

    log(f"[bench] n={n} edges={edges} warmup={warm} steps={steps}")
    for k in range(warm):
        step(k, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warm, warm + steps):
        step(k, True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    status = L.lskum_status(plan)
    h = hist.cpu().numpy()
    flux_ms = float(np.mean([a.elapsed_time(b) for a, b in ev])) if ev else float("nan")
    log(f"[bench] {sec:.3f} s, flux mean {flux_ms:.4f} ms, status {status}, "
        f"hist first {h[0]:.6e} last {h[warm + steps - 1]:.6e}")
    # the timed launch is the flux with the SSP stage in its epilogue, or
    # (rk4) the plain flux; the FP64 count per edge is the default residual's
    flops = costs.flux_flops(n, edges, stage=not rk4)
    achieved = flops / (flux_ms * 1e-3) / 1e12
    if options & (L.FIRST_ORDER | L.MINMAX):
        achieved = None
    stage_gb = costs.stage_bytes(n, cloud.k_pad, n_inner, fused=not rk4) / 1e9
    return {
        "plan": plan, "U": U, "U0_host": U0_host, "sec": sec, "flux_ms": flux_ms, "hist": h,
        "status": status, "edges": edges,
        "roofline": {"bound": "alu", "kernel": "k_flux" + ("" if rk4 else " + SSP stage"),
                     "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": None if achieved is None else achieved / FP64_PEAK_TFLOPS,
                     "traffic": None, "flops_per_launch": flops, "avg_launch_ms": flux_ms,
                     "algorithmic_bytes_per_launch": costs.flux_bytes(n, cloud.k_pad,
                                                                      stage=not rk4)},
        "hbm_compulsory": {"GB_per_stage": stage_gb,
                           "achieved_GBs": stage_gb * 4 * steps / sec,
                           "frac": stage_gb * 4 * steps / sec / HBM_PEAK_GBS},
    }


def main():
    global GEN_WORKERS
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed iterations (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="1m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward ratio in the 1m line")
    ap.add_argument("--no-sustained", action="store_true",
                    help="skip the 1000-iteration sustained figure of the default 1m line "
                         "(e.g. under a per-dispatch counter profiler)")
    ap.add_argument("--no-16m", action="store_true",
                    help="skip the 16m object (10 timed iterations) of the default 1m line")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch object (64 clouds, batched vs looped) of the default "
                         "1m line")
    ap.add_argument("--n-inner", type=int, default=None,
                    help="inner least-squares sweeps (default: the workload's)")
    ap.add_argument("--scheme", default="default",
                    choices=("default", "first-order", "minmax", "rk4"),
                    help="scheme variant of the sweep (default: the paper's second-order "
                         "scheme with the Venkatakrishnan limiter and SSPRK(4,3); rk4: the "
                         "same residual with classical RK4 stages)")
    ap.add_argument("--prepare", type=int, default=PREPARE_ITERS,
                    help="untimed iterations that develop the flow before the warm-up "
                         "(the timed input state); 0 times from the free stream")
    ap.add_argument("--prepare-16m", type=int, default=PREPARE_ITERS_16M,
                    help="the same for the 16m object of the default 1m line")
    ap.add_argument("--save-input", default=None,
                    help="save the timed input state (after --prepare) as .npy")
    ap.add_argument("--load-input", default=None,
                    help="take the timed input state from a .npy saved by --save-input "
                         "(no --prepare iterations)")
    ap.add_argument("--tuning", default=None,
                    help="launch tuning of the timed plan as block/xcd_contiguous/flux_block, "
                         "e.g. 256/1/64 (default: the library's)")
    ap.add_argument("--gen-workers", type=int, default=GEN_WORKERS,
                    help="worker processes that build the clouds (1: in this process)")
    ap.add_argument("--converge", type=int, default=0,
                    help="--workload adjoint: also advance the flow until the residual has "
                         "fallen 10 orders (at most this many iterations) and time the "
                         "adjoint ratio there")
    ap.add_argument("--save-state", default=None,
                    help="--workload adjoint --converge: save the state reached (.npy)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of the sweep, run 5 plain device copies of this many bytes "
                         "(calibrates the HBM traffic counters)")
    ap.add_argument("--calibrate-elementary", action="store_true",
                    help="instead of the sweep, run the FP64 elementary-function calibration "
                         "kernels once each over 2^24 inputs (profile with rocprofv3 --pmc)")
    args = ap.parse_args()
    GEN_WORKERS = max(1, args.gen_workers)
    if args.calibrate_elementary:
        return calibrate_elementary()
    if args.copy_bytes:
        import torch
        torch.cuda.set_device(0)
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "copies": 5}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the sweep is not "
              "sharded across GPUs in this build", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "ksweep":
        return bench_ksweep(args)

    import numpy as np
    import torch

    from cloudgen.workloads import WORKLOADS
    from paper_2403_13287_amd import lskum as L

    wl = WORKLOADS[args.workload]
    steps = wl.iters if args.steps is None else args.steps
    warm = args.warmup
    options = {"default": 0, "first-order": L.FIRST_ORDER, "minmax": L.MINMAX,
               "rk4": L.RK4}[args.scheme]
    n_inner = wl.n_inner if args.n_inner is None else args.n_inner
    headline = wl.name == "1m" and args.scheme == "default" and args.n_inner is None
    # every cloud is built (in worker processes) before the GPU is touched
    log(f"[bench] generating the {wl.name} cloud ({wl.W} x {wl.L})")
    cloud = wl.cloud(workers=GEN_WORKERS)
    cloud16 = bclouds = None
    if headline and not args.no_16m:
        w16 = WORKLOADS["16m"]
        log(f"[bench] generating the 16m cloud ({w16.W} x {w16.L})")
        cloud16 = w16.cloud(workers=GEN_WORKERS)
    if headline and not args.no_batch:
        bclouds, draws = batch_clouds()
    torch.cuda.set_device(0)

    tuning = None
    if args.tuning:
        b, x, fb = (int(v) for v in args.tuning.split("/"))
        tuning = L.Tuning(b, x, fb)
    r = run_sweep(cloud, wl, steps, warm, options, n_inner, tuning=tuning, prepare=args.prepare,
                  save_input=args.save_input, load_input=args.load_input)
    plan, U, sec, flux_ms, h, status = (r[k] for k in ("plan", "U", "sec", "flux_ms", "hist",
                                                       "status"))
    n, edges = cloud.n, r["edges"]
    out = {
        "metric": METRIC,
        "value": n * 4.0 * steps / sec,
        "unit": "point-stage updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": sec * 1e3 / max(steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: NACA 0012 O-type airfoil cloud {wl.W} x {wl.L}, "
                               f"k_max {wl.k_max}, M {wl.mach}, AoA {wl.aoa_deg} deg, "
                               f"n_inner {n_inner}, CFL {wl.cfl}, Venkatakrishnan K {wl.venkat_k}"
                               + ("" if args.scheme == "default" else f", scheme {args.scheme}"),
                   "points": n, "edges": edges, "k_pad": cloud.k_pad, "iterations": steps,
                   "stages_per_iteration": 4,
                   "input_state": (f"loaded from {args.load_input}" if args.load_input else
                                   f"free stream advanced {args.prepare} iterations (untimed) "
                                   "before the warm-up"),
                   "tuning": (tuning or L.Tuning()).key()},
        "roofline": r["roofline"],
        "hbm_compulsory": r["hbm_compulsory"],
        "status": L.strerror(status),
        "residual_history": {"first": float(h[0]), "last": float(h[warm + steps - 1])},
    }
    if wl.name == "1m" and args.scheme == "default":  # the profiled launch
        from paper_2403_13287_amd import costs
        out["roofline"]["traffic"] = costs.stored_flux_traffic(
            os.path.join(ROOT, "profiles", "k_flux_1m.txt"))
    ok = status == L.OK and bool(np.all(np.isfinite(h[:warm + steps])))
    if headline and not args.no_sustained:
        # the same iteration over 1000 more iterations through the library's
        # own loop: the rate a long run settles to
        ws = L.workspace(plan)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.lskum_iterate(plan, SUSTAINED_ITERS, U, None, ws)
        torch.cuda.synchronize()
        t_s = time.perf_counter() - t0
        out["sustained"] = {"iterations": SUSTAINED_ITERS, "ms_per_step": t_s * 1e3 / SUSTAINED_ITERS,
                            "value": n * 4.0 * SUSTAINED_ITERS / t_s, "driver": "lskum_iterate",
                            "status": L.strerror(L.lskum_status(plan))}
        log(f"[bench] sustained: {out['sustained']}")
        del ws
    # the headline's second figure: the residual VJP against the forward
    # residual, on this plan at the state the timed iterations reached
    if wl.name == "1m" and not args.no_adjoint and not options & (L.FIRST_ORDER | L.MINMAX):
        log("[bench] timing the residual VJP against the forward residual")
        adj = time_adjoint(plan, U, reps=20, warmup=5)
        adj["state"] = (f"the {wl.name} state after the input state's {args.prepare} iterations, "
                        f"the {warm + steps} above"
                        + (f" and {SUSTAINED_ITERS} more" if headline and not args.no_sustained
                           else ""))
        adj["cotangents"] = "N(0, 1), seed 7"
        adj["status"] = L.strerror(L.lskum_status(plan))
        out["adjoint"] = adj
        log(f"[bench] forward {adj['forward_ms']:.4f} ms, vjp {adj['vjp_ms']:.4f} ms, "
            f"ratio {adj['ratio']:.3f}")
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle (one thread, then all cores)")
        out["cpu_baseline"] = cpu_baseline(
            cloud, wl, r["U0_host"], options, n_inner,
            state=f"the GPU's input state (free stream + {args.prepare} iterations)")
    del plan, U, r
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if cloud16 is not None:
        w16 = WORKLOADS["16m"]
        log(f"[bench] 16m: prepare {args.prepare_16m}, 2 warm-up + 10 timed iterations")
        r16 = run_sweep(cloud16, w16, 10, 2, 0, w16.n_inner, keep_initial=False,
                        prepare=args.prepare_16m)
        out["16m"] = {
            "workload": f"16m: NACA 0012 O-type airfoil cloud {w16.W} x {w16.L}, k_max "
                        f"{w16.k_max}, M {w16.mach}, AoA {w16.aoa_deg} deg, n_inner {w16.n_inner}",
            "points": cloud16.n, "edges": r16["edges"], "iterations": 10, "warmup": 2,
            "input_state": f"free stream advanced {args.prepare_16m} iterations (untimed)",
            "ms_per_step": r16["sec"] * 1e3 / 10,
            "value": cloud16.n * 4.0 * 10 / r16["sec"], "unit": "point-stage updates/s",
            "roofline": r16["roofline"], "hbm_compulsory": r16["hbm_compulsory"],
            "status": L.strerror(r16["status"])}
        ok = ok and r16["status"] == L.OK
        log(f"[bench] 16m: {out['16m']['value']:.4g} point-stage updates/s")
        del r16, cloud16
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if bclouds is not None:
        rb = run_batch(bclouds, draws, BATCH_ITERS)
        rb["workload"] = BATCH_CONFIG
        out["batch"] = rb
        ok = ok and rb["batched_equals_looped"] and rb["status"] == L.strerror(L.OK)
        log(f"[bench] batch: {rb['value']:.4g} point-stage updates/s, "
            f"{rb['speedup_vs_loop']:.2f}x the loop")
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
