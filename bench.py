#!/usr/bin/env python3
"""Projection benchmark on one MI355X.

One step = one pass of the whole ghost-cell projection on the multi-body 256^3 workload
(8 perturbed icospheres of 20,480 triangles on a stretched grid): cell classification,
ghost-cell stencils and multigrid hierarchy, divergence right-hand side, pressure Poisson
solve from p = 0 to relative residual 1e-10, velocity correction.  The body mesh is uploaded
and validated once; every timed step's input fields are resident in HBM before timing starts.

Prints one JSON line: metric, value (projections/s), ms_per_step, the workload config, the
fine sweep's roofline (live HIP-event timing, counter traffic) and the oracle's CPU
baseline, plus the other forms (mixed, momentum, paper solver, moving bodies, serving).
--gpus N > 1 is not supported.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SWEEP_BYTES = {"fp64": 25.0, "fp32": 13.0}  # algorithmic bytes per cell of one fused sweep
HBM_PEAK_GBS = 8000.0
SWEEP_SRC = os.path.join(ROOT, "paper_2505_17287_amd", "csrc", "sweep.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rbgs_fused_fp64_multibody256_pmc.txt")


def recorded_traffic(workload):
    """HBM bytes per launch of the FP64 fused sweep from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by its plain-copy calibration factor), or None
    when the summary is missing, is for another workload, or was taken on a different
    version of the kernel source."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith(("#", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        src = hashlib.sha256(open(SWEEP_SRC, "rb").read()).hexdigest()
        if kv.get("kernel_source_sha256") != src or kv.get("workload") != workload:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def oracle_reference(wl):
    """The oracle as it stands, on the same workload, as the CPU baseline and as the accuracy
    reference of the timed results.  Timed: classification, ghost stencils and multigrid
    hierarchy (once), then the whole projection (right-hand side, BiCGStab preconditioned by
    one V-cycle to relative residual 1e-10 from p = 0, the same solver and tolerance as the GPU
    step, correction), median of 3.  Not timed: a converged solve (1e-12) as the accuracy
    reference, one BiCGStab step on one thread (per-step time against all threads), and the
    host's STREAM triad bandwidth.  The converged solve starts from the 1e-10 result."""
    import numpy as np
    from oracle import OracleProblem
    from oracle.oracle import set_threads, stream_triad_gbs, threads
    nthr = threads()
    u, v, w = wl.velocity()
    t0 = time.perf_counter()
    P = OracleProblem(wl.xf, wl.yf, wl.zf)
    P.set_mesh(wl.verts, wl.tris)
    P.classify()
    P.build_stencils()
    P.levels()  # the multigrid hierarchy
    t_setup = time.perf_counter() - t0
    runs = []
    for _ in range(3):
        t1 = time.perf_counter()
        u1, v1, w1, p10, st10, f = P.project(u, v, w, dt=1.0, rel_tol=1e-10, method="bicgstab")
        runs.append(time.perf_counter() - t1)
    t_proj = float(np.median(runs))
    pc, stc = P.solve(f, p0=p10, rel_tol=1e-12, max_cycles=400, method="bicgstab")
    t2 = time.perf_counter()
    P.solve(f, fixed_cycles=1, method="bicgstab")
    t_step_all = time.perf_counter() - t2
    set_threads(1)
    try:
        t3 = time.perf_counter()
        P.solve(f, fixed_cycles=1, method="bicgstab")
        t_step_one = time.perf_counter() - t3
    finally:
        set_threads(nthr)
    triad = stream_triad_gbs()
    t_step = t_setup + t_proj
    base = {"value": round(1.0 / t_step, 4), "unit": "projections/s", "cores": nthr, "kind": "oracle",
            "sample": "the oracle's whole projection of the same %s workload: classification, ghost stencils and "
                      "hierarchy %.2fs (once), then right-hand side + BiCGStab to rel-res 1e-10 (%d steps, V-cycle "
                      "preconditioner) + correction, median of 3 runs %.2fs (runs %s)"
                      % (wl.name, t_setup, st10.cycles, t_proj, ", ".join("%.2f" % r for r in runs)),
            "setup_s": round(t_setup, 3), "projection_s_median": round(t_proj, 3), "steps": st10.cycles,
            "one_thread": {"bicgstab_step_s": round(t_step_one, 3), "all_threads_step_s": round(t_step_all, 3),
                           "speedup": round(t_step_one / t_step_all, 2)},
            "stream_triad_GBs": round(triad, 1)}
    refs = {"types": P.types(), "p10": p10, "u10": (u1, v1, w1), "steps10": st10.cycles, "pconv": pc,
            "steps_conv": stc.cycles, "rel_conv": stc.rel_residual}
    return base, refs


def rel_err(p, pr, act):
    """Max-norm relative difference of two pressures after aligning their gauges on the
    active (fluid and ghost) cells."""
    import numpy as np
    a = p - p[act].mean()
    b = pr - pr[act].mean()
    return float(np.max(np.abs(a[act] - b[act])) / np.max(np.abs(b[act])))


def probe(args):
    """Fixed kernel sequence for rocprofv3 counter runs: a 512 MiB device-to-device copy
    (calibration: 512 MiB read + 512 MiB written), four level-0 fused sweeps in FP64 on the
    workload, then one projection with a single BiCGStab step (every solver kernel once or
    a few times)."""
    import numpy as np
    import torch

    from paper_2505_17287_amd import ibm
    from paper_2505_17287_amd import inputs as I

    dev = torch.device("cuda:0")
    src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log("probe: copy of %d bytes done" % (src.numel() * 8))
    wl = I.multibody(args.n)
    g = ibm.Grid(wl.xf, wl.yf, wl.zf, precision="fp64")
    g.setup(wl.verts, wl.tris)
    rng = np.random.default_rng(0)
    p = torch.from_numpy(rng.standard_normal(g.shape)).to(dev)
    f = torch.from_numpy(rng.standard_normal(g.shape)).to(dev)
    torch.cuda.synchronize()
    g.debug_sweep(p, f, lam=0.0, n=4, refresh=False)
    torch.cuda.synchronize()
    log("probe: 4 fused FP64 sweeps on %s done" % wl.name)
    u, v, w = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in wl.velocity())
    g.project(u, v, w, dt=1.0, fixed_cycles=1)
    torch.cuda.synchronize()
    log("probe: one projection with a single BiCGStab step done")
    print(json.dumps({"probe": wl.name, "cells": wl.ncells, "copy_bytes": int(src.numel() * 8)}), flush=True)


def fresh_inputs(u0, v0, w0, n):
    """n device copies of the velocity fields, one per projection: the projection corrects
    its input in place, so each timed step takes a copy made before the timed region."""
    return [(u0.clone(), v0.clone(), w0.clone()) for _ in range(n)]


def mixed_form(wl, u0, v0, w0, args):
    """The same projection with FP32 V-cycles inside FP64 BiCGStab: projections/s and the
    FP32 fine sweep's algorithmic bandwidth."""
    import numpy as np
    import torch

    from paper_2505_17287_amd import ibm

    dev = u0.device
    g = ibm.Grid(wl.xf, wl.yf, wl.zf, precision="mixed")
    g.set_geometry(wl.verts, wl.tris)
    p = torch.empty(g.shape, dtype=torch.float64, device=dev)

    def step(uvw):
        g.classify()
        g.build_ghost_stencils()
        return g.project(*uvw, dt=1.0, p=p, rel_tol=1e-10, precision="mixed", method=args.method)[1]

    steps = max(1, min(args.steps, 5))
    require_ok("mixed warmup", [step(fresh_inputs(u0, v0, w0, 1)[0])])
    inputs = fresh_inputs(u0, v0, w0, steps)
    torch.cuda.synchronize()
    g.set_profiling(True, stride=PROFILE_STRIDE)
    t0 = time.perf_counter()
    sts = [step(inputs[q]) for q in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    prof = g.profile()
    g.set_profiling(False)
    require_ok("mixed timed", sts)
    last = None if args.no_cpu_baseline else (p.cpu().numpy(), inputs[-1][0].cpu().numpy())
    avg = prof["ms_fp32"] / max(prof["n_fp32"], 1)
    ach = SWEEP_BYTES["fp32"] * wl.ncells / (avg * 1e-3) / 1e9
    g.close()
    return {"value": round(1000.0 / ms, 3), "unit": "projections/s", "ms_per_step": round(ms, 3), "steps": steps,
            "dtype": "f32+f64", "outer_steps": int(np.median([s.cycles for s in sts])),
            "vcycles": int(np.median([s.vcycles for s in sts])),
            "max_rel_residual": max(s.rel_residual for s in sts), "all_status_ok": True,
            "sweep_fp32": {"achieved_GBs": round(ach, 1), "avg_launch_ms": round(avg, 5),
                           "frac": round(ach / HBM_PEAK_GBS, 4), "launches_timed": prof["n_fp32"]}}, last


def require_ok(what, sts):
    """Every projection of a timed (or warm-up) run must have converged: a failed solve is
    not a measurement."""
    bad = [(i, s.status, s.rel_residual) for i, s in enumerate(sts) if s.status != 0]
    if bad:
        raise SystemExit("bench: %s projections did not converge (index, status, rel-res): %s" % (what, bad))


def tolerance_sweep(g, u0, v0, w0, tols=(1e-10, 1e-11, 1e-12), steps=3):
    """The headline projection (FP64 grid) at tighter tolerances: outer steps, ms per
    projection (median of `steps`, driver-timed) and the pressure of the last run, to set
    the error against the converged oracle beside the cost."""
    import numpy as np
    import torch
    p = torch.empty(g.shape, dtype=torch.float64, device=u0.device)
    out = []
    for tol in tols:
        ts, sts = [], []
        for uvw in fresh_inputs(u0, v0, w0, steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.classify()
            g.build_ghost_stencils()
            _, st = g.project(*uvw, dt=1.0, p=p, rel_tol=tol, precision="fp64", max_cycles=400)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            sts.append(st)
        require_ok("tolerance %.0e" % tol, sts)
        out.append(({"rel_tol": tol, "ms_per_step": round(1000.0 * float(np.median(ts)), 3),
                     "outer_steps": int(np.median([s.cycles for s in sts])),
                     "rel_residual": max(s.rel_residual for s in sts)}, p.cpu().numpy()))
        log("tolerance %.0e: %.2f ms, %d steps" % (tol, out[-1][0]["ms_per_step"], out[-1][0]["outer_steps"]))
    return out


def large_form(args, n=384, steps=3):
    """The same projection on the multi-body 384^3 workload (56.6M cells), FP64 and mixed:
    projections/s timed by the driver (synchronised wall clock around `steps` projections)
    and the fine sweep's algorithmic bandwidth from its HIP events."""
    import numpy as np
    import torch

    from paper_2505_17287_amd import ibm
    from paper_2505_17287_amd import inputs as I

    dev = torch.device("cuda:0")
    wl = I.multibody(n)
    u0, v0, w0 = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in wl.velocity())
    out = {"workload": wl.name, "cells": wl.ncells}
    for prec in ("fp64", "mixed"):
        g = ibm.Grid(wl.xf, wl.yf, wl.zf, precision=prec)
        g.set_geometry(wl.verts, wl.tris)
        p = torch.empty(g.shape, dtype=torch.float64, device=dev)

        def step(uvw):
            g.classify()
            g.build_ghost_stencils()
            return g.project(*uvw, dt=1.0, p=p, rel_tol=1e-10, precision=prec)[1]

        require_ok("%d^3 %s warmup" % (n, prec), [step(fresh_inputs(u0, v0, w0, 1)[0])])
        inputs = fresh_inputs(u0, v0, w0, steps)
        torch.cuda.synchronize()
        g.set_profiling(True, stride=PROFILE_STRIDE)
        t0 = time.perf_counter()
        sts = [step(inputs[q]) for q in range(steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        prof = g.profile()
        g.set_profiling(False)
        require_ok("%d^3 %s timed" % (n, prec), sts)
        del inputs
        kind = "fp64" if prec == "fp64" else "fp32"
        avg = prof["ms_" + kind] / max(prof["n_" + kind], 1)
        ach = SWEEP_BYTES[kind] * wl.ncells / (avg * 1e-3) / 1e9
        out[prec] = {"value": round(1000.0 / ms, 3), "unit": "projections/s", "ms_per_step": round(ms, 3),
                     "steps": steps, "outer_steps": int(np.median([s.cycles for s in sts])),
                     "max_rel_residual": max(s.rel_residual for s in sts),
                     "sweep_" + kind: {"achieved_GBs": round(ach, 1), "avg_launch_ms": round(avg, 5),
                                       "frac": round(ach / HBM_PEAK_GBS, 4), "launches_timed": prof["n_" + kind]}}
        log("%d^3 %s: %.2f ms/projection, sweep %.0f GB/s" % (n, prec, ms, ach))
        g.close()
    return out


# Every PROFILE_STRIDE-th level-0 sweep of the timed steps is bracketed by HIP events (on its
# launch stream).  Bracketing every sweep costs about 0.6 ms per 256^3 projection in event
# overhead; 7 is coprime to the four sweeps of a V(2,2) cycle, so the sample visits every
# sweep position.
PROFILE_STRIDE = 7

MOM_SWEEP_BYTES = 73.0  # algorithmic bytes per cell of one SRJ sweep: read 3 x 8 + 3 x 8 (b) + 1, write 3 x 8


def momentum_form(wl, args, steps=None):
    """The advection-diffusion half-step on the same grid and bodies (Re = 1000, dt = half the
    smallest width, 8 Chebyshev factors per cycle, rel-res 1e-10): steps/s, and the scheduled
    Jacobi sweep's algorithmic bandwidth, from the time difference between runs of 3 and 1
    fixed cycles (each sweep with its ghost-row pass)."""
    import numpy as np
    import torch

    from paper_2505_17287_amd import ibm

    dev = torch.device("cuda:0")
    g = ibm.Grid(wl.xf, wl.yf, wl.zf)
    g.setup(wl.verts, wl.tris)
    U0n, H0n = wl.cell_fields()
    U0 = torch.from_numpy(np.ascontiguousarray(U0n)).to(dev)
    H0 = torch.from_numpy(np.ascontiguousarray(H0n)).to(dev)
    del U0n, H0n
    U, H = U0.clone(), H0.clone()
    nu, dt, m = 1e-3, 0.5 * float(np.min(np.diff(wl.xf))), 8

    def step(**kw):
        U.copy_(U0)
        H.copy_(H0)
        torch.cuda.synchronize()
        code, st = g.momentum_step(U, H, nu, dt, m=m, **kw)
        return st

    steps = steps or max(1, min(args.steps, 5))
    step()
    sts = [step(rel_tol=1e-10) for _ in range(steps)]
    t_step = float(np.median([s.t_step for s in sts]))
    t1 = float(np.median([step(fixed_cycles=1).t_step for _ in range(3)]))
    t3 = float(np.median([step(fixed_cycles=3).t_step for _ in range(3)]))
    per_sweep = (t3 - t1) / (2 * m)
    ach = MOM_SWEEP_BYTES * wl.ncells / per_sweep / 1e9
    g.close()
    return {"value": round(1.0 / t_step, 3), "unit": "steps/s", "ms_per_step": round(1000.0 * t_step, 3),
            "steps": steps, "dtype": "f64", "nu": nu, "dt": dt, "srj_factors": m,
            "cycles": int(np.median([s.cycles for s in sts])), "sweeps": int(np.median([s.sweeps for s in sts])),
            "rho": round(sts[0].rho, 6), "max_rel_residual": max(s.rel_residual for s in sts),
            "srj_sweep": {"achieved_GBs": round(ach, 1), "ms_per_sweep": round(1000.0 * per_sweep, 4),
                          "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_cell": MOM_SWEEP_BYTES}}


def paper_solver_form(wl, u0, v0, w0, args, max_steps=5000):
    """The same projection with the paper's pressure solver: BiCGStab preconditioned by 16
    scheduled relaxed Jacobi sweeps (Chebyshev factors) instead of one V-cycle.  One timed
    projection (the kernels are warm from the headline run)."""
    import torch

    from paper_2505_17287_amd import ibm

    dev = u0.device
    g = ibm.Grid(wl.xf, wl.yf, wl.zf)
    g.set_geometry(wl.verts, wl.tris)
    u, v, w = u0.clone(), v0.clone(), w0.clone()
    p = torch.empty(g.shape, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.classify()
    g.build_ghost_stencils()
    _, st = g.project(u, v, w, dt=1.0, p=p, rel_tol=1e-10, method="bicgstab_srj", srj_sweeps=16,
                      max_cycles=max_steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0
    g.close()
    return {"value": round(1000.0 / ms, 4), "unit": "projections/s", "ms_per_step": round(ms, 1),
            "method": "bicgstab + 16 SRJ sweeps", "outer_steps": st.cycles, "status": st.status,
            "rel_residual": st.rel_residual, "jacobi_sweeps": 32 * st.cycles}


def momentum_cpu_baseline(wl, m=8):
    """The advection-diffusion oracle (numpy) on the same workload: ghost rows of u^n,
    convective term and right-hand side timed in full, one scheduled-Jacobi sweep timed and
    scaled to the m sweeps of the GPU step (the Dirichlet weights, a one-off per geometry,
    are not timed)."""
    import numpy as np
    from oracle import OracleProblem
    from oracle.momentum import MomentumOracle, srj_rho, srj_schedule
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    mo = MomentumOracle(OracleProblem.from_workload(wl))
    U0, H0 = wl.cell_fields()
    nu, dt = 1e-3, 0.5 * float(np.min(np.diff(wl.xf)))
    a = 0.5 * nu * dt
    t0 = time.perf_counter()
    U = np.array(U0, copy=True)
    U[:, mo.types == 2] = 0.0
    U = mo.ghost_rows(U, None, src=U.copy())
    H = mo.convective(U)
    b = mo.cn_rhs(U, H, H0, nu, dt, False)
    t1 = time.perf_counter()
    w = srj_schedule(srj_rho(mo.m, a), m)[0]
    mo.srj_sweep(U, b, a, w)
    t2 = time.perf_counter()
    t_step = (t1 - t0) + m * (t2 - t1)
    return {"value": round(1.0 / t_step, 4), "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": "ghost rows, convection and right-hand side (%.2fs) in full, one of the %d sweeps timed "
                      "(%.2fs) and scaled" % (t1 - t0, m, t2 - t1)}


def moving_cpu_baseline(wl):
    """The oracle on one move of the same workload: classification of the moved bodies, the
    fresh list with intercepts and weights, and the fill."""
    import numpy as np
    from oracle import OracleProblem
    from oracle.fresh import FreshOracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    h = float(np.min(np.diff(wl.xf)))
    P0 = OracleProblem(wl.xf, wl.yf, wl.zf)
    P0.set_mesh(wl.verts, wl.tris)
    P0.classify()
    U0, _ = wl.cell_fields()
    t0 = time.perf_counter()
    P1 = OracleProblem(wl.xf, wl.yf, wl.zf)
    P1.set_mesh(wl.verts + np.array([0.3 * h, -0.2 * h, 0.1 * h]), wl.tris)
    P1.classify()
    P1.build_stencils()
    t1 = time.perf_counter()
    n_sample = 200
    F = FreshOracle(P0.types(), P1, limit=n_sample)
    F.fill(U0)
    t2 = time.perf_counter()
    nf = F.n_all
    t = (t1 - t0) + (t2 - t1) * nf / max(len(F.cells), 1)
    return {"value": round(1.0 / t, 4), "unit": "moves/s", "cores": threads, "kind": "oracle",
            "sample": "one move: classification and ghost stencils of the moved bodies (%.2fs) in full, "
                      "%d of the %d fresh cells (intercept, weights, fill) timed (%.2fs) and scaled"
                      % (t1 - t0, len(F.cells), nf, t2 - t1)}


def moving_form(wl, args, moves=5):
    """Moving bodies on the same workload: every body translated by (0.3, -0.2, 0.1) of the
    smallest cell width per move; a move re-classifies, rebuilds the ghost stencils and the
    hierarchy, lists the fresh cells with their intercepts and weights (ibm_move_geometry),
    and sets the fresh cells of the three velocity components (ibm_fill_fresh)."""
    import numpy as np
    import torch

    from paper_2505_17287_amd import ibm

    dev = torch.device("cuda:0")
    g = ibm.Grid(wl.xf, wl.yf, wl.zf)
    g.setup(wl.verts, wl.tris)
    U0, _ = wl.cell_fields()
    U = torch.from_numpy(np.ascontiguousarray(U0)).to(dev)
    del U0
    h = float(np.min(np.diff(wl.xf)))
    step = np.array([0.3 * h, -0.2 * h, 0.1 * h])
    verts = wl.verts.copy()
    verts = verts + step
    g.move_geometry(verts, wl.tris)  # warm-up move
    g.fill_fresh(U)
    torch.cuda.synchronize()
    ts, nfs = [], []
    for _ in range(moves):
        verts = verts + step
        t0 = time.perf_counter()
        counts, nf = g.move_geometry(verts, wl.tris)
        g.fill_fresh(U)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        nfs.append(nf)
    g.close()
    t = float(np.median(ts))
    return {"value": round(1.0 / t, 2), "unit": "moves/s", "ms_per_move": round(1000.0 * t, 3), "moves": moves,
            "fresh_cells": int(np.median(nfs)), "ghosts": int(counts[1]), "dtype": "f64",
            "includes": "classification, ghost stencils, multigrid hierarchy, fresh list + weights, fresh fill"}


def serving_form(args):
    """Continuous batching of whole projections (grids 64^3..256^3, 1-4 bodies) against the
    same requests served one at a time in plain FP64: saturation throughput, then p50/p99
    latency at Poisson arrival rates of 0.5, 0.9 and 1.5 x the sequential capacity."""
    from paper_2505_17287_amd import serve

    R = args.serve_requests
    log("serving: generating %d requests" % R)
    base = serve.make_trace(R, qps=None)
    warm = []
    for n in (64, 128, 192, 256):
        warm += [q for q in base if q.shape[0] == n][:1]
    seq = serve.Server(slots=1, precision="fp64")
    srv = serve.Server(slots=args.serve_slots, precision="mixed")
    try:
        seq.run(warm)
        for _ in range(args.serve_slots):
            srv.run(warm)
        out = {"requests": R, "sizes": [64, 128, 192, 256], "slots": args.serve_slots,
               "budget_GB": srv.budget / 2 ** 30, "served_precision": "mixed", "baseline": "one at a time, fp64"}
        r, mk = seq.run(base)
        out["sequential_fp64_saturation"] = serve.summarize(r, mk)
        mu = out["sequential_fp64_saturation"]["solves_per_s"]
        r, mk = srv.run(base)
        out["served_saturation"] = serve.summarize(r, mk)
        sweep = []
        for x in (0.5, 0.9, 1.5):
            tr = serve.make_trace(0, qps=x * mu, requests=base)
            point = {"qps": round(x * mu, 3), "load_vs_seq_capacity": x}
            for name, server in (("served", srv), ("sequential_fp64", seq)):
                try:
                    rr, mm = server.run(tr)
                    point[name] = serve.summarize(rr, mm)
                except Exception as e:  # a failed request ends this point; it is reported, not retried
                    point[name] = {"error": "%s: %s" % (type(e).__name__, e)}
                    log("serving qps %.2f (%s) failed: %s" % (x * mu, name, e))
            sweep.append(point)
            if "error" not in point["served"] and "error" not in point["sequential_fp64"]:
                log("serving qps %.2f: served p50 %.1f p99 %.1f ms, sequential p50 %.1f p99 %.1f ms"
                    % (x * mu, point["served"]["p50_ms"], point["served"]["p99_ms"],
                       point["sequential_fp64"]["p50_ms"], point["sequential_fp64"]["p99_ms"]))
        out["qps_sweep"] = sweep
        out["resident_GB"] = round((srv.resident_bytes() + seq.resident_bytes()) / 2 ** 30, 2)
        return out
    finally:
        seq.close()
        srv.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--method", default="bicgstab", choices=["bicgstab", "vcycle"])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision and serving forms (headline FP64 line only)")
    ap.add_argument("--serve-requests", type=int, default=32,
                    help="requests per serving run (sizes 64^3..256^3, 1-4 bodies each)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--momentum", action="store_true",
                    help="only the advection-diffusion half-step form (3 steps), one JSON line")
    ap.add_argument("--moving", action="store_true",
                    help="only the moving-body form (translated bodies, fresh cells), one JSON line")
    ap.add_argument("--paper-solver", action="store_true",
                    help="only the projection with the paper's pressure solver (BiCGStab + SRJ), one JSON line")
    ap.add_argument("--probe", action="store_true",
                    help="kernel probe for hardware counters: a plain device copy of known size for "
                         "calibration, 4 fused FP64 sweeps of level 0, one single-step projection")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        probe(args)
        return
    if args.paper_solver:
        import numpy as np
        import torch
        from paper_2505_17287_amd import inputs as I
        wl = I.multibody(args.n)
        u0, v0, w0 = (torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in wl.velocity())
        print(json.dumps({"workload": wl.name, "paper_solver": paper_solver_form(wl, u0, v0, w0, args)}), flush=True)
        return
    if args.moving:
        from paper_2505_17287_amd import inputs as I
        wl = I.multibody(args.n)
        print(json.dumps({"workload": wl.name, "moving": moving_form(wl, args)}), flush=True)
        return
    if args.momentum:
        from paper_2505_17287_amd import inputs as I
        wl = I.multibody(args.n)
        print(json.dumps({"workload": wl.name, "momentum": momentum_form(wl, args, steps=3)}), flush=True)
        return

    import numpy as np
    import torch

    from paper_2505_17287_amd import ibm
    from paper_2505_17287_amd import inputs as I

    dev = torch.device("cuda:0")
    wl = I.multibody(args.n)
    log("workload", wl.name, wl.shape, "triangles", len(wl.tris))
    g = ibm.Grid(wl.xf, wl.yf, wl.zf, precision=args.precision)
    g.set_geometry(wl.verts, wl.tris)
    u0, v0, w0 = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in wl.velocity())
    p = torch.empty(g.shape, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(uvw):
        counts = g.classify()
        ng = g.build_ghost_stencils()
        _, st = g.project(*uvw, dt=1.0, p=p, rel_tol=1e-10, precision=args.precision, method=args.method)
        return counts, ng, st

    for q in range(args.warmup):
        counts, ng, st = step(fresh_inputs(u0, v0, w0, 1)[0])
        log("warmup", q, "steps", st.cycles, "vcycles", st.vcycles, "rel", st.rel_residual, "status", st.status)
        require_ok("warmup", [st])
    inputs = fresh_inputs(u0, v0, w0, args.steps)
    torch.cuda.synchronize()
    g.set_profiling(True, stride=PROFILE_STRIDE)
    t0 = time.perf_counter()
    sts = []
    for q in range(args.steps):
        counts, ng, st = step(inputs[q])
        sts.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile()
    g.set_profiling(False)
    require_ok("timed", sts)
    cyc, vcyc = [s.cycles for s in sts], [s.vcycles for s in sts]
    # the last timed projection's results, compared with the oracle below (copied to the
    # host only when the oracle runs)
    last, types_gpu = None, None
    if not args.no_cpu_baseline:
        last = (p.cpu().numpy(), inputs[-1][0].cpu().numpy())
        types_gpu = g.cell_types().cpu().numpy()
    del inputs
    ms = (t1 - t0) * 1000.0 / args.steps
    value = 1000.0 / ms

    # dominant kernel: the fused red-black sweep of level 0
    kind = "fp64" if args.precision == "fp64" else "fp32"
    n_sw = prof["n_fp64"] if kind == "fp64" else prof["n_fp32"]
    ms_sw = prof["ms_fp64"] if kind == "fp64" else prof["ms_fp32"]
    avg_ms = ms_sw / max(n_sw, 1)
    bytes_per_launch = SWEEP_BYTES[kind] * wl.ncells
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "k_rbgs_fused<%s>" % ("double" if kind == "fp64" else "float"),
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic(wl.name) if kind == "fp64" else None,
                "avg_launch_ms": round(avg_ms, 5), "launches_timed": int(n_sw),
                "timed_every": PROFILE_STRIDE, "bytes_per_launch": bytes_per_launch}
    out = {
        "metric": "Poisson solves/s + HBM GB/s at 256^3, rel-res 1e-10; p50/p99 serve latency",
        "value": round(value, 3),
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": wl.ncells, "triangles": int(len(wl.tris)),
                   "fluid_ghost_dead": [int(x) for x in counts], "ghosts": int(ng),
                   "method": args.method, "outer_steps": int(np.median(cyc)), "vcycles": int(np.median(vcyc)),
                   "rel_tol": 1e-10, "precision": args.precision, "all_status_ok": True,
                   "max_rel_residual": max(s.rel_residual for s in sts),
                   "parallelism": "1 GPU"},
        "roofline": roofline,
    }
    mixed_last, sweep = None, []
    if not args.no_forms:
        out["forms"] = {}
        out["forms"]["mixed"], mixed_last = mixed_form(wl, u0, v0, w0, args)
        if args.precision == "fp64":
            sweep = tolerance_sweep(g, u0, v0, w0)
        out["forms"]["momentum"] = momentum_form(wl, args)
        out["forms"]["paper_solver"] = paper_solver_form(wl, u0, v0, w0, args)
        out["forms"]["moving"] = moving_form(wl, args)
        out["forms"]["serving"] = None
        try:
            out["forms"]["serving"] = serving_form(args)
        except Exception as e:  # reported in the JSON line; the other forms stand
            out["forms"]["serving"] = {"error": "%s: %s" % (type(e).__name__, e)}
            log("serving form failed: %s" % e)
        g.close()
        del u0, v0, w0, p
        torch.cuda.empty_cache()
        if args.n == 256:
            out["forms"]["large_384"] = large_form(args)
    if not args.no_cpu_baseline:
        log("cpu baseline and accuracy reference (oracle) ...")
        base, refs = oracle_reference(wl)
        out["cpu_baseline"] = base
        act = refs["types"] != 2
        uref = refs["u10"][0]

        def errs(pu):
            pg, ug = pu
            return {"p_vs_oracle_same_tol": rel_err(pg, refs["p10"], act),
                    "p_vs_oracle_converged": rel_err(pg, refs["pconv"], act),
                    "u_vs_oracle_same_tol": float(np.max(np.abs(ug - uref)) / np.max(np.abs(uref)))}

        out["err_vs_oracle"] = errs(last)
        out["err_vs_oracle"].update({"types_equal": bool(np.array_equal(types_gpu, refs["types"])),
                                     "oracle_steps_same_tol": refs["steps10"],
                                     "oracle_converged": {"rel_tol": 1e-12, "rel_residual": refs["rel_conv"],
                                                          "extra_steps_from_1e-10": refs["steps_conv"]}})
        if mixed_last is not None:
            out["forms"]["mixed"]["err_vs_oracle"] = errs(mixed_last)
        if sweep:
            out["tolerance_sweep"] = [dict(row, p_vs_oracle_converged=rel_err(pt, refs["pconv"], act))
                                      for row, pt in sweep]
        log("accuracy:", json.dumps(out["err_vs_oracle"]))
        if not args.no_forms:
            log("cpu baselines of the forms (oracle) ...")
            out["forms"]["momentum"]["cpu_baseline"] = momentum_cpu_baseline(wl)
            out["forms"]["moving"]["cpu_baseline"] = moving_cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
