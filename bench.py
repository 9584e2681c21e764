#!/usr/bin/env python
"""Benchmark of the EBIT elliptic hot path on one MI355X.

A step is one pass of the whole hot path over the workload: cut fractions
and multigrid hierarchies from the markers (ebit_build_coeffs), the implicit
heat solve (cold start, to the workload's relative residual), the mass flux,
and the ghost-fluid projection (cold start, same target).  T* = T^n and
u* = u^n: the advection and momentum predictor are outside the path.  The
default workload is the largest single-GPU one, the 3D film: 256^3 cells,
interface y = 0.25 + 0.02 cos(2 pi x) cos(2 pi z) + 1e-3 noise (PCG64(5)),
heated wall T = 1 at y = 0, outflow at y = 1, periodic in x and z, density
ratio 200, conductivity ratio 0.2, mixed precision, rtol 1e-9.

Prints ONE JSON line.  value = fine cells advanced through one full step per
second (cell-steps/s).  Progress lines go to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "bubble2d_256": (1, None),
    "stefan2d_64": (0, None),
    "bubble3d_128": (2, None),
    "film3d_256": (4, None),
    "batch64_2d": (3, None),
}
# relative residual target of each workload's solves
RTOL = {"stefan2d_64": 1e-10}
DEFAULT_RTOL = 1e-9


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)

HBM_PEAK_GBS = 8000.0
KERNEL_CLASSES = ["fine_smooth", "fine_restrict", "coarse", "outer_apply", "outer_update", "tail"]
# the HIP kernels of each class (names as rocprofv3 reports them): 2D grids,
# and 3D grids (colour-split fine level, streaming p-update and A p)
KERNEL_NAMES = {
    "fine_smooth": "kb_rb_fine",
    "fine_restrict": "kb_fine_restrict",
    "coarse": "kb_rb_coarse",
    "tail": "kb_tail",
    "outer_apply": "kb_p_update_apply",
    "outer_update": "kb_update_xr",
}
KERNEL_NAMES_3D = dict(KERNEL_NAMES, fine_smooth="kb_half3", fine_restrict="kb_fine_restrict_split",
                       outer_apply="kb_p_update3 + kb_apply_q3")


def algorithmic_bytes_per_cell(kclass, precision, dim):
    """Bytes one launch of a kernel class must move per fine cell (sparse
    theta reads on cut links, O(interface), are not counted).  sx: size of
    the inner iterate and of the right-hand side the V-cycle smooths against
    (4 in mixed precision, 8 in FP64).  The coarse-level and tail classes
    work on levels of varying size and have no per-fine-cell model (None)."""
    sx = 4 if precision == "mixed" else 8
    agg = 2 ** dim
    if kclass == "fine_smooth":      # per full red-black sweep: read x, r, flags; write x
        return sx + sx + 1 + sx
    if kclass == "fine_restrict":    # read x (all cells), r and flags (colour-0 cells); write coarse b, clear coarse x
        return sx + (sx + 1) / 2 + 2 * sx / agg
    if kclass == "outer_apply":      # read z, p_old, flags; write p_new and q (FP64)
        return sx + 8 + 1 + 8 + 8 if dim == 2 else sx + 8 + 8 + 8 + 1 + 8  # 3D: p_new written, then read back
    if kclass == "outer_update":     # read x, p, r, q; write x, r (FP64)
        return 48.0
    return None


def solve_model_bytes_per_iteration(precision, dim, schedule):
    """Algorithmic bytes per fine cell of one outer iteration (one V-cycle
    plus the outer update), by the table of the design: a full red-black
    sweep 2 sx + sx + 1 (read x, r, flag; write x), residual + restriction
    and prolongation + correction 18 (FP64) / 9.5 (FP32) each, all levels
    x 8/7 (3D) or x 4/3 (2D), plus the FP64 outer residual and correction
    (about 33 B)."""
    sx = 4 if precision == "mixed" else 8
    sch = schedule or {"nu1": 2, "nu2": 2}
    sweep = 3 * sx + 1
    transfer = 9.5 if precision == "mixed" else 18.0
    fine = (sch["nu1"] + sch["nu2"]) * sweep + 2 * transfer
    levels = 8.0 / 7.0 if dim == 3 else 4.0 / 3.0
    return fine * levels + 33.0


SOLVE_SOURCES = ("ebit_internal.h", "solver.hip")


def kernel_source_digest():
    """Digest of the sources of the solve kernels (the roofline kernel is
    one of them): the committed counter traffic is reported only while they
    are unchanged since it was measured."""
    import hashlib
    h = hashlib.sha256()
    cdir = os.path.join(ROOT, "paper_2402_13677_amd", "csrc")
    for name in SOLVE_SOURCES:
        h.update(open(os.path.join(cdir, name), "rb").read())
    return h.hexdigest()[:16]


def make_case(name):
    import ebit_inputs as ei
    idx, n = WORKLOADS[name]
    return ei.config(idx, n)


def autotune(ctx, dc, case):
    """Untimed set-up: let the library pick the solve schedule on the first
    step's heat and pressure right-hand sides."""
    import torch
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    bh = torch.empty_like(dc.T0)
    ctx.heat_rhs(dc.T0, bh)
    m = torch.zeros_like(dc.T0)
    ctx.mass_flux(dc.T0, m)
    bp = torch.empty_like(dc.T0)
    ctx.project_rhs([u.clone() for u in dc.u_l], [u.clone() for u in dc.u_v], m, bp)
    chosen, _ = ctx.autotune(bh, bp)
    return {k: chosen[k] for k in ("nu1", "nu2", "tail_cells", "check_every")}


def parse_schedule(text):
    nu, tail, k = (int(v) for v in text.split(","))
    return {"nu1": nu, "nu2": nu, "tail_cells": tail, "check_every": k}


def workload_rtol(case):
    return RTOL.get(case.name, DEFAULT_RTOL)


def run_gpu(case, precision, steps, warmup, profile=False, tune=True, warm=False):
    """Time `steps` full steps after `warmup` untimed ones (and, with tune,
    the untimed schedule autotuning).  With profile, the library also times
    every launch of each kernel class with hipEvents on its stream; with
    warm, each solve starts from the previous step's T and p instead of
    zero.  Returns (elapsed, records, per-class (launches, ms), schedule);
    the records also hold the level sizes."""
    import torch
    from paper_2402_13677_amd import ebit

    fixed = tune if isinstance(tune, dict) else {}
    opts = ebit.default_opts(rtol=workload_rtol(case), precision=ebit.MIXED if precision == "mixed" else ebit.FP64,
                             **fixed)
    ctx, dc = ebit.context_for(case, opts)
    schedule = autotune(ctx, dc, case) if tune is True else (fixed or None)
    T = dc.T0.clone()
    mdot = torch.zeros_like(T)
    p = torch.zeros_like(T)
    u_l = [u.clone() for u in dc.u_l]
    u_v = [u.clone() for u in dc.u_v]
    rec = {"heat_ms": [], "proj_ms": [], "heat_it": [], "proj_it": [], "heat_res": [], "proj_res": [],
           "div": [], "fallbacks": []}

    def step(record):
        ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
        sh = ctx.heat_solve(T, T, use_guess=warm)
        ctx.mass_flux(T, mdot, stats=False)
        sp = ctx.project(u_l, u_v, mdot, p, use_guess=warm)
        if record:
            rec["heat_ms"].append(sh["seconds"] * 1e3)
            rec["proj_ms"].append(sp["seconds"] * 1e3)
            rec["heat_it"].append(sh["iters"])
            rec["proj_it"].append(sp["iters"])
            rec["heat_res"].append(sh["rel_res"])
            rec["proj_res"].append(sp["rel_res"])
            rec["div"].append(sp["div_max"])

    for _ in range(warmup):
        step(False)
    if profile:
        ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern = {}
    if profile:
        for kc, name in enumerate(KERNEL_CLASSES):
            kern[name] = ctx.profile_read(kc)
        ctx.profile(False)
    # the fallback count of the stencil, read once after the timed steps
    rec["fallbacks"].append(ctx.mass_flux(T, torch.zeros_like(T))["fallbacks"])
    rec["levels"] = [a * b * c for a, b, c in ctx.levels()]
    ctx.close()
    return elapsed, rec, kern, schedule


def cell_updates(rec, schedule, ms_step):
    """Smoother cell updates per second: per V-cycle nu1 + nu2 sweeps of
    every level above the exactly solved one (at most 64 cells), over the
    whole step's time and over the solves' time alone."""
    sch = schedule or {"nu1": 2, "nu2": 2}
    per_cycle = (sch["nu1"] + sch["nu2"]) * sum(n for n in rec["levels"] if n > 64)
    cycles = statistics.mean(h + p for h, p in zip(rec["heat_it"], rec["proj_it"]))
    solve_ms = statistics.mean(h + p for h, p in zip(rec["heat_ms"], rec["proj_ms"]))
    upd = cycles * per_cycle
    return {"per_step": upd, "over_step": upd / (ms_step * 1e-3), "over_solves": upd / (solve_ms * 1e-3)}


def run_gpu_batch(cases, precision, steps, warmup, batched=True, schedule=None, keep_solves=None):
    """The uneven batch: one step = build + heat + mass flux + projection
    of every case; batched (one launch per solve kernel over all cases, the
    schedule autotuned untimed on the first step's right-hand sides) or one
    context after another with a given schedule.  Returns (elapsed,
    iterations, schedule)."""
    import torch
    from paper_2402_13677_amd import ebit

    opts = ebit.default_opts(rtol=DEFAULT_RTOL, precision=ebit.MIXED if precision == "mixed" else ebit.FP64,
                             **(schedule or {}))
    ctxs, dcs = [], []
    for c in cases:
        ctx, dc = ebit.context_for(c, opts)
        ctxs.append(ctx)
        dcs.append(dc)
    T = [d.T0.clone() for d in dcs]
    m = [torch.zeros_like(t) for t in T]
    p = [torch.zeros_like(t) for t in T]
    u_l = [[u.clone() for u in d.u_l] for d in dcs]
    u_v = [[u.clone() for u in d.u_v] for d in dcs]
    b = ebit.Batch(ctxs) if batched else None
    its = []
    if batched and schedule is None:
        b.build_coeffs([d.markers for d in dcs], [d.vcol for d in dcs], [d.ccol for d in dcs],
                       [c.dt for c in cases])
        bh, bp = [], []
        for ctx, d in zip(ctxs, dcs):
            x = torch.empty_like(d.T0)
            ctx.heat_rhs(d.T0, x)
            bh.append(x)
            mm = torch.zeros_like(d.T0)
            ctx.mass_flux(d.T0, mm)
            y = torch.empty_like(d.T0)
            ctx.project_rhs([u.clone() for u in d.u_l], [u.clone() for u in d.u_v], mm, y)
            bp.append(y)
        chosen, _ = b.autotune(bh, bp)
        schedule = {k: chosen[k] for k in ("nu1", "nu2", "tail_cells", "check_every")}

    solve = {"heat_s": [], "proj_s": [], "heat_iters": [], "proj_iters": []}

    def step():
        if batched:
            b.build_coeffs([d.markers for d in dcs], [d.vcol for d in dcs], [d.ccol for d in dcs],
                           [c.dt for c in cases])
            sh = b.heat_solve(T, T)
            b.mass_flux(T, m, stats=False)
            sp = b.project(u_l, u_v, m, p)
            its.append((max(x["iters"] for x in sh), max(x["iters"] for x in sp)))
            solve["heat_s"].append(sh[0]["seconds"])
            solve["proj_s"].append(sp[0]["seconds"])
            solve["heat_iters"].append([x["iters"] for x in sh])
            solve["proj_iters"].append([x["iters"] for x in sp])
        else:
            hs, ps, hi, pi = [], [], [], []
            for i, (ctx, d, c) in enumerate(zip(ctxs, dcs, cases)):
                ctx.build_coeffs(d.markers, d.vcol, d.ccol, c.dt)
                st = ctx.heat_solve(T[i], T[i])
                hs.append(st["seconds"])
                hi.append(st["iters"])
                ctx.mass_flux(T[i], m[i], stats=False)
                st = ctx.project(u_l[i], u_v[i], m[i], p[i])
                ps.append(st["seconds"])
                pi.append(st["iters"])
            solve["heat_s"].append(hs)
            solve["proj_s"].append(ps)
            solve["heat_iters"].append(hi)
            solve["proj_iters"].append(pi)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if b is not None:
        b.close()
    for c in ctxs:
        c.close()
    if keep_solves is not None:
        keep_solves.update({k: v[warmup:] for k, v in solve.items()})
    return el, its, schedule


def gpu_first_step(case, precision, schedule):
    """The first step of the workload from its seeded inputs, solved to the
    workload's rtol as benchmarked: host copies of T, mdot, p, u_l, u_v."""
    import torch
    from paper_2402_13677_amd import ebit

    opts = ebit.default_opts(rtol=workload_rtol(case), precision=ebit.MIXED if precision == "mixed" else ebit.FP64,
                             **(schedule or {}))
    ctx, dc = ebit.context_for(case, opts)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    T = torch.zeros_like(dc.T0)
    ctx.heat_solve(dc.T0, T)
    m = torch.zeros_like(T)
    ctx.mass_flux(T, m)
    p = torch.zeros_like(T)
    ctx.project(dc.u_l, dc.u_v, m, p)
    torch.cuda.synchronize()
    out = {"T": T.cpu().numpy().ravel(), "mdot": m.cpu().numpy().ravel(), "p": p.cpu().numpy().ravel(),
           "u_l": [u.cpu().numpy() for u in dc.u_l], "u_v": [u.cpu().numpy() for u in dc.u_v]}
    ctx.close()
    del dc
    torch.cuda.empty_cache()
    return out


def _oracle_step(case, threads):
    """One full step of the oracle (plain FP64) on the workload's seeded
    inputs: geometry, heat solve, mass flux, ghost velocities, pressure
    solve, face update; the solves by its multigrid (oracle/mg.c) on
    `threads` OpenMP threads.  Returns (fields, seconds per phase)."""
    from oracle import flux, geometry, heat, mg, project
    t = {}
    t0 = time.perf_counter()
    geo = geometry.build(case)
    opH = heat.operator(case, geo)
    bH = heat.rhs(case, geo, case.T0)
    t["setup"] = time.perf_counter() - t0
    t1 = time.perf_counter()
    T = mg.solve_op(opH, bH, threads=threads)
    t["heat_solve"] = time.perf_counter() - t1
    del opH
    t1 = time.perf_counter()
    mdot, _ = flux.mass_flux(case, geo, T)
    ulg, uvg = project.ghost_velocities(case, geo, mdot, case.u_l, case.u_v)
    rhs = project.divergence(case, ulg, uvg) - project.bc_rhs(case, geo)
    opP = project.operator(case, geo)
    t["flux_and_rhs"] = time.perf_counter() - t1
    t1 = time.perf_counter()
    p = mg.solve_op(opP, -rhs, threads=threads)
    t["pressure_solve"] = time.perf_counter() - t1
    del opP
    ul1, uv1 = project.face_update(case, geo, p, ulg, uvg)
    t["step"] = time.perf_counter() - t0
    return {"T": T, "mdot": mdot, "p": p, "u_l": ul1, "u_v": uv1}, t


def cpu_baseline_leg(case, gpu_steps, one_thread=True):
    """The oracle timed on the host's cores, and the GPU's first step against
    it.  (1) one full oracle step with as many OpenMP threads as the host has
    cores: the reported baseline (cell-steps/s) and the reference for the
    error of each GPU precision at the benchmarked rtol; (2) the oracle on
    one thread over a bounded sample: the full step on grids up to 2^21
    cells, the heat solve alone above."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    cores = os.cpu_count() or 1
    log(f"oracle step on {cores} threads")
    ref, t = _oracle_step(case, cores)
    base = {"value": case.ncells / t["step"], "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"one full step of the workload ({t['step']:.1f} s: geometry, multigrid heat and pressure "
                      f"solves to the discrete solution, mass flux, projection) on {cores} threads of {host_cpu()}",
            "phases_s": t}

    def rel(a, b):
        a = np.concatenate([np.ravel(x) for x in a]) if isinstance(a, list) else np.ravel(a)
        b = np.concatenate([np.ravel(x) for x in b]) if isinstance(b, list) else np.ravel(b)
        nb = np.linalg.norm(b)
        return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))

    err = {prec: {k: rel(g[k], ref[k]) for k in ("T", "p", "mdot", "u_l", "u_v")} for prec, g in gpu_steps.items()}
    del ref
    if one_thread:
        if case.ncells <= (1 << 21):
            log("oracle step on 1 thread")
            _, t1 = _oracle_step(case, 1)
            base["one_thread"] = {"value": case.ncells / t1["step"], "unit": "cell-steps/s", "cores": 1,
                                  "sample": f"one full step ({t1['step']:.1f} s)"}
        else:
            log("oracle heat solve on 1 thread")
            from oracle import geometry, heat, mg
            geo = geometry.build(case)
            opH = heat.operator(case, geo)
            bH = heat.rhs(case, geo, case.T0)
            t0 = time.perf_counter()
            mg.solve_op(opH, bH, threads=1)
            el = time.perf_counter() - t0
            base["one_thread"] = {"heat_solve_s": el, "cells_per_s": case.ncells / el, "cores": 1,
                                  "sample": f"the heat solve of one step alone ({el:.1f} s; the full step on one "
                                            "thread would take minutes)"}
    return base, err


def host_cpu():
    """The host CPU's model name and logical core count."""
    name = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return f"{name}, {os.cpu_count()} logical cores"


def half_sweep_mix(schedule):
    """Launches of each form of the 3D colour-split half-sweep in one
    V-cycle: form 1 (the first half-sweep, from a zero guess: no iterate
    read), form 2 (the first post-smoothing half-sweep: the other colour
    takes its parent's coarse correction) and form 0 (the rest)."""
    nu1, nu2 = (schedule or {}).get("nu1", 2), (schedule or {}).get("nu2", 2)
    return {0: 2 * (nu1 + nu2) - 2, 1: 1, 2: 1}


def half_sweep_bytes_per_cell(form, precision):
    """Algorithmic bytes of one half-sweep launch per fine cell: half the
    cells are updated, each reading the other colour's iterate (not in form
    1), r and the flag and writing its iterate; form 2 also reads the level-1
    correction (one coarse value per 8 fine cells)."""
    sx = 4 if precision == "mixed" else 8
    b = (sx + sx + 1 + sx) / 2.0 if form != 1 else (sx + 1 + sx) / 2.0
    return b + (sx / 8.0 if form == 2 else 0.0)


def sweeps_per_launch(dim, schedule):
    """Red-black sweeps one fine smoothing launch performs: on 2D grids the
    library runs the sweeps of a smoothing run in pairs (a run of nu sweeps
    takes ceil(nu/2) launches); in 3D a launch is one colour of a sweep (the
    colour-split half-sweeps)."""
    if dim != 2:
        return 0.5
    nu1, nu2 = (schedule or {}).get("nu1", 2), (schedule or {}).get("nu2", 2)
    return (nu1 + nu2) / ((nu1 + 1) // 2 + (nu2 + 1) // 2)


def roofline(case, precision, steps, tune=True):
    """Profiled timed pass: average launch duration of each kernel class,
    measured with hipEvents on the library's stream; the class with the most
    device time is the dominant kernel.  Algorithmic bytes per launch = the
    per-sweep-per-cell figure x the sweeps x cells one launch processes."""
    _, _, kern, sched = run_gpu(case, precision, steps, 1, profile=True, tune=tune)
    spl = sweeps_per_launch(case.dim, sched)
    rows = {}
    for name, (n, ms) in kern.items():
        if n == 0:
            continue
        bpc = algorithmic_bytes_per_cell(name, precision, case.dim)
        avg_s = ms * 1e-3 / n
        rows[name] = {"launches": n, "total_ms": ms, "avg_us": avg_s * 1e6}
        if bpc is not None:
            units = spl if name == "fine_smooth" else 1.0
            bytes_launch = bpc * case.ncells * units
            if name == "fine_smooth" and case.dim == 3:
                # the launch-weighted mean of the three half-sweep forms
                mix = half_sweep_mix(sched)
                bytes_launch = case.ncells * sum(n * half_sweep_bytes_per_cell(f, precision)
                                                 for f, n in mix.items()) / sum(mix.values())
            rows[name]["algorithmic_bytes_per_launch"] = bytes_launch
            rows[name]["achieved_GBps"] = bytes_launch / avg_s / 1e9
            if name == "fine_smooth":
                rows[name]["sweeps_per_launch"] = spl
    modelled = [k for k in rows if "achieved_GBps" in rows[k]]
    dom = max(modelled, key=lambda k: rows[k]["total_ms"])
    r = rows[dom]
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        key = f"{case.name}:{precision}:{(KERNEL_NAMES_3D if case.dim == 3 else KERNEL_NAMES)[dom]}"
        ent = t.get("kernels", {}).get(key)
        if ent and t.get("source_digest") == kernel_source_digest():
            if "hbm_bytes_per_launch_by_form" in ent:
                # measured per form, weighted like the algorithmic bytes
                mix = half_sweep_mix(sched)
                by = ent["hbm_bytes_per_launch_by_form"]
                traffic = sum(n * by[str(f)] for f, n in mix.items()) / sum(mix.values())
            else:
                traffic = ent["hbm_bytes_per_launch"]
    names = KERNEL_NAMES_3D if case.dim == 3 else KERNEL_NAMES
    ro = {"bound": "hbm", "kernel": names[dom], "achieved": r["achieved_GBps"], "peak": HBM_PEAK_GBS,
          "unit": "GB/s", "frac": r["achieved_GBps"] / HBM_PEAK_GBS, "traffic": traffic,
          "traffic_source": ("stored profile value: rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of this kernel on this "
                             "workload (profiles/traffic.json), scaled by a plain copy of known size; reported only "
                             "while the kernel sources match the digest it was taken with") if traffic else None,
          "avg_launch_us": r["avg_us"], "algorithmic_bytes_per_launch": r["algorithmic_bytes_per_launch"]}
    if "sweeps_per_launch" in r:
        ro["sweeps_per_launch"] = r["sweeps_per_launch"]
    return ro, rows


def extension_bench(case, steps=40, reps=5):
    """Eq. extrapolation (ebit_extend) on the workload's geometry, each mode
    with `steps` pseudo-time steps, timed with events on the library's stream
    (the current torch stream).  Per step: the call's time less that of a
    call with no steps (the band set-up), over the steps.  Algorithmic bytes
    of one step, per changing cell: its list entry (8 B), dim weights (8 B
    each), its value and result (16 B) and up to dim upwind values (8 B
    each; counted as dim)."""
    import numpy as np
    import torch
    from paper_2402_13677_amd import ebit

    ctx, dc = ebit.context_for(case)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    rng = np.random.default_rng(11)
    q0 = torch.from_numpy(rng.uniform(-1.0, 1.0, case.ncells)).to("cuda")
    names = {ebit.EXT_LIQ_TO_VAP: "liq_to_vap", ebit.EXT_VAP_TO_LIQ: "vap_to_liq",
             ebit.EXT_IFACE_TO_BAND: "iface_to_band"}
    out = {"steps": steps}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(q, mode, t):
        ms = []
        for _ in range(reps):
            q.copy_(q0)
            ev[0].record()
            ctx.extend(q, mode, t)
            ev[1].record()
            ev[1].synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        return statistics.median(ms)

    q = q0.clone()
    for mode, name in names.items():
        ctx.extend(q, mode, 1)
        moved = int((q != q0).sum().item())
        t_full, t_set = timed(q, mode, steps), timed(q, mode, 0)
        step_s = max(t_full - t_set, 1e-9) * 1e-3 / steps
        byts = moved * (24.0 + 16.0 * case.dim)
        out[name] = {"changing_cells": moved, "call_ms": t_full, "setup_ms": t_set, "step_us": step_s * 1e6,
                     "algorithmic_bytes_per_step": byts, "achieved_GBps": byts / step_s / 1e9,
                     "frac": byts / step_s / 1e9 / HBM_PEAK_GBS}
    out["ghost_band"] = ghost_band_bench(case, ctx, reps)
    ctx.close()
    return out


def ghost_band_bench(case, ctx, reps):
    """Eq. ghost_velocity over the narrow band (ebit_ghost_band) from a
    band-extended mass flux, on the workload's geometry: median ms per call.
    Algorithmic bytes per call: the band (dim dilation passes of one byte
    read and one written per cell, then one byte read per cell), the facet
    normals of the interface cells (8 B per axis), and per ghost face its
    theta, the two cells' mass fluxes, the real value read and the ghost
    written (40 B)."""
    import numpy as np
    import torch
    from paper_2402_13677_amd import ebit

    rng = np.random.default_rng(12)
    m = torch.from_numpy(rng.uniform(0.5, 1.5, case.ncells)).to("cuda")
    ctx.extend(m, ebit.EXT_IFACE_TO_BAND, 10)
    shapes = [int(np.prod(case.u_l[a].shape)) for a in range(case.dim)]
    l0 = [torch.from_numpy(rng.normal(0.0, 1.0, k)).to("cuda") for k in shapes]
    v0 = [torch.from_numpy(rng.normal(0.0, 1.0, k)).to("cuda") for k in shapes]
    ul, uv = [x.clone() for x in l0], [x.clone() for x in v0]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    for _ in range(reps):
        for a in range(case.dim):
            ul[a].copy_(l0[a])
            uv[a].copy_(v0[a])
        ev[0].record()
        ctx.ghost_band(ul, uv, m)
        ev[1].record()
        ev[1].synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    faces = sum(int((ul[a] != l0[a]).sum().item()) + int((uv[a] != v0[a]).sum().item()) for a in range(case.dim))
    flags = torch.empty(case.ncells, dtype=torch.uint8, device="cuda")
    ctx.get_geometry(flags=flags)
    n_if = int(((flags >> 7) & 1).sum().item())
    t = statistics.median(ms) * 1e-3
    byts = case.ncells * (2.0 * case.dim + 1.0) + n_if * 8.0 * case.dim + faces * 40.0
    return {"ghost_faces": faces, "interface_cells": n_if, "call_ms": t * 1e3, "algorithmic_bytes": byts,
            "achieved_GBps": byts / t / 1e9, "frac": byts / t / 1e9 / HBM_PEAK_GBS}


def extension_cpu_baseline(case, steps=40):
    """The oracle's extension on the same geometry (1 thread): ms per call."""
    import numpy as np
    import oracle
    geo = oracle.geometry.build(case)
    q0 = np.random.default_rng(11).uniform(-1.0, 1.0, case.ncells)
    t0 = time.perf_counter()
    for mode in (0, 1, 2):
        oracle.extend.extend(case, geo, q0, mode, steps)
    el = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.project.ghost_velocities_band(case, geo, q0, case.u_l, case.u_v)
    gb = time.perf_counter() - t0
    return {"ms_per_call": el / 3 * 1e3, "ghost_band_ms": gb * 1e3, "cores": 1, "kind": "oracle",
            "sample": f"the three modes once each, {steps} steps, and the band ghost velocities once, "
                      "on the workload's geometry"}


def one_fluid_bench(case, precision, schedule, reps=10):
    """The one-fluid projection (ebit_project_one_fluid) beside the
    ghost-fluid one on the workload: median ms per call (right-hand side,
    solve to 1e-9, face update, divergence check) and outer iterations, with
    the mass flux of the input temperature."""
    import torch
    from paper_2402_13677_amd import ebit

    opts = ebit.default_opts(rtol=workload_rtol(case), precision=ebit.MIXED if precision == "mixed" else ebit.FP64,
                             **(schedule or {}))
    ctx, dc = ebit.context_for(case, opts)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    m = torch.zeros_like(dc.T0)
    ctx.mass_flux(dc.T0, m)
    out = {}
    for name in ("one_fluid", "ghost_fluid"):
        ms, its, div = [], [], []
        for r in range(reps + 1):
            p = torch.zeros_like(dc.T0)
            ul = [u.clone() for u in dc.u_l]
            if name == "one_fluid":
                st = ctx.project_one_fluid(ul, m, p)
            else:
                st = ctx.project(ul, [u.clone() for u in dc.u_v], m, p)
            if r:
                ms.append(st["seconds"] * 1e3)
                its.append(st["iters"])
                div.append(st["div_max"])
        out[name] = {"ms": statistics.median(ms), "iters": statistics.median(its), "div_max": max(div)}
    ctx.close()
    return out


def one_fluid_cpu_baseline(case):
    """The oracle's one-fluid projection (SuperLU direct solve, 1 thread)."""
    import oracle
    from oracle import onefluid
    geo = oracle.geometry.build(case)
    mdot, _ = oracle.flux.mass_flux(case, geo, case.T0)
    t0 = time.perf_counter()
    onefluid.project_one_fluid(case, geo, mdot, case.u_l, oracle.solve.direct)
    el = time.perf_counter() - t0
    return {"ms_per_call": el * 1e3, "cores": 1, "kind": "oracle",
            "sample": "one call on the workload (SciPy SuperLU direct solve)"}


def iface_velocity_bytes_per_cell(dim):
    """Algorithmic bytes of ebit_interface_velocity per cell: the own
    phase's face velocity per axis (8 B, each face shared by two cells),
    the flags (1 B), the mass flux (8 B) and the dim outputs (8 B each); the
    facet normals of the few interface cells are not counted."""
    return 8 * dim + 1 + 8 + 8 * dim


def marker_motion_bytes(ncells_x, ncells_y, markers):
    """Algorithmic bytes of one ebit_advect_markers step on an nx x ny grid:
    one read of both marker arrays (8 B per edge, the only part that grows
    with the grid: the markers have to be found), and per marker 64 B (its
    old and new coordinates, the vertex colours of its edge, the cells it
    bounds)."""
    edges = ncells_x * (ncells_y + 1) + (ncells_x + 1) * ncells_y
    return 8 * edges + 64 * markers


def marker_motion_bench(names=("bubble2d_256", "bubble2d_4096"), reps=20):
    """The interfacial velocity (ebit_interface_velocity) and one marker
    step (ebit_advect_markers) on 2D bubbles: the mass flux of the initial
    temperature carried into the band, the interfacial velocity of the
    workload's face fields, dt for a CFL number of 0.5.  Median of `reps`
    calls timed with events on the library's stream (the marker step
    includes its status read-back); the markers are restored between
    calls outside the timed region."""
    import torch
    import ebit_inputs as ei
    from paper_2402_13677_amd import ebit

    out = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for name in names:
        n = int(name.split("_")[1])
        case = ei.config(1, n=n)
        ctx, dc = ebit.context_for(case)
        ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
        N = case.ncells
        mdot = torch.zeros(N, dtype=torch.float64, device="cuda")
        ctx.mass_flux(dc.T0, mdot)
        ctx.extend(mdot, ebit.EXT_IFACE_TO_BAND, 8)
        ug = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(2)]
        ctx.interface_velocity(dc.u_l, dc.u_v, mdot, ug)
        torch.cuda.synchronize()
        umax = max(float(u.abs().max()) for u in ug)
        dt = 0.5 * case.h / umax
        mk0 = [m.clone() for m in dc.markers]
        vc0 = dc.vcol.clone()
        cc = torch.empty_like(dc.ccol)
        t_iv, t_mv = [], []
        for r in range(reps + 2):
            ev[0].record()
            ctx.interface_velocity(dc.u_l, dc.u_v, mdot, ug)
            ev[1].record()
            ev[1].synchronize()
            t_iv.append(ev[0].elapsed_time(ev[1]))
            for m, m0 in zip(dc.markers, mk0):
                m.copy_(m0)
            dc.vcol.copy_(vc0)
            torch.cuda.synchronize()
            ev[0].record()
            ctx.advect_markers(ug, dc.markers, dc.vcol, cc, dt)
            ev[1].record()
            ev[1].synchronize()
            t_mv.append(ev[0].elapsed_time(ev[1]))
        nmark = sum(int((~torch.isnan(m)).sum()) for m in dc.markers)
        frac = torch.empty(N, dtype=torch.float64, device="cuda")
        t_vf = []
        for r in range(reps + 2):
            ev[0].record()
            ctx.volume_fraction(dc.markers, dc.vcol, frac)
            ev[1].record()
            ev[1].synchronize()
            t_vf.append(ev[0].elapsed_time(ev[1]))
        vf = statistics.median(t_vf[2:])
        # per cell: its two own edges' markers (8 B each), its vertex byte,
        # the fraction written (8 B)
        b_vf = 25.0 * N
        iv = statistics.median(t_iv[2:])
        mv = statistics.median(t_mv[2:])
        b_iv = iface_velocity_bytes_per_cell(2) * N
        b_mv = marker_motion_bytes(n, n, nmark)
        out[name] = {"cells": N, "markers": nmark, "dt": dt,
                     "interface_velocity": {"us": iv * 1e3, "algorithmic_bytes": b_iv,
                                            "achieved_GBps": b_iv / (iv * 1e-3) / 1e9,
                                            "frac": b_iv / (iv * 1e-3) / 1e9 / HBM_PEAK_GBS},
                     "advect_markers": {"us": mv * 1e3, "algorithmic_bytes": b_mv,
                                        "achieved_GBps": b_mv / (mv * 1e-3) / 1e9,
                                        "frac": b_mv / (mv * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                        "launches": 10, "note": "whole call: ten launches and the status "
                                        "read-back; the scan of the marker arrays is the only grid-sized part"},
                     "volume_fraction": {"us": vf * 1e3, "algorithmic_bytes": b_vf,
                                         "achieved_GBps": b_vf / (vf * 1e-3) / 1e9,
                                         "frac": b_vf / (vf * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                         "liquid_area": float(frac.sum()) * case.h ** 2,
                                         "note": "whole call: the error-word clear, the kernel and the status "
                                         "read-back"}}
        ctx.close()
    return out


def time_loop_bench(n=256, steps=20, warmup=3, U=0.5):
    """The whole time step of Sec. 2.5 on the GPU, on the translating vapour
    disc of ebit_inputs at n^2 (periodic in x, walls in y, a uniform flow U
    along x, CFL 0.1): per-phase extension of T, the energy advection and
    the extension of T*, the interfacial velocity and the marker step, the
    build, the heat solve, the mass flux and its band extension, the band
    ghost velocities and the projection (u* = u^n: no momentum predictor).
    Median of the steps timed with events on the library's stream, the torch
    glue between the calls included."""
    import torch
    import ebit_inputs as ei
    from paper_2402_13677_amd import ebit

    dt = 0.1 / (n * U)
    case = ei.translating_bubble(n, U, dt)
    ctx, dc = ebit.context_for(case)
    N = case.ncells
    T = dc.T0.reshape(-1).clone()
    mk, vc, cc = dc.markers, dc.vcol, dc.ccol
    ul, uv = dc.u_l, dc.u_v
    mdot = torch.zeros(N, dtype=torch.float64, device="cuda")
    p = torch.zeros(N, dtype=torch.float64, device="cuda")
    ug = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(2)]
    Tstar = torch.empty_like(T)
    ext = 8
    ctx.build_coeffs(mk, vc, cc, dt)
    ctx.mass_flux(T, mdot)
    mb = mdot.clone()
    ctx.extend(mb, ebit.EXT_IFACE_TO_BAND, ext)
    ctx.ghost_band(ul, uv, mb)
    ctx.project(ul, uv, mdot, p)
    names = ("energy_advection_and_extensions", "interface_velocity_and_markers", "build", "heat_solve",
             "mass_flux_and_extension", "ghost_band", "projection")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
    ms, iters = [], []
    parts = {k: [] for k in names}
    for s in range(warmup + steps):
        ev[0].record()
        Tl = T.clone()
        ctx.extend(Tl, ebit.EXT_LIQ_TO_VAP, ext)
        Tv = T.clone()
        ctx.extend(Tv, ebit.EXT_VAP_TO_LIQ, ext)
        ctx.advect_energy(Tl, Tv, ul, uv, cc, dt, Tstar)
        Tl = Tstar.clone()
        ctx.extend(Tl, ebit.EXT_LIQ_TO_VAP, ext)
        Tv = Tstar.clone()
        ctx.extend(Tv, ebit.EXT_VAP_TO_LIQ, ext)
        ev[1].record()
        ctx.interface_velocity(ul, uv, mb, ug)
        old = cc.reshape(-1).clone()
        ctx.advect_markers(ug, mk, vc, cc, dt)
        new = cc.reshape(-1)
        Ts = torch.where(new == old, Tstar, torch.where(new == 1, Tl, Tv))
        ev[2].record()
        ctx.build_coeffs(mk, vc, cc, dt)
        ev[3].record()
        sh = ctx.heat_solve(Ts, T)
        ev[4].record()
        ctx.mass_flux(T, mdot)
        mb = mdot.clone()
        ctx.extend(mb, ebit.EXT_IFACE_TO_BAND, ext)
        ev[5].record()
        ctx.ghost_band(ul, uv, mb)
        ev[6].record()
        sp = ctx.project(ul, uv, mdot, p)
        ev[7].record()
        ev[7].synchronize()
        if s >= warmup:
            ms.append(ev[0].elapsed_time(ev[7]))
            iters.append((sh["iters"], sp["iters"]))
            for q, k in enumerate(names):
                parts[k].append(ev[q].elapsed_time(ev[q + 1]))
    nmark = sum(int((~torch.isnan(m)).sum()) for m in mk)
    ctx.close()
    t = statistics.median(ms)
    return {"workload": case.name, "cells": N, "steps": steps, "dt": dt, "ms_per_step": t,
            "cell_steps_per_s": N / (t * 1e-3), "markers_after": nmark,
            "outer_iters_heat_projection": [statistics.median([a for a, _ in iters]),
                                            statistics.median([b for _, b in iters])],
            "extension_steps": ext, "ms_by_phase": {k: statistics.median(v) for k, v in parts.items()}}


def time_loop_cpu_baseline(n=256, U=0.5):
    """The oracle's time step on the same case (1 thread, SuperLU solves):
    one step."""
    import dataclasses
    import numpy as np
    import ebit_inputs as ei
    import oracle
    from oracle import advect, energy, extend, flux, geometry, heat, project, solve
    dt = 0.1 / (n * U)
    case = ei.translating_bubble(n, U, dt)
    ext = 8
    geo = geometry.build(case)
    T = case.T0.ravel().copy()
    mdot, _ = flux.mass_flux(case, geo, T)
    mb = extend.extend(case, geo, mdot, extend.IFACE_TO_BAND, ext)
    ul, uv = project.ghost_velocities_band(case, geo, mb, case.u_l, case.u_v)
    pr = project.project(case, geo, mdot, ul, uv, solve.direct)
    ul, uv = pr["u_l"], pr["u_v"]
    t0 = time.perf_counter()
    Tl = extend.extend(case, geo, T, extend.LIQ_TO_VAP, ext)
    Tv = extend.extend(case, geo, T, extend.VAP_TO_LIQ, ext)
    T = energy.advect_energy(case, Tl, Tv, ul, uv, dt)
    Tl = extend.extend(case, geo, T, extend.LIQ_TO_VAP, ext)
    Tv = extend.extend(case, geo, T, extend.VAP_TO_LIQ, ext)
    mk, vc, cc = advect.advect(case, geo, ul, uv, mb, dt)
    old, new = case.ccol.ravel(), cc.ravel()
    Ts = np.where(new == old, T, np.where(new == 1, Tl, Tv))
    case = dataclasses.replace(case, markers=list(mk), vcol=vc, ccol=cc, T0=Ts.reshape(case.T0.shape))
    geo = geometry.build(case)
    A, b = heat.assemble(case, geo, Ts)
    T = solve.direct(A, b, heat.operator(case, geo))
    mdot, _ = flux.mass_flux(case, geo, T)
    mb = extend.extend(case, geo, mdot, extend.IFACE_TO_BAND, ext)
    ul, uv = project.ghost_velocities_band(case, geo, mb, ul, uv)
    project.project(case, geo, mdot, ul, uv, solve.direct)
    el = time.perf_counter() - t0
    return {"ms_per_step": el * 1e3, "value": case.ncells / el, "unit": "cell-steps/s", "cores": 1,
            "kind": "oracle", "sample": f"one step on {case.name} (direct solves)"}


def marker_motion_cpu_baseline():
    """The oracle's interfacial velocity and marker step on bubble2d_256
    (1 thread): ms per call."""
    import numpy as np
    import ebit_inputs as ei
    import oracle
    case = ei.config(1)
    geo = oracle.geometry.build(case)
    inb, _ = oracle.extend.band(case, geo)
    mdot = np.where(inb, 1.0, 0.0)
    t0 = time.perf_counter()
    ug = oracle.advect.cell_interface_velocity(case, geo, case.u_l, case.u_v, mdot)
    t1 = time.perf_counter()
    dt = 0.5 * case.h / np.max(np.abs(ug))
    mk, vc = case.markers, case.vcol
    for a in range(2):
        mk, vc = oracle.advect.advect_pass(case, mk, vc, ug, dt, a)
    oracle.advect.cell_colours(case, mk, vc)
    t2 = time.perf_counter()
    oracle.volume.volume_fraction(case)
    t3 = time.perf_counter()
    return {"interface_velocity_ms": (t1 - t0) * 1e3, "advect_markers_ms": (t2 - t1) * 1e3,
            "volume_fraction_ms": (t3 - t2) * 1e3, "cores": 1,
            "kind": "oracle", "sample": "one call each on bubble2d_256 (mdot = 1 in the band)"}


def energy_bytes_per_cell(dim):
    """Algorithmic bytes of one energy-advection call per cell: the colour
    byte, the cell's own-phase T and its phase's face per axis (each face
    read once), the T* write; the stencil neighbours come from the caches."""
    return 1 + 8 + 8 * dim + 8


def _energy_inputs(case, seed=41):
    """Per-phase fields carried across the interface (Eq. extrapolation, 8
    steps each way) from the workload's initial T, and smooth face
    velocities of both signs (the workloads' own fields are zero or nearly
    so): u_a = 1e-2 sin(2 pi (k . x) / L + phi_a) at the face centres, k and
    phi seeded per axis and phase; dt for a CFL number of 0.5."""
    import torch
    from paper_2402_13677_amd import ebit
    ctx, dc = ebit.context_for(case)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    Tl, Tv = dc.T0.clone(), dc.T0.clone()
    ctx.extend(Tl, ebit.EXT_LIQ_TO_VAP, 8)
    ctx.extend(Tv, ebit.EXT_VAP_TO_LIQ, 8)
    import numpy as np
    import ebit_inputs as ei
    rng = np.random.Generator(np.random.PCG64(seed))
    L = case.n[0] * case.h

    def smooth(a):
        shp = ei.face_shape(case.dim, case.n, a)             # (nz, ny, nx) order, one more along a
        ax = [torch.arange(m, dtype=torch.float64, device="cuda") for m in reversed(shp[-case.dim:])]
        xs = [(ax[b] + (0.0 if b == a else 0.5)) * case.h for b in range(case.dim)]
        k = rng.integers(1, 4, case.dim)
        arg = sum(float(k[b]) * xs[b].view([-1 if q == case.dim - 1 - b else 1 for q in range(case.dim)])
                  for b in range(case.dim))
        return (1e-2 * torch.sin(2 * math.pi * arg / L + float(rng.uniform(0, 2 * math.pi)))).reshape(-1)

    ul = [smooth(a) for a in range(case.dim)]
    uv = [smooth(a) for a in range(case.dim)]
    torch.cuda.synchronize()
    vmax = max(float(u.abs().max()) for u in ul + uv)
    return ctx, dc, Tl, Tv, ul, uv, 0.5 * case.h / vmax


def energy_bench(case, reps=20):
    """ebit_advect_energy (Eq. energy_advection) on the workload's grid:
    median of `reps` calls timed with events on the library's stream."""
    import torch
    ctx, dc, Tl, Tv, ul, uv, dt = _energy_inputs(case)
    out = torch.empty_like(Tl)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ts = []
    for _ in range(reps + 2):
        ev[0].record()
        ctx.advect_energy(Tl, Tv, ul, uv, dc.ccol, dt, out)
        ev[1].record()
        ev[1].synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    ms = statistics.median(ts[2:])
    b = energy_bytes_per_cell(case.dim) * case.ncells
    ctx.close()
    return {"cells": case.ncells, "us": ms * 1e3, "algorithmic_bytes": b, "achieved_GBps": b / (ms * 1e-3) / 1e9,
            "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "cell_updates_per_s": case.ncells / (ms * 1e-3),
            "inputs": "per-phase T extended 8 steps across the interface, smooth face velocities "
                      "1e-2 sin(2 pi k.x / L + phi) of both signs, CFL 0.5"}


def energy_cpu_baseline(case, sample_cells=1 << 20):
    """The oracle's energy advection (NumPy, one process) on a sample of
    the workload's cells with the same inputs: cells per second."""
    import numpy as np
    import oracle
    import torch
    ctx, dc, Tl, Tv, ul, uv, dt = _energy_inputs(case)
    h = lambda t: t.cpu().numpy()
    Tl, Tv, ul, uv = h(Tl), h(Tv), [h(u) for u in ul], [h(u) for u in uv]
    ctx.close()
    rng = np.random.Generator(np.random.PCG64(42))
    n = min(sample_cells, case.ncells)
    cells = rng.choice(case.ncells, n, replace=False) if n < case.ncells else None
    t0 = time.perf_counter()
    oracle.energy.advect_energy(case, Tl, Tv, ul, uv, dt, cells=cells)
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} cells of {case.name} ({el:.1f} s, NumPy)"}


def copy_calibration(nbytes=1 << 30):
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}))


def repeats(case, precision, schedule, reps=5, steps=4):
    """Time-to-rtol of each solve in `reps` separate timed runs of `steps`
    steps (fresh context each, fixed schedule): the median per run and the
    median of those medians."""
    out = {"heat": [], "projection": [], "ms_per_step": []}
    for _ in range(reps):
        el, rec, _, _ = run_gpu(case, precision, steps, 1, tune=schedule or False)
        out["heat"].append(statistics.median(rec["heat_ms"]))
        out["projection"].append(statistics.median(rec["proj_ms"]))
        out["ms_per_step"].append(el / steps * 1e3)
        its = (statistics.median(rec["heat_it"]), statistics.median(rec["proj_it"]))
    return {"time_to_rtol_ms": {k: statistics.median(out[k]) for k in ("heat", "projection")},
            "ms_per_step": statistics.median(out["ms_per_step"]),
            "spread_ms": {k: [min(out[k]), max(out[k])] for k in ("heat", "projection")},
            "outer_iters": {"heat": its[0], "projection": its[1]}, "runs": reps, "steps_per_run": steps}


def solve_roofline(case, precision, schedule, rep):
    """Whole-solve figure: the design's algorithmic bytes of every outer
    iteration (V-cycle on all levels plus the outer update) over the
    measured time-to-rtol, against the HBM peak."""
    bpc = solve_model_bytes_per_iteration(precision, case.dim, schedule)
    out = {"model_bytes_per_cell_per_iteration": bpc}
    for k in ("heat", "projection"):
        byts = bpc * case.ncells * rep["outer_iters"][k]
        gbs = byts / (rep["time_to_rtol_ms"][k] * 1e-3) / 1e9
        out[k] = {"algorithmic_GB": byts / 1e9, "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="film3d_256", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--compare", action="store_true", default=True,
                    help="also time the plain FP64 solve (reported beside the value)")
    ap.add_argument("--no-compare", dest="compare", action="store_false")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-one-thread", action="store_true", help="skip the one-thread oracle sample")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-repeats", action="store_true", help="skip the five repeated timed runs")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default solve schedule")
    ap.add_argument("--schedule", default=None,
                    help="fixed schedule nu,tail_cells,check_every (nu1 = nu2 = nu) instead of autotuning")
    ap.add_argument("--no-extension", action="store_true", help="skip the narrow-band extension timing")
    ap.add_argument("--no-one-fluid", action="store_true", help="skip the one-fluid projection timing")
    ap.add_argument("--no-energy", action="store_true", help="skip the energy-advection timing")
    ap.add_argument("--no-time-loop", action="store_true", help="skip the whole-time-step timing (2D)")
    ap.add_argument("--no-marker-motion", action="store_true",
                    help="skip the interfacial-velocity and marker-motion timing")
    ap.add_argument("--marker-motion-only", action="store_true",
                    help="run only the interfacial-velocity and marker-motion timing (2D bubbles)")
    ap.add_argument("--energy-only", action="store_true",
                    help="run only the energy-advection timing on the workload (for profiling it)")
    ap.add_argument("--extras-only", action="store_true",
                    help="time only the extras: the narrow-band extension with the band ghost velocities, the "
                         "one-fluid projection, the energy advection, the marker motion and the whole 2D time step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the path runs and is measured on a single GPU; "
                                   "sharding across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.marker_motion_only:
        print(json.dumps({"marker_motion": marker_motion_bench()}))
        return
    case = make_case(args.workload)
    if isinstance(case, list):
        return main_batch(args, case)
    if args.energy_only:
        print(json.dumps({"workload": case.name, "energy_advection": energy_bench(case, reps=5)}))
        return
    if args.extras_only:
        sched = parse_schedule(args.schedule) if args.schedule else None
        print(json.dumps({"workload": case.name, "extension": extension_bench(case),
                          "one_fluid": one_fluid_bench(case, args.precision, sched),
                          "energy_advection": energy_bench(case),
                          "marker_motion": marker_motion_bench(),
                          "time_loop": time_loop_bench()}))
        return
    rtol = workload_rtol(case)
    tune = parse_schedule(args.schedule) if args.schedule else (not args.no_autotune)
    log(f"{case.name}: {case.ncells} cells, {args.precision}, rtol {rtol:g}; timed steps")
    elapsed, rec, _, schedule = run_gpu(case, args.precision, args.steps, args.warmup, tune=tune)
    ms_per_step = elapsed / args.steps * 1e3
    med = lambda v: statistics.median(v) if v else None
    extra = {
        "time_to_rtol_ms": {"heat": med(rec["heat_ms"]), "projection": med(rec["proj_ms"])},
        "outer_iters": {"heat": med(rec["heat_it"]), "projection": med(rec["proj_it"])},
        "rel_res_max": {"heat": max(rec["heat_res"]), "projection": max(rec["proj_res"])},
        "div_max": max(rec["div"]),
        "mass_flux_fallbacks": max(rec["fallbacks"]),
    }
    extra["cell_updates_per_s"] = cell_updates(rec, schedule, ms_per_step)
    fixed = schedule or False
    if not args.no_repeats:
        log("five repeated runs per precision")
        extra["repeats"] = {args.precision: repeats(case, args.precision, fixed)}
        if args.compare:
            other = "fp64" if args.precision == "mixed" else "mixed"
            extra["repeats"][other] = repeats(case, other, fixed)
            mine, theirs = extra["repeats"][args.precision], extra["repeats"][other]
            mixed, fp64 = (mine, theirs) if args.precision == "mixed" else (theirs, mine)
            extra["mixed_over_fp64_speedup"] = {
                k: fp64["time_to_rtol_ms"][k] / mixed["time_to_rtol_ms"][k] for k in ("heat", "projection")}
            extra["mixed_over_fp64_speedup"]["step"] = fp64["ms_per_step"] / mixed["ms_per_step"]
        extra["solve_roofline"] = solve_roofline(case, args.precision, schedule, extra["repeats"][args.precision])
    log("warm-start run")
    _, recw, _, _ = run_gpu(case, args.precision, max(5, args.steps // 5), 1, tune=fixed, warm=True)
    extra["warm_start"] = {"time_to_rtol_ms": {"heat": med(recw["heat_ms"]), "projection": med(recw["proj_ms"])},
                           "outer_iters": {"heat": med(recw["heat_it"]), "projection": med(recw["proj_it"])}}
    out = {
        "metric": "time-to-1e-9 residual per solve (mixed vs FP64) + cell-updates/s, % HBM peak",
        "value": case.ncells * args.steps / elapsed,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": case.ncells, "precision": args.precision,
                   "rtol": rtol, "parallelism": "single GPU", "schedule": schedule},
        "extra": extra,
        "roofline": None,
    }
    if not args.no_roofline:
        log("profiled pass (hipEvents per kernel class)")
        out["roofline"], extra["kernels"] = roofline(case, args.precision, max(5, args.steps // 5), tune=fixed)
    if not args.no_extension:
        log("narrow-band extension")
        extra["extension"] = extension_bench(case)
        if not args.no_cpu_baseline and case.dim == 2:
            extra["extension"]["cpu_oracle"] = extension_cpu_baseline(case)
    if not args.no_one_fluid:
        log("one-fluid projection")
        extra["one_fluid"] = one_fluid_bench(case, args.precision, schedule)
        if not args.no_cpu_baseline and case.dim == 2:
            extra["one_fluid"]["cpu_oracle"] = one_fluid_cpu_baseline(case)
    if not args.no_energy:
        log("energy advection")
        extra["energy_advection"] = energy_bench(case)
        if not args.no_cpu_baseline:
            extra["energy_advection"]["cpu_oracle"] = energy_cpu_baseline(case)
    if not args.no_marker_motion:
        log("interfacial velocity and marker motion (2D bubbles)")
        extra["marker_motion"] = marker_motion_bench()
        if not args.no_cpu_baseline:
            extra["marker_motion"]["cpu_oracle"] = marker_motion_cpu_baseline()
    if not args.no_time_loop:
        log("the whole time step (2D translating bubble)")
        extra["time_loop"] = time_loop_bench()
        if not args.no_cpu_baseline:
            extra["time_loop"]["cpu_oracle"] = time_loop_cpu_baseline()
    if not args.no_cpu_baseline:
        log("first step of each precision for the error against the oracle")
        gsteps = {"mixed": gpu_first_step(case, "mixed", schedule), "fp64": gpu_first_step(case, "fp64", schedule)}
        out["cpu_baseline"], errs = cpu_baseline_leg(case, gsteps, one_thread=not args.no_one_thread)
        extra["error_vs_oracle_at_rtol"] = errs
        extra["mixed_error_vs_oracle"] = errs["mixed"]
    print(json.dumps(out))


def batch_cpu_baseline(cases, one_thread_cases=8):
    """The oracle on the batch: one full step of every case (multigrid solves
    to the discrete solution) with as many OpenMP threads as the host has
    cores, and the first `one_thread_cases` cases on one thread."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    cores = os.cpu_count() or 1
    log(f"oracle steps of the {len(cases)} cases on {cores} threads")
    tot = 0.0
    for c in cases:
        _, t = _oracle_step(c, cores)
        tot += t["step"]
    ncells = sum(c.ncells for c in cases)
    base = {"value": ncells / tot, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"one full step of each of the {len(cases)} cases ({tot:.1f} s in all: geometry, multigrid "
                      f"heat and pressure solves to the discrete solution, mass flux, projection) on {cores} "
                      f"threads of {host_cpu()}"}
    log(f"oracle steps of {one_thread_cases} cases on 1 thread")
    t1, n1 = 0.0, 0
    for c in cases[:one_thread_cases]:
        _, t = _oracle_step(c, 1)
        t1 += t["step"]
        n1 += c.ncells
    base["one_thread"] = {"value": n1 / t1, "unit": "cell-steps/s", "cores": 1,
                          "sample": f"one full step of the first {one_thread_cases} cases ({t1:.1f} s)"}
    return base


def main_batch(args, cases):
    """The 64-case uneven 2D batch (sides 64..256): batched solves, with the
    same cases one context after another beside it, in the benchmarked
    precision and in FP64.  The roofline is the design's algorithmic bytes
    of every outer iteration of every case (a V-cycle on all levels plus the
    outer update, per fine cell) over the batched solve time: the batch's
    solves are single launches over all cases, so no one kernel stands for
    them."""
    import statistics
    ncells = sum(c.ncells for c in cases)
    log(f"batch of {len(cases)} cases, {ncells} cells: batched steps")
    bs = {}
    el, its, schedule = run_gpu_batch(cases, args.precision, args.steps, args.warmup, batched=True, keep_solves=bs)
    seq_steps = max(2, args.steps // 5)
    log("the same cases one context after another")
    ss = {}
    el_seq, _, _ = run_gpu_batch(cases, args.precision, seq_steps, 1, batched=False, schedule=schedule,
                                 keep_solves=ss)
    other = "fp64" if args.precision == "mixed" else "mixed"
    s64 = {}
    el_seq64, _, _ = run_gpu_batch(cases, other, seq_steps, 1, batched=False, schedule=schedule, keep_solves=s64)
    med = statistics.median
    per_step_sum = lambda lst: med([sum(x) for x in lst])
    per_case = lambda lst: med([v for x in lst for v in x])
    extra = {
        "sequential_ms_per_step": el_seq / seq_steps * 1e3,
        "batched_speedup": (el_seq / seq_steps) / (el / args.steps),
        "max_outer_iters": {"heat": max(i[0] for i in its), "projection": max(i[1] for i in its)},
        "time_to_rtol_ms": {
            "batched": {"heat": med(bs["heat_s"]) * 1e3, "projection": med(bs["proj_s"]) * 1e3,
                        "note": "one solve call over all 64 cases"},
            f"sequential_{args.precision}": {
                "heat_all_cases": per_step_sum(ss["heat_s"]) * 1e3,
                "projection_all_cases": per_step_sum(ss["proj_s"]) * 1e3,
                "heat_median_case": per_case(ss["heat_s"]) * 1e3,
                "projection_median_case": per_case(ss["proj_s"]) * 1e3},
            f"sequential_{other}": {
                "heat_all_cases": per_step_sum(s64["heat_s"]) * 1e3,
                "projection_all_cases": per_step_sum(s64["proj_s"]) * 1e3,
                "heat_median_case": per_case(s64["heat_s"]) * 1e3,
                "projection_median_case": per_case(s64["proj_s"]) * 1e3},
        },
        f"sequential_{other}_ms_per_step": el_seq64 / seq_steps * 1e3,
    }
    bpc = solve_model_bytes_per_iteration(args.precision, 2, schedule)
    sizes = [c.ncells for c in cases]
    ro = {}
    for k, sk, ik in (("heat", "heat_s", "heat_iters"), ("projection", "proj_s", "proj_iters")):
        byts = med([sum(n * it for n, it in zip(sizes, its_)) for its_ in bs[ik]]) * bpc
        gbs = byts / med(bs[sk]) / 1e9
        ro[k] = {"algorithmic_GB": byts / 1e9, "achieved_GBps": gbs}
    dom = max(ro, key=lambda k: med(bs["heat_s" if k == "heat" else "proj_s"]))
    roofline = {"bound": "hbm", "kernel": f"batched {dom} solve (every solve kernel, design byte model)",
                "achieved": ro[dom]["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ro[dom]["achieved_GBps"] / HBM_PEAK_GBS, "traffic": None,
                "model_bytes_per_cell_per_iteration": bpc, "solves": ro}
    out = {
        "metric": "time-to-1e-9 residual per solve (mixed vs FP64) + cell-updates/s, % HBM peak",
        "value": ncells * args.steps / el,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "batch64_2d", "cases": len(cases), "cells": ncells, "precision": args.precision,
                   "rtol": DEFAULT_RTOL, "parallelism": "single GPU", "schedule": schedule},
        "extra": extra,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(cases)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
