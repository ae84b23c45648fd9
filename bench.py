#!/usr/bin/env python3
"""Benchmark of the level-by-level implicit FLD solve with adaptive time-stepping.

One step = one coarse step of the base level with the fine-first schedule over
the whole hierarchy (15 level solves: 8 on level 9, 4 on 8, 2 on 7, 1 on 6),
each solve = cell diffusivity, face coefficients and right-hand side, Jacobi
PCG to a 1e-10 relative residual, post-solve; restriction between levels.

Workload: flux-limited radiative diffusion on a density-refined hierarchy,
levels 6..9 (64^3 base, 4.01 M cells), log-normal density (sigma 1.5, k^-4),
Levermore-Pomraning limiter, Dirichlet level interfaces.  Every step starts
from the same initial fields (reset inside the timed region), so every step
does the same work.

Output: one JSON line (metric: PCG cell-iterations per second = sum over solves
of leaf cells x iterations / wall time), with the roofline of the dominant
kernel (the fused CG iteration sweep) from HIP events its launches record, the
same for the sweeps of the HBM-streaming workloads (the 512-patch batch and the
collapse hierarchy), and the CPU FP64 oracle timed on a bounded sample of the same
workload on one thread and on all host threads.
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

HBM_PEAK_GBS = 8000.0
# the method's own bytes per cell and CG iteration, each array element counted once
# per iteration (the two sweeps of Jacobi PCG: r, p, d, 3 face coefficients, the
# neighbour table, p and q written; x, r, p, q, d read, x and r written): FP64 125 B,
# the FP32 inner solve of the mixed form 65 B.  The rooflines are quoted against them.
ALG_BYTES_FP64 = 125
ALG_BYTES_FP32 = 65
# what the fused iteration sweep itself moves per slot: reads p, s, w, x, r, rs
# (48 B), three scaled face coefficients (24 B) and the per-oct neighbour table (24 B
# per oct = 3 B per slot); writes p, s, x, r, w (40 B)
SWEEP_BYTES = 6 * 8 + 3 * 8 + 3 + 5 * 8
# with the coefficients formed from K: K (8 B) and the face mask (1 B) instead
SWEEP_BYTES_FORMED = 6 * 8 + 8 + 1 + 3 + 5 * 8
SWEEP_BYTES_FP32 = 6 * 4 + 3 * 4 + 3 + 5 * 4
METRIC = "PCG cell-iterations/s + HBM GB/s vs peak; FP64 vs mixed+batched at 1e-10"


def kernel_source_sha() -> str:
    """Hash prefix of the sources the PCG sweep kernels are compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("pcg.hip", "common.h", "device.h"):
        h.update(open(os.path.join(ROOT, "paper_1401_1112_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _measured_traffic(kernel: str, max_blocks: int, profile: str = "fld_lognormal_L6-9_fp64_hbm_counters.txt"):
    """Fabric-side bytes per dispatch of `kernel` (L2-to-fabric reads and writes, which
    include Infinity Cache hits) from a committed rocprofv3 counter summary, or None
    when the kernel source or the launch shape differ from those the counters were
    taken with."""
    prof = os.path.join(ROOT, "profiles", profile)
    try:
        kv = dict(line.split(": ", 1) for line in open(prof).read().splitlines()
                  if line.startswith("traffic_"))
    except OSError:
        return None
    cur = kernel_source_sha()
    if kv.get("traffic_kernel") != kernel or kv.get("traffic_source_sha256_prefix") != cur:
        return None
    if kv.get("traffic_max_blocks") != str(max_blocks):
        return None
    return float(kv["traffic_kib_per_dispatch"]) * 1024.0


class _gc_paused:
    """No garbage-collector pauses inside a timed region (Python objects are made per
    step there)."""

    def __enter__(self):
        import gc
        gc.collect()
        gc.disable()

    def __exit__(self, *exc):
        import gc
        gc.enable()
        return False


def _copy_bandwidth(mib=1024, reps=5):
    """Achievable HBM bandwidth: a plain device-to-device copy of `mib` MiB (read + write
    bytes over the event-timed duration, best of `reps`)."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * mib * (1 << 20) / (best * 1e-3) / 1e9


def _problem():
    from synth.configs import config_fld_lognormal
    return config_fld_lognormal()


def _schedule(p):
    """The operations of one coarse step in the driver's order (Sect. 2.2): finer levels
    first, nsub = 2, restriction after their substeps."""
    ops = []

    def walk(level, dt):
        if level < p.hierarchy.max_level:
            for _ in range(2):
                walk(level + 1, dt / 2)
            ops.append(("restrict", level + 1, None))
        ops.append(("solve", level, dt))

    walk(p.hierarchy.base_level, p.dt_coarse)
    return ops


def _align(level, cells_a, vals_a, cells_b):
    """Values given in cell order cells_a, reordered into cell order cells_b."""
    import numpy as np
    n = np.int64(1) << level

    def key(c):
        c = np.asarray(c, dtype=np.int64)
        return (c[:, 0] * n + c[:, 1]) * n + c[:, 2]

    ka, kb = key(cells_a), key(cells_b)
    o = np.argsort(ka)
    return np.asarray(vals_a)[o[np.searchsorted(ka[o], kb)]]


def _mixed_per_solve(p, init, n_solves):
    """The mixed-precision form run solve by solve through the C ABI in the driver's
    order (level solves and restrictions), its result after each of the first
    n_solves solves: (level, cells, E)."""
    from paper_1401_1112_amd import BC_DIRICHLET, MIXED
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    s = solver_from_problem(p, precision=MIXED)
    for lvl in s.levels:
        rho, E = init[lvl]
        s.set_fields(lvl, rho, E, kmode=1)
    out = []
    for kind, lvl, dt in _schedule(p):
        if len(out) >= n_solves:
            break
        if kind == "restrict":
            s.restrict(lvl)
        else:
            s.solve_level(lvl, dt, BC_DIRICHLET, p.tol)
            out.append((lvl, s.cells(lvl), to_numpy(s.E(lvl))))
    s.close()
    return out


def _cpu_baseline(p, budget_s=30.0, threads=1, mixed=None):
    """Oracle on the first solves of one coarse step (finest level first), timed on the
    solve region only, with BLAS limited to `threads` (None: all of them).  `mixed`:
    results of the mixed-precision GPU form after the same solves, compared per solve
    (outside the timed region)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    import oracle as ora
    o = ora.Oracle(p.hierarchy.base_level, p.hierarchy.octs, kmode=p.kmode, robin_alpha=p.robin_alpha,
                   abs_floor=p.abs_floor, linf_test=p.linf_test, max_iter=p.max_iter)
    for lvl in p.hierarchy.levels:
        c = o.cells(lvl)
        o.set_fields(lvl, p.rho(lvl, c), p.E(lvl, c))
    done, cell_it, t_solve, errs = [], 0, 0.0, []
    with threadpool_limits(limits=threads):
        n_threads = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
        for kind, lvl, dt in _schedule(p):
            if kind == "restrict":
                o.restrict(lvl)
                continue
            t0 = time.perf_counter()
            st = o.solve_level(lvl, dt, ora.DIRICHLET, p.tol)
            t_solve += time.perf_counter() - t0
            cell_it += st["n_leaf"] * st["iters"]
            done.append(f"L{lvl}:{st['iters']}it")
            k = len(done) - 1
            if mixed is not None and k < len(mixed) and mixed[k][0] == lvl:
                _, cells, e = mixed[k]
                ref = _align(lvl, o.cells(lvl), o.E[lvl], cells)
                errs.append({"solve": k, "level": lvl, "max_rel": float(np.abs(e - ref).max() / np.abs(ref).max()),
                             "l2_rel": float(np.linalg.norm(e - ref) / np.linalg.norm(ref))})
            if t_solve >= budget_s:
                break
    model = ""
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    out = {"value": cell_it / t_solve, "unit": "cell-iterations/s", "cores": int(n_threads), "kind": "oracle",
           "host_cpu": f"{model} ({os.cpu_count()} logical CPUs visible)",
           "sample": (f"first {len(done)} of 15 level solves of one coarse step ({', '.join(done)}), "
                      f"{cell_it:.3e} cell-iterations in {t_solve:.1f} s, numpy/scipy CSR, BLAS on {n_threads} "
                      f"thread(s) (the CSR operator product of scipy runs on one)"),
           "seconds": t_solve}
    if errs:
        out["mixed_err_vs_fp64_oracle_per_solve"] = errs
    return out


def _patch_oracle_job(args):
    from threadpoolctl import threadpool_limits

    from oracle.patch_oracle import patch_advance
    q, p, alpha, tol = args
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, hist = patch_advance(p.rho, p.E, p.dx, p.dt, p.face_mode, p.face_ghost, p.face_flux, 1, tol, alpha=alpha)
        el = time.perf_counter() - t0
    return q, int(p.n) ** 3 * hist[0]["iters"], el


def _batch_cpu_baseline(patches, alpha, tol, n_sample=32, workers=None):
    """The patch oracle on a seeded sample of the batch's patches, one step each, the
    independent patches spread over all host threads (one process each)."""
    import multiprocessing as mp

    import numpy as np
    rng = np.random.default_rng(2024)
    sample = sorted(int(i) for i in rng.choice(len(patches), min(n_sample, len(patches)), replace=False))
    workers = workers or min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    # fresh interpreters (spawn), which never touch the GPU
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_patch_oracle_job, [(q, patches[q], alpha, tol) for q in sample])
    el = time.perf_counter() - t0
    ci = sum(r[1] for r in res)
    return {"value": ci / el, "unit": "cell-iterations/s", "cores": workers, "kind": "oracle",
            "solves_per_s": len(sample) / el,
            "sample": f"{len(sample)} seeded patches of the batch, one step each, {ci:.3e} cell-iterations in "
                      f"{el:.1f} s on {workers} processes (one thread each)"}


def _roofline(stats, bytes_per_cell, kernel, note, traffic=None, active=None):
    """Roofline of the CG iteration sweep from the start/stop events its launches
    recorded: the method's bytes per cell x the cells of each timed launch over the
    summed launch time.  active(st) -> cells of one timed launch (default: the solve's
    leaves)."""
    ms = sum(st["sweep_ms"] for st in stats)
    n = sum(st["n_timed"] for st in stats)
    if ms <= 0 or n == 0:
        return None
    byts = sum(bytes_per_cell * (active(st) if active else st["n_leaf"] * st["n_timed"]) for st in stats)
    achieved = byts / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "alg_bytes_per_cell": bytes_per_cell, "alg_bytes_per_launch": round(byts / n),
            "timed_launches": n, "avg_launch_us": round(ms * 1e3 / n, 2), "note": note}


def _rel_err(a, b):
    import numpy as np
    d = np.abs(a - b)
    return float(d.max() / max(np.abs(b).max(), 1e-300)), float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _residual_gate(stats, tol, abs_floor=1e-14):
    """True residuals ||b - A x|| against the stopping threshold in force,
    max(tol ||r0||, abs_floor ||b||).  Solves whose threshold is tol ||r0|| report the
    largest ||b - A x|| / (tol ||r0||) (the FP64 stop is on the recursive residual, so
    this may exceed 1 by the recursion's rounding drift); solves that stop on the floor
    (r0 already below 1e-4 ||b||, e.g. a patch near its steady state) report the largest
    ||b - A x|| / (abs_floor ||b||), which FP64 rounding bounds from below."""
    tol_ratio, floor_ratio, worst_rel, floor = 0.0, 0.0, 0.0, 0
    for st in stats:
        r0, bn = st["rnorm0"], st["bnorm"]
        true = st["true_rel_res"] * r0
        worst_rel = max(worst_rel, st["true_rel_res"])
        if abs_floor * bn > tol * r0:
            floor += 1
            floor_ratio = max(floor_ratio, true / (abs_floor * bn))
        elif r0 > 0:
            tol_ratio = max(tol_ratio, true / (tol * r0))
    return {"tol_bound_max_true_over_tol_r0": tol_ratio, "floor_bound_solves": int(floor),
            "floor_bound_max_true_over_floor_b": floor_ratio, "max_true_rel_res": worst_rel,
            "solves": len(stats)}


def _mixed_form(p, s64, init, ms64, args):
    """The precision form on the same workload: FP32 inner CG inside FP64 refinement to
    the same 1e-10 relative residual, host-driven and as one persistent launch per
    solve captured with the whole step in a hipGraph; error against the FP64 GPU solve
    of the same step (the error against the FP64 oracle, per solve, is in the
    cpu_baseline record)."""
    import numpy as np
    import torch
    from paper_1401_1112_amd import BC_DIRICHLET, MIXED
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy

    def timed(s, steps):
        def step():
            for lvl in s.levels:
                rho, E = init[lvl]
                s.set_fields(lvl, rho, E, kmode=1)
            s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
            return s.stats()
        step()
        torch.cuda.synchronize()
        with _gc_paused():
            t0 = time.perf_counter()
            sts = [step() for _ in range(steps)]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        return el, sts, step

    s = solver_from_problem(p, precision=MIXED, max_blocks=args.max_blocks)
    inner = {"inner_tol": 3e-3, "tuned": False}
    if not args.no_tune:
        # the inner tolerance: the split between FP32 inner iterations and FP64 refinement
        from paper_1401_1112_amd.autotune import tune_refinement

        def one():
            for lvl in s.levels:
                rho, E = init[lvl]
                s.set_fields(lvl, rho, E, kmode=1)
            s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
        best, times, cached = tune_refinement(s, one, [s.info(l)[0] for l in s.levels], "levels")
        inner = {"inner_tol": best["inner_tol"], "tuned": True, "source": cached, "candidate_ms_per_step": times}
    el, sts, _ = timed(s, args.steps)
    cell_it = sum(st["n_leaf"] * st["iters"] for x in sts for st in x)
    res_polled = {l: to_numpy(s.E(l)) for l in s.levels}
    s.close()
    ms_g, res_graph = None, None
    if not args.no_persistent:
        # the whole step as a graph of persistent solves, each one cooperative launch
        g = solver_from_problem(p, precision=MIXED, max_blocks=args.max_blocks, persistent=True, graph=True,
                                inner_tol=inner["inner_tol"])
        el_g, sts_g, _ = timed(g, args.steps)
        res_graph = {l: to_numpy(g.E(l)) for l in g.levels}
        g.close()
        ms_g = el_g * 1e3 / args.steps
    # the FP64 reference: the same step from the same state (s64 may hold another form's result)
    for lvl in s64.levels:
        rho, E = init[lvl]
        s64.set_fields(lvl, rho, E, kmode=1)
    s64.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
    worst_max, worst_l2 = 0.0, 0.0
    for lvl in s64.levels:
        a, b = res_polled[lvl], to_numpy(s64.E(lvl))
        m, l2 = _rel_err(a, b)
        worst_max, worst_l2 = max(worst_max, m), max(worst_l2, l2)
    last = sts[-1]
    ms = el * 1e3 / args.steps
    out = {"value": cell_it / el, "unit": "inner cell-iterations/s", "ms_per_step": ms,
           "speedup_vs_fp64": ms64 / ms,
           "persistent_graph_ms_per_step": ms_g,
           "persistent_graph_speedup_vs_fp64": ms64 / ms_g if ms_g else None,
           "persistent_graph_equals_host_driven_bitwise":
               all(np.array_equal(res_polled[l], res_graph[l]) for l in res_polled) if res_graph else None,
           "inner_iterations_per_step": sum(st["iters"] for st in last),
           "outer_sweeps_per_step": sum(st["outer_iters"] for st in last),
           "residual": _residual_gate([st for x in sts for st in x], p.tol),
           "err_vs_fp64_gpu": {"max_rel": worst_max, "l2_rel": worst_l2},
           "inner_tol": inner}
    return out


def _unique_form(p, s, init, ms_ats, args):
    """The comparison the paper makes: the same coarse step with the unique time step of
    the finest level, all levels coupled in one composite system per fine step (8 solves
    over all 4.0 M cells), against the adaptive level-by-level step (15 level solves)."""
    import torch
    from paper_1401_1112_amd import BC_DIRICHLET
    from paper_1401_1112_amd.solver import to_numpy

    def reset():
        for lvl in s.levels:
            rho, E = init[lvl]
            s.set_fields(lvl, rho, E, kmode=1)

    reset()
    s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
    ats = {l: to_numpy(s.E(l)) for l in s.levels}
    reset()
    s.advance_unique(p.dt_coarse, p.tol)  # warm-up (composite tables and workspace)
    steps = max(1, min(args.steps, 3))
    torch.cuda.synchronize()
    with _gc_paused():
        t0 = time.perf_counter()
        sts = []
        for _ in range(steps):
            reset()
            s.advance_unique(p.dt_coarse, p.tol)
            sts.append(s.stats())
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
    st = sts[-1]
    dtu = {l: to_numpy(s.E(l)) for l in s.levels}
    diff = max(_rel_err(dtu[l], ats[l])[1] for l in s.levels)
    ci = sum(x["n_leaf"] * x["iters"] for x in st)
    return {"ms_per_step": round(el * 1e3, 2), "composite_solves": len(st),
            "pcg_iterations": sum(x["iters"] for x in st), "cells_per_solve": st[0]["n_leaf"],
            "cell_iterations_per_s": ci / el, "residual": _residual_gate(st, p.tol),
            "adaptive_ms_per_step": round(ms_ats, 2), "adaptive_speedup": el * 1e3 / ms_ats,
            "rel_l2_unique_vs_adaptive": diff}


def _dirac_form(args):
    """The paper's linear diffusion test (Sect. 4.1) in 3D plane-parallel form: an energy
    pulse (E0 = 1e5 per unit area on a background of 1) through refined slabs, levels 5..8
    (2.79 M cells), up to t = 2e-3 (K = 1), with Dirichlet, Robin and Neumann interfaces:
    total-energy gain and L2 error against the heat kernel, and the time per coarse step.
    Two step sizes: the paper's coarse step (3.125e-5, 64 steps) and one 16x larger (4
    steps), at which the finest level's diffusion number K dt / dx^2 is ~4 as the paper
    also states."""
    import numpy as np
    import torch
    from paper_1401_1112_amd import BC_DIRICHLET, BC_NEUMANN, BC_ROBIN
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    from synth.configs import config_dirac_slab
    modes = {1.0: BC_DIRICHLET, 0.5: BC_ROBIN, 0.0: BC_NEUMANN}
    E0, K = 1e5, 1.0
    out = {}
    for tag, dt, steps in (("paper_dt", 3.125e-5, 64), ("cfl4_dt", 5e-4, 4)):
        out[tag] = {}
        for alpha, mode in modes.items():
            p = config_dirac_slab(dt_coarse=dt, n_coarse_steps=steps, robin_alpha=alpha)
            s = solver_from_problem(p)
            leaf = {}
            for l in p.hierarchy.levels:
                c = s.cells(l)
                m = np.ones(len(c), dtype=bool)
                if l + 1 in p.hierarchy.octs:
                    par = np.asarray(p.hierarchy.octs[l + 1], dtype=np.int64)
                    n = np.int64(1) << l
                    m = ~np.isin((c[:, 0].astype(np.int64) * n + c[:, 1]) * n + c[:, 2],
                                 (par[:, 0] * n + par[:, 1]) * n + par[:, 2])
                leaf[l] = (m, c)

            def total():
                return sum(float(to_numpy(s.E(l))[leaf[l][0]].sum()) / float(1 << (3 * l)) for l in leaf)

            e0 = total()
            gains, its = [], 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            el = 0.0
            for _ in range(steps):
                t1 = time.perf_counter()
                s.advance(p.dt_coarse, mode, p.tol)
                torch.cuda.synchronize()
                el += time.perf_counter() - t1
                its += sum(x["iters"] for x in s.stats())
                gains.append((total() - e0) / e0)
            T = dt * steps
            tt = T + (2.0 * p.info["pulse_half"]) ** 2 / (24.0 * K)
            e2 = n2 = 0.0
            for l, (m, c) in leaf.items():
                x = (c[m, 0] + 0.5) / (1 << l)
                a = 1.0 + E0 / np.sqrt(4.0 * np.pi * K * tt) * np.exp(-(x - 0.5) ** 2 / (4.0 * K * tt))
                e = to_numpy(s.E(l))[m]
                e2 += float(np.sum((e - a) ** 2)) / float(1 << (3 * l))
                n2 += float(np.sum((a - 1.0) ** 2)) / float(1 << (3 * l))
            s.close()
            out[tag][f"alpha_{alpha}"] = {"energy_gain_end": gains[-1], "energy_gain_max": max(gains, key=abs),
                                          "l2_error_vs_heat_kernel": float(np.sqrt(e2 / n2)),
                                          "ms_per_coarse_step": round(el * 1e3 / steps, 2), "pcg_iterations": its}
        out[tag]["workload"] = (f"levels 5..8 (2,785,280 cells), {steps} coarse steps of {dt}, "
                                f"finest K dt/dx^2 = {K * dt / 8 * 256 ** 2:.2f}, tol 1e-8")
    return out


def _equilibrium_form(args):
    """The paper's equilibrium test with a nonlinear diffusivity (Sect. 4.2): K = E^1.5,
    E held at 4 (x = 0) and 0.5 (x = 1), relaxed from a step to the stationary profile
    (E^2.5 linear in x), plane-parallel in 3D.  As in the paper's convergence study:
    uniform grids of 8..128 cells per side, and 8 coarse cells with 1..4 more levels
    refined where the profile changes by more than 10% per cell (28 cells along x at 4
    levels), adaptive (Dirichlet interfaces) and unique time step.  Per run: coarse steps
    to the steady state, L2 error against the profile (volume-weighted; and the form the
    paper prints, with dx inside the square, over the effective cell count), the boundary
    flux imbalance, and the time per coarse step."""
    import numpy as np
    import torch
    from paper_1401_1112_amd import BC_DIRICHLET
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    from synth.configs import config_equilibrium, equilibrium_profile
    a, lo, hi = 1.5, 4.0, 0.5
    exact_flux = (lo ** (a + 1) - hi ** (a + 1)) / (a + 1)

    def run(base, top, unique):
        p = config_equilibrium(base_level=base, max_level=top, a=a, E_left=lo, E_right=hi, tol=1e-8)
        s = solver_from_problem(p)
        leaf = {}
        for l in p.hierarchy.levels:
            c = s.cells(l).astype(np.int64)
            m = np.ones(len(c), dtype=bool)
            if l + 1 in p.hierarchy.octs:
                par = np.asarray(p.hierarchy.octs[l + 1], dtype=np.int64)
                n = np.int64(1) << l
                m = ~np.isin((c[:, 0] * n + c[:, 1]) * n + c[:, 2], (par[:, 0] * n + par[:, 1]) * n + par[:, 2])
            leaf[l] = (m, c[m])

        def leaves():
            return {l: to_numpy(s.E(l))[m] for l, (m, _) in leaf.items()}

        prev, steps, el, its = leaves(), 0, 0.0, 0
        while steps < 1000:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if unique:
                s.advance_unique(p.dt_coarse, p.tol)
            else:
                s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            its += sum(x["iters"] for x in s.stats())
            steps += 1
            cur = leaves()
            done = max(float(np.abs(cur[l] - prev[l]).max()) for l in cur) < 1e-10
            prev = cur
            if done:
                break
        s.close()
        e2 = lit = 0.0
        flux = [0.0, 0.0]
        n_eff = 1 << top
        for l, e in prev.items():
            c = leaf[l][1]
            dx = 1.0 / (1 << l)
            err = e - equilibrium_profile((c[:, 0] + 0.5) * dx, a, lo, hi)
            e2 += float(np.sum(err ** 2)) * dx ** 3
            lit += float(np.sum((err * dx) ** 2)) * dx ** 2  # one term per cell along x
            for k, (face, v) in enumerate(((0, lo), ((1 << l) - 1, hi))):
                on = c[:, 0] == face
                Ki, Kb = e[on] ** a, v ** a
                flux[k] += float(np.sum(4.0 * Ki * Kb / (Ki + Kb) * (v - e[on]) / dx)) * dx * dx
        return {"cells_along_x": int(sum(len(np.unique(leaf[l][1][:, 0])) for l in leaf)),
                "slots": int(sum(len(m) for m, _ in leaf.values())), "steps_to_steady": steps,
                "pcg_iterations": its, "ms_per_coarse_step": round(el * 1e3 / steps, 3),
                "l2_error": float(np.sqrt(e2)), "l2_error_paper_form": float(np.sqrt(lit / n_eff)),
                "flux_in_rel_exact": flux[0] / exact_flux - 1.0,
                "flux_imbalance_rel": (flux[0] + flux[1]) / flux[0]}

    out = {"workload": "K = E^1.5, E(0) = 4, E(1) = 0.5, rho = 1, dt 0.05, tol 1e-8, steady when no leaf "
                       "moves by 1e-10 in a coarse step"}
    out["uniform"] = {str(1 << lv): run(lv, lv, False) for lv in (3, 4, 5, 6, 7)}
    out["adaptive"] = {str(8 << k): run(3, 3 + k, False) for k in (1, 2, 3, 4)}
    out["unique"] = {str(8 << k): run(3, 3 + k, True) for k in (1, 2, 3, 4)}
    return out


def _batched_form(args):
    """The batching form: independent patches with log-uniform sizes 8^3..128^3, own
    log-normal density, mixed Dirichlet / Neumann / Robin faces, 16 backward-Euler steps,
    all patches in shared sweeps; against a loop of one-patch launches."""
    import numpy as np
    import torch
    from paper_1401_1112_amd import MIXED
    from paper_1401_1112_amd.solver import BatchSolver
    from synth.configs import patch_batch
    t_gen = time.perf_counter()
    patches, alpha = patch_batch(4000, args.batch_patches)
    t_gen = time.perf_counter() - t_gen
    steps, tol = args.batch_steps, 1e-10
    cells = sum(int(p.n) ** 3 for p in patches)
    out = {"workload": f"{len(patches)} patches, n in [{min(p.n for p in patches)}, {max(p.n for p in patches)}], "
                       f"{cells} cells, {steps} steps, tol 1e-10", "generation_s": round(t_gen, 1)}

    def timed(solver, h, precision):
        solver.run(h, 1, tol, precision)  # warm-up (layout, allocations)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.run(h, steps, tol, precision)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = solver.stats()
        ci = sum(x["n_leaf"] * x["iters"] for x in st)
        return el, ci, st

    from paper_1401_1112_amd import AmrfldError
    # the host-polled FP64 run also times every form_time_period-th iteration sweep (roofline)
    forms = [("fp64_polled", {"time_sweeps": args.form_time_period}, 0),
             ("fp64_persistent_graph", {"persistent": True, "graph": True}, 0),
             ("mixed_polled", {}, MIXED),
             ("mixed_persistent_graph", {"persistent": True, "graph": True}, MIXED)]
    if not args.no_tune:
        # launch shape of the FP64 batch: host-polled, or a persistent launch with its
        # resident blocks per compute unit, each timed on one step
        from paper_1401_1112_amd.autotune import tune_batch
        print("bench: tuning the batch launch shape", file=sys.stderr, flush=True)
        bs = BatchSolver(robin_alpha=alpha, graph=True)
        h = bs.upload(patches)
        best, times, cached = tune_batch(bs, lambda: bs.run(h, 1, tol), [p.n for p in patches], 0)
        bs.close()
        del h
        torch.cuda.empty_cache()
        out["tuned_shape"] = {"best": best, "source": cached, "candidate_ms_per_step": times}
        forms.append(("fp64_tuned", {"persistent": bool(best["persistent"]), "graph": True,
                                     "persistent_per_cu": best["persistent_per_cu"],
                                     "form_coefs": bool(best.get("form_coefs", 0))}, 0))
        # the mixed form's inner tolerance, host-polled sweeps
        from paper_1401_1112_amd.autotune import tune_refinement
        print("bench: tuning the batch inner tolerance", file=sys.stderr, flush=True)
        bs = BatchSolver(robin_alpha=alpha, form_coefs=bool(best.get("form_coefs", 0)))
        h = bs.upload(patches)
        best_in, times_in, cached_in = tune_refinement(bs, lambda: bs.run(h, 1, tol, MIXED),
                                                       [p.n for p in patches], "batch")
        bs.close()
        del h
        torch.cuda.empty_cache()
        out["tuned_inner_tol"] = {"best": best_in, "source": cached_in, "candidate_ms_per_step": times_in}
        # launch shape of the mixed batch at that inner tolerance
        print("bench: tuning the mixed batch launch shape", file=sys.stderr, flush=True)
        bs = BatchSolver(robin_alpha=alpha, graph=True, inner_tol=best_in["inner_tol"])
        h = bs.upload(patches)
        best_m, times_m, cached_m = tune_batch(bs, lambda: bs.run(h, 1, tol, MIXED), [p.n for p in patches], 1)
        bs.close()
        del h
        torch.cuda.empty_cache()
        out["tuned_shape_mixed"] = {"best": best_m, "source": cached_m, "candidate_ms_per_step": times_m}
        forms.append(("mixed_tuned", {"persistent": bool(best_m["persistent"]), "graph": True,
                                      "persistent_per_cu": best_m["persistent_per_cu"],
                                      "form_coefs": bool(best_m.get("form_coefs", 0)),
                                      "inner_tol": best_in["inner_tol"]}, MIXED))
    results = {}
    for name, kw, prec in forms:
        print(f"bench: batched form {name}", file=sys.stderr, flush=True)
        bs = BatchSolver(robin_alpha=alpha, **kw)
        h = bs.upload(patches)
        try:
            el, ci, st = timed(bs, h, prec)
        except AmrfldError as e:
            # report the failing patches instead of dropping the whole line
            st = bs.stats()
            bad = [(q, x["status"], x["iters"], x["rel_res"]) for q, x in enumerate(st) if x["status"] != 0]
            out[name] = {"error": str(e), "n_bad": len(bad), "first_bad": bad[:8]}
            bs.close()
            del h
            torch.cuda.empty_cache()
            continue
        results[name] = (bs.result(h), st)
        out[name] = {"seconds": round(el, 3), "solves_per_s": len(patches) * steps / el,
                     "cell_iterations_per_s": ci / el,
                     "residual": _residual_gate(st, tol),
                     "launch_mode": max(x.get("launch_mode", 0) for x in st)}
        bs.close()
        del h
        torch.cuda.empty_cache()
    if len(results) < len(forms):
        return out
    # baseline: one patch per launch sequence (each patch its own context, warmed up)
    singles = []
    for p in patches:
        bs = BatchSolver(robin_alpha=alpha)
        h = bs.upload([p])
        bs.run(h, 1, tol)
        singles.append((bs, h))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for bs, h in singles:
        bs.run(h, steps, tol)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    single_res = [bs.result(h)[0] for bs, h in singles]
    for bs, _ in singles:
        bs.close()
    out["fp64_single_patch_loop"] = {"seconds": round(el, 3), "solves_per_s": len(patches) * steps / el}
    out["batched_speedup_vs_single_loop"] = {k: el / out[k]["seconds"] for k, _, prec in forms if prec == 0}
    a = results["fp64_polled"][0]
    b = results["fp64_persistent_graph"][0]
    m = results["mixed_polled"][0]
    mg = results["mixed_persistent_graph"][0]
    out["persistent_equals_polled_bitwise"] = all(np.array_equal(x, y) for x, y in zip(a, b))
    out["mixed_persistent_equals_polled_bitwise"] = all(np.array_equal(x, y) for x, y in zip(m, mg))
    out["mixed_persistent_graph_speedup_vs_fp64_polled"] = out["fp64_polled"]["seconds"] / \
        out["mixed_persistent_graph"]["seconds"]
    out["max_rel_l2_batch_vs_single"] = max(_rel_err(x, y)[1] for x, y in zip(a, single_res))
    out["mixed_err_vs_fp64_gpu"] = {"max_rel": max(_rel_err(x, y)[0] for x, y in zip(m, a)),
                                    "l2_rel": max(_rel_err(x, y)[1] for x, y in zip(m, a))}
    if "mixed_tuned" in results:
        mt = results["mixed_tuned"][0]
        out["mixed_tuned_err_vs_fp64_gpu"] = {"max_rel": max(_rel_err(x, y)[0] for x, y in zip(mt, a)),
                                              "l2_rel": max(_rel_err(x, y)[1] for x, y in zip(mt, a))}
    # roofline of the FP64 iteration sweep on this HBM-streaming workload: the timed
    # sweeps of each step (every form_time_period-th iteration) move the method's bytes of the
    # cells of the patches still iterating
    st = results["fp64_polled"][1]
    n = len(patches)
    sizes3 = [int(p.n) ** 3 for p in patches]
    ms = byts = 0.0
    launches = 0
    for k in range(steps):
        its = [st[k * n + q]["iters"] for q in range(n)]
        rec = st[k * n]
        if rec["n_timed"] == 0:
            continue
        ms += rec["sweep_ms"]
        for j in range(1, rec["n_timed"] + 1):
            it = j * args.form_time_period
            byts += ALG_BYTES_FP64 * sum(c for c, i in zip(sizes3, its) if i >= it)
            launches += 1
    if ms > 0:
        ach = byts / (ms * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(ach / HBM_PEAK_GBS, 4),
                           "traffic": _measured_traffic("k_cg_sweep<double>", 0,
                                                        "patch_batch_512_fp64_polled_hbm_counters.txt"),
                           "kernel": "k_cg_sweep<double> (fused CG iteration sweep), host-polled FP64 batch",
                           "alg_bytes_per_cell": ALG_BYTES_FP64, "alg_bytes_per_launch": round(byts / launches),
                           "timed_launches": launches, "avg_launch_us": round(ms * 1e3 / launches, 2),
                           "note": "cells of the patches still iterating in each timed sweep; the 17 GB batch "
                                   "streams from HBM"}
    if not args.no_cpu_baseline:
        print("bench: batch oracle on the host cores", file=sys.stderr, flush=True)
        out["cpu_baseline"] = _batch_cpu_baseline(patches, alpha, tol)
    return out


def _collapse_form(args):
    """Collapse-like hierarchy: levels 6..13 Jeans-refined around a softened singular
    isothermal sphere (contrast 1e6), radiation coupled to the gas energy, levels 6..9
    sharing the coarse dt and 10..13 subcycling (34 solves per coarse step, 16 on level 13).
    Mixed precision (FP32 inner CG, FP64 refinement to 1e-10) with the whole refinement
    loop of each solve in one persistent launch (and the coarse step captured in a
    hipGraph), against mixed and FP64 host-driven sweeps; every variant advances one
    coarse step from the same state.  The host-driven runs also time their iteration
    sweeps (rooflines on this HBM-streaming workload)."""
    import torch
    from paper_1401_1112_amd import BC_DIRICHLET, FP64, MIXED
    from paper_1401_1112_amd.solver import HierarchySolver, solver_from_problem
    from synth.configs import config_collapse
    t_gen = time.perf_counter()
    p = config_collapse()
    first = solver_from_problem(p, precision=MIXED, persistent=True, max_blocks=args.max_blocks)
    t_gen = time.perf_counter() - t_gen
    fields = {l: tuple(t.clone() for t in first._fields[l]) for l in first.levels}
    slots = {l: first.info(l)[0] for l in first.levels}
    out = {"workload": f"collapse levels 6..13: {sum(slots.values())} cells "
                       f"({', '.join(f'L{l} {slots[l]}' for l in first.levels)}), Jeans J = 0.14, "
                       "coupled E-T, nsub 1 on levels 7..9 and 2 on 10..13, Dirichlet interfaces, tol 1e-10",
           "generation_s": round(t_gen, 1)}

    def reset(s):
        for l in s.levels:
            rho, E, T = fields[l]
            s.set_fields(l, rho, E, T, kmode=1)

    tuned = None
    if not args.no_tune:
        from paper_1401_1112_amd.autotune import tune_level_shapes

        def tune_step():
            reset(first)
            first.advance(p.dt_coarse, BC_DIRICHLET, p.tol)

        print("bench: tuning the collapse launch shape", file=sys.stderr, flush=True)
        best, times, cached = tune_level_shapes(first, tune_step, list(slots.values()), MIXED)
        out["tuned_shape_mixed"] = {"best": best, "source": cached, "candidate_ms_per_step": times}
        tuned = best
        first.set_launch(args.max_blocks, True, 0)

    results, stats = {}, {}
    shapes = [("mixed_persistent", MIXED, {"persistent": True}),
              ("mixed_persistent_graph", MIXED, {"persistent": True, "graph": True}),
              ("mixed_polled", MIXED, {"time_sweeps": args.form_time_period}),
              ("fp64_polled", FP64, {"time_sweeps": args.form_time_period})]
    if tuned is not None:
        shapes.append(("mixed_tuned", MIXED, tuned))
    for name, prec, pers in shapes:
        print(f"bench: collapse form {name}", file=sys.stderr, flush=True)
        if first is not None:
            s, first = first, None
        elif name == "mixed_tuned":  # the tuned shape and inner tolerance
            s = HierarchySolver(p.hierarchy.base_level, p.hierarchy.octs, precision=prec, nsub=p.nsub)
            s.set_launch(pers["max_blocks"], bool(pers["persistent"]), pers["persistent_per_cu"],
                         bool(pers.get("form_coefs", 0)))
            from paper_1401_1112_amd.autotune import tune_refinement

            def tune_step():
                reset(s)
                s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)

            best_in, times_in, cached_in = tune_refinement(s, tune_step, list(slots.values()), "collapse")
            out["tuned_inner_tol"] = {"best": best_in, "source": cached_in, "candidate_ms_per_step": times_in}
        else:
            s = HierarchySolver(p.hierarchy.base_level, p.hierarchy.octs, precision=prec, nsub=p.nsub,
                                max_blocks=args.max_blocks, **pers)
        reset(s)
        s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)  # warm-up
        reset(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = s.stats()
        stats[name] = st
        ci = sum(x["n_leaf"] * x["iters"] for x in st)
        results[name] = {l: s.E(l, with_T=True) for l in s.levels}
        out[name] = {"ms_per_step": round(el * 1e3, 1), "solves": len(st),
                     "pcg_iterations": sum(x["iters"] for x in st),
                     "outer_sweeps": sum(x["outer_iters"] for x in st),
                     "cell_iterations_per_s": ci / el,
                     "launch_modes": sorted({x["launch_mode"] for x in st}),
                     "residual": _residual_gate(st, p.tol), "min_E": min(x["min_E"] for x in st)}
        s.close()
    if not args.no_unique:
        # the same coarse step with the unique time step of level 13 (16 composite solves)
        print("bench: collapse form unique_fp64", file=sys.stderr, flush=True)
        u = HierarchySolver(p.hierarchy.base_level, p.hierarchy.octs, precision=FP64, nsub=p.nsub,
                            max_blocks=args.max_blocks)
        reset(u)
        u.advance_unique(p.dt_coarse, p.tol)
        reset(u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u.advance_unique(p.dt_coarse, p.tol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = u.stats()
        ref64 = results["fp64_polled"]
        out["unique_fp64"] = {
            "ms_per_step": round(el * 1e3, 1), "composite_solves": len(st),
            "pcg_iterations": sum(x["iters"] for x in st), "residual": _residual_gate(st, p.tol),
            "cell_iterations_per_s": sum(x["n_leaf"] * x["iters"] for x in st) / el,
            "adaptive_fp64_speedup": el * 1e3 / out["fp64_polled"]["ms_per_step"],
            "rel_l2_vs_adaptive_fp64": max(float(torch.linalg.vector_norm(u.E(l) - ref64[l][0])
                                                 / torch.linalg.vector_norm(ref64[l][0])) for l in u.levels)}
        u.close()
    ref = results["fp64_polled"]
    for name in [n for n in ("mixed_persistent", "mixed_polled", "mixed_tuned") if n in results]:
        worst_e = max(float(torch.linalg.vector_norm(results[name][l][0] - ref[l][0])
                            / torch.linalg.vector_norm(ref[l][0])) for l in ref)
        worst_t = max(float(torch.linalg.vector_norm(results[name][l][1] - ref[l][1])
                            / torch.linalg.vector_norm(ref[l][1])) for l in ref)
        out[name]["rel_l2_vs_fp64_gpu"] = {"E": worst_e, "T": worst_t}
    out["mixed_persistent_equals_polled_bitwise"] = all(
        bool(torch.equal(results[k][l][0], results["mixed_polled"][l][0]))
        for k in ("mixed_persistent", "mixed_persistent_graph") for l in ref)
    out["mixed_speedup_vs_fp64"] = {k: out["fp64_polled"]["ms_per_step"] / out[k]["ms_per_step"]
                                    for k in ("mixed_persistent", "mixed_persistent_graph", "mixed_polled",
                                              "mixed_tuned") if k in out}
    # rooflines of the iteration sweeps on this HBM-streaming workload (levels of 2-6.5 M
    # cells, coupled E-T): FP64 and the FP32 inner sweep of the mixed form
    out["roofline"] = {
        "fp64_sweep": _roofline(stats["fp64_polled"], ALG_BYTES_FP64, "k_cg_sweep<double>, host-driven FP64",
                                "leaves of the level of each timed sweep",
                                traffic=_measured_traffic("k_cg_sweep<double>", args.max_blocks,
                                                          "collapse_L6-13_fp64_polled_hbm_counters.txt")),
        "fp32_inner_sweep": _roofline(stats["mixed_polled"], ALG_BYTES_FP32, "k_cg_sweep<float>, inner solves of "
                                      "the host-driven mixed form", "leaves of the level of each timed sweep",
                                      traffic=_measured_traffic("k_cg_sweep<float>", args.max_blocks,
                                                                "collapse_L6-13_mixed_polled_hbm_counters.txt"))}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--time-period", type=int, default=32,
                    help="bracket the sweep of every N-th CG iteration of the headline step with HIP events "
                         "(0: off; the per-sweep event handling is host work inside the timed region)")
    ap.add_argument("--form-time-period", type=int, default=16,
                    help="the same for the batch and collapse forms, whose solves are shorter")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--max-blocks", type=int, default=0, help="blocks per PCG sweep (0: library default)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision form")
    ap.add_argument("--no-unique", action="store_true", help="skip the unique-time-step comparison")
    ap.add_argument("--no-dirac", action="store_true", help="skip the pulse-diffusion test of the paper")
    ap.add_argument("--no-equilibrium", action="store_true",
                    help="skip the nonlinear equilibrium test of the paper")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched form")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the persistent (cooperative) launches of the mixed level form (profiling runs)")
    ap.add_argument("--batch-patches", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=16)
    ap.add_argument("--no-collapse", action="store_true",
                    help="skip the collapse-like form (levels 6..13, ~41 M cells; ~1 min of setup)")
    ap.add_argument("--form-coefs", action="store_true",
                    help="level solves form the face coefficients from K in every sweep instead of reading them")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape autotuner (level solves: --max-blocks or the default)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the level solve shards by Morton range across GPUs only in design)", file=sys.stderr)
        return 2

    import torch

    from paper_1401_1112_amd import BC_DIRICHLET
    from paper_1401_1112_amd.solver import solver_from_problem

    t_gen = time.perf_counter()
    p = _problem()
    t_gen = time.perf_counter() - t_gen
    s = solver_from_problem(p, time_sweeps=args.time_period, max_blocks=args.max_blocks,
                            form_coefs=args.form_coefs)
    init = {lvl: (s._fields[lvl][0].clone(), s._fields[lvl][1].clone()) for lvl in s.levels}
    kmode = 1

    def reset():
        for lvl in s.levels:
            rho, E = init[lvl]
            s.set_fields(lvl, rho, E, kmode=kmode)

    def one_step():
        reset()
        s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
        return s.stats()

    launch = {"max_blocks": args.max_blocks, "tuned": False}
    if not args.no_tune and args.max_blocks == 0:
        from paper_1401_1112_amd.autotune import tune_levels
        best, times, cached = tune_levels(s, one_step, [s.info(l)[0] for l in s.levels], 0)
        args.max_blocks = best["max_blocks"]
        args.form_coefs = bool(best.get("form_coefs", 0))
        launch = {"max_blocks": args.max_blocks, "form_coefs": int(args.form_coefs), "tuned": True,
                  "source": cached, "candidate_ms_per_step": times}
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    with _gc_paused():
        t0 = time.perf_counter()
        all_stats, marks = [], []
        for _ in range(args.steps):
            all_stats.append(one_step())  # returns after the step's last solve has finished
            marks.append(time.perf_counter())
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    step_ms = sorted((b - a) * 1e3 for a, b in zip([t0] + marks[:-1], marks))

    cell_it = sum(st["n_leaf"] * st["iters"] for sts in all_stats for st in sts)
    slots = {lvl: s.info(lvl)[0] for lvl in s.levels}
    pcg_ms = sum(st["pcg_ms"] for sts in all_stats for st in sts)
    solve_ms = sum(st["ms"] for sts in all_stats for st in sts)
    per_step = all_stats[-1]
    flat = [st for sts in all_stats for st in sts]
    roofline = _roofline(flat, ALG_BYTES_FP64, "k_cg_sweep<double> (fused CG iteration: p, s, x, r updates and "
                         "the 7-point operator on the new r, two dot products)",
                         "the levels (about 150 MB each) sit in the 256 MB Infinity Cache: cache-assisted, the "
                         "HBM gate is judged on the batch and collapse workloads (roofline_gate)")
    if roofline is not None:
        n_a = roofline["timed_launches"]
        a_ms = sum(st["sweep_ms"] for st in flat)
        moved = sum((SWEEP_BYTES_FORMED if args.form_coefs else SWEEP_BYTES) * slots[st["level"]] * st["n_timed"]
                    for st in flat)
        traffic = _measured_traffic("k_cg_sweep<double>", args.max_blocks if args.max_blocks > 0 else 1024)
        roofline.update({
            "traffic": None if (traffic is None or args.form_coefs) else round(traffic),
            "traffic_note": "fabric-side bytes per sweep dispatch from rocprofv3 (FETCH_SIZE x fetch scale + "
                            "WRITE_SIZE, both scales from a device copy of known size): reads that hit the "
                            "Infinity Cache count too; profiles/fld_lognormal_L6-9_fp64_hbm_counters.txt",
            "coefficients": "formed from K in the sweep (bitwise the stored ones)" if args.form_coefs
                            else "stored (3 scaled coefficients per slot)",
            "bytes_per_slot_moved": SWEEP_BYTES_FORMED if args.form_coefs else SWEEP_BYTES,
            "moved_GBs": round(moved / (a_ms * 1e-3) / 1e9, 1),
            "timing": f"HIP start/stop events recorded by the launches themselves (hipExtLaunchKernelGGL) of "
                      f"the sweep of every {args.time_period}th CG iteration",
            "copy_GBs_achievable": round(_copy_bandwidth(), 1)})
    out = {
        "metric": METRIC,
        "value": cell_it / elapsed,
        "unit": "cell-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "fld_lognormal levels 6..9: 64^3 base, 4,012,144 cells "
                        f"({', '.join(f'L{l} {slots[l]}' for l in s.levels)} slots), LP limiter, "
                        "Dirichlet interfaces, tol 1e-10, one coarse step = 15 level solves",
            "precision": "fp64",
            "solves_per_step": len(per_step),
            "pcg_iterations_per_step": sum(st["iters"] for st in per_step),
            "cell_iterations_per_step": sum(st["n_leaf"] * st["iters"] for st in per_step),
        },
        "pcg_only_cell_it_per_s": cell_it / (pcg_ms * 1e-3) if pcg_ms > 0 else None,
        "residual": _residual_gate([st for sts in all_stats for st in sts], p.tol),
        "device_solve_ms_per_step": solve_ms / args.steps,
        "step_ms": {"min": round(step_ms[0], 2), "median": round(step_ms[len(step_ms) // 2], 2),
                    "max": round(step_ms[-1], 2)},
        "generation_s": round(t_gen, 1),
        "launch": launch,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    out["forms"] = {}
    if not args.no_unique:
        out["forms"]["unique_time_step"] = _unique_form(p, s, init, elapsed * 1e3 / args.steps, args)
    mixed_solves = None
    if not args.no_mixed:
        out["forms"]["mixed"] = _mixed_form(p, s, init, elapsed * 1e3 / args.steps, args)
        if not args.no_cpu_baseline:
            # the mixed form solve by solve, for its per-solve error against the oracle
            mixed_solves = _mixed_per_solve(p, init, 15)
    s.close()
    if not args.no_batch:
        import torch as _t
        _t.cuda.empty_cache()
        out["forms"]["batched"] = _batched_form(args)
    if not args.no_dirac:
        out["forms"]["dirac_pulse"] = _dirac_form(args)
    if not args.no_equilibrium:
        out["forms"]["equilibrium"] = _equilibrium_form(args)
    if not args.no_collapse:
        import torch as _t
        _t.cuda.empty_cache()
        out["forms"]["collapse"] = _collapse_form(args)
    # the rooflines of the HBM-streaming workloads, on which the bandwidth gate is judged
    gate = {}
    if isinstance(out["forms"].get("batched", {}).get("roofline"), dict):
        gate["patch_batch_fp64_sweep"] = out["forms"]["batched"]["roofline"]
    for k, v in (out["forms"].get("collapse", {}).get("roofline") or {}).items():
        if v is not None:
            gate["collapse_" + k] = v
    out["roofline_gate"] = gate or None
    if not args.no_cpu_baseline:
        # the oracle on all host threads (BLAS) and on one, each on a bounded sample
        print("bench: oracle on the host cores", file=sys.stderr, flush=True)
        one = _cpu_baseline(p, args.cpu_budget / 2, threads=1, mixed=mixed_solves)
        allc = _cpu_baseline(p, args.cpu_budget / 2, threads=None)
        errs = one.pop("mixed_err_vs_fp64_oracle_per_solve", None)
        if errs and "mixed" in out["forms"]:
            out["forms"]["mixed"]["err_vs_fp64_oracle"] = {
                "per_solve": errs, "max_rel": max(e["max_rel"] for e in errs),
                "l2_rel": max(e["l2_rel"] for e in errs),
                "note": "the mixed form run solve by solve in the driver's order (amrfld_solve_level, "
                        "amrfld_restrict_level) against the FP64 oracle after the same solves"}
        one.pop("seconds", None)
        allc.pop("seconds", None)
        allc["one_core"] = one
        out["cpu_baseline"] = allc
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
