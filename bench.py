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
kernel (the operator sweep, pass A) from HIP events around its launches and the
CPU FP64 oracle timed on a bounded sample of the same workload.
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
# algorithmic bytes per slot (FP64): pass A reads r, p_old, diag, 3 face
# coefficients and the per-oct neighbour table (24 B per oct = 3 B per slot),
# writes p_new and q; pass B reads x, r, p, q, diag and writes x, r.
PASS_A_BYTES = 3 * 8 + 3 * 8 + 3 + 2 * 8
PASS_B_BYTES = 5 * 8 + 2 * 8
METRIC = "PCG cell-iterations/s + HBM GB/s vs peak; FP64 vs mixed+batched at 1e-10"


def _measured_traffic(kernel: str):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "fld_lognormal_L6-9_fp64_hbm_counters.txt")
    src = os.path.join(ROOT, "paper_1401_1112_amd", "csrc", "pcg.hip")
    try:
        kv = dict(line.split(": ", 1) for line in open(prof).read().splitlines()
                  if line.startswith("traffic_"))
    except OSError:
        return None
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if kv.get("traffic_kernel") != kernel or kv.get("traffic_source_sha256_prefix") != cur:
        return None
    return float(kv["traffic_kib_per_dispatch"]) * 1024.0


def _problem():
    from synth.configs import config_fld_lognormal
    return config_fld_lognormal()


def _cpu_baseline(p, budget_s=30.0):
    """Oracle on the first solves of one coarse step (finest level first), timed on the
    solve region only; BLAS limited to one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as ora
    o = ora.Oracle(p.hierarchy.base_level, p.hierarchy.octs, kmode=p.kmode, robin_alpha=p.robin_alpha,
                   abs_floor=p.abs_floor, linf_test=p.linf_test, max_iter=p.max_iter)
    for lvl in p.hierarchy.levels:
        c = o.cells(lvl)
        o.set_fields(lvl, p.rho(lvl, c), p.E(lvl, c))
    # schedule of one coarse step, finest first (levels base..max, nsub = 2)
    sched = []

    def walk(level, dt):
        if level < p.hierarchy.max_level:
            for _ in range(2):
                walk(level + 1, dt / 2)
            sched.append(("restrict", level + 1, None))
        sched.append(("solve", level, dt))

    walk(p.hierarchy.base_level, p.dt_coarse)
    done, cell_it, t_solve = [], 0, 0.0
    with threadpool_limits(limits=1):
        for kind, lvl, dt in sched:
            if kind == "restrict":
                o.restrict(lvl)
                continue
            t0 = time.perf_counter()
            st = o.solve_level(lvl, dt, ora.DIRICHLET, p.tol)
            t_solve += time.perf_counter() - t0
            cell_it += st["n_leaf"] * st["iters"]
            done.append(f"L{lvl}:{st['iters']}it")
            if t_solve >= budget_s:
                break
    return {"value": cell_it / t_solve, "unit": "cell-iterations/s", "cores": 1, "kind": "oracle",
            "sample": (f"first {len(done)} of 15 level solves of one coarse step ({', '.join(done)}), "
                       f"{cell_it:.3e} cell-iterations in {t_solve:.1f} s, numpy/scipy CSR, 1 thread"),
            "seconds": t_solve}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--time-period", type=int, default=16,
                    help="bracket the two sweeps of every N-th PCG iteration with HIP events (0: off)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--max-blocks", type=int, default=0, help="blocks per PCG sweep (0: library default)")
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
    s = solver_from_problem(p, time_sweeps=args.time_period, max_blocks=args.max_blocks)
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

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_stats = []
    for _ in range(args.steps):
        all_stats.append(one_step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    cell_it = sum(st["n_leaf"] * st["iters"] for sts in all_stats for st in sts)
    slots = {lvl: s.info(lvl)[0] for lvl in s.levels}
    a_bytes = sum(PASS_A_BYTES * slots[st["level"]] * st["n_timed"] for sts in all_stats for st in sts)
    b_bytes = sum(PASS_B_BYTES * slots[st["level"]] * st["n_timed"] for sts in all_stats for st in sts)
    a_ms = sum(st["pass_a_ms"] for sts in all_stats for st in sts)
    b_ms = sum(st["pass_b_ms"] for sts in all_stats for st in sts)
    n_a = sum(st["n_timed"] for sts in all_stats for st in sts)
    pcg_ms = sum(st["pcg_ms"] for sts in all_stats for st in sts)
    solve_ms = sum(st["ms"] for sts in all_stats for st in sts)
    per_step = all_stats[-1]
    roofline = None
    if a_ms > 0:
        achieved = a_bytes / (a_ms * 1e-3) / 1e9
        traffic = _measured_traffic("k_pass_a<double>")
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else round(traffic),
                    "traffic_note": "measured HBM bytes per pass-A dispatch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, "
                                    "copy-calibrated), profiles/fld_lognormal_L6-9_fp64_hbm_counters.txt",
                    "alg_bytes_per_launch": round(a_bytes / max(n_a, 1)),
                    "kernel": "k_pass_a (p update + 7-point operator + (p,q) partials)",
                    "bytes_per_slot": PASS_A_BYTES, "timed_launches": n_a,
                    "timing": f"HIP events around the sweeps of every {args.time_period}th PCG iteration",
                    "avg_launch_us": round(a_ms * 1e3 / max(n_a, 1), 2),
                    "pass_b_GBs": round(b_bytes / (b_ms * 1e-3) / 1e9, 1) if b_ms > 0 else None,
                    "pass_b_bytes_per_slot": PASS_B_BYTES}
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
        "device_solve_ms_per_step": solve_ms / args.steps,
        "generation_s": round(t_gen, 1),
        "roofline": roofline,
        "cpu_baseline": None,
    }
    s.close()
    if not args.no_cpu_baseline:
        cb = _cpu_baseline(p, args.cpu_budget)
        cb.pop("seconds", None)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
