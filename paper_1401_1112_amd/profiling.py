"""Helpers for counter runs under rocprofv3.

``python -m paper_1401_1112_amd.profiling copy --mib 1024 --reps 4`` runs a plain
device-to-device copy of a known size, whose FETCH_SIZE / WRITE_SIZE readings
calibrate the per-dispatch HBM byte counters of the solver kernels.

``python -m paper_1401_1112_amd.profiling batch --patches 512 --steps 2 --mode polled``
runs the batched workload alone (for kernel traces of the batch form);
``... collapse --mode polled --precision mixed`` likewise the collapse-like hierarchy, and
``... unique --steps 1`` the unique-time-step composite solves of the lognormal hierarchy,
and ``... levels --precision mixed --steps 2`` its adaptive coarse steps alone.

``python -m paper_1401_1112_amd.profiling summarize DIR`` prints a per-kernel
summary (count, average duration, and the averages of any counters) from the
CSV files rocprofv3 writes with ``--output-format csv``.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import sys
from collections import defaultdict


def run_copy(mib: int, reps: int) -> None:
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}", flush=True)


def run_batch(patches: int, steps: int, mode: str, per_cu: int, form_coefs: bool = False,
              precision: str = "fp64") -> None:
    """The batched workload (seeded patches, n in [8, 128]) for one warm-up step and
    `steps` timed steps, host-polled or as persistent launches (optionally in a graph),
    in FP64 or mixed precision."""
    import time

    import torch

    from synth.configs import patch_batch

    from . import _lib as L
    from .solver import BatchSolver
    prec = L.MIXED if precision == "mixed" else L.FP64
    ps, alpha = patch_batch(4000, patches)
    kw = {} if mode == "polled" else {"persistent": True, "graph": mode == "graph", "persistent_per_cu": per_cu}
    kw["form_coefs"] = form_coefs
    bs = BatchSolver(robin_alpha=alpha, **kw)
    h = bs.upload(ps)
    bs.run(h, 1, 1e-10, prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs.run(h, steps, 1e-10, prec)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = bs.stats()
    ci = sum(x["n_leaf"] * x["iters"] for x in st)
    print(f"batch {precision} {mode}{' formed' if form_coefs else ''}: {patches} patches, {steps} steps in {el:.3f} s, {ci / el:.3e} cell-iterations/s, "
          f"{st[0]['sweep_blocks']} sweep blocks, {st[0]['launch_blocks']} launch blocks", flush=True)
    bs.close()


def run_collapse(steps: int, mode: str, precision: str, form_coefs: bool = False, max_blocks: int = 0) -> None:
    """The collapse-like hierarchy (levels 6..13, ~41 M cells, coupled E-T): one warm-up
    and `steps` timed coarse steps from the same state, host-polled or one persistent
    launch per solve."""
    import time

    import torch

    from synth.configs import config_collapse

    from . import _lib as L
    from .solver import solver_from_problem
    p = config_collapse()
    prec = L.MIXED if precision == "mixed" else L.FP64
    s = solver_from_problem(p, precision=prec, persistent=(mode == "persistent"), form_coefs=form_coefs,
                            max_blocks=max_blocks)
    fields = {lv: tuple(t.clone() for t in s._fields[lv]) for lv in s.levels}

    def step():
        for lv in s.levels:
            rho, E, T = fields[lv]
            s.set_fields(lv, rho, E, T, kmode=1)
        s.advance(p.dt_coarse, L.BC_DIRICHLET, p.tol)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    st = s.stats()
    print(f"collapse {precision} {mode}{' formed' if form_coefs else ''}: {el * 1e3:.1f} ms per coarse step, {len(st)} solves, "
          f"{sum(x['iters'] for x in st)} PCG iterations, {sum(x['outer_iters'] for x in st)} refinement sweeps",
          flush=True)
    s.close()


def run_levels(steps: int, mode: str, precision: str, max_blocks: int, form_coefs: bool = False) -> None:
    """The lognormal hierarchy (levels 6..9, 4.0 M cells, 15 level solves per coarse
    step) in FP64 or mixed precision: one warm-up and `steps` timed coarse steps from
    the same state, host-polled or one persistent launch per solve."""
    import time

    import torch

    from synth.configs import config_fld_lognormal

    from . import _lib as L
    from .solver import solver_from_problem
    p = config_fld_lognormal()
    prec = L.MIXED if precision == "mixed" else L.FP64
    s = solver_from_problem(p, precision=prec, persistent=(mode == "persistent"), form_coefs=form_coefs,
                            max_blocks=max_blocks)
    fields = {lv: tuple(t.clone() for t in s._fields[lv][:2]) for lv in s.levels}

    def step():
        for lv in s.levels:
            rho, E = fields[lv]
            s.set_fields(lv, rho, E, kmode=1)
        s.advance(p.dt_coarse, L.BC_DIRICHLET, p.tol)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    st = s.stats()
    print(f"levels {precision} {mode}{' formed' if form_coefs else ''}: {el * 1e3:.2f} ms per coarse step, "
          f"{len(st)} solves, {sum(x['iters'] for x in st)} CG iterations, "
          f"{sum(x['outer_iters'] for x in st)} refinement sweeps, {st[0]['sweep_blocks']} sweep blocks",
          flush=True)
    s.close()


def run_unique(steps: int) -> None:
    """The unique-time-step comparison on the lognormal hierarchy (levels 6..9, 4.0 M
    cells): one warm-up and `steps` timed coarse steps, each 8 composite solves over all
    levels, from the same state."""
    import time

    import torch

    from synth.configs import config_fld_lognormal

    from .solver import solver_from_problem
    p = config_fld_lognormal()
    s = solver_from_problem(p)
    fields = {lv: tuple(t.clone() for t in s._fields[lv][:2]) for lv in s.levels}

    def step():
        for lv in s.levels:
            rho, E = fields[lv]
            s.set_fields(lv, rho, E, kmode=1)
        s.advance_unique(p.dt_coarse, p.tol)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    st = s.stats()
    print(f"unique: {el * 1e3:.1f} ms per coarse step, {len(st)} composite solves, "
          f"{sum(x['iters'] for x in st)} PCG iterations over {st[0]['n_leaf']} cells", flush=True)
    s.close()


def _short(name: str) -> str:
    for pre in ("amrfld::(anonymous namespace)::", "void "):
        name = name.replace(pre, "")
    return name.split("(")[0][:60]


def summarize(d: str) -> str:
    lines = []
    kt = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if kt:
        agg = defaultdict(lambda: [0, 0.0])
        for path in kt:
            with open(path) as f:
                for row in csv.DictReader(f):
                    k = _short(row.get("Kernel_Name", ""))
                    dur = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3
                    agg[k][0] += 1
                    agg[k][1] += dur
        lines.append("kernel trace (durations in us):")
        lines.append(f"{'kernel':60s} {'calls':>7s} {'total_us':>12s} {'avg_us':>10s}")
        for k, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
            lines.append(f"{k:60s} {c:7d} {t:12.1f} {t / c:10.2f}")
    cc = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if cc:
        vals = defaultdict(lambda: defaultdict(list))
        for path in cc:
            with open(path) as f:
                for row in csv.DictReader(f):
                    k = _short(row.get("Kernel_Name", ""))
                    vals[k][row["Counter_Name"]].append((int(row.get("Dispatch_Id", 0)), float(row["Counter_Value"])))
        lines.append("counters (per dispatch: sum over the dispatch's records, then averaged over dispatches):")
        for k in sorted(vals):
            for cn, recs in sorted(vals[k].items()):
                per = defaultdict(float)
                for disp, v in recs:
                    per[disp] += v
                avg = sum(per.values()) / max(len(per), 1)
                lines.append(f"{k:60s} {cn:20s} dispatches {len(per):6d} avg {avg:14.1f}")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=4)
    s = sub.add_parser("summarize")
    s.add_argument("dir")
    b = sub.add_parser("batch")
    b.add_argument("--patches", type=int, default=512)
    b.add_argument("--steps", type=int, default=2)
    b.add_argument("--mode", choices=("polled", "persistent", "graph"), default="polled")
    b.add_argument("--per-cu", type=int, default=0)
    b.add_argument("--form-coefs", action="store_true")
    b.add_argument("--precision", choices=("mixed", "fp64"), default="fp64")
    cl = sub.add_parser("collapse")
    cl.add_argument("--steps", type=int, default=1)
    cl.add_argument("--mode", choices=("polled", "persistent"), default="polled")
    cl.add_argument("--precision", choices=("mixed", "fp64"), default="mixed")
    cl.add_argument("--form-coefs", action="store_true")
    cl.add_argument("--max-blocks", type=int, default=512)
    lv = sub.add_parser("levels")
    lv.add_argument("--steps", type=int, default=2)
    lv.add_argument("--mode", choices=("polled", "persistent"), default="polled")
    lv.add_argument("--precision", choices=("mixed", "fp64"), default="fp64")
    lv.add_argument("--max-blocks", type=int, default=512)
    lv.add_argument("--form-coefs", action="store_true")
    u = sub.add_parser("unique")
    u.add_argument("--steps", type=int, default=1)
    a = ap.parse_args(argv)
    if a.cmd == "unique":
        run_unique(a.steps)
    elif a.cmd == "levels":
        run_levels(a.steps, a.mode, a.precision, a.max_blocks, a.form_coefs)
    elif a.cmd == "collapse":
        run_collapse(a.steps, a.mode, a.precision, a.form_coefs, a.max_blocks)
    elif a.cmd == "copy":
        run_copy(a.mib, a.reps)
    elif a.cmd == "batch":
        run_batch(a.patches, a.steps, a.mode, a.per_cu, a.form_coefs, a.precision)
    else:
        print(summarize(a.dir))
    return 0


if __name__ == "__main__":
    sys.exit(main())
