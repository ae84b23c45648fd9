"""Launch-shape autotuning of the PCG sweeps.

Candidate shapes are timed on the device (events on the solver's stream, median of a
few runs after a warm-up run) and the fastest is kept in a JSON cache keyed by the
device and a signature of the workload; a later call with the same key applies the
cached choice without timing.  A shape only changes how the sweeps are dealt to the
GPU (blocks per sweep, i.e. 256-slot tiles per block; host-polled sweeps or one
persistent launch and its resident blocks per compute unit) and whether the sweeps
read stored face coefficients or form them from K (fewer bytes, more arithmetic:
faster where the levels stream from HBM, slower where they sit in the Infinity
Cache): results of one shape are bitwise reproducible, and between shapes they differ
at most in the last bits, since the block partials are summed in other groupings.

The cache lives at ``$AMRFLD_TUNE_CACHE`` or ``~/.cache/amrfld/tune.json``.  Below it
sits a table shipped with the package (``tuned_gfx950.json``): shapes measured on MI355X
for the benchmark workloads, keyed by workload and applied on devices of that
architecture, so that those workloads run a fixed, profiled shape; a workload in
neither is timed (``AMRFLD_TUNE_SHIPPED=0`` skips the table).
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
import tempfile

import torch

LEVEL_BLOCKS = (256, 512, 1024, 2048, 4096)
LEVEL_CANDIDATES = tuple({"max_blocks": b, "form_coefs": f} for b in LEVEL_BLOCKS for f in (0, 1))
LEVEL_SHAPES = (
    {"max_blocks": 512, "persistent": 0, "persistent_per_cu": 0, "form_coefs": 0},
    {"max_blocks": 1024, "persistent": 0, "persistent_per_cu": 0, "form_coefs": 0},
    {"max_blocks": 2048, "persistent": 0, "persistent_per_cu": 0, "form_coefs": 0},
    {"max_blocks": 512, "persistent": 0, "persistent_per_cu": 0, "form_coefs": 1},
    {"max_blocks": 1024, "persistent": 0, "persistent_per_cu": 0, "form_coefs": 1},
    {"max_blocks": 1024, "persistent": 1, "persistent_per_cu": 0, "form_coefs": 0},
    {"max_blocks": 1024, "persistent": 1, "persistent_per_cu": 1, "form_coefs": 0},
)
INNER_TOLS = (3e-2, 1e-2, 3e-3, 1e-3)
BATCH_SHAPES = (
    {"persistent": 0, "persistent_per_cu": 0, "form_coefs": 0},
    {"persistent": 0, "persistent_per_cu": 0, "form_coefs": 1},
    {"persistent": 1, "persistent_per_cu": 0, "form_coefs": 0},
    {"persistent": 1, "persistent_per_cu": 0, "form_coefs": 1},
    {"persistent": 1, "persistent_per_cu": 2, "form_coefs": 0},
    {"persistent": 1, "persistent_per_cu": 1, "form_coefs": 0},
)


def cache_path() -> str:
    return os.environ.get("AMRFLD_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "amrfld",
                                                               "tune.json")


def device_key() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def workload_key(kind: str, sizes, precision: int) -> str:
    h = hashlib.sha1(json.dumps([int(x) for x in sizes]).encode()).hexdigest()[:16]
    return f"{kind}|{len(sizes)}|{h}|prec{int(precision)}"


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


def _shipped(key: str, arch: str = None):
    """Entry of the shipped table for a workload key, if it applies to this device
    (``AMRFLD_TUNE_SHIPPED=0`` ignores the table, so that its workloads are timed)."""
    if os.environ.get("AMRFLD_TUNE_SHIPPED") == "0":
        return None
    try:
        with open(SHIPPED) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if arch is None:
        arch = getattr(torch.cuda.get_device_properties(torch.cuda.current_device()), "gcnArchName", "")
    if not arch.startswith(d.get("arch", "?")):
        return None
    return d.get("entries", {}).get(key)


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    """Write the cache atomically; an unwritable location only loses the cache."""
    path = cache_path()
    tmp = None
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path), suffix=".tmp")
        with os.fdopen(fd, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        if tmp is not None and os.path.exists(tmp):
            try:
                os.unlink(tmp)
            except OSError:
                pass


def time_candidates(candidates, apply, run, repeats=3, stream=None):
    """Device time (ms, median of `repeats`) of run() under each candidate shape."""
    stream = stream or torch.cuda.current_stream()
    out = {}
    for c in candidates:
        apply(c)
        run()  # warm-up: layouts, workspaces, code paths
        ts = []
        for _ in range(repeats):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            run()
            b.record(stream)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        out[json.dumps(c, sort_keys=True)] = statistics.median(ts)
    return out


def tune(key, candidates, apply, run, repeats=3, stream=None, use_cache=True, timer=None, device=None,
         arch=None):
    """Apply the fastest candidate for `key`; returns (shape, timings in ms, source) with
    source "timed", "cache" or "shipped".  `timer` (default: time_candidates on the
    device), `device` and `arch` (default: the current GPU's) can be replaced, e.g. to
    exercise the cache without a GPU."""
    full = (device or device_key()) + "|" + key
    cache = _load()
    if use_cache and full in cache:
        best = cache[full]["best"]
        apply(best)
        return best, cache[full]["ms"], "cache"
    if use_cache:
        entry = _shipped(key, arch)
        if entry is not None:
            apply(entry["best"])
            return entry["best"], entry.get("ms"), "shipped"
    times = (timer or time_candidates)(candidates, apply, run, repeats, stream)
    best = json.loads(min(times, key=times.get))
    cache[full] = {"best": best, "ms": times}
    _store(cache)
    apply(best)
    return best, times, "timed"


def tune_levels(solver, run, sizes, precision, repeats=3, use_cache=True):
    """Blocks per sweep and coefficient form of a hierarchy's level solves; `run`
    advances one step from the same state every time (the caller resets the fields
    inside it)."""
    return tune(workload_key("levels", sizes, precision), list(LEVEL_CANDIDATES),
                lambda c: solver.set_launch(max_blocks=c["max_blocks"], form_coefs=c.get("form_coefs", 0)), run,
                repeats, solver.stream, use_cache)


def tune_batch(solver, run, sizes, precision, repeats=2, use_cache=True):
    """Host-polled sweeps or a persistent launch (and its resident blocks per compute unit)
    for a batch of patches of the given sizes."""
    return tune(workload_key("batch", sizes, precision), list(BATCH_SHAPES),
                lambda c: solver.set_launch(0, c["persistent"], c["persistent_per_cu"], c.get("form_coefs", 0)),
                run, repeats,
                solver.stream, use_cache)


def tune_level_shapes(solver, run, sizes, precision, repeats=2, use_cache=True):
    """Blocks per sweep and host-polled or persistent launches of a hierarchy's level
    solves; `run` advances one step from the same state every time."""
    return tune(workload_key("level-shapes", sizes, precision), list(LEVEL_SHAPES),
                lambda c: solver.set_launch(c["max_blocks"], c["persistent"], c["persistent_per_cu"],
                                            c.get("form_coefs", 0)), run,
                repeats, solver.stream, use_cache)


def tune_refinement(solver, run, sizes, kind="levels", repeats=2, use_cache=True):
    """Inner tolerance of the mixed-precision form (FP32 inner solves inside FP64
    refinement): every candidate meets the same FP64 stopping rule, and the split of the
    work that is fastest depends on the workload."""
    return tune(workload_key("refinement-" + kind, sizes, 1), [{"inner_tol": t} for t in INNER_TOLS],
                lambda c: solver.set_refinement(c["inner_tol"]), run, repeats, solver.stream, use_cache)
