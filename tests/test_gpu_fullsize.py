"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

Protocol (as for the small cases): with equal iteration counts in every solve the
results agree to 1e-12 relative L2; where a count differs (a near-tie of a residual with
its stopping threshold, the two sides summing in different orders) both sides are run
again with every solve fixed at the largest count seen (tol 0, no absolute floor) and
that comparison is gated at 1e-12.

* fld_lognormal (levels 6..9, 4,012,144 cells): one coarse step (15 level solves) on the
  GPU and in the oracle, at every block count the tuner may pick.
* the mixed-precision form of the same step: every solve meets its threshold on the FP64
  true residual; its error against the FP64 oracle (max and L2, per level) is reported
  and bounded.
* the 512-patch batch: three steps of all patches in shared sweeps; a seeded sample of 16
  patches (the smallest and the largest among them) against the patch oracle step by
  step, every patch's true residual against its threshold, and the persistent launch
  bitwise equal to the polled one.
"""
import numpy as np
import pytest

from _util import align, oracle_from_problem
import oracle as ora
from oracle.patch_oracle import patch_advance
from synth.configs import config_fld_lognormal, patch_batch

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def lognormal():
    return config_fld_lognormal()


@pytest.fixture(scope="module")
def oracle_step(lognormal):
    p = lognormal
    o = oracle_from_problem(p)
    o.advance_subcycled(p.dt_coarse, ora.DIRICHLET, p.tol)
    return o, [(h["level"], h["iters"]) for h in o.history]


@pytest.fixture(scope="module")
def gpu_solver(lognormal):
    from paper_1401_1112_amd.solver import solver_from_problem
    s = solver_from_problem(lognormal)
    yield s
    s.close()


def _gpu_step(s, p, max_blocks):
    """One coarse step from the initial fields with the given blocks per sweep."""
    from paper_1401_1112_amd import BC_DIRICHLET
    from paper_1401_1112_amd.solver import sample_problem_fields, to_numpy
    sample_problem_fields(s, p)
    s.set_launch(max_blocks=max_blocks)
    s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
    gpu = {l: (to_numpy(s.E(l)), s.cells(l)) for l in p.hierarchy.levels}
    return gpu, [(st["level"], st["iters"]) for st in s.stats()], s.stats()


_FIXED = {}


def _oracle_fixed(p, n_fix):
    """The oracle's coarse step with every solve run for exactly n_fix iterations."""
    if n_fix not in _FIXED:
        o = oracle_from_problem(p, max_iter=n_fix, abs_floor=0.0)
        o.advance_subcycled(p.dt_coarse, ora.DIRICHLET, 0.0)
        _FIXED[n_fix] = o
    return _FIXED[n_fix]


def _worst_vs_oracle(p, o, gpu):
    worst = 0.0
    for l in p.hierarchy.levels:
        e, cells = gpu[l]
        worst = max(worst, _rel(e, align(l, o.cells(l), o.E[l], cells)))
    return worst


# every launch shape the autotuner may pick for the level solves
@pytest.mark.parametrize("max_blocks", [256, 512, 1024, 2048, 4096])
def test_lognormal_full_step_parity(lognormal, oracle_step, gpu_solver, max_blocks):
    o, counts_o = oracle_step
    gpu, counts_g, _ = _gpu_step(gpu_solver, lognormal, max_blocks)
    assert [l for l, _ in counts_g] == [l for l, _ in counts_o]
    worst = _worst_vs_oracle(lognormal, o, gpu)
    print(f"max_blocks {max_blocks}: iteration counts {counts_g} (oracle {counts_o}); "
          f"worst relative L2 {worst:.3e}")
    if counts_g == counts_o:
        assert worst <= 1e-12
        return
    # near-tie at a stopping threshold: both sides with every solve at the largest count
    from paper_1401_1112_amd import BC_DIRICHLET
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    n_fix = max(it for _, it in counts_g + counts_o)
    of = _oracle_fixed(lognormal, n_fix)
    s = solver_from_problem(lognormal, max_iter=n_fix, abs_floor=0.0, max_blocks=max_blocks)
    s.advance(lognormal.dt_coarse, BC_DIRICHLET, 0.0, raise_on_error=False)
    g2 = {l: (to_numpy(s.E(l)), s.cells(l)) for l in lognormal.hierarchy.levels}
    c2 = [st["iters"] for st in s.stats()]
    s.close()
    assert c2 == [h["iters"] for h in of.history] == [n_fix] * len(c2)
    worst2 = _worst_vs_oracle(lognormal, of, g2)
    print(f"max_blocks {max_blocks}: fixed count {n_fix}, worst relative L2 {worst2:.3e}")
    assert worst2 <= 1e-12


@pytest.fixture(scope="module")
def fp64_step(lognormal, gpu_solver):
    return _gpu_step(gpu_solver, lognormal, 0)


def test_lognormal_full_step_residuals(lognormal, fp64_step):
    # every FP64 solve of the step meets its threshold on the true residual, up to the
    # recursion's rounding drift
    _, _, stats = fp64_step
    for st in stats:
        thr = max(lognormal.tol * st["rnorm0"], lognormal.abs_floor * st["bnorm"])
        assert st["converged"] == 1 and st["true_rel_res"] * st["rnorm0"] <= 1.05 * thr, st


def test_lognormal_mixed_full_step(lognormal, fp64_step, oracle_step):
    # the precision form: every solve stops on the FP64 true residual; its error
    # against the FP64 oracle and against the FP64 GPU solve, per level after the step
    from paper_1401_1112_amd import BC_DIRICHLET, MIXED
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    gpu, _, _ = fp64_step
    o, _ = oracle_step
    p = lognormal
    s = solver_from_problem(p, precision=MIXED)
    s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
    for st in s.stats():
        thr = max(p.tol * st["rnorm0"], p.abs_floor * st["bnorm"])
        assert st["converged"] == 1 and st["true_rel_res"] * st["rnorm0"] <= thr * (1 + 1e-12), st
    for l in p.hierarchy.levels:
        e, cells = gpu[l]
        assert np.array_equal(s.cells(l), cells)
        m = to_numpy(s.E(l))
        ref = align(l, o.cells(l), o.E[l], cells)
        err_max = float(np.abs(m - ref).max() / np.abs(ref).max())
        err_l2 = _rel(m, ref)
        print(f"mixed level {l}: vs FP64 oracle max {err_max:.3e} L2 {err_l2:.3e}; "
              f"vs FP64 GPU L2 {_rel(m, e):.3e}")
        assert err_l2 <= 1e-8 and _rel(m, e) <= 1e-8
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lognormal_persistent_equals_polled(lognormal, precision):
    # one persistent launch per solve at full size gives the host-polled results bitwise
    from paper_1401_1112_amd import BC_DIRICHLET, FP64, MIXED
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    p = lognormal
    prec = MIXED if precision == "mixed" else FP64
    out = []
    for kw in ({}, {"persistent": True}):
        s = solver_from_problem(p, precision=prec, **kw)
        s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
        st = s.stats()
        out.append(({l: to_numpy(s.E(l)) for l in p.hierarchy.levels}, [x["iters"] for x in st],
                    {x["launch_mode"] for x in st}))
        s.close()
    (a, ia, ma), (b, ib, mb) = out
    assert ma == {0} and mb == {1}
    assert ia == ib
    assert all(np.array_equal(a[l], b[l]) for l in a)


@pytest.fixture(scope="module")
def batch512():
    return patch_batch(4000, 512)


def _batch_sample_vs_oracle(patches, alpha, sample, steps, tol, max_iter, abs_floor):
    """The whole batch on the GPU for `steps` steps, the sampled patches in the patch
    oracle; per sampled patch: per-step counts of both sides and the relative L2
    difference at the end, plus the GPU stats."""
    from paper_1401_1112_amd.solver import BatchSolver
    bs = BatchSolver(robin_alpha=alpha, max_iter=max_iter, abs_floor=abs_floor)
    h = bs.upload(patches)
    bs.run(h, steps, tol, raise_on_error=False)
    res = bs.result(h)
    st = bs.stats()
    bs.close()
    n = len(patches)
    out = {}
    for q in sample:
        p = patches[q]
        e, hist = patch_advance(p.rho, p.E, p.dx, p.dt, p.face_mode, p.face_ghost, p.face_flux, steps, tol,
                                alpha=alpha, max_iter=max_iter, abs_floor=abs_floor)
        out[q] = ([st[k * n + q]["iters"] for k in range(steps)], [x["iters"] for x in hist], _rel(res[q], e))
    return out, st


def test_patch_batch_full_size_sampled(batch512):
    patches, alpha = batch512
    steps = 3
    sizes = np.array([p.n for p in patches])
    rng = np.random.default_rng(512)
    sample = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))}
                    | set(int(i) for i in rng.choice(len(patches), 14, replace=False)))
    out, st = _batch_sample_vs_oracle(patches, alpha, sample, steps, 1e-10, 10000, 1e-14)
    for k, x in enumerate(st):
        thr = max(1e-10 * x["rnorm0"], 1e-14 * x["bnorm"])
        assert x["converged"] == 1 and x["true_rel_res"] * x["rnorm0"] <= 2.5 * thr, (k, x)
    for q, (ig, io, r) in out.items():
        print(f"patch {q} n={patches[q].n}: iterations gpu {ig} oracle {io}, rel L2 {r:.3e}")
    if all(ig == io for ig, io, _ in out.values()):
        assert max(r for _, _, r in out.values()) <= 1e-12
        return
    # near-tie at a stopping threshold: every solve fixed at the largest count seen
    n_fix = max(max(ig + io) for ig, io, _ in out.values())
    out2, _ = _batch_sample_vs_oracle(patches, alpha, sample, steps, 0.0, n_fix, 0.0)
    for q, (ig, io, r) in out2.items():
        print(f"patch {q} fixed count {n_fix}: rel L2 {r:.3e}")
        assert ig == io == [n_fix] * steps
    assert max(r for _, _, r in out2.values()) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_patch_batch_full_size_persistent_bitwise(batch512, precision):
    # every batch launch shape the autotuner may pick gives the polled results bitwise;
    # in mixed precision the persistent launch runs each step's whole refinement loop
    from paper_1401_1112_amd import FP64, MIXED
    from paper_1401_1112_amd.solver import BatchSolver
    patches, alpha = batch512
    prec = MIXED if precision == "mixed" else FP64
    out = []
    for kw in ({}, {"persistent": True, "graph": True}, {"persistent": True, "persistent_per_cu": 1},
               {"persistent": True, "graph": True, "persistent_per_cu": 2}):
        print(f"batch 512 {precision} {kw}", flush=True)
        bs = BatchSolver(robin_alpha=alpha, **kw)
        h = bs.upload(patches)
        bs.run(h, 2, 1e-10, prec)
        st = bs.stats()
        out.append((bs.result(h), [(x["iters"], x["outer_iters"]) for x in st], {x["launch_mode"] for x in st}))
        bs.close()
    a, ia, ma = out[0]
    assert ma == {0}
    for b, ib, mode in out[1:]:
        assert mode in ({1}, {2})
        assert ia == ib
        assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_lognormal_formed_coefficients_equal_stored_bitwise(lognormal, fp64_step):
    # face coefficients formed from K in every sweep against the stored ones (the
    # benchmark's default), at full size: same counts, same bits
    from paper_1401_1112_amd import BC_DIRICHLET
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    gpu, counts, _ = fp64_step
    p = lognormal
    s = solver_from_problem(p, form_coefs=True)
    s.advance(p.dt_coarse, BC_DIRICHLET, p.tol)
    assert [(st["level"], st["iters"]) for st in s.stats()] == counts
    for l in p.hierarchy.levels:
        e, cells = gpu[l]
        assert np.array_equal(s.cells(l), cells)
        assert np.array_equal(to_numpy(s.E(l)), e)
    s.close()
