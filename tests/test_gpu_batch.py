"""The batch form (amrfld_solve_batch) against the CPU patch oracle."""
import numpy as np
import pytest

from oracle.patch_oracle import patch_advance
from synth.configs import patch_batch

pytestmark = pytest.mark.gpu


def _solver(**kw):
    from paper_1401_1112_amd.solver import BatchSolver
    return BatchSolver(**kw)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


class _P:
    def __init__(self, p, E):
        self.n, self.dx, self.dt = p.n, p.dx, p.dt
        self.rho, self.E = p.rho, E
        self.face_mode, self.face_ghost, self.face_flux = p.face_mode, p.face_ghost, p.face_flux


def _oracle_step(p, E, tol, alpha, max_iter=10000):
    return patch_advance(p.rho, E, p.dx, p.dt, p.face_mode, p.face_ghost, p.face_flux, 1, tol,
                         alpha=alpha, max_iter=max_iter)


def _batch_steps(patches, steps, tol, alpha, max_iter):
    """Advance GPU batch and oracle step by step; per step: counts (gpu, oracle) per patch and the
    worst relative L2 difference."""
    s = _solver(robin_alpha=alpha, max_iter=max_iter)
    Eg = [p.E for p in patches]
    Eo = [p.E for p in patches]
    out = []
    for _ in range(steps):
        res, _ = s.solve([_P(p, e) for p, e in zip(patches, Eg)], 1, tol, raise_on_error=False)
        st = s.stats()
        it_g = [x["iters"] for x in st]
        it_o, worst = [], 0.0
        new_o = []
        for q, p in enumerate(patches):
            e, h = _oracle_step(p, Eo[q], tol, alpha, max_iter)
            it_o.append(h[0]["iters"])
            new_o.append(e)
            worst = max(worst, _rel(res[q], e))
        out.append((it_g, it_o, worst))
        Eg, Eo = res, new_o
    s.close()
    return out


@pytest.mark.parametrize("seed", [4100, 4200])
def test_batch_fp64_parity_per_step(seed):
    patches, alpha = patch_batch(seed, 10, n_min=4, n_max=20)
    res = _batch_steps(patches, 3, 1e-12, alpha, 10000)
    if all(g == o for g, o, _ in res):
        assert max(w for _, _, w in res) <= 1e-12, res
        return
    # near-tie at the stopping threshold: both sides with the larger count, tol = 0
    n_fix = max(max(g + o) for g, o, _ in res)
    res2 = _batch_steps(patches, 3, 0.0, alpha, n_fix)
    assert max(w for _, _, w in res2) <= 1e-12, res2


def test_batch_uneven_sizes_and_modes():
    # sizes from 2 to 32 in one batch, every face mode present
    patches, alpha = patch_batch(4300, 14, n_min=2, n_max=32)
    modes = {int(m) for p in patches for m in p.face_mode}
    assert modes == {0, 1, 2}
    res = _batch_steps(patches, 2, 1e-11, alpha, 10000)
    for g, o, w in res:
        assert w <= 1e-10, res


def test_batch_matches_single_patch_calls():
    from paper_1401_1112_amd import OK
    patches, alpha = patch_batch(4400, 6, n_min=4, n_max=16)
    s = _solver(robin_alpha=alpha)
    batch, st = s.solve(patches, 2, 1e-12)
    assert st == OK
    for q, p in enumerate(patches):
        one, _ = s.solve([p], 2, 1e-12)
        assert _rel(batch[q], one[0]) <= 1e-12
    s.close()


def test_batch_deterministic():
    patches, alpha = patch_batch(4500, 8, n_min=4, n_max=24)
    s = _solver(robin_alpha=alpha)
    a, _ = s.solve(patches, 2, 1e-12)
    b, _ = s.solve(patches, 2, 1e-12)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    s.close()


def test_batch_mixed_precision_reaches_tolerance():
    from paper_1401_1112_amd import MIXED
    patches, alpha = patch_batch(4600, 10, n_min=4, n_max=24)
    s = _solver(robin_alpha=alpha)
    res, _ = s.solve(patches, 2, 1e-10, precision=MIXED)
    for st in s.stats():
        assert st["converged"] == 1 and st["true_rel_res"] <= 1e-10 * (1 + 1e-6), st
    for q, p in enumerate(patches):
        e, _ = patch_advance(p.rho, p.E, p.dx, p.dt, p.face_mode, p.face_ghost, p.face_flux, 2, 1e-13,
                             alpha=alpha)
        assert _rel(res[q], e) <= 1e-8
    s.close()


def test_batch_rejects_bad_patch():
    from paper_1401_1112_amd import AmrfldError
    patches, alpha = patch_batch(4700, 2, n_min=4, n_max=8)
    patches[1].n = 5  # odd sizes are rejected before any device work
    s = _solver()
    with pytest.raises(AmrfldError):
        s.solve(patches, 1, 1e-10)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("graph,big", [(False, False), (True, False), (False, True), (True, True)])
def test_batch_persistent_launch_equals_polled(graph, big, precision):
    # one cooperative launch per step (and all steps in one hipGraph) runs the same
    # sweep bodies over the same block plan: results and counts are bitwise equal.
    # In mixed precision that launch runs the whole refinement loop of every patch,
    # its decisions made on the device.  The big case spreads each patch over many
    # blocks of up to 16 tiles, so the grid barrier must make neighbour values visible
    # across XCDs.
    from paper_1401_1112_amd import FP64, MIXED
    prec = MIXED if precision == "mixed" else FP64
    tol = 1e-10 if precision == "mixed" else 1e-12
    if big:
        patches, alpha = patch_batch(4900, 48, n_min=24, n_max=96)
    else:
        patches, alpha = patch_batch(4800, 12, n_min=4, n_max=24)
    print(f"batch persistent vs polled: {precision}, graph {graph}, {len(patches)} patches", flush=True)
    s = _solver(robin_alpha=alpha)
    a, _ = s.solve(patches, 3, tol, precision=prec)
    it_a = [(x["iters"], x["outer_iters"]) for x in s.stats()]
    s.close()
    sp = _solver(robin_alpha=alpha, persistent=True, graph=graph)
    b, st = sp.solve(patches, 3, tol, precision=prec)
    stats = sp.stats()
    sp.close()
    assert {x["launch_mode"] for x in stats} == ({2} if graph else {1})
    assert [(x["iters"], x["outer_iters"]) for x in stats] == it_a
    assert all(x["converged"] == 1 for x in stats)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_set_launch_rejects_negative_values():
    from paper_1401_1112_amd import AmrfldError
    patches, alpha = patch_batch(4950, 3, n_min=4, n_max=8)
    s = _solver(robin_alpha=alpha)
    with pytest.raises(AmrfldError):
        s.set_launch(-1, False, 0)
    with pytest.raises(AmrfldError):
        s.set_launch(0, True, -2)
    # the shape is unchanged and the solver still works
    res, st = s.solve(patches, 1, 1e-10)
    assert st == 0
    s.set_launch(64, True, 1)
    res2, _ = s.solve(patches, 1, 1e-10)
    assert [x["launch_mode"] for x in s.stats()] == [1] * len(patches)
    for a, b in zip(res, res2):
        assert _rel(a, b) <= 1e-13
    s.close()
