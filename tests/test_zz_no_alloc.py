"""amrfld_solve_level_noalloc (PCG workspace in the library's static device array)
against amrfld_solve_level, through the C ABI: the same energies bit for bit and the
same stats, on calls in a row whose later ones are smaller (they run on what the
earlier calls left in the array), and its rejections."""
import numpy as np
import pytest

from synth.configs import config_tiny, config_uniform
from synth.hierarchy import Hierarchy, uniform_hierarchy

pytestmark = pytest.mark.gpu

SCRATCH_SLOTS = 1 << 20


def _at_the_limit():
    """Uniform level 6 and a level 7 over the half box x < 1/2: exactly 2^20 slots."""
    p = config_uniform(6, kmode="lp", seed=3)
    g = np.arange(64, dtype=np.int32)
    I, J, K = np.meshgrid(np.arange(32, dtype=np.int32), g, g, indexing="ij")
    slab = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    p.hierarchy = Hierarchy(6, {6: p.hierarchy.octs[6], 7: slab})
    assert 8 * len(slab) == SCRATCH_SLOTS
    return p


def _mods():
    import torch
    from paper_1401_1112_amd import _lib as L
    from paper_1401_1112_amd import solver as S
    return torch, L, S


def _both(p, level, dt, mode, tol, **kw):
    """Solve `level` once with each entry point on two contexts built from the same
    inputs; returns (E regular, E no-alloc, stats regular, stats no-alloc)."""
    torch, L, S = _mods()
    a = S.solver_from_problem(p, **kw)
    b = S.solver_from_problem(p, **kw)
    print(f"no-alloc pair: {p.name} level {level} ({a.info(level)[0]} slots) mode {mode} {kw}", flush=True)
    st_a = L.amrfld_solve_level(a.ctx, level, dt, mode, tol)
    st_b = L.amrfld_solve_level_noalloc(b.ctx, level, dt, mode, tol)
    assert st_a == L.OK, L.amrfld_last_error(a.ctx)
    assert st_b == L.OK, L.amrfld_last_error(b.ctx)
    out = (S.to_numpy(a.E(level)), S.to_numpy(b.E(level)), a.stats(), b.stats())
    a.close()
    b.close()
    return out


def _same(res):
    ea, eb, sa, sb = res
    assert np.array_equal(ea, eb)
    assert len(sa) == len(sb) == 1
    for k in ("iters", "converged", "status", "rel_res", "true_rel_res", "linf_change", "min_E", "rnorm0",
              "bnorm", "sweep_blocks", "launch_mode"):
        assert sa[0][k] == sb[0][k], k


def test_noalloc_matches_solve_level_on_calls_in_a_row():
    # largest level first (exactly the scratch limit), then smaller ones on the
    # scratch contents the earlier calls left behind
    big = _at_the_limit()
    dx = 1.0 / 128
    _same(_both(big, 7, 8.0 * dx * dx, 0, 1e-10))
    small = config_tiny(2, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-12)
    for level in (5, 4):
        _same(_both(small, level, small.dt_coarse / 4, 0, small.tol))


def test_noalloc_persistent_launch_and_robin_interfaces():
    torch, L, S = _mods()
    p = config_tiny(3, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-12)
    # one persistent launch per solve: its barrier words live in the scratch too
    _same(_both(p, 5, p.dt_coarse / 4, 0, p.tol, persistent=True))
    # Robin mode once the flux registers exist (a Robin solve of level l creates level
    # l-1's): level 4 reads the register that the level-5 solve before it filled
    a = S.solver_from_problem(p)
    b = S.solver_from_problem(p)
    for s in (a, b):
        for lvl, dt in ((5, p.dt_coarse / 4), (4, p.dt_coarse / 2), (5, p.dt_coarse / 4)):
            assert L.amrfld_solve_level(s.ctx, lvl, dt, 2, p.tol) == L.OK
    print("no-alloc Robin pair: level 4 after a level-5 Robin solve", flush=True)
    assert L.amrfld_solve_level(a.ctx, 4, p.dt_coarse / 2, 2, p.tol) == L.OK
    assert L.amrfld_solve_level_noalloc(b.ctx, 4, p.dt_coarse / 2, 2, p.tol) == L.OK, L.amrfld_last_error(b.ctx)
    for lvl in (4, 5):
        assert np.array_equal(S.to_numpy(a.E(lvl)), S.to_numpy(b.E(lvl)))
    assert a.stats()[0]["iters"] == b.stats()[0]["iters"]
    a.close()
    b.close()


def test_noalloc_rejections_leave_the_context_usable():
    torch, L, S = _mods()
    p = config_tiny(4, base_level=3, max_level=4, p_refine=0.5, kmode="lp", tol=1e-12)
    # Neumann before any call created the coarser level's flux register
    s = S.solver_from_problem(p)
    assert L.amrfld_solve_level_noalloc(s.ctx, 4, p.dt_coarse / 2, 1, p.tol) == L.E_STATE
    assert "flux register" in L.amrfld_last_error(s.ctx)
    assert L.amrfld_solve_level_noalloc(s.ctx, 9, p.dt_coarse, 0, p.tol) == L.E_INVALID
    assert L.amrfld_solve_level_noalloc(s.ctx, 4, -1.0, 0, p.tol) == L.E_INVALID
    assert L.amrfld_solve_level_noalloc(s.ctx, 4, p.dt_coarse / 2, 0, p.tol) == L.OK
    s.close()
    # mixed precision needs FP32 workspace
    from paper_1401_1112_amd import MIXED
    m = S.solver_from_problem(p, precision=MIXED)
    assert L.amrfld_solve_level_noalloc(m.ctx, 4, p.dt_coarse / 2, 0, p.tol) == L.E_INVALID
    assert "FP64" in L.amrfld_last_error(m.ctx)
    m.close()
    # a level above the scratch limit (no fields needed: the size is checked first)
    h = uniform_hierarchy(7)
    big = S.HierarchySolver(h.base_level, h.octs)
    assert big.info(7)[0] > SCRATCH_SLOTS
    assert L.amrfld_solve_level_noalloc(big.ctx, 7, 1e-5, 0, 1e-10) == L.E_INVALID
    assert "scratch limit" in L.amrfld_last_error(big.ctx)
    big.close()
