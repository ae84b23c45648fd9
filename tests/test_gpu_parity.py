"""Parity of the HIP library (through its C ABI) with the CPU FP64 oracle.

Bar: relative L2 difference per level <= 1e-12 after every compared step, with
the same PCG iteration counts; where a count differs by a near-tie at the
stopping threshold both sides are re-run with the larger count and tol = 0.
"""
import numpy as np
import pytest
import scipy.fft

from _util import align, oracle_from_problem
import oracle as ora
from synth.configs import config_heat_gaussian, config_tiny, config_uniform

pytestmark = pytest.mark.gpu

MODES = {"dirichlet": ora.DIRICHLET, "neumann": ora.NEUMANN, "robin": ora.ROBIN}


def _gpu():
    import torch
    from paper_1401_1112_amd import solver as S
    return torch, S


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def _compare_levels(s, o, levels, tol=1e-12, label=""):
    torch, S = _gpu()
    worst = 0.0
    for lvl in levels:
        g = S.to_numpy(s.E(lvl))
        e = align(lvl, o.cells(lvl), o.E[lvl], s.cells(lvl))
        r = _rel(g, e)
        worst = max(worst, r)
        assert r <= tol, f"{label} level {lvl}: relative L2 {r:.3e}"
    return worst


def _iters_gpu(s):
    return [(st["level"], st["iters"]) for st in s.stats()]


def _iters_oracle(o, start):
    return [(h["level"], h["iters"]) for h in o.history[start:]]


@pytest.mark.parametrize("level,dtfac", [(4, 4.0), (5, 16.0), (6, 4.0)])
def test_uniform_level_closed_form(level, dtfac):
    torch, S = _gpu()
    p = config_uniform(level, kmode="const", seed=level)
    dx = 1.0 / (1 << level)
    dt = dtfac * dx * dx
    s = S.solver_from_problem(p, abs_floor=1e-16)
    c = s.cells(level)
    n = 1 << level
    b = np.zeros((n, n, n))
    b[c[:, 0], c[:, 1], c[:, 2]] = p.E(level, c)
    s.solve_level(level, dt, 0, 1e-14)
    x = S.to_numpy(s.E(level))
    lam1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    ref = scipy.fft.idctn(scipy.fft.dctn(b, type=2, norm="ortho") / (1 + dt / dx ** 2 * lam),
                          type=2, norm="ortho")[c[:, 0], c[:, 1], c[:, 2]]
    assert _rel(x, ref) < 1e-13
    o = oracle_from_problem(p, abs_floor=1e-16)
    o.solve_level(level, dt, ora.DIRICHLET, 1e-14)
    assert s.stats()[0]["iters"] == o.history[-1]["iters"]
    _compare_levels(s, o, [level])
    s.close()


def _spd_start(p, o):
    """The level systems are SPD when K > 0: always for constant K, and in LP mode while
    every energy is positive.  Neumann interfaces can drive energies negative (the
    failure mode of Sect. 3.3.5); steps from such a state are outside the parity gate."""
    return p.kmode == "const" or all(np.all(o.E[l] > 0) for l in o.lev)


def _run_pair(p, mode, steps, tol, max_iter):
    """Advance GPU and oracle side by side over the steps that start from an SPD state;
    returns per-step iteration lists and the largest per-level relative L2 difference.
    tol = 0 runs every solve for exactly max_iter iterations (no absolute floor either).

    A solve inside a step can still meet a diagonal entry <= 0 (energies gone negative
    earlier in the step): CG on the Jacobi-scaled system is undefined there, and the GPU
    must report E_NONFINITE for exactly that solve after the same counts on the solves
    before it; the comparison ends at that step."""
    torch, S = _gpu()
    floor = {} if tol > 0 else {"abs_floor": 0.0}
    s = S.solver_from_problem(p, max_iter=max_iter, **floor)
    o = oracle_from_problem(p, max_iter=max_iter, **floor)
    counts, diffs = [], []
    for _ in range(steps):
        if not _spd_start(p, o):
            break
        start = len(o.history)
        status = s.advance(p.dt_coarse, mode, tol, raise_on_error=False)
        o.advance_subcycled(p.dt_coarse, mode, tol)
        g, r = _iters_gpu(s), _iters_oracle(o, start)
        bad = [k for k, h in enumerate(o.history[start:]) if h["min_diag"] <= 0.0]
        # a fixed-count run (tol = 0) ends every solve at its cap: E_NOCONV by design
        fine = {S.L.OK} if tol > 0 else {S.L.OK, S.L.E_NOCONV}
        st = s.stats()
        if bad:
            k = bad[0]
            assert status != S.L.OK and len(st) == k + 1, (status, len(st), k)
            assert st[k]["status"] == S.L.E_NONFINITE and st[k]["level"] == r[k][0]
            assert all(x["status"] in fine for x in st[:k])
            if k:
                counts.append((g[:k], r[:k]))
            break
        assert status in fine and all(x["status"] in fine for x in st), status
        counts.append((g, r))
        diffs.append(_compare_levels(s, o, p.hierarchy.levels, tol=np.inf))
    s.close()
    return counts, diffs


def _parity_protocol(p, mode, steps, tol=1e-12):
    """Gate: same iteration counts and <= 1e-12 relative L2 per level and step.  Where a
    count differs (a near-tie at the stopping threshold) both sides are re-run with the
    largest count fixed and tol = 0, and that comparison is gated at 1e-12."""
    counts, diffs = _run_pair(p, mode, steps, p.tol, p.max_iter)
    assert counts and diffs, "no step started from an SPD state"
    if all(g == o for g, o in counts):
        assert max(diffs) <= tol, diffs
        return "same-count"
    n_fix = max(it for g, o in counts for _, it in g + o)
    counts2, diffs2 = _run_pair(p, mode, steps, 0.0, n_fix)
    assert all(g == o for g, o in counts2), counts2
    assert diffs2 and max(diffs2) <= tol, diffs2
    return "fixed-count"


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("mode", ["dirichlet", "neumann", "robin"])
@pytest.mark.parametrize("kmode", ["lp", "const"])
def test_tiny_amr_advance_parity(seed, mode, kmode):
    p = config_tiny(seed, base_level=3, max_level=5, p_refine=0.5, kmode=kmode, tol=1e-12)
    how = _parity_protocol(p, MODES[mode], steps=2)
    print(f"seed {seed} {mode} {kmode}: {how}")


def test_heat_gaussian_parity_every_step():
    p = config_heat_gaussian()
    how = _parity_protocol(p, ora.DIRICHLET, steps=p.n_coarse_steps)
    print(f"heat gaussian: {how}")


def _leaf_mask(p, lvl, cells):
    if lvl + 1 not in p.hierarchy.octs:
        return np.ones(len(cells), dtype=bool)
    n = np.int64(1) << lvl
    par = p.hierarchy.octs[lvl + 1].astype(np.int64)
    keys = set(((par[:, 0] * n + par[:, 1]) * n + par[:, 2]).tolist())
    k = (cells[:, 0].astype(np.int64) * n + cells[:, 1]) * n + cells[:, 2]
    return np.array([kk not in keys for kk in k.tolist()])


def _total_energy(s, p):
    torch, S = _gpu()
    tot = 0.0
    for lvl in p.hierarchy.levels:
        c = s.cells(lvl)
        e = S.to_numpy(s.E(lvl))
        tot += np.sum(e[_leaf_mask(p, lvl, c)]) / float(1 << lvl) ** 3
    return tot


def test_neumann_conserves_dirichlet_drifts_on_gpu():
    torch, S = _gpu()
    out = {}
    for mode in (ora.NEUMANN, ora.DIRICHLET):
        p = config_tiny(2, base_level=3, max_level=5, p_refine=0.5, tol=1e-13)
        s = S.solver_from_problem(p)
        e0 = _total_energy(s, p)
        s.advance(p.dt_coarse, mode, p.tol)
        out[mode] = abs(_total_energy(s, p) - e0) / e0
        s.close()
    assert out[ora.NEUMANN] < 1e-12
    assert out[ora.DIRICHLET] > 1e-6


def test_negative_energy_reported_like_oracle():
    # Neumann interfaces on a steep field: the coarse solve ends with negative energies
    # (Sect. 3.3.5, Fig. 2); the GPU stats report the same minimum as the oracle.
    torch, S = _gpu()
    p = config_tiny(0, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-12)
    s = S.solver_from_problem(p)
    o = oracle_from_problem(p)
    s.advance(p.dt_coarse, ora.NEUMANN, p.tol)
    o.advance_subcycled(p.dt_coarse, ora.NEUMANN, p.tol)
    g = [st["min_E"] for st in s.stats()]
    r = [h["min_E"] for h in o.history]
    assert min(r) < 0 and min(g) < 0
    assert np.allclose(g, r, rtol=1e-10, atol=1e-12)
    s.close()


def test_noconv_returns_status_and_iterate():
    torch, S = _gpu()
    from paper_1401_1112_amd import E_NOCONV
    p = config_tiny(0, base_level=3, max_level=4, tol=1e-12)
    s = S.solver_from_problem(p, max_iter=1)
    st = s.solve_level(3, p.dt_coarse, 0, 1e-12, raise_on_error=False)
    assert st == E_NOCONV
    assert s.stats()[0]["iters"] == 1 and s.stats()[0]["converged"] == 0
    o = oracle_from_problem(p, max_iter=1)
    o.solve_level(3, p.dt_coarse, ora.DIRICHLET, 1e-12)
    _compare_levels(s, o, [3])
    s.close()


def test_nan_density_is_nonfinite():
    torch, S = _gpu()
    from paper_1401_1112_amd import E_NONFINITE
    p = config_uniform(3, kmode="lp")
    s = S.solver_from_problem(p)
    c = s.cells(3)
    rho = p.rho(3, c)
    rho[5] = np.nan
    s.set_fields(3, rho, p.E(3, c))
    assert s.solve_level(3, p.dt_coarse, 0, 1e-10, raise_on_error=False) == E_NONFINITE
    s.close()


def test_unbalanced_level_rejected():
    torch, S = _gpu()
    from paper_1401_1112_amd import AmrfldError
    octs = {2: np.array([[i, j, k] for i in range(2) for j in range(2) for k in range(2)], dtype=np.int32),
            3: np.array([[0, 0, 0]], dtype=np.int32),
            4: np.array([[0, 0, 0], [1, 0, 0]], dtype=np.int32)}
    # oct (1,0,0) at level 4 has parent cell (1,0,0) at level 3, which exists; its +x
    # neighbour cell (2,0,0) at level 3 is absent -> unbalanced
    with pytest.raises(AmrfldError):
        S.HierarchySolver(2, octs)


def test_constant_state_zero_iterations():
    torch, S = _gpu()
    p = config_tiny(4, base_level=2, max_level=4, p_refine=0.5)
    s = S.solver_from_problem(p)
    for lvl in p.hierarchy.levels:
        ns, _ = s.info(lvl)
        s.set_fields(lvl, np.linspace(0.5, 2.0, ns), np.full(ns, 3.25))
    for mode in (0, 1, 2):
        s.advance(0.05, mode, 1e-10)
        assert all(st["iters"] == 0 for st in s.stats())
    for lvl in p.hierarchy.levels:
        assert np.all(S.to_numpy(s.E(lvl)) == 3.25)
    s.close()


def test_deterministic_bitwise():
    torch, S = _gpu()
    res = []
    for _ in range(2):
        p = config_tiny(3, base_level=3, max_level=5, p_refine=0.5)
        s = S.solver_from_problem(p)
        s.advance(p.dt_coarse, 2, 1e-12)
        res.append([S.to_numpy(s.E(l)).copy() for l in p.hierarchy.levels])
        s.close()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_coupled_temperature_parity():
    torch, S = _gpu()
    p = config_tiny(5, base_level=3, max_level=4, p_refine=0.5, tol=1e-12)
    p.T = lambda lvl, c: (p.E(lvl, c) ** 0.25) * 1.05
    p.kappa_P = 2.0
    s = S.solver_from_problem(p)
    o = oracle_from_problem(p)
    s.advance(p.dt_coarse, 0, p.tol)
    o.advance_subcycled(p.dt_coarse, ora.DIRICHLET, p.tol)
    _compare_levels(s, o, p.hierarchy.levels)
    for lvl in p.hierarchy.levels:
        _, t = s.E(lvl, with_T=True)
        tt = align(lvl, o.cells(lvl), o.T[lvl], s.cells(lvl))
        assert _rel(S.to_numpy(t), tt) < 1e-12
    s.close()


# ------------------------------------------------------------- mixed precision
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("mode", ["dirichlet", "robin"])
def test_mixed_precision_refinement_reaches_fp64_tolerance(seed, mode):
    # FP32 inner PCG + FP64 refinement: every solve must reach a true FP64 relative
    # residual <= tol; lambda_min(A) >= 1 then bounds the error by the residual.
    torch, S = _gpu()
    from paper_1401_1112_amd import MIXED
    p = config_tiny(seed, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-10)
    s = S.solver_from_problem(p, precision=MIXED)
    o = oracle_from_problem(p)
    s.advance(p.dt_coarse, MODES[mode], p.tol)
    o.advance_subcycled(p.dt_coarse, MODES[mode], 1e-13)
    for st in s.stats():
        assert st["converged"] == 1
        assert st["true_rel_res"] <= p.tol * (1 + 1e-6), st
        assert st["outer_iters"] >= 1
    worst = _compare_levels(s, o, p.hierarchy.levels, tol=1e-8)
    print(f"mixed seed {seed} {mode}: max relative L2 vs FP64 oracle {worst:.2e}")
    s.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_mixed_precision_inner_iterations_track_fp64_cg(seed):
    # After a refinement sweep the FP32 CG continues its search direction from the
    # replaced residual: its iterations over a step stay within a few per cent of FP64
    # CG's (restarting it from zero after every refinement costs about a third more).
    torch, S = _gpu()
    from paper_1401_1112_amd import FP64, MIXED
    p = config_tiny(seed, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-10)
    its = {}
    for name, prec in (("fp64", FP64), ("mixed", MIXED)):
        s = S.solver_from_problem(p, precision=prec)
        s.advance(p.dt_coarse, MODES["dirichlet"], p.tol)
        st = s.stats()
        assert all(x["converged"] == 1 for x in st)
        its[name] = (sum(x["iters"] for x in st), len(st))
        s.close()
    (n64, k), (nmx, _) = its["fp64"], its["mixed"]
    print(f"seed {seed}: FP64 CG {n64} iterations, mixed inner {nmx} over {k} solves")
    assert nmx <= 1.15 * n64 + 2 * k, its


def test_mixed_precision_uniform_closed_form():
    torch, S = _gpu()
    from paper_1401_1112_amd import MIXED
    level = 5
    p = config_uniform(level, kmode="const", seed=level)
    dx = 1.0 / (1 << level)
    dt = 16.0 * dx * dx
    s = S.solver_from_problem(p, precision=MIXED, abs_floor=0.0)
    c = s.cells(level)
    n = 1 << level
    b = np.zeros((n, n, n))
    b[c[:, 0], c[:, 1], c[:, 2]] = p.E(level, c)
    s.solve_level(level, dt, 0, 1e-12)
    x = S.to_numpy(s.E(level))
    lam1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    ref = scipy.fft.idctn(scipy.fft.dctn(b, type=2, norm="ortho") / (1 + dt / dx ** 2 * lam),
                          type=2, norm="ortho")[c[:, 0], c[:, 1], c[:, 2]]
    st = s.stats()[0]
    assert st["true_rel_res"] <= 1e-12 * (1 + 1e-6)
    assert _rel(x, ref) < 1e-11
    s.close()


# ------------------------------------------------------------- persistent launch
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("mode", ["dirichlet", "robin"])
def test_persistent_level_solves_equal_polled(precision, mode):
    # one cooperative launch per solve (per inner solve in mixed precision) runs the same
    # sweep bodies over the same block plan as the host-polled sweeps: results and
    # iteration counts are bitwise equal
    torch, S = _gpu()
    from paper_1401_1112_amd import FP64, MIXED
    prec = MIXED if precision == "mixed" else FP64
    p = config_tiny(2, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-10)
    out = []
    for kw in ({}, {"persistent": True}, {"persistent": True, "persistent_per_cu": 1}):
        s = S.solver_from_problem(p, precision=prec, **kw)
        s.advance(p.dt_coarse, MODES[mode], p.tol)
        s.advance(p.dt_coarse, MODES[mode], p.tol)
        st = s.stats()
        out.append(([S.to_numpy(s.E(l)) for l in p.hierarchy.levels],
                    [(x["iters"], x["outer_iters"]) for x in st], {x["launch_mode"] for x in st}))
        s.close()
    base, counts, modes = out[0]
    assert modes == {0}
    for e, c, m in out[1:]:
        assert m == {1}
        assert c == counts
        assert all(np.array_equal(a, b) for a, b in zip(e, base))


def test_own_schedule_with_restrict_equals_advance():
    # a caller's own schedule of amrfld_solve_level and amrfld_restrict_level calls in
    # the driver's order (Sect. 2.2: finer levels first, restriction after their
    # substeps) gives the subcycled step bit for bit
    torch, S = _gpu()
    from paper_1401_1112_amd import E_INVALID, _lib as L
    p = config_tiny(5, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-12)
    a = S.solver_from_problem(p)
    a.advance(p.dt_coarse, 0, p.tol)
    b = S.solver_from_problem(p)

    def step(level, dt):
        if level < p.hierarchy.max_level:
            for _ in range(2):
                step(level + 1, dt / 2)
            b.restrict(level + 1)
        b.solve_level(level, dt, 0, p.tol)

    step(p.hierarchy.base_level, p.dt_coarse)
    for lvl in p.hierarchy.levels:
        assert np.array_equal(S.to_numpy(a.E(lvl)), S.to_numpy(b.E(lvl))), lvl
    assert L.amrfld_restrict_level(b.ctx, p.hierarchy.base_level) == E_INVALID
    assert L.amrfld_restrict_level(b.ctx, p.hierarchy.max_level + 1) == E_INVALID
    a.close()
    b.close()
