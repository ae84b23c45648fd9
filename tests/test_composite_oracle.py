"""Pins of the oracle's unique-time-step composite solve (all levels coupled in one
system with the finest time step, the method the paper compares its adaptive one with),
against facts that do not come from its own formulas: a closed form, exact reductions,
an invariant of the volume-scaled system, a direct solve, hand-derived entries and the
analytic heat kernel."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft

from _util import oracle_from_problem
from oracle import DIRICHLET, Oracle, dense_solve
from synth.configs import config_collapse, config_heat_gaussian, config_tiny, config_uniform


def _grid_of(o, level, v):
    n = 1 << level
    g = np.zeros((n, n, n))
    c = o.cells(level)
    g[c[:, 0], c[:, 1], c[:, 2]] = v
    return g


def _dct_solution(b, C):
    n = b.shape[0]
    lam1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    return scipy.fft.idctn(scipy.fft.dctn(b, type=2, norm="ortho") / (1.0 + C * lam), type=2, norm="ortho")


def test_uniform_level_composite_is_the_level_solve_bitwise():
    # one level: the composite rows are the level rows times V = dx^3, an exact power of
    # two, so Jacobi-PCG takes bitwise the same iterates; and both are the DCT solution
    p = config_uniform(4, kmode="const", seed=3)
    a = oracle_from_problem(p, abs_floor=1e-16)
    b = oracle_from_problem(p, abs_floor=1e-16)
    dt = 8.0 / 256
    b0 = _grid_of(a, 4, a.E[4])
    sa = a.solve_composite(dt, tol=1e-14)
    sb = b.solve_level(4, dt, DIRICHLET, tol=1e-14)
    assert sa["iters"] == sb["iters"]
    assert np.array_equal(a.E[4], b.E[4])
    ref = _dct_solution(b0, dt * 256)
    x = _grid_of(a, 4, a.E[4])
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("kmode", ["lp", "const"])
def test_composite_matrix_symmetric_and_bounded_below(seed, kmode):
    # V-scaled rows: symmetric, and V^-1/2 A V^-1/2 = I + (symmetric PSD coupling) >= 1
    p = config_tiny(seed, base_level=3, max_level=5, p_refine=0.5, kmode=kmode)
    o = oracle_from_problem(p)
    A, b, _, off = o.assemble_composite(p.dt_coarse / 4)
    M = A.toarray()
    assert np.max(np.abs(M - M.T)) <= 1e-14 * np.max(np.abs(M))
    vol = np.concatenate([np.full(len(o.lev[l].leaf_slots), o.lev[l].vol) for l in sorted(o.lev)])
    S = M / np.sqrt(vol)[:, None] / np.sqrt(vol)[None, :]
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() >= 1.0 - 1e-12
    # every off-diagonal entry is a coupling of two leaves that share a face
    assert np.all(M[~np.eye(len(M), dtype=bool)] <= 0.0)


def test_composite_pcg_within_certificate_of_cholesky():
    p = config_tiny(2, base_level=3, max_level=5, p_refine=0.5)
    o = oracle_from_problem(p)
    A, b, _, _ = o.assemble_composite(p.dt_coarse / 4)
    xs = dense_solve(A, b)
    from oracle import pcg_jacobi
    x0 = np.concatenate([o.E[l][o.lev[l].leaf_slots] for l in sorted(o.lev)])
    x, st = pcg_jacobi(A, b, x0, 1e-12, 10000, 0.0, True)
    vol = np.concatenate([np.full(len(o.lev[l].leaf_slots), o.lev[l].vol) for l in sorted(o.lev)])
    # lambda_min(V^-1/2 A V^-1/2) >= 1 gives ||x - x*||_V <= ||r||_{V^-1}
    err_v = np.sqrt(np.sum(vol * (x - xs) ** 2))
    res_v = np.sqrt(np.sum((b - A @ x) ** 2 / vol))
    assert err_v <= res_v * (1 + 1e-9) + 1e-300


@pytest.mark.parametrize("kmode", ["const", "lp"])
def test_composite_conserves_total_energy(kmode):
    # zero-flux outer boundary, no coupling: the flux between two leaves enters both rows
    # with opposite signs, so sum V E is unchanged by every composite solve
    p = config_tiny(4, base_level=3, max_level=5, p_refine=0.5, kmode=kmode)
    o = oracle_from_problem(p, abs_floor=0.0)
    e0 = o.total_energy()
    o.advance_unique(p.dt_coarse, tol=1e-14)
    assert abs(o.total_energy() - e0) <= 1e-12 * abs(e0)
    # the level-by-level method with Dirichlet interfaces does not conserve
    q = oracle_from_problem(p, abs_floor=0.0)
    q.advance_subcycled(p.dt_coarse, DIRICHLET, tol=1e-14)
    assert abs(q.total_energy() - e0) > 1e3 * abs(o.total_energy() - e0)


def test_composite_interface_entries_hand_derived():
    # heat_gaussian grid: base 16^3 (level 4), level 5 over coarse cells 4..11; K = 1,
    # dt = 1/128 (the fine step).  Coarse leaf (3, 6, 6) faces the refined cell (4, 6, 6):
    # V_c * dt / (3 dx_c^2) per facing fine cell = (1/16)^3 (1/128) / (3 (1/16)^2) = 1/6144.
    # Fine leaf (8, 12, 12): V_f (2/3) dt / dx_f^2 towards (3, 6, 6) = 1/6144 as well, and
    # its diagonal is V_f (1 + 5 * 8 + (2/3) * 8) with dt / dx_f^2 = 8.
    p = config_heat_gaussian()
    o = oracle_from_problem(p)
    A, _, _, off = o.assemble_composite(Fraction(1, 128).__float__())
    M = A.tocsr()

    def gidx(level, ijk):
        L = o.lev[level]
        s = L.lookup(np.array([ijk]))[0]
        return off[level] + L.leaf_of[s]

    c = gidx(4, (3, 6, 6))
    fines = [gidx(5, (8, j, k)) for j in (12, 13) for k in (12, 13)]
    expect = -float(Fraction(1, 6144))
    for f in fines:
        assert M[c, f] == pytest.approx(expect, rel=1e-15)
        assert M[f, c] == pytest.approx(expect, rel=1e-15)
    f0 = gidx(5, (8, 12, 12))
    assert M[f0, f0] == pytest.approx(float(Fraction(1, 32) ** 3 * (1 + 40 + Fraction(16, 3))), rel=1e-15)
    # the coarse row holds exactly the four facing fine cells across that face
    row = M.getrow(c)
    lvl5 = set(range(off[5], off[5] + len(o.lev[5].leaf_slots)))
    assert sorted(j for j in row.indices if j in lvl5) == sorted(fines)


def test_composite_schedule_counts():
    p = config_heat_gaussian()
    o = oracle_from_problem(p)
    assert o.advance_unique(p.dt_coarse, p.tol) == 2
    q = config_collapse(base_level=3, max_level=7, jeans=2.5, contrast=1e4, field_n=64, shared_dt_levels=2)
    o = oracle_from_problem(q)
    assert o.advance_unique(q.dt_coarse, q.tol) == 8
    assert [h["level"] for h in o.history] == [-1] * 8


def _gaussian_with_images(x, t, s0=0.05, K=1.0):
    s2 = s0 * s0 + 2.0 * K * t
    out = np.full(len(x), (s0 * s0 / s2) ** 1.5)
    for d in range(3):
        g = np.zeros(len(x))
        for m in range(-4, 5):  # mirror images for the zero-flux walls at 0 and 1
            g += np.exp(-(x[:, d] - 0.5 - m) ** 2 / (2.0 * s2))
        out *= g
    return out + 1e-3


def _unique_error(k):
    p = config_heat_gaussian(n_coarse_steps=k, dt_scale=1.0 / k)
    o = oracle_from_problem(p)
    for _ in range(p.n_coarse_steps):
        o.advance_unique(p.dt_coarse, p.tol)
    t = p.dt_coarse * p.n_coarse_steps
    e2 = n2 = 0.0
    for l, L in o.lev.items():
        x = (L.cells[L.leaf_slots] + 0.5) / L.n
        a = _gaussian_with_images(x, t)
        e2 += np.sum((o.E[l][L.leaf_slots] - a) ** 2) * L.vol
        n2 += np.sum(a * a) * L.vol
    return np.sqrt(e2 / n2)


def test_composite_heat_pulse_first_order_in_time():
    errs = [_unique_error(k) for k in (1, 2, 4, 8)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 1.7 < r < 2.3, (errs, ratios)
    assert errs[-1] < 0.06
