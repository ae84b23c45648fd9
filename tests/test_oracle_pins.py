"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a closed form,
a hand-derived fixture, an invariant, a textbook routine, or brute force.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft
import scipy.linalg

from _util import oracle_from_problem
from oracle import (C2F, DIRICHLET, F2C, NEUMANN, OUTER, ROBIN, SAME, Oracle, dense_solve,
                    lp_limiter, pcg_jacobi)
from synth.configs import config_heat_gaussian, config_tiny, config_uniform
from synth.hierarchy import Hierarchy, random_balanced_hierarchy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid_of(o, level, v):
    n = 1 << level
    g = np.zeros((n, n, n))
    c = o.cells(level)
    g[c[:, 0], c[:, 1], c[:, 2]] = v
    return g


def _dct_solution(b_grid, C):
    """Exact solution of (I + C L) x = b for the cell-centred zero-flux Laplacian L."""
    n = b_grid.shape[0]
    lam1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    bh = scipy.fft.dctn(b_grid, type=2, norm="ortho")
    return scipy.fft.idctn(bh / (1.0 + C * lam), type=2, norm="ortho")


# ---------------------------------------------------------------- P1: closed form
@pytest.mark.parametrize("level,dtfac", [(3, 4.0), (4, 4.0), (4, 0.3), (5, 16.0)])
def test_uniform_level_matches_dct_closed_form(level, dtfac):
    p = config_uniform(level, kmode="const", seed=level)
    dx = 1.0 / (1 << level)
    dt = dtfac * dx * dx
    o = oracle_from_problem(p, abs_floor=1e-16)
    b = _grid_of(o, level, o.E[level])
    st = o.solve_level(level, dt, DIRICHLET, tol=1e-14)
    assert st["converged"]
    x = _grid_of(o, level, o.E[level])
    ref = _dct_solution(b, dt / dx ** 2)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-13


def test_constant_K_value_enters_as_scale():
    # K = 2.5 with dt is the same system as K = 1 with 2.5 dt.
    level = 4
    dx = 1.0 / (1 << level)
    p = config_uniform(level, kmode="const", seed=3)
    o = oracle_from_problem(p, K_const=2.5, abs_floor=1e-16)
    b = _grid_of(o, level, o.E[level])
    o.solve_level(level, 2.0 * dx * dx, DIRICHLET, tol=1e-14)
    ref = _dct_solution(b, 2.5 * 2.0)
    assert np.linalg.norm(_grid_of(o, level, o.E[level]) - ref) / np.linalg.norm(ref) < 1e-13


def test_face_mean_exact_for_layered_diffusivity():
    # Series conduction: with K constant inside each cell and the face value the harmonic
    # mean, the cell-centred scheme is exact, each cell adding dx / K to the resistance.
    # A slab with seeded K per x column and energies held at x = 0 and 1 (LP law with
    # rho kappa_R = 1e10 keeps lambda at 1/3 to ~1e-10, so K = c / (3 rho kappa_R) is set
    # per cell through rho) must reach the series-resistance profile at the cell centres.
    level, n = 3, 8
    ijk = np.array([(i, j, k) for k in range(4) for j in range(4) for i in range(4)], dtype=np.int32)
    Kx = 0.25 + 0.75 * np.random.default_rng(7).random(n)
    scale = 1e10
    o = Oracle(level, {level: ijk}, kmode="lp", kappa_R=1.0, c_light=3.0 * scale, outer={0: 4.0, 1: 0.5})
    c = o.cells(level)
    o.set_fields(level, scale / Kx[c[:, 0]], np.ones(len(c)))
    o.solve_level(level, 1e12, DIRICHLET, solver="dense")  # dt far beyond the relaxation time
    half = 0.5 / n / Kx  # resistance of half a cell
    F = (4.0 - 0.5) / (2.0 * half.sum())
    centre = 4.0 - F * (np.cumsum(2.0 * half) - half)
    got = _grid_of(o, level, o.E[level])
    assert np.max(np.abs(got - centre[:, None, None])) <= 1e-8 * 4.0


def test_lp_diffusivity_is_c_over_3_rho_kappa_in_the_diffusion_limit():
    # Optically thick limit of the LP law (R -> 0, lambda -> 1/3): K = c / (3 rho kappa_R).
    # With rho kappa_R = 2e10 and c = 6e10 (K = 1 to ~1e-10) one backward-Euler step of a
    # seeded field on a uniform level is the DCT closed form with C = dt / dx^2.
    level = 3
    dx = 1.0 / (1 << level)
    ijk = np.array([(i, j, k) for k in range(4) for j in range(4) for i in range(4)], dtype=np.int32)
    o = Oracle(level, {level: ijk}, kmode="lp", kappa_R=2.0, c_light=6e10, abs_floor=1e-16)
    c = o.cells(level)
    E0 = 1.0 + 0.1 * np.random.default_rng(11).random(len(c))
    o.set_fields(level, np.full(len(c), 1e10), E0)
    b = _grid_of(o, level, o.E[level])
    o.solve_level(level, 4.0 * dx * dx, DIRICHLET, tol=1e-14)
    ref = _dct_solution(b, 4.0)
    assert np.linalg.norm(_grid_of(o, level, o.E[level]) - ref) / np.linalg.norm(ref) < 1e-9


# ------------------------------------------------------- P2: hand-derived rows
def _two_level_oracle():
    octs = {1: np.array([[0, 0, 0]], dtype=np.int32), 2: np.array([[0, 0, 0]], dtype=np.int32)}
    o = Oracle(1, octs, kmode="const", K_const=1.0, robin_alpha=0.5)
    for l in (1, 2):
        c = o.cells(l)
        if l == 2:
            E = 1.0 + c[:, 0] + 2 * c[:, 1] + 4 * c[:, 2]
        else:
            E = 10.0 + c[:, 0] + 2 * c[:, 1] + 4 * c[:, 2]
            E[np.all(c == 0, axis=1)] = 20.0
        o.set_fields(l, np.ones(len(c)), E)
    return o


def _row_dict(o, level, A, b):
    L = o.lev[level]
    cells = L.cells[L.leaf_slots]
    names = [",".join(str(int(v)) for v in c) for c in cells]
    out = {}
    A = A.tocsr()
    for i, nm in enumerate(names):
        row = A.getrow(i)
        off = {names[j]: v for j, v in zip(row.indices, row.data) if j != i}
        out[nm] = (A[i, i], off, b[i])
    return out


def _frac(pair):
    return float(Fraction(pair[0], pair[1]))


def test_two_level_rows_match_hand_derivation():
    gold = json.load(open(os.path.join(GOLDEN, "two_level_rows.json")))
    o = _two_level_oracle()
    for mode in (DIRICHLET, NEUMANN, ROBIN):
        A, b, _ = o.assemble(2, gold["fine"]["dt"], mode)
        rows = _row_dict(o, 2, A, b)
        assert set(rows) == set(gold["fine"]["rows"])
        for nm, g in gold["fine"]["rows"].items():
            diag, off, bi = rows[nm]
            assert diag == pytest.approx(_frac(g["diag"]), rel=1e-15)
            assert bi == pytest.approx(_frac(g["b"]), rel=1e-15)
            assert set(off) == set(g["off"])
            for k, v in g["off"].items():
                assert off[k] == pytest.approx(v, rel=1e-15)
    cg = gold["coarse"]
    s = o.lev[1].lookup(np.array([[1, 0, 0]]))[0]
    o.reg[1][s, cg["register"]["1,0,0"]["dir"]] = cg["register"]["1,0,0"]["value"]
    for key, mode in (("dirichlet", DIRICHLET), ("neumann", NEUMANN), ("robin_0.5", ROBIN)):
        A, b, _ = o.assemble(1, cg["dt"], mode)
        rows = _row_dict(o, 1, A, b)
        for nm, g in cg["rows"][key].items():
            diag, off, bi = rows[nm]
            assert diag == pytest.approx(_frac(g["diag"]), rel=1e-15), (key, nm)
            assert bi == pytest.approx(_frac(g["b"]), rel=1e-14), (key, nm)
            assert set(off) == set(g["off"]), (key, nm)


# ------------------------------------------------------ brute-force face types
def _brute_face_types(h: Hierarchy):
    """For every leaf and direction, locate the cell just across the face by scanning
    every cell of every level (pure Python)."""
    cells = {}
    for l, octs in h.octs.items():
        for o in octs:
            for c in range(2):
                for b in range(2):
                    for a in range(2):
                        cells[(l, 2 * o[0] + a, 2 * o[1] + b, 2 * o[2] + c)] = True
    refined = set()
    for l, octs in h.octs.items():
        if l > h.base_level:
            for o in octs:
                refined.add((l - 1, int(o[0]), int(o[1]), int(o[2])))
    out = {}
    offs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    for (l, i, j, k) in cells:
        if (l, i, j, k) in refined:
            continue
        n = 1 << l
        for d, (a, b, c) in enumerate(offs):
            # a point just across the face centre, in units of the finest possible cell
            px = (i + 0.5 + 0.51 * a) / n
            py = (j + 0.5 + 0.51 * b) / n
            pz = (k + 0.5 + 0.51 * c) / n
            if not (0 <= px < 1 and 0 <= py < 1 and 0 <= pz < 1):
                out[(l, i, j, k, d)] = OUTER
                continue
            found = None
            for (m, x, y, z) in cells:
                s = 1 << m
                if (m, x, y, z) in refined:
                    continue
                if x <= px * s < x + 1 and y <= py * s < y + 1 and z <= pz * s < z + 1:
                    found = m
                    break
            if found == l:
                out[(l, i, j, k, d)] = SAME
            elif found == l + 1:
                out[(l, i, j, k, d)] = C2F
            elif found == l - 1:
                out[(l, i, j, k, d)] = F2C
            else:
                out[(l, i, j, k, d)] = -1
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_face_classification_matches_brute_force(seed):
    h = random_balanced_hierarchy(seed, 1, 4, p_refine=0.6)
    o = Oracle(h.base_level, h.octs, kmode="const")
    brute = _brute_face_types(h)
    for l, L in o.lev.items():
        for s in L.leaf_slots:
            i, j, k = (int(v) for v in L.cells[s])
            for d in range(6):
                assert L.ftype[s, d] == brute[(l, i, j, k, d)], (l, i, j, k, d)


# ------------------------------------------------ P3 symmetry and definiteness
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("mode", [DIRICHLET, NEUMANN, ROBIN])
def test_matrix_symmetric_spd_lambda_min_ge_1(seed, mode):
    p = config_tiny(seed, base_level=2, max_level=4, p_refine=0.5)
    o = oracle_from_problem(p)
    for l in o.lev:
        A, b, _ = o.assemble(l, p.dt_coarse / 2 ** (l - o.base), mode)
        if A.shape[0] == 0:
            continue
        M = A.toarray()
        assert np.array_equal(M, M.T)
        scipy.linalg.cholesky(M)
        assert np.linalg.eigvalsh(M).min() >= 1.0 - 1e-12
        off = M - np.diag(np.diag(M))
        assert np.all(off <= 0.0)
        assert np.all(np.diag(M) - 1.0 >= -off.sum(axis=1) * (1 - 1e-13))


# ---------------------------------------------- P2 / P7 dense solve certificate
@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_pcg_matches_cholesky_within_certificate(seed):
    p = config_tiny(seed, base_level=3, max_level=5, p_refine=0.4)
    o = oracle_from_problem(p)
    for l in o.lev:
        A, b, _ = o.assemble(l, p.dt_coarse / 2 ** (l - o.base), DIRICHLET)
        n = A.shape[0]
        if n == 0 or n > 3000:
            continue
        xs = dense_solve(A, b)
        x0 = o.E[l][o.lev[l].leaf_slots]
        x, st = pcg_jacobi(A, b, x0, 1e-13, 10000)
        assert st["converged"]
        res = np.linalg.norm(b - A @ x)
        # lambda_min(A) >= 1 gives ||x - x*|| <= ||b - A x||
        assert np.linalg.norm(x - xs) <= res * (1 + 1e-8) + 1e-14 * np.linalg.norm(xs)
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-12


# ------------------------------------------------------------ P4 conservation
def test_single_level_conserves_energy():
    p = config_uniform(4, kmode="lp", seed=5)
    o = oracle_from_problem(p)
    e0 = o.total_energy()
    st = o.solve_level(4, p.dt_coarse, DIRICHLET, tol=1e-13)
    n = st["n_leaf"]
    vol = (1.0 / 16) ** 3
    assert abs(o.total_energy() - e0) <= np.sqrt(n) * st["true_res"] * vol * 2 + 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_neumann_interfaces_conserve_dirichlet_drifts(seed):
    drift = {}
    for mode in (NEUMANN, DIRICHLET):
        p = config_tiny(seed, base_level=3, max_level=5, p_refine=0.5)
        o = oracle_from_problem(p)
        e0 = o.total_energy()
        o.advance_subcycled(p.dt_coarse, mode, tol=1e-13)
        drift[mode] = abs(o.total_energy() - e0) / e0
    assert drift[NEUMANN] < 1e-12
    assert drift[DIRICHLET] > 1e-6


def test_heat_pulse_neumann_conserves_over_steps():
    p = config_heat_gaussian(n_coarse_steps=2)
    o = oracle_from_problem(p)
    e0 = o.total_energy()
    for _ in range(2):
        o.advance_subcycled(p.dt_coarse, NEUMANN, tol=1e-13)
    assert abs(o.total_energy() - e0) / e0 < 1e-12


# --------------------------------------------------------- P5 fixed point
@pytest.mark.parametrize("mode", [DIRICHLET, NEUMANN, ROBIN])
@pytest.mark.parametrize("kmode", ["const", "lp"])
def test_constant_state_is_fixed_point(mode, kmode):
    h = random_balanced_hierarchy(4, 2, 4, p_refine=0.5)
    o = Oracle(h.base_level, h.octs, kmode=kmode)
    for l in o.lev:
        n = o.lev[l].n_slots
        rng = np.random.default_rng(l)
        o.set_fields(l, rng.uniform(0.5, 2.0, n), np.full(n, 3.25))
    o.advance_subcycled(0.05, mode, tol=1e-10)
    for st in o.history:
        assert st["iters"] == 0
    for l in o.lev:
        assert np.all(o.E[l] == 3.25)


# ------------------------------------------------------------ P6 Robin limits
@pytest.mark.parametrize("seed", [0, 1])
def test_robin_limits_equal_dirichlet_and_neumann(seed):
    p = config_tiny(seed, base_level=3, max_level=5, p_refine=0.5)
    o = oracle_from_problem(p)
    rng = np.random.default_rng(seed)
    for l in o.lev:
        o.reg[l][:] = rng.uniform(-1e-3, 1e-3, size=o.reg[l].shape)
    for l in o.lev:
        dt = p.dt_coarse / 2 ** (l - o.base)
        o.alpha = 1.0
        Ar, br, _ = o.assemble(l, dt, ROBIN)
        Ad, bd, _ = o.assemble(l, dt, DIRICHLET)
        assert np.array_equal(Ar.toarray(), Ad.toarray()) and np.array_equal(br, bd)
        o.alpha = 0.0
        Ar, br, _ = o.assemble(l, dt, ROBIN)
        An, bn, _ = o.assemble(l, dt, NEUMANN)
        assert np.array_equal(Ar.toarray(), An.toarray()) and np.array_equal(br, bn)


# ---------------------------------------------------- P8 analytic heat kernel
def _gaussian_with_images(x, t, s0=0.05, K=1.0):
    s2 = s0 * s0 + 2.0 * K * t
    out = np.full(len(x), (s0 * s0 / s2) ** 1.5)
    for d in range(3):
        g = np.zeros(len(x))
        for m in range(-4, 5):  # mirror images for the zero-flux walls at 0 and 1
            g += np.exp(-(x[:, d] - 0.5 - m) ** 2 / (2.0 * s2))
        out *= g
    return out + 1e-3


def _heat_error(k, steps, mode):
    p = config_heat_gaussian(n_coarse_steps=steps * k, dt_scale=1.0 / k)
    o = oracle_from_problem(p)
    for _ in range(p.n_coarse_steps):
        o.advance_subcycled(p.dt_coarse, mode, p.tol)
    t = p.dt_coarse * p.n_coarse_steps
    e2 = n2 = 0.0
    for l, L in o.lev.items():
        x = (L.cells[L.leaf_slots] + 0.5) / L.n
        a = _gaussian_with_images(x, t)
        e2 += np.sum((o.E[l][L.leaf_slots] - a) ** 2) * L.vol
        n2 += np.sum(a * a) * L.vol
    return np.sqrt(e2 / n2)


@pytest.mark.parametrize("mode", [DIRICHLET, NEUMANN])
def test_heat_pulse_first_order_in_time(mode):
    errs = [_heat_error(k, 1, mode) for k in (1, 2, 4, 8)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 1.7 < r < 2.3, (errs, ratios)
    assert errs[-1] < 0.06


# ------------------------------------------------------------ P9 the driver
def test_driver_without_refinement_is_one_solve():
    p = config_uniform(4, kmode="lp", seed=2)
    a = oracle_from_problem(p)
    b = oracle_from_problem(p)
    a.advance_subcycled(p.dt_coarse, DIRICHLET, tol=1e-12)
    b.solve_level(4, p.dt_coarse, DIRICHLET, tol=1e-12)
    assert np.array_equal(a.E[4], b.E[4])


def test_driver_fully_refined_base_is_two_half_steps():
    base = 3
    octs8 = np.array([[i, j, k] for i in range(4) for j in range(4) for k in range(4)], dtype=np.int32)
    octs16 = np.array([[i, j, k] for i in range(8) for j in range(8) for k in range(8)], dtype=np.int32)
    o = Oracle(base, {3: octs8, 4: octs16}, kmode="const", abs_floor=1e-16)
    for l in (3, 4):
        c = o.cells(l)
        x = (c + 0.5) / (1 << l)
        o.set_fields(l, np.ones(len(c)), 1.0 + np.sin(3 * x[:, 0]) * np.cos(2 * x[:, 1]) + x[:, 2] ** 2)
    b0 = _grid_of(o, 4, o.E[4])
    dt = 0.01
    o.advance_subcycled(dt, DIRICHLET, tol=1e-14)
    assert o.lev[3].leaf_slots.size == 0
    dx = 1.0 / 16
    ref = _dct_solution(_dct_solution(b0, 0.5 * dt / dx ** 2), 0.5 * dt / dx ** 2)
    x = _grid_of(o, 4, o.E[4])
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-13
    assert [h["level"] for h in o.history] == [4, 4, 3]


# ----------------------------------------------- P11 Levermore-Pomraning limiter
def test_lp_limiter_values_and_limits():
    for R, frac in ((0.0, Fraction(1, 3)), (1.0, Fraction(3, 10)), (3.0, Fraction(5, 24)),
                    (2.0, Fraction(4, 16))):
        assert lp_limiter(R) == pytest.approx(float(frac), rel=2e-16)
    R = np.logspace(-6, 8, 400)
    lam = lp_limiter(R)
    assert np.all(np.diff(lam) < 0)
    assert np.all(lam <= 1.0 / 3.0)
    assert abs(R[-1] * lam[-1] - 1.0) < 1e-7       # free streaming |F| -> c E
    # close to the exact Levermore-Pomraning form (coth R - 1/R) / R
    Rm = np.logspace(-2, 3, 200)
    exact = (1.0 / np.tanh(Rm) - 1.0 / Rm) / Rm
    assert np.max(np.abs(lp_limiter(Rm) / exact - 1.0)) < 0.08


# ----------------------------------------- gradient stencil on linear fields
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_gradient_exact_for_single_axis_linear_field_on_amr(seed, axis):
    # A field linear along one axis: across a coarser neighbour the centre-to-centre
    # distance along that axis is 3 dx / 2, so the difference quotient is exact there
    # too (transverse offsets of the coarse centre do not matter for such a field).
    h = random_balanced_hierarchy(seed, 2, 5, p_refine=0.6)
    o = Oracle(h.base_level, h.octs, kmode="lp")
    g = 0.7 - 0.5 * axis
    for l in o.lev:
        c = o.cells(l)
        x = (c + 0.5) / (1 << l)
        o.set_fields(l, np.full(len(c), 2.0), 5.0 + g * x[:, axis])
    n_f2c = 0
    for l, L in o.lev.items():
        grad = o.grad_E(l)
        interior = np.all(L.ftype[:, 2 * axis:2 * axis + 2] != OUTER, axis=1)
        n_f2c += np.sum(np.any(L.ftype[interior, 2 * axis:2 * axis + 2] == F2C, axis=1))
        assert np.allclose(grad[interior, axis], g, rtol=0, atol=1e-12)
        for b in range(3):
            if b != axis:
                # without a coarser neighbour along b the field is constant along b
                m = np.all(L.ftype[:, 2 * b:2 * b + 2] != F2C, axis=1)
                assert np.allclose(grad[m, b], 0.0, rtol=0, atol=1e-12)
        K = o.cell_K(l)
        m = interior & np.all((L.ftype != F2C) | (np.arange(6) // 2 == axis)[None, :], axis=1)
        R = abs(g) / (2.0 * o.E[l][m])
        assert np.allclose(K[m], (2 + R) / (6 + 3 * R + R * R) / 2.0, rtol=1e-13)
    assert n_f2c > 0


def test_restriction_of_linear_field_is_parent_centre_value():
    h = random_balanced_hierarchy(7, 2, 4, p_refine=0.6)
    o = Oracle(h.base_level, h.octs, kmode="const")
    g = np.array([0.3, 0.2, -0.9])
    for l in o.lev:
        c = o.cells(l)
        o.set_fields(l, np.ones(len(c)), np.zeros(len(c)) if l < o.max_level else 1.0 + ((c + 0.5) / (1 << l)) @ g)
    o.restrict(o.max_level)
    Lc = o.lev[o.max_level - 1]
    xc = (Lc.cells[Lc.refined] + 0.5) / Lc.n
    assert np.allclose(o.E[o.max_level - 1][Lc.refined], 1.0 + xc @ g, rtol=0, atol=1e-14)


# -------------------------------------------------- two-temperature coupling
def test_coupling_uniform_cell_matches_linearised_two_equation_backward_euler():
    # With uniform fields there is no diffusion; the reduced E equation plus the T
    # update must equal backward Euler of the two coupled ODEs with the emission
    # term linearised about T^n, solved as a 2x2 linear system.
    o = Oracle(2, {2: np.array([[i, j, k] for i in range(2) for j in range(2) for k in range(2)])},
               kmode="lp", kappa_P=3.0, c_light=2.0, a_rad=0.7, c_v=1.5)
    rho, E0, T0, dt = 1.3, 2.0, 1.1, 0.4
    n = o.lev[2].n_slots
    o.set_fields(2, np.full(n, rho), np.full(n, E0), np.full(n, T0))
    o.solve_level(2, dt, DIRICHLET, tol=1e-14)
    eta = 3.0 * rho * 2.0 * dt
    bT = 4 * 0.7 * T0 ** 3
    # unknowns (E', T'):  E' - E0 = eta (a T0^4 + bT (T' - T0) - E')
    #                     rho c_v (T' - T0) = -eta (a T0^4 + bT (T' - T0) - E')
    M = np.array([[1 + eta, -eta * bT], [-eta, rho * 1.5 + eta * bT]])
    rhs = np.array([E0 + eta * (0.7 * T0 ** 4 - bT * T0),
                    rho * 1.5 * T0 - eta * (0.7 * T0 ** 4 - bT * T0)])
    Ex, Tx = np.linalg.solve(M, rhs)
    assert np.allclose(o.E[2], Ex, rtol=1e-13)
    assert np.allclose(o.T[2], Tx, rtol=1e-13)
    # total energy E + rho c_v T is conserved by the linearised update
    assert abs((o.E[2][0] + rho * 1.5 * o.T[2][0]) - (E0 + rho * 1.5 * T0)) < 1e-13
