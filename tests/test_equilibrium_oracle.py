"""Pins of the oracle's nonlinear equilibrium test (Sect. 4.2): power-law diffusivity,
Dirichlet values held at two faces of the box, relaxation to the stationary profile.

Against facts that do not come from the oracle's formulas: an exact reduction (exponent
0 is the constant-K law), an exact discrete solution (a linear profile is reproduced by
every consistent interface treatment, so it must be a fixed point of the adaptive and
the unique-time-step schemes), the closed-form stationary profile (E^(a+1) linear in x)
approached at close to second order on uniform grids, and the flux balance of a
conservative scheme at steady state."""
import numpy as np
import pytest

from _util import oracle_from_problem
import oracle as ora
from synth.configs import config_equilibrium, equilibrium_profile


def _leaves(o):
    return np.concatenate([o.E[l][o.lev[l].leaf_slots] for l in sorted(o.lev)])


def _steady(o, p, unique=False, mode=ora.DIRICHLET, max_steps=400, eps=1e-12):
    """Coarse steps until no leaf energy moves by more than eps; returns the step count."""
    prev = _leaves(o)
    for k in range(max_steps):
        if unique:
            o.advance_unique(p.dt_coarse, p.tol)
        else:
            o.advance_subcycled(p.dt_coarse, mode, p.tol)
        cur = _leaves(o)
        if np.abs(cur - prev).max() < eps:
            return k + 1
        prev = cur
    raise AssertionError("no steady state")


def _l2(o, a=1.5, E_left=4.0, E_right=0.5):
    """Volume-weighted L2 error of the leaves against the stationary profile."""
    e2 = 0.0
    for l, L in o.lev.items():
        x = (L.cells[L.leaf_slots, 0] + 0.5) / L.n
        e = o.E[l][L.leaf_slots] - equilibrium_profile(x, a, E_left, E_right)
        e2 += float(np.sum(e * e)) * L.vol
    return np.sqrt(e2)


def _boundary_fluxes(o, p):
    """Energy per unit time entering through the x = 0 face and through the x = 1 face,
    from the leaves on those faces: 2 K_f (E_b - E_i) / dx per unit area, K_f the
    harmonic mean of the cell's and the held value's K."""
    out = []
    for d in (0, 1):
        v, F = p.outer[d], 0.0
        for l, L in o.lev.items():
            m = (L.ftype[:, d] == ora.fld_oracle.OUTER) & ~L.refined
            Ki = p.K_const * o.E[l][m] ** p.K_exp
            Kb = p.K_const * v ** p.K_exp
            Kf = 2.0 * Ki * Kb / (Ki + Kb)
            F += float(np.sum(2.0 * Kf * (v - o.E[l][m]) / L.dx)) * L.dx ** 2
        out.append(F)
    return out


def test_zero_exponent_is_the_constant_law_bitwise():
    p = config_equilibrium(max_level=5, a=0.0, n_coarse_steps=2)
    a = oracle_from_problem(p)
    p.kmode, p.K_exp = "const", 0.0
    b = oracle_from_problem(p)
    for o in (a, b):
        o.advance_subcycled(p.dt_coarse, ora.DIRICHLET, p.tol)
    for l in a.lev:
        assert np.array_equal(a.E[l], b.E[l])


@pytest.mark.parametrize("method", ["dirichlet", "neumann", "robin", "unique"])
def test_linear_profile_is_a_fixed_point(method):
    # K = 1, E = 4 - 3.5 x on the refined mesh of the test: the held faces at dx / 2, the
    # fine-to-coarse faces at 3 dx / 2, restriction and the flux register are all exact
    # for a linear profile, so no step may move it
    p = config_equilibrium(max_level=5, tol=1e-13)
    p.K_exp = 0.0
    p.E = lambda level, ijk: 4.0 - 3.5 * (ijk[:, 0] + 0.5) / (1 << level)
    o = oracle_from_problem(p, abs_floor=1e-16)
    e0 = {l: o.E[l].copy() for l in o.lev}
    if method == "unique":
        o.advance_unique(p.dt_coarse, p.tol)
    else:
        o.advance_subcycled(p.dt_coarse, {"dirichlet": ora.DIRICHLET, "neumann": ora.NEUMANN,
                                          "robin": ora.ROBIN}[method], p.tol)
    for l, L in o.lev.items():
        s = L.leaf_slots
        assert np.max(np.abs(o.E[l][s] - e0[l][s])) <= 1e-11, (method, l)


@pytest.mark.parametrize("a", [1.5, -1.5])
def test_uniform_grids_approach_the_closed_form_at_near_second_order(a):
    # a = 1.5: the profile the paper prints; a = -1.5: K = E^-1.5, the power an opacity
    # kappa_R proportional to E^1.5 gives in the diffusion limit; both have E^(a+1)
    # linear in x
    errs = []
    for lv in (3, 4, 5):
        p = config_equilibrium(base_level=lv, max_level=lv, a=a, E_left=4.0, E_right=0.5)
        o = oracle_from_problem(p)
        _steady(o, p)
        errs.append(_l2(o, a))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(r > 2.8 for r in ratios), (errs, ratios)
    assert errs[-1] < 0.02, errs


@pytest.fixture(scope="module")
def amr_steady():
    out = {}
    for unique in (False, True):
        p = config_equilibrium(max_level=5, tol=1e-10)
        o = oracle_from_problem(p)
        _steady(o, p, unique=unique)
        out[unique] = (o, p)
    return out


def test_unique_step_balances_the_boundary_fluxes(amr_steady):
    # the composite system is conservative: at steady state what enters at x = 0
    # leaves at x = 1; the level-by-level scheme with Dirichlet interfaces is not
    o, p = amr_steady[True]
    f_in, f_out = _boundary_fluxes(o, p)
    assert abs(f_in + f_out) <= 1e-8 * abs(f_in)
    exact = (4.0 ** 2.5 - 0.5 ** 2.5) / 2.5  # flux of the stationary profile
    assert abs(f_in - exact) <= 0.02 * exact
    q, p = amr_steady[False]
    g_in, g_out = _boundary_fluxes(q, p)
    assert abs(g_in + g_out) > 1e-4 * abs(g_in)
    assert abs(g_in - exact) <= 0.02 * exact


def test_adaptive_and_unique_steady_states_agree(amr_steady):
    # both methods settle within the discretisation error of the profile, and close to
    # each other (the same mesh, the same stationary problem but for the interface
    # fluxes); the refined mesh does as well as the uniform grid of its finest cells
    (o, _), (q, _) = amr_steady[True], amr_steady[False]
    eu, ea = _l2(o), _l2(q)
    assert eu < 0.02 and ea < 0.02
    assert abs(eu - ea) <= 0.15 * eu
    diff = np.sqrt(sum(float(np.sum((o.E[l] - q.E[l])[L.leaf_slots] ** 2)) * L.vol for l, L in o.lev.items()))
    assert diff <= 0.5 * eu
