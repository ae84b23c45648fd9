"""The paper's linear diffusion test (Sect. 4.1, an energy pulse diffusing through
refined levels with Dirichlet, Robin and Neumann interfaces), run in 3D plane-parallel
form on the oracle at reduced size, against what the paper and the mathematics fix: the
solution does not depend on y and z; Neumann interfaces (alpha = 0) conserve the total
energy; Dirichlet and Robin interfaces gain a few percent, Robin less than Dirichlet
(Fig. 4 of the paper: up to ~8%); the profile stays within a few percent of the 1D heat
kernel of the pulse (Fig. 3)."""
import numpy as np
import pytest

from _util import oracle_from_problem
import oracle as ora
from synth.configs import config_dirac_slab

MODES = {1.0: ora.DIRICHLET, 0.5: ora.ROBIN, 0.0: ora.NEUMANN}


def analytic(x, t, E0, half, K=1.0):
    """1D heat kernel of E0 per unit area released at x = 0.5 on a background of 1; the
    uniform initial slab of width 2 half has the variance of the kernel at t0 = w^2/(24 K)."""
    tt = t + (2.0 * half) ** 2 / (24.0 * K)
    return 1.0 + E0 / np.sqrt(4.0 * np.pi * K * tt) * np.exp(-(x - 0.5) ** 2 / (4.0 * K * tt))


def _run(alpha, steps=16, scale=4.0):
    p = config_dirac_slab(base_level=3, max_level=6, dt_coarse=3.125e-5 * scale, n_coarse_steps=steps,
                          robin_alpha=alpha)
    o = oracle_from_problem(p, robin_alpha=alpha)
    e0 = o.total_energy()
    gains = []
    for _ in range(steps):
        o.advance_subcycled(p.dt_coarse, MODES[alpha], p.tol)
        gains.append((o.total_energy() - e0) / e0)
    return p, o, np.array(gains)


@pytest.fixture(scope="module")
def runs():
    return {a: _run(a) for a in (1.0, 0.5, 0.0)}


def test_solution_is_plane_parallel(runs):
    # the same to the solver tolerance at every y, z (boundary cells have fewer face
    # terms, so rounding differs per cell; a y or z indexing mistake would be O(1))
    p, o, _ = runs[1.0]
    for l, L in o.lev.items():
        x = L.cells[:, 0]
        e = o.E[l]
        for xi in np.unique(x):
            v = e[x == xi]
            assert np.max(np.abs(v - v[0])) <= 10 * p.tol * np.max(np.abs(v))


def test_neumann_conserves_dirichlet_and_robin_gain(runs):
    g1, g05, g0 = runs[1.0][2], runs[0.5][2], runs[0.0][2]
    assert np.max(np.abs(g0)) < 1e-8
    assert 0.0 < g1[-1] < 0.1
    assert 0.0 < g05[-1] < g1[-1]
    assert np.all(np.abs(g05) <= np.abs(g1) + 1e-12)


@pytest.mark.parametrize("alpha", [1.0, 0.5, 0.0])
def test_profile_close_to_heat_kernel(runs, alpha):
    p, o, _ = runs[alpha]
    T = p.dt_coarse * p.n_coarse_steps
    e2 = n2 = 0.0
    for l, L in o.lev.items():
        x = (L.cells[L.leaf_slots, 0] + 0.5) / L.n
        a = analytic(x, T, p.info["E0"], p.info["pulse_half"])
        e2 += np.sum((o.E[l][L.leaf_slots] - a) ** 2) * L.vol
        n2 += np.sum((a - 1.0) ** 2) * L.vol
    assert np.sqrt(e2 / n2) < 0.06
