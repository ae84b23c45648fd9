"""The paper's linear diffusion test (Sect. 4.1) on the GPU: the plane-parallel energy
pulse through refined slabs with Dirichlet, Robin and Neumann interfaces.

Reduced size: parity with the oracle at every coarse step (the protocol of the level
tests: equal counts and 1e-12, else fixed counts).  Full size (levels 5..8, 2.79 M cells,
64 coarse steps of the paper's 3.125e-5): Neumann conserves the total energy, Dirichlet
and Robin gain a few percent with Robin below Dirichlet, the profile is within a few
percent of the heat kernel, and the solution does not depend on y and z."""
import numpy as np
import pytest

import oracle as ora
from synth.configs import config_dirac_slab
from test_dirac_oracle import analytic
from test_gpu_parity import _parity_protocol

pytestmark = pytest.mark.gpu

MODES = {1.0: ora.DIRICHLET, 0.5: ora.ROBIN, 0.0: ora.NEUMANN}


@pytest.mark.parametrize("alpha", [1.0, 0.5, 0.0])
def test_dirac_parity_reduced(alpha):
    p = config_dirac_slab(base_level=3, max_level=6, dt_coarse=1.25e-4, n_coarse_steps=16, robin_alpha=alpha)
    how = _parity_protocol(p, MODES[alpha], steps=16)
    print(f"alpha {alpha}: {how}")


def _leaf_sum(s, p, l, v):
    c = s.cells(l)
    leaf = np.ones(len(c), dtype=bool)
    if l + 1 in p.hierarchy.octs:
        par = np.asarray(p.hierarchy.octs[l + 1], dtype=np.int64)
        n = np.int64(1) << l
        kc = (c[:, 0].astype(np.int64) * n + c[:, 1]) * n + c[:, 2]
        kp = (par[:, 0] * n + par[:, 1]) * n + par[:, 2]
        leaf = ~np.isin(kc, kp)
    return leaf


def test_dirac_full_size():
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    res = {}
    for alpha in (1.0, 0.5, 0.0):
        p = config_dirac_slab(robin_alpha=alpha)
        s = solver_from_problem(p)
        leaves = {l: _leaf_sum(s, p, l, None) for l in p.hierarchy.levels}

        def total():
            return sum(float(to_numpy(s.E(l))[leaves[l]].sum()) / float(1 << (3 * l)) for l in p.hierarchy.levels)

        e0 = total()
        gains = []
        for k in range(p.n_coarse_steps):
            s.advance(p.dt_coarse, MODES[alpha], p.tol)
            if k % 8 == 7:
                gains.append((total() - e0) / e0)
        T = p.dt_coarse * p.n_coarse_steps
        e2 = n2 = 0.0
        for l in p.hierarchy.levels:
            e = to_numpy(s.E(l))
            c = s.cells(l)
            m = leaves[l]
            x = (c[m, 0] + 0.5) / (1 << l)
            a = analytic(x, T, p.info["E0"], p.info["pulse_half"])
            e2 += np.sum((e[m] - a) ** 2) / float(1 << (3 * l))
            n2 += np.sum((a - 1.0) ** 2) / float(1 << (3 * l))
            for xi in np.unique(c[:, 0]):
                v = e[c[:, 0] == xi]
                assert np.max(np.abs(v - v[0])) <= 10 * p.tol * np.max(np.abs(v))
        s.close()
        res[alpha] = (np.array(gains), float(np.sqrt(e2 / n2)))
        print(f"alpha {alpha}: energy gain {gains[-1]:+.3e} (max {max(gains, key=abs):+.3e}), "
              f"L2 error vs heat kernel {res[alpha][1]:.3e}")
    g1, g05, g0 = res[1.0][0], res[0.5][0], res[0.0][0]
    assert np.max(np.abs(g0)) < 1e-7
    assert 0.0 < g05[-1] < g1[-1] < 0.1
    for a in res:
        assert res[a][1] < 0.06
