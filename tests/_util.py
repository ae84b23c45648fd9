"""Helpers shared by the tests: glue between the input generators and the oracle."""
from __future__ import annotations

import numpy as np

from oracle import Oracle
from synth.configs import BC_MODES


def oracle_from_problem(p, **over):
    kw = dict(kmode=p.kmode, K_const=p.K_const, kappa_R=p.kappa_R, kappa_P=p.kappa_P,
              c_light=p.c_light, a_rad=p.a_rad, c_v=p.c_v, robin_alpha=p.robin_alpha,
              abs_floor=p.abs_floor, linf_test=p.linf_test, max_iter=p.max_iter, nsub=p.nsub,
              theta=getattr(p, "theta", 1.0), K_exp=getattr(p, "K_exp", 0.0), outer=getattr(p, "outer", None))
    kw.update(over)
    o = Oracle(p.hierarchy.base_level, p.hierarchy.octs, **kw)
    for l in p.hierarchy.levels:
        c = o.cells(l)
        o.set_fields(l, p.rho(l, c), p.E(l, c), None if p.T is None else p.T(l, c))
    return o


def mode_of(p):
    return BC_MODES[p.bc_mode]


def cell_key(level, ijk):
    n = np.int64(1) << level
    ijk = np.asarray(ijk, dtype=np.int64)
    return (ijk[:, 0] * n + ijk[:, 1]) * n + ijk[:, 2]


def align(level, cells_a, vals_a, cells_b):
    """Reorder values given in cell order ``cells_a`` into cell order ``cells_b``."""
    ka, kb = cell_key(level, cells_a), cell_key(level, cells_b)
    oa = np.argsort(ka)
    pos = np.searchsorted(ka[oa], kb)
    assert np.all(ka[oa][pos] == kb)
    return np.asarray(vals_a)[oa[pos]]
