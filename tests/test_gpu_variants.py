"""The Minerbo limiter and the theta-weighted (Crank-Nicolson) step on the GPU against
the oracle: per-step parity on AMR hierarchies (equal counts and 1e-12, else fixed
counts), the theta step against its DCT closed form, and the rejected combinations."""
import numpy as np
import pytest
import scipy.fft

import oracle as ora
from oracle.patch_oracle import patch_advance
from synth.configs import config_tiny, config_uniform, patch_batch
from test_gpu_parity import MODES, _parity_protocol

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("mode", ["dirichlet", "neumann", "robin"])
def test_minerbo_amr_parity(seed, mode):
    p = config_tiny(seed, base_level=3, max_level=5, p_refine=0.5, kmode="minerbo", tol=1e-12)
    print(f"minerbo seed {seed} {mode}: {_parity_protocol(p, MODES[mode], steps=2)}")


def _minerbo_batch(patches, alpha, tol, max_iter, abs_floor):
    from paper_1401_1112_amd import K_MINERBO
    from paper_1401_1112_amd.solver import BatchSolver
    s = BatchSolver(robin_alpha=alpha, max_iter=max_iter, abs_floor=abs_floor)
    res, _ = s.solve(patches, 1, tol, kmode=K_MINERBO, raise_on_error=False)
    it = [x["iters"] for x in s.stats()]
    s.close()
    out = []
    for q, p in enumerate(patches):
        e, h = patch_advance(p.rho, p.E, p.dx, p.dt, p.face_mode, p.face_ghost, p.face_flux, 1, tol, alpha=alpha,
                             kmode="minerbo", max_iter=max_iter, abs_floor=abs_floor)
        out.append((it[q], h[0]["iters"], float(np.linalg.norm(res[q] - e) / np.linalg.norm(e))))
    return out


def test_minerbo_batch_parity():
    # same counts and 1e-12; where a count differs, every solve at the largest count, tol 0
    patches, alpha = patch_batch(5100, 6, n_min=4, n_max=16)
    out = _minerbo_batch(patches, alpha, 1e-12, 10000, 1e-14)
    if any(g != o for g, o, _ in out):
        n_fix = max(max(g, o) for g, o, _ in out)
        out = _minerbo_batch(patches, alpha, 0.0, n_fix, 0.0)
        assert all(g == o == n_fix for g, o, _ in out), out
    assert max(r for _, _, r in out) <= 1e-12, out


@pytest.mark.parametrize("seed", [0, 2])
@pytest.mark.parametrize("kmode", ["lp", "const"])
def test_crank_nicolson_amr_parity(seed, kmode):
    p = config_tiny(seed, base_level=3, max_level=5, p_refine=0.5, kmode=kmode, tol=1e-12)
    p.theta = 0.5
    print(f"theta 0.5 seed {seed} {kmode}: {_parity_protocol(p, ora.DIRICHLET, steps=2)}")


def test_crank_nicolson_closed_form():
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    level, theta = 5, 0.5
    p = config_uniform(level, kmode="const", seed=7)
    p.theta = theta
    s = solver_from_problem(p, abs_floor=1e-16)
    n = 1 << level
    c = s.cells(level)
    b = np.zeros((n, n, n))
    b[c[:, 0], c[:, 1], c[:, 2]] = p.E(level, c)
    dt = 12.0 / n ** 2
    s.solve_level(level, dt, 0, 1e-14)
    lam1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    C = dt * n * n
    g = (1.0 - (1.0 - theta) * C * lam) / (1.0 + theta * C * lam)
    ref = scipy.fft.idctn(scipy.fft.dctn(b, type=2, norm="ortho") * g, type=2, norm="ortho")[c[:, 0], c[:, 1], c[:, 2]]
    x = to_numpy(s.E(level))
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-13
    s.close()


def test_theta_rejections():
    from paper_1401_1112_amd import AmrfldError, BC_NEUMANN
    from paper_1401_1112_amd.solver import HierarchySolver, solver_from_problem
    p = config_tiny(0, base_level=3, max_level=4, p_refine=0.5)
    p.theta = 0.5
    s = solver_from_problem(p)
    with pytest.raises(AmrfldError):
        s.advance(p.dt_coarse, BC_NEUMANN, 1e-10)
    with pytest.raises(AmrfldError):
        s.advance_unique(p.dt_coarse, 1e-10)
    s.close()
    with pytest.raises(AmrfldError):
        HierarchySolver(p.hierarchy.base_level, p.hierarchy.octs, theta=0.3)


def test_crank_nicolson_persistent_and_mixed():
    # the theta-weighted step through the other solve forms: one persistent launch per
    # solve gives the host-polled result bitwise; FP32 inner solves with FP64 refinement
    # meet the threshold on the FP64 true residual and agree with FP64
    from paper_1401_1112_amd import MIXED
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    p = config_tiny(1, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-10)
    p.theta = 0.5
    out = {}
    for name, kw in (("polled", {}), ("persistent", {"persistent": True}), ("mixed", {"precision": MIXED})):
        s = solver_from_problem(p, **kw)
        for _ in range(2):
            s.advance(p.dt_coarse, 0, p.tol)
            for st in s.stats():
                thr = max(p.tol * st["rnorm0"], p.abs_floor * st["bnorm"])
                assert st["converged"] == 1 and st["true_rel_res"] * st["rnorm0"] <= 1.05 * thr, (name, st)
        out[name] = ({l: to_numpy(s.E(l)) for l in p.hierarchy.levels}, [x["iters"] for x in s.stats()])
        s.close()
    a, ia = out["polled"]
    b, ib = out["persistent"]
    assert ia == ib and all(np.array_equal(a[l], b[l]) for l in a)
    m, _ = out["mixed"]
    for l in a:
        assert np.linalg.norm(m[l] - a[l]) <= 1e-8 * np.linalg.norm(a[l])
