"""Pins of the oracle's variants: the Minerbo flux limiter (the paper's collapse runs,
Sect. 5.1) and the theta-weighted step (Crank-Nicolson, named in Sect. 3.3.6 as the
remedy for the first-order time error), against closed forms and exact values."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft

from _util import oracle_from_problem
from oracle import DIRICHLET, lp_limiter, minerbo_limiter
from synth.configs import config_tiny, config_uniform


# ------------------------------------------------------------ Minerbo limiter
def test_minerbo_exact_values():
    assert minerbo_limiter(0.0) == pytest.approx(1.0 / 3.0, rel=1e-15)
    # both branches meet at R = 3/2: 2 / (3 + sqrt(36)) = 1 / (1 + 3/2 + sqrt(4)) = 2/9
    assert float(minerbo_limiter(1.5)) == pytest.approx(float(Fraction(2, 9)), rel=1e-15)
    assert float(minerbo_limiter(1.5 + 1e-12)) == pytest.approx(float(Fraction(2, 9)), rel=1e-11)
    # R = 2: 1 / (3 + sqrt(5)); R = 1/2: 2 / (3 + sqrt(12))
    assert float(minerbo_limiter(2.0)) == pytest.approx(1.0 / (3.0 + np.sqrt(5.0)), rel=1e-15)
    assert float(minerbo_limiter(0.5)) == pytest.approx(2.0 / (3.0 + np.sqrt(12.0)), rel=1e-15)


def test_minerbo_slope_continuous_at_the_junction():
    # d lambda / dR = -2/27 from both sides of R = 3/2
    h = 1e-6
    left = (minerbo_limiter(1.5) - minerbo_limiter(1.5 - h)) / h
    right = (minerbo_limiter(1.5 + h) - minerbo_limiter(1.5)) / h
    assert left == pytest.approx(-2.0 / 27.0, rel=1e-5)
    assert right == pytest.approx(-2.0 / 27.0, rel=1e-5)


def test_minerbo_limits_and_monotone():
    R = np.logspace(-6, 8, 2000)
    lam = minerbo_limiter(R)
    assert np.all(np.diff(lam) < 0)
    assert R[-1] * lam[-1] == pytest.approx(1.0, rel=1e-3)  # free streaming: lambda R -> 1
    # both limiters reduce to 1/3 in the diffusion limit and to 1/R in free streaming
    assert lam[0] == pytest.approx(float(lp_limiter(R[0])), rel=1e-5)
    assert R[-1] * float(lp_limiter(R[-1])) == pytest.approx(R[-1] * lam[-1], rel=1e-3)


# --------------------------------------------------------- theta-weighted step
def _dct_step(b, C, theta):
    n = b.shape[0]
    lam1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    g = (1.0 - (1.0 - theta) * C * lam) / (1.0 + theta * C * lam)
    return scipy.fft.idctn(scipy.fft.dctn(b, type=2, norm="ortho") * g, type=2, norm="ortho")


def _grid(o, level, v):
    n = 1 << level
    g = np.zeros((n, n, n))
    c = o.cells(level)
    g[c[:, 0], c[:, 1], c[:, 2]] = v
    return g


@pytest.mark.parametrize("theta", [0.5, 0.75])
def test_theta_step_is_the_dct_closed_form(theta):
    p = config_uniform(4, kmode="const", seed=5)
    o = oracle_from_problem(p, theta=theta, abs_floor=1e-16)
    b0 = _grid(o, 4, o.E[4])
    dt = 6.0 / 256
    o.solve_level(4, dt, DIRICHLET, tol=1e-14)
    ref = _dct_step(b0, dt * 256, theta)
    x = _grid(o, 4, o.E[4])
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-13


def test_theta_one_is_backward_euler_bitwise():
    p = config_tiny(3, base_level=3, max_level=5, p_refine=0.5)
    a = oracle_from_problem(p, theta=1.0)
    b = oracle_from_problem(p)
    a.advance_subcycled(p.dt_coarse, DIRICHLET, 1e-12)
    b.advance_subcycled(p.dt_coarse, DIRICHLET, 1e-12)
    for l in a.lev:
        assert np.array_equal(a.E[l], b.E[l])


def _semi_discrete_error(theta, k):
    # error at T against the exact solution of the spatially discrete system, exp(-T L)
    level, T = 4, 0.02
    p = config_uniform(level, kmode="const", seed=6)
    o = oracle_from_problem(p, theta=theta, abs_floor=0.0)
    b0 = _grid(o, level, o.E[level])
    n = 1 << level
    for _ in range(k):
        o.solve_level(level, T / k, DIRICHLET, tol=1e-14)
    lam1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    exact = scipy.fft.idctn(scipy.fft.dctn(b0, type=2, norm="ortho") * np.exp(-T * n * n * lam),
                            type=2, norm="ortho")
    return np.linalg.norm(_grid(o, level, o.E[level]) - exact) / np.linalg.norm(exact)


def test_crank_nicolson_second_order_backward_euler_first():
    cn = [_semi_discrete_error(0.5, k) for k in (8, 16, 32)]
    be = [_semi_discrete_error(1.0, k) for k in (8, 16, 32)]
    for i in range(2):
        assert 3.6 < cn[i] / cn[i + 1] < 4.4, cn
        assert 1.8 < be[i] / be[i + 1] < 2.2, be
    assert cn[-1] < 0.1 * be[-1]


def test_theta_system_symmetric_positive_definite_on_amr():
    p = config_tiny(4, base_level=3, max_level=5, p_refine=0.5)
    o = oracle_from_problem(p, theta=0.5)
    A1, b1, _ = o.assemble(5, p.dt_coarse / 4, DIRICHLET)
    A, b = o.theta_scheme(A1, b1, o.E[5][o.lev[5].leaf_slots])
    M = A.toarray()
    assert np.max(np.abs(M - M.T)) <= 1e-15 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(M).min() >= 1.0 - 1e-12
