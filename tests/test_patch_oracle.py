"""Pins of the batch-form patch oracle against closed forms and invariants."""
import numpy as np
import pytest
import scipy.fft

from oracle.patch_oracle import DIRICHLET, NEUMANN, ROBIN, patch_advance, patch_system


def _dct_solution(b, C):
    n = b.shape[0]
    lam1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    return scipy.fft.idctn(scipy.fft.dctn(b, type=2, norm="ortho") / (1.0 + C * lam), type=2, norm="ortho")


def _fields(n, seed):
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    E = 1.0 + 0.3 * np.sin(2 * np.pi * X + seed) * np.cos(np.pi * Y) + 0.1 * Z
    rho = np.exp(0.5 * rng.standard_normal((n, n, n)) * 0.2)
    return rho, E


@pytest.mark.parametrize("n", [6, 10])
def test_zero_flux_constant_K_is_dct_closed_form(n):
    rho, E = _fields(n, 1)
    dx, dt = 1.0 / n, 3.0 / n ** 2
    Ex, hist = patch_advance(rho, E, dx, dt, [NEUMANN] * 6, [0.0] * 6, [0.0] * 6, 1, 1e-14,
                             kmode="const", K_const=1.0, abs_floor=1e-16)
    ref = _dct_solution(E, dt / dx ** 2)
    assert np.linalg.norm(Ex - ref) / np.linalg.norm(ref) < 1e-13


def test_neumann_inflow_enters_exactly():
    n = 8
    rho, E = _fields(n, 2)
    flux = [0.01, -0.02, 0.005, 0.0, 0.03, -0.01]
    Ex, hist = patch_advance(rho, E, 1.0 / n, 2.0 / n ** 2, [NEUMANN] * 6, [0.0] * 6, flux, 3, 1e-13)
    expected = E.sum() + 3 * n * n * sum(flux)
    assert abs(Ex.sum() - expected) < 1e-9


def test_dirichlet_steady_state_is_linear():
    n = 8
    rho, E = _fields(n, 3)
    g0, g1 = 2.0, 0.5
    modes = [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN]
    Ex, _ = patch_advance(rho, E, 1.0 / n, 1e9, modes, [g0, g1, 0, 0, 0, 0], [0.0] * 6, 1, 1e-15,
                          kmode="const", K_const=1.0, abs_floor=0.0, linf_test=False)
    i = np.arange(n)
    prof = g0 + (g1 - g0) * (i + 1) / (n + 1)
    assert np.allclose(Ex, prof[:, None, None], rtol=0, atol=1e-7)


@pytest.mark.parametrize("mode", [DIRICHLET, NEUMANN, ROBIN])
def test_constant_state_fixed_point(mode):
    n = 6
    rho, _ = _fields(n, 4)
    E = np.full((n, n, n), 1.7)
    Ex, hist = patch_advance(rho, E, 1.0 / n, 0.3, [mode] * 6, [1.7] * 6, [0.0] * 6, 2, 1e-10)
    assert all(h["iters"] == 0 for h in hist)
    assert np.all(Ex == 1.7)


def test_robin_limits():
    n = 6
    rho, E = _fields(n, 5)
    modes = [ROBIN] * 6
    g = [1.1, 0.9, 1.0, 1.05, 0.95, 1.2]
    f = [0.01, -0.01, 0.02, 0.0, -0.03, 0.004]
    A1, b1 = patch_system(rho, E, 1 / n, 0.1, modes, g, f, alpha=1.0)
    Ad, bd = patch_system(rho, E, 1 / n, 0.1, [DIRICHLET] * 6, g, f)
    assert np.array_equal(A1.toarray(), Ad.toarray()) and np.array_equal(b1, bd)
    A0, b0 = patch_system(rho, E, 1 / n, 0.1, modes, g, f, alpha=0.0)
    An, bn = patch_system(rho, E, 1 / n, 0.1, [NEUMANN] * 6, g, f)
    assert np.array_equal(A0.toarray(), An.toarray()) and np.array_equal(b0, bn)


def test_patch_matrix_spd():
    n = 6
    rho, E = _fields(n, 6)
    A, _ = patch_system(rho, E, 1 / n, 0.2, [ROBIN, DIRICHLET, NEUMANN, ROBIN, DIRICHLET, NEUMANN],
                        [1.0] * 6, [0.0] * 6, alpha=0.3)
    M = A.toarray()
    assert np.array_equal(M, M.T)
    assert np.linalg.eigvalsh(M).min() >= 1.0 - 1e-12
