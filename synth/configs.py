"""Workload definitions: hierarchy, sampled fields and run parameters.

Each builder returns a :class:`Problem`.  Fields are callables
``f(level, cell_ijk) -> float64 array`` so that each consumer can sample them
in its own cell order.  Every value comes from seeded random numbers or closed
-form profiles; nothing here computes any part of the diffusion solve.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache
from typing import Callable, Optional

import numpy as np

from .fields import PowerLawField, cell_centres, gaussian_pulse
from .hierarchy import (Hierarchy, budgeted_hierarchy, centred_box_hierarchy,
                        random_balanced_hierarchy, uniform_hierarchy)

BC_MODES = {"dirichlet": 0, "neumann": 1, "robin": 2}


@dataclass
class Problem:
    name: str
    hierarchy: Hierarchy
    rho: Callable
    E: Callable
    T: Optional[Callable] = None
    kmode: str = "lp"            # "const" or "lp"
    K_const: float = 1.0
    kappa_R: float = 1.0
    kappa_P: float = 1.0
    c_light: float = 1.0
    a_rad: float = 1.0
    c_v: float = 1.0
    dt_coarse: float = 1.0
    bc_mode: str = "dirichlet"
    robin_alpha: float = 0.5
    tol: float = 1e-10
    n_coarse_steps: int = 1
    nsub: dict = field(default_factory=dict)   # level -> substeps per parent step (default 2)
    abs_floor: float = 1e-14
    linf_test: bool = True
    max_iter: int = 10000
    theta: float = 1.0           # 1: backward Euler, 1/2: Crank-Nicolson
    K_exp: float = 0.0           # kmode "power": K = K_const E^K_exp
    outer: Optional[dict] = None  # outer face direction -> Dirichlet value (others zero flux)
    info: dict = field(default_factory=dict)

    def nsub_of(self, level: int) -> int:
        return int(self.nsub.get(level, 2))


@lru_cache(maxsize=8)
def _field(n: int, slope: float, seed: int) -> PowerLawField:
    return PowerLawField(n, slope, seed)


def config_heat_gaussian(n_coarse_steps: int = 4, dt_scale: float = 1.0) -> Problem:
    """3D heat equation, constant K = 1, on a 16^3 base with the central 8^3 coarse
    cells refined once (512 octs).  Gaussian pulse (sigma 0.05) plus 1e-3 background;
    coarse dt = 4 dx^2 / K; Dirichlet interfaces; tolerance 1e-12."""
    h = centred_box_hierarchy(4, 4, 12, seed=11)

    def E(level, ijk):
        return gaussian_pulse(cell_centres(level, ijk))

    def rho(level, ijk):
        return np.ones(len(ijk))

    return Problem("heat_gaussian_16c_2lev", h, rho, E, kmode="const", K_const=1.0,
                   dt_coarse=dt_scale * 4.0 / 256.0, bc_mode="dirichlet", tol=1e-12,
                   n_coarse_steps=n_coarse_steps)


def _lognormal_rho(field_n: int, sigma: float, seed: int):
    g = _field(field_n, 4.0, seed)
    mu = -0.5 * sigma * sigma

    def rho(level, ijk):
        return np.exp(mu + sigma * g.sample(cell_centres(level, ijk)))

    def criterion(level, ijk):
        x = cell_centres(level, ijk)
        dx = 1.0 / (1 << level)
        s = np.zeros(len(x))
        for d in range(3):
            e = np.zeros(3)
            e[d] = dx
            s += (0.5 * sigma * (g.sample(x + e) - g.sample(x - e))) ** 2
        return np.sqrt(s)

    return rho, criterion


def _perturbed_E(field_n: int, seed: int, amp: float = 0.1):
    g = _field(field_n, 4.0, seed)

    def E(level, ijk):
        return 1.0 + amp * np.clip(g.sample(cell_centres(level, ijk)), -3.0, 3.0)

    return E


def config_fld_lognormal(base_level: int = 6, max_level: int = 9, field_n: int = 256,
                         quota: int = 156250, threshold: float = 0.2, sigma: float = 1.5,
                         rho_seed: int = 1401, E_seed: int = 1112, tol: float = 1e-10,
                         bc_mode: str = "dirichlet", robin_alpha: float = 0.5) -> Problem:
    """Flux-limited radiative diffusion on a density-gradient-refined hierarchy.

    Log-normal density (sigma_ln = ``sigma``, k^-4 spectrum, mean 1), kappa = c = 1,
    Levermore-Pomraning limited diffusivity, E = 1 + 10% k^-4 perturbation.  Levels
    ``base_level..max_level``; at each level the eligible cells with the largest
    |grad rho| dx / rho above ``threshold`` are refined, at most ``quota`` per level.
    Coarse dt = 4 dx_base^2 / K_thick with K_thick = c / (3 rho kappa) = 1/3."""
    rho, crit = _lognormal_rho(field_n, sigma, rho_seed)
    h, counts = budgeted_hierarchy(base_level, max_level, crit, threshold, quota, seed=rho_seed)
    E = _perturbed_E(field_n, E_seed)
    dxb = 1.0 / (1 << base_level)
    return Problem(f"fld_lognormal_L{base_level}-{max_level}", h, rho, E, kmode="lp",
                   dt_coarse=4.0 * dxb * dxb * 3.0, bc_mode=bc_mode, robin_alpha=robin_alpha,
                   tol=tol, n_coarse_steps=1, info={"refined_per_level": counts})


def _collapse_rho(contrast: float, field_n: int, seed: int, amp: float = 0.05):
    """Softened singular isothermal sphere at the box centre, rho_e (R_c^2 + eps^2) /
    (r^2 + eps^2) with rho_e = 1 and R_c = sqrt(3)/2 (centre to corner), eps set so that
    the centre-to-corner contrast is ``contrast``; times (1 + amp g) with g a clipped
    unit-variance k^-4 field."""
    g = _field(field_n, 4.0, seed)
    rc2 = 0.75
    eps2 = rc2 / (contrast - 1.0)

    def rho(level, ijk):
        x = cell_centres(level, ijk)
        r2 = np.sum((x - 0.5) ** 2, axis=1)
        return (rc2 + eps2) / (r2 + eps2) * (1.0 + amp * np.clip(g.sample(x), -3.0, 3.0))

    return rho, np.sqrt(rc2)


def config_collapse(base_level: int = 6, max_level: int = 13, jeans: float = 0.14, contrast: float = 1e6,
                    field_n: int = 256, rho_seed: int = 5000, E_seed: int = 5001, shared_dt_levels: int = 4,
                    tol: float = 1e-10) -> Problem:
    """Collapse-like hierarchy with coupled radiation and gas energy.

    Density: softened singular isothermal sphere (contrast ``contrast``) with a 5% k^-4
    perturbation.  A cell of level l is refined while dx_l > lambda_J / 8 with the Jeans
    length lambda_J = J (rho / rho_e)^(-1/2) R_c (2:1 balance kept), J = ``jeans``.
    E = 1 + 10% k^-4 perturbation, T = (E / a)^(1/4) (radiation and gas in equilibrium),
    kappa_R = kappa_P = c = c_v = a = 1, LP limiter, Dirichlet interfaces.  The first
    ``shared_dt_levels`` levels share the coarse dt (nsub = 1), the finer ones halve it
    (nsub = 2).  Coarse dt = 4 dx_base^2 / K_thick with K_thick = 1/3."""
    rho, rc = _collapse_rho(contrast, field_n, rho_seed)

    def criterion(level, ijk):
        return 8.0 * np.sqrt(rho(level, ijk)) / ((1 << level) * jeans * rc)

    h, counts = budgeted_hierarchy(base_level, max_level, criterion, 1.0, 1 << 62, seed=rho_seed)
    E = _perturbed_E(field_n, E_seed)

    def T(level, ijk):
        return E(level, ijk) ** 0.25

    top = max(h.levels)
    nsub = {l: (1 if l < base_level + shared_dt_levels else 2) for l in range(base_level + 1, top + 1)}
    dxb = 1.0 / (1 << base_level)
    return Problem(f"collapse_L{base_level}-{top}", h, rho, E, T=T, kmode="lp", dt_coarse=4.0 * dxb * dxb * 3.0,
                   bc_mode="dirichlet", tol=tol, n_coarse_steps=1, nsub=nsub,
                   info={"refined_per_level": counts, "jeans": jeans, "contrast": contrast})


def config_dirac_slab(base_level: int = 5, max_level: int = 8, widths=(0.25, 0.125, 0.0625), E0: float = 1e5,
                      dt_coarse: float = 3.125e-5, n_coarse_steps: int = 64, tol: float = 1e-8,
                      bc_mode: str = "dirichlet", robin_alpha: float = 0.5) -> Problem:
    """Plane-parallel energy pulse diffusing through nested refined slabs.

    E = 1 plus a pulse of E0 per unit area spread uniformly over the two central cell
    planes (x) of the finest level, each field value the cell average (so restriction
    reproduces it).  Level l + 1 covers the level-l cells whose centre lies within
    ``widths[l - base]`` of x = 0.5, over the whole y-z extent.  Constant K = 1,
    zero-flux outer faces, ``n_coarse_steps`` steps of ``dt_coarse``."""
    widths = list(widths)

    def criterion(level, ijk):
        k = level - base_level
        if k >= len(widths):
            return np.zeros(len(ijk))
        x = (ijk[:, 0] + 0.5) / (1 << level)
        return (np.abs(x - 0.5) < widths[k]).astype(np.float64)

    h, counts = budgeted_hierarchy(base_level, max_level, criterion, 0.5, 1 << 62, seed=17)
    top = max(h.levels)
    half = 1.0 / (1 << top)  # the pulse spans [0.5 - dx_f, 0.5 + dx_f]

    def E(level, ijk):
        dx = 1.0 / (1 << level)
        x0 = ijk[:, 0] * dx
        overlap = np.clip(np.minimum(x0 + dx, 0.5 + half) - np.maximum(x0, 0.5 - half), 0.0, None)
        return 1.0 + E0 * overlap / (2.0 * half) / dx

    def rho(level, ijk):
        return np.ones(len(ijk))

    return Problem(f"dirac_slab_L{base_level}-{top}", h, rho, E, kmode="const", K_const=1.0,
                   dt_coarse=dt_coarse, bc_mode=bc_mode, robin_alpha=robin_alpha, tol=tol,
                   n_coarse_steps=n_coarse_steps, info={"refined_per_level": counts, "E0": E0, "pulse_half": half})


def equilibrium_profile(x, a: float = 1.5, E_left: float = 4.0, E_right: float = 0.5):
    """Stationary solution of d/dx (E^a dE/dx) = 0 on [0, 1] with E(0) = E_left and
    E(1) = E_right: E^(a+1) is linear in x (Sect. 4.2)."""
    lo, hi = E_left ** (a + 1.0), E_right ** (a + 1.0)
    return ((hi - lo) * np.asarray(x, dtype=np.float64) + lo) ** (1.0 / (a + 1.0))


def config_equilibrium(base_level: int = 3, max_level: int = 7, a: float = 1.5, E_left: float = 4.0,
                       E_right: float = 0.5, threshold: float = 0.1, dt_coarse: float = 0.05,
                       n_coarse_steps: int = 200, tol: float = 1e-8, bc_mode: str = "dirichlet") -> Problem:
    """Equilibrium test with a nonlinear diffusivity (Sect. 4.2), plane-parallel in 3D.

    rho = 1, K = E^a (the diffusivity the stationary profile of the paper belongs to),
    Dirichlet values E_left at x = 0 and E_right at x = 1 held at the faces, zero flux
    through the y and z faces, and a step E = E_left for x < 1/2, E_right above as the
    initial state.  The mesh is the one the run settles on: a level-l cell is refined where
    the relative change of the stationary profile over one cell, dx |E'| / E, exceeds
    ``threshold`` at the cell or at one of its x neighbours (one buffer cell), over the
    whole y-z extent.  base_level == max_level gives a uniform grid."""

    def rel_change(level, x):
        dx = 1.0 / (1 << level)
        lo, hi = E_left ** (a + 1.0), E_right ** (a + 1.0)
        u = (hi - lo) * x + lo
        return dx * np.abs((hi - lo) / (a + 1.0) / u)

    def criterion(level, ijk):
        dx = 1.0 / (1 << level)
        x = (ijk[:, 0] + 0.5) * dx
        c = rel_change(level, x)
        for s in (-1.0, 1.0):
            xn = x + s * dx
            ok = (xn > 0.0) & (xn < 1.0)
            c = np.where(ok, np.maximum(c, rel_change(level, np.clip(xn, 0.0, 1.0))), c)
        return c

    h, counts = budgeted_hierarchy(base_level, max_level, criterion, threshold, 1 << 62, seed=23)
    top = max(h.levels)

    def E(level, ijk):
        return np.where((ijk[:, 0] + 0.5) / (1 << level) < 0.5, E_left, E_right)

    def rho(level, ijk):
        return np.ones(len(ijk))

    return Problem(f"equilibrium_L{base_level}-{top}", h, rho, E, kmode="power", K_const=1.0, K_exp=a,
                   outer={0: E_left, 1: E_right}, dt_coarse=dt_coarse, bc_mode=bc_mode, tol=tol,
                   n_coarse_steps=n_coarse_steps,
                   info={"refined_per_level": counts, "a": a, "E_left": E_left, "E_right": E_right})


def config_tiny(seed: int, base_level: int = 2, max_level: int = 4, kmode: str = "lp",
                bc_mode: str = "dirichlet", dt_scale: float = 1.0, p_refine: float = 0.35,
                tol: float = 1e-12, robin_alpha: float = 0.5) -> Problem:
    """Small random balanced hierarchy with a smooth log-normal density and a smooth
    positive energy field; sized so that dense direct solves are cheap."""
    h = random_balanced_hierarchy(seed, base_level, max_level, p_refine=p_refine)
    rho, _ = _lognormal_rho(16, 1.0, 7000 + seed)
    E = _perturbed_E(16, 8000 + seed, amp=0.3)
    dxb = 1.0 / (1 << base_level)
    return Problem(f"tiny_{seed}", h, rho, E, kmode=kmode, K_const=1.0,
                   dt_coarse=dt_scale * 4.0 * dxb * dxb * 3.0, bc_mode=bc_mode,
                   robin_alpha=robin_alpha, tol=tol, n_coarse_steps=1)


def config_uniform(level: int, kmode: str = "const", seed: int = 0, dt: float = None,
                   tol: float = 1e-12) -> Problem:
    """A single uniform level (no refinement)."""
    h = uniform_hierarchy(level, seed=seed)
    rho, _ = _lognormal_rho(16, 1.0, 9000 + seed)
    E = _perturbed_E(16, 9100 + seed, amp=0.3)
    dx = 1.0 / (1 << level)
    return Problem(f"uniform_L{level}", h, rho, E, kmode=kmode, K_const=1.0,
                   dt_coarse=dt if dt is not None else 4.0 * dx * dx, tol=tol)


@dataclass
class Patch:
    """One independent single-level problem on an n^3 box of cell size 1/n."""
    n: int
    dx: float
    dt: float
    rho: np.ndarray          # (n, n, n), x-major: index [i, j, k]
    E: np.ndarray
    face_mode: np.ndarray    # int32[6]: -x,+x,-y,+y,-z,+z ; 0 Dirichlet, 1 Neumann, 2 Robin
    face_ghost: np.ndarray   # float64[6] Dirichlet / Robin outside value
    face_flux: np.ndarray    # float64[6] inflow per face cell per step in E units (Neumann / Robin)


def patch_sizes(seed: int, n_patches: int, n_min: int = 8, n_max: int = 128):
    rng = np.random.default_rng(seed)
    u = rng.uniform(np.log(n_min), np.log(n_max), size=n_patches)
    return (2 * np.round(0.5 * np.exp(u))).astype(int)


def patch_batch(base_seed: int = 4000, n_patches: int = 512, n_min: int = 8, n_max: int = 128,
                sigma: float = 1.0, robin_alpha: float = 0.5):
    """Independent patches with log-uniform sizes, own log-normal density and energy,
    and a boundary mode drawn per face."""
    sizes = patch_sizes(base_seed, n_patches, n_min, n_max)
    out = []
    for i, n in enumerate(sizes):
        rng = np.random.default_rng(base_seed + i)
        n = int(max(2, n))
        fld = PowerLawField(n, 4.0, base_seed + i)
        rho = np.exp(-0.5 * sigma * sigma + sigma * fld.grid)
        e = PowerLawField(n, 4.0, base_seed + 100000 + i)
        E = 1.0 + 0.1 * np.clip(e.grid, -3.0, 3.0)
        dx = 1.0 / n
        dt = 4.0 * dx * dx * 3.0
        modes = rng.integers(0, 3, size=6).astype(np.int32)
        ghost = rng.uniform(0.9, 1.1, size=6)
        phi = rng.uniform(-0.05, 0.05, size=6)
        out.append(Patch(n, dx, dt, rho, E, modes, ghost, phi * dt / dx))
    return out, robin_alpha
