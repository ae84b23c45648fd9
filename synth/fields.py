"""Seeded scalar fields sampled at AMR cell centres."""
from __future__ import annotations

import numpy as np


def cell_centres(level: int, ijk: np.ndarray) -> np.ndarray:
    """Cell-centre positions in the unit box of level-``level`` cells ``ijk``."""
    return (np.asarray(ijk, dtype=np.float64) + 0.5) / float(1 << level)


class PowerLawField:
    """Periodic Gaussian random field on an ``n^3`` grid with power spectrum
    ``P(k) ~ k**-slope`` (zero mean, unit variance), sampled anywhere in the unit
    box by periodic trilinear interpolation between grid-cell centres."""

    def __init__(self, n: int, slope: float, seed: int):
        rng = np.random.default_rng(seed)
        white = rng.standard_normal((n, n, n))
        spec = np.fft.rfftn(white)
        kx = np.fft.fftfreq(n) * n
        kz = np.fft.rfftfreq(n) * n
        k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
        amp = np.zeros_like(k2)
        nz = k2 > 0
        amp[nz] = k2[nz] ** (-slope / 4.0)  # sqrt(P(k)) = k^(-slope/2)
        spec *= amp
        g = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
        g -= g.mean()
        g /= g.std()
        self.n = n
        self.grid = g

    def sample(self, x: np.ndarray) -> np.ndarray:
        """Trilinear periodic interpolation at positions ``x`` (shape (m, 3))."""
        n = self.n
        u = np.asarray(x, dtype=np.float64) * n - 0.5
        i0 = np.floor(u).astype(np.int64)
        w = u - i0
        i0 %= n
        i1 = (i0 + 1) % n
        g = self.grid
        out = np.zeros(len(u))
        for a in (0, 1):
            ia = i1[:, 0] if a else i0[:, 0]
            wa = w[:, 0] if a else 1.0 - w[:, 0]
            for b in (0, 1):
                ib = i1[:, 1] if b else i0[:, 1]
                wb = w[:, 1] if b else 1.0 - w[:, 1]
                for c in (0, 1):
                    ic = i1[:, 2] if c else i0[:, 2]
                    wc = w[:, 2] if c else 1.0 - w[:, 2]
                    out += wa * wb * wc * g[ia, ib, ic]
        return out


def gaussian_pulse(x: np.ndarray, centre=(0.5, 0.5, 0.5), sigma: float = 0.05,
                   background: float = 1e-3) -> np.ndarray:
    """``exp(-r^2 / (2 sigma^2)) + background`` at positions ``x``."""
    r2 = np.sum((np.asarray(x) - np.asarray(centre)) ** 2, axis=1)
    return np.exp(-r2 / (2.0 * sigma * sigma)) + background
