"""CPU FP64 oracle of the batch form: one independent patch (TEST INFRASTRUCTURE).

A patch is a box of n^3 cells of size dx advanced by backward Euler (Sect. 3.1,
eq. Er_imp1).  Interior faces are same-level faces with C = K_f dt / dx^2
(harmonic face diffusivity).  Each of the six boundary faces takes one of the
level-interface rows of Sect. 3.2 with a given outside energy g and inflow F:
Dirichlet diag += C, b += C g; Neumann b += F; Robin diag += alpha C,
b += alpha C g + (1 - alpha) F, where C = K_i dt / dx^2 (the outside cell is
taken with the boundary cell's own diffusivity, so the harmonic mean is K_i).
The diffusivity and the gradient for R follow the level oracle (the boundary
neighbour is the cell itself at distance dx).  Arrays are indexed [i, j, k]
with i along x.

Parity unpinned: the boundary coefficient C = K_i dt / dx^2 with the cell's own
diffusivity (patches are not in the paper; the closed forms pin the rows, not this
choice of the outside diffusivity).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fld_oracle import harmonic_mean, lp_limiter, minerbo_limiter, pcg_jacobi

DIRICHLET, NEUMANN, ROBIN = 0, 1, 2


def patch_K(rho, E, dx, kmode="lp", K_const=1.0, kappa_R=1.0, c_light=1.0):
    if kmode == "const":
        return np.full(E.shape, float(K_const))
    g2 = np.zeros(E.shape)
    for ax in range(3):
        Ep = np.concatenate([np.take(E, np.arange(1, E.shape[ax]), axis=ax),
                             np.take(E, [E.shape[ax] - 1], axis=ax)], axis=ax)
        Em = np.concatenate([np.take(E, [0], axis=ax),
                             np.take(E, np.arange(0, E.shape[ax] - 1), axis=ax)], axis=ax)
        g = (Ep - Em) / (dx + dx)
        g2 += g * g
    R = np.sqrt(g2) / (rho * kappa_R * E)
    lam = minerbo_limiter(R) if kmode == "minerbo" else lp_limiter(R)
    return c_light * lam / (rho * kappa_R)


def patch_system(rho, E, dx, dt, modes, ghosts, fluxes, alpha=0.5, kmode="lp", K_const=1.0,
                 kappa_R=1.0, c_light=1.0):
    """CSR matrix and right-hand side over the cells in [i, j, k] C order."""
    n = E.shape[0]
    K = patch_K(rho, E, dx, kmode, K_const, kappa_R, c_light)
    coef = dt / (dx * dx)
    idx = np.arange(n ** 3).reshape(n, n, n)
    diag = np.ones((n, n, n))
    b = E.copy()
    rows, cols, vals = [], [], []
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        lo, hi = tuple(lo), tuple(hi)
        C = harmonic_mean(K[lo], K[hi]) * coef
        diag[lo] += C
        diag[hi] += C
        rows += [idx[lo].ravel(), idx[hi].ravel()]
        cols += [idx[hi].ravel(), idx[lo].ravel()]
        vals += [-C.ravel(), -C.ravel()]
        for side in (0, 1):
            face = [slice(None)] * 3
            face[ax] = 0 if side == 0 else n - 1
            face = tuple(face)
            d = 2 * ax + side
            m = int(modes[d])
            w = {DIRICHLET: 1.0, NEUMANN: 0.0, ROBIN: alpha}[m]
            Cb = K[face] * coef
            diag[face] += w * Cb
            b[face] += w * Cb * ghosts[d] + (1.0 - w) * fluxes[d]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n ** 3, n ** 3))
    A.sum_duplicates()
    A.sort_indices()
    return A, b.ravel()


def patch_advance(rho, E, dx, dt, modes, ghosts, fluxes, n_steps, tol, alpha=0.5, kmode="lp",
                  max_iter=10000, abs_floor=1e-14, linf_test=True, **kw):
    """n_steps backward-Euler steps; returns the final E and the per-step stats."""
    E = np.array(E, dtype=np.float64)
    hist = []
    for _ in range(n_steps):
        A, b = patch_system(rho, E, dx, dt, modes, ghosts, fluxes, alpha, kmode, **kw)
        x, st = pcg_jacobi(A, b, E.ravel(), tol, max_iter, abs_floor, linf_test)
        st["true_res"] = float(np.linalg.norm(b - A @ x))
        hist.append(st)
        E = x.reshape(E.shape)
    return E, hist
