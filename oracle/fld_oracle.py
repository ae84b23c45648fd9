"""Plain CPU FP64 oracle of the level-by-level implicit diffusion solve.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import or call this
module; it exists so that the GPU library can be checked against an obviously
correct, independent implementation of the method.

What it computes (Commercon, Debout & Teyssier 2014):

* Backward-Euler finite-volume update of dE/dt = div(K grad E) on one AMR level
  at a time (Sect. 3.1, eqs. Er_diff, Er_imp, Er_imp1): for every leaf cell
  ``(1 + sum_f C_f) E_i^{n+1} - sum_f C_f E_nb^{n+1} = E_i^n`` with
  ``C_f = K_f dt / dx^2``.
* Face coefficients by neighbour type (Sect. 3.1): same level and coarse-to-fine
  faces use ``A = K dt / dx^2``; a face towards a coarser neighbour, whose
  centre is 3 dx / 2 away, uses ``(2/3) A``.
* Level-interface conditions (Sect. 3.2 and 3.3): the face towards a coarser
  leaf is always Dirichlet with the coarse energy at the start of the coarse
  step; the face towards a refined neighbour is Dirichlet (ghost = restriction
  of the fine leaves), Neumann (imposed inflow from the stored fine flux) or
  Robin (weight alpha on the Dirichlet part, 1 - alpha on the stored flux).
* The stored interface flux of eq. mean_flux: the energy that crossed each
  fine-to-coarse face, summed over the fine substeps (dt is inside C).
* Conjugate gradient with a diagonal (Jacobi) preconditioner and the stopping
  test of Sect. 3.3.4: relative L2 residual and relative L-infinity change of
  the iterate, both below the tolerance.
* Adaptive time-stepping (Sect. 2.2): the level step equals the sum of two
  fine steps; finer levels are advanced first; after its substeps a fine level
  is restricted into the refined cells of its parent level.
* Two-temperature coupling term kappa_P rho c (a T^4 - E) (Sect. 2.1), reduced
  to one equation in E by linearising the emission term in T.
* For comparison, the unique-time-step method (Sect. 1, end of Sect. 3.1): all
  levels coupled in one system advanced with the finest time step, a coarse
  cell coupled to each finer cell of a refined neighbour's face with
  2^(3-ndim) A / 3, rows scaled by the cell volume.
* Levermore-Pomraning limited diffusivity ``K = c lambda(R) / (rho kappa_R)``
  with ``R = |grad E| / (rho kappa_R E)`` (Sect. 2.1); the Minerbo limiter of the
  collapse runs (Sect. 5.1) as an option.
* Optionally a theta-weighted step (Crank-Nicolson at theta = 1/2, Sect. 3.3.6).
* Optionally a power-law diffusivity K = K_const E^K_exp (the nonlinear
  equilibrium test, Sect. 4.2) and Dirichlet values held at outer faces
  (C = 2 K_f dt / dx^2 with the face dx / 2 away).

Readings where the paper is silent or ambiguous:

* lambda(R) = (2 + R) / (6 + 3R + R^2) (rational Levermore-Pomraning form).
* Face diffusivity: harmonic mean of the two cell diffusivities.
* grad E per cell: per axis, (E_+ - E_-) / (d_+ + d_-) with the neighbour at
  distance dx (same level, refined cells hold restricted values), 3 dx / 2
  (coarser leaf) or, across the outer boundary, the cell itself at distance dx.
* A refined neighbour's diffusivity comes from its restricted E and its density.
* Neumann inflow F is the energy entering the cell in E units; at a coarse
  refined face it is minus the stored fine flux divided by the coarse volume.
* Stopping: ``||r_j|| <= max(tol ||r_0||, floor ||b||)`` AND (optional)
  ``max |x_j - x_{j-1}| / |x_{j-1}| < tol``; ``x_0 = E^n``; the recursive
  residual is used.
* Outer boundary: zero flux.

Every function below is a direct statement of one of these steps, with no
blocking, fusion or reordering; numpy and scipy primitives (sparse matrix
products, Cholesky) serve as single steps.

Parity unpinned (readings that no closed form, invariant or printed value fixes;
the library makes the same choice, so only self-consistency is checked):

* ``grad_E``: the coarser neighbour taken as uniform over its cell (no transverse
  interpolation) when it enters the gradient at 3 dx / 2.
* ``cell_K`` on a refined neighbour: its diffusivity from the restricted E and the
  density sampled at its centre.
* ``K_of_value`` / ``_outer_C`` for a non-constant law: the diffusivity of the
  value held at a box face (the factor 2 and the half-cell distance are pinned by
  the linear fixed point, the harmonic mean with the law's value only by the
  near-second-order approach to the stationary profile).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp

SAME, C2F, F2C, OUTER = 0, 1, 2, 3
DIRICHLET, NEUMANN, ROBIN = 0, 1, 2
# direction d = 2*axis + side, side 0 is the minus face, side 1 the plus face
_OFF = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], dtype=np.int64)


def opposite(d: int) -> int:
    return d ^ 1


def lp_limiter(R):
    """Levermore-Pomraning flux limiter, rational form; lambda(0) = 1/3 (Sect. 2.1, 4.1)."""
    R = np.asarray(R, dtype=np.float64)
    return (2.0 + R) / (6.0 + 3.0 * R + R * R)


def minerbo_limiter(R):
    """Minerbo (1978) flux limiter, the limiter of the paper's collapse runs (Sect. 5.1):
    2 / (3 + sqrt(9 + 12 R^2)) up to R = 3/2, 1 / (1 + R + sqrt(1 + 2R)) beyond."""
    R = np.asarray(R, dtype=np.float64)
    low = 2.0 / (3.0 + np.sqrt(9.0 + 12.0 * R * R))
    high = 1.0 / (1.0 + R + np.sqrt(1.0 + 2.0 * R))
    return np.where(R <= 1.5, low, high)


def harmonic_mean(a, b):
    """Face diffusivity 2 a b / (a + b); zero when both sides are zero."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = a + b
    out = np.zeros(np.broadcast(a, b).shape)
    nz = s != 0.0
    out[nz] = (2.0 * a * b)[nz] / s[nz]
    return out


class _Level:
    """Cells of one level in the oracle's own order (octs as listed, x fastest)."""

    def __init__(self, level: int, octs: np.ndarray):
        self.level = level
        self.n = 1 << level
        self.dx = 1.0 / self.n
        self.vol = self.dx ** 3
        octs = np.asarray(octs, dtype=np.int64).reshape(-1, 3)
        child = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=np.int64)
        self.cells = (2 * octs[:, None, :] + child[None, :, :]).reshape(-1, 3)
        self.n_slots = len(self.cells)
        keys = self.key(self.cells)
        self._order = np.argsort(keys, kind="stable")
        self._sorted = keys[self._order]
        if len(self._sorted) > 1 and np.any(self._sorted[1:] == self._sorted[:-1]):
            raise ValueError(f"duplicate cells at level {level}")
        self.refined = np.zeros(self.n_slots, dtype=bool)

    def key(self, ijk):
        ijk = np.asarray(ijk, dtype=np.int64)
        return (ijk[:, 0] * self.n + ijk[:, 1]) * self.n + ijk[:, 2]

    def lookup(self, ijk):
        """Slot index of each cell in ``ijk`` at this level, or -1 where absent."""
        k = self.key(ijk)
        pos = np.searchsorted(self._sorted, k)
        pos = np.minimum(pos, max(len(self._sorted) - 1, 0))
        found = self._sorted[pos] == k
        return np.where(found, self._order[pos], -1)


class Oracle:
    """Level-by-level backward-Euler diffusion on an oct hierarchy, FP64."""

    def __init__(self, base_level, octs, *, kmode="lp", K_const=1.0, kappa_R=1.0, kappa_P=1.0,
                 c_light=1.0, a_rad=1.0, c_v=1.0, robin_alpha=0.5, abs_floor=1e-14,
                 linf_test=True, max_iter=10000, nsub=None, theta=1.0, K_exp=0.0, outer=None):
        self.base = int(base_level)
        self.theta = float(theta)
        self.K_exp = float(K_exp)
        # outer faces: direction -> Dirichlet value held at the face (others: zero flux)
        self.outer = {int(d): float(v) for d, v in (outer or {}).items()}
        self.max_level = max(octs)
        self.kmode = kmode
        self.K_const = float(K_const)
        self.kappa_R, self.kappa_P = float(kappa_R), float(kappa_P)
        self.c, self.a, self.c_v = float(c_light), float(a_rad), float(c_v)
        self.alpha = float(robin_alpha)
        self.abs_floor = float(abs_floor)
        self.linf_test = bool(linf_test)
        self.max_iter = int(max_iter)
        self.nsub = dict(nsub or {})
        self.lev = {}
        for l in range(self.base, self.max_level + 1):
            self.lev[l] = _Level(l, octs[l])
        n0 = 1 << self.base
        if self.lev[self.base].n_slots != n0 ** 3:
            raise ValueError("base level must cover the box")
        # refined flags: a slot is refined when an oct of the next level has it as parent
        for l in range(self.base + 1, self.max_level + 1):
            parents = np.asarray(octs[l], dtype=np.int64).reshape(-1, 3)
            ps = self.lev[l - 1].lookup(parents)
            if np.any(ps < 0):
                raise ValueError(f"oct at level {l} without parent")
            self.lev[l - 1].refined[ps] = True
        self._classify()
        self.E, self.rho, self.T = {}, {}, {}
        self.reg = {l: np.zeros((self.lev[l].n_slots, 6)) for l in self.lev}
        self.history = []

    # ------------------------------------------------------------------ geometry
    def _classify(self):
        """Face type and neighbour of every slot and direction (Fig. 1, Sect. 3.1)."""
        for l, L in self.lev.items():
            ftype = np.full((L.n_slots, 6), OUTER, dtype=np.int8)
            fnb = np.full((L.n_slots, 6), -1, dtype=np.int64)
            for d in range(6):
                nb = L.cells + _OFF[d]
                inside = np.all((nb >= 0) & (nb < L.n), axis=1)
                idx = np.full(L.n_slots, -1, dtype=np.int64)
                idx[inside] = L.lookup(nb[inside])
                same = idx >= 0
                ftype[same, d] = np.where(L.refined[idx[same]], C2F, SAME)
                fnb[same, d] = idx[same]
                need = inside & ~same
                if need.any():
                    if l == self.base:
                        raise ValueError("base level must cover the box")
                    c = self.lev[l - 1].lookup(nb[need] >> 1)
                    if np.any(c < 0) or np.any(self.lev[l - 1].refined[c]):
                        raise ValueError(f"level {l}: neighbour two levels coarser (unbalanced)")
                    ftype[need, d] = F2C
                    fnb[need, d] = c
            L.ftype, L.fnb = ftype, fnb
            L.leaf_slots = np.nonzero(~L.refined)[0]
            L.leaf_of = np.full(L.n_slots, -1, dtype=np.int64)
            L.leaf_of[L.leaf_slots] = np.arange(len(L.leaf_slots))

    def cells(self, level):
        return self.lev[level].cells

    def set_fields(self, level, rho, E, T=None):
        n = self.lev[level].n_slots
        self.rho[level] = np.array(rho, dtype=np.float64).reshape(n)
        self.E[level] = np.array(E, dtype=np.float64).reshape(n)
        self.T[level] = None if T is None else np.array(T, dtype=np.float64).reshape(n)

    # ------------------------------------------------------------- diffusivity
    def K_of_value(self, E, rho):
        """Diffusivity of a boundary value: K_const, K_const E^K_exp, or c lambda(0) /
        (rho kappa_R) = c / (3 rho kappa_R) (no gradient at a held value)."""
        if self.kmode == "const":
            return np.full(np.shape(rho), self.K_const)
        if self.kmode == "power":
            return np.full(np.shape(rho), self.K_const * E ** self.K_exp)
        return self.c / (3.0 * rho * self.kappa_R)

    def grad_E(self, level):
        """Per-slot gradient of E with the neighbour distances of the stencil reading."""
        L = self.lev[level]
        E = self.E[level]
        g = np.zeros((L.n_slots, 3))
        for axis in range(3):
            vals, dist = [], []
            for side in (0, 1):
                d = 2 * axis + side
                t, nb = L.ftype[:, d], L.fnb[:, d]
                v = E.copy()
                h = np.full(L.n_slots, L.dx)
                m = (t == SAME) | (t == C2F)
                v[m] = E[nb[m]]
                m = t == F2C
                if m.any():
                    v[m] = self.E[level - 1][nb[m]]
                    h[m] = 1.5 * L.dx
                if d in self.outer:  # Dirichlet value held at the outer face, dx / 2 away
                    m = t == OUTER
                    v[m] = self.outer[d]
                    h[m] = 0.5 * L.dx
                vals.append(v)
                dist.append(h)
            g[:, axis] = (vals[1] - vals[0]) / (dist[0] + dist[1])
        return g

    def cell_K(self, level):
        """Cell diffusivity K = c lambda(R) / (rho kappa_R) (Sect. 2.1); constant in heat mode."""
        L = self.lev[level]
        if self.kmode == "const":
            return np.full(L.n_slots, self.K_const)
        if self.kmode == "power":
            return self.K_const * self.E[level] ** self.K_exp
        rho, E = self.rho[level], self.E[level]
        g = self.grad_E(level)
        gn = np.sqrt(np.sum(g * g, axis=1))
        R = gn / (rho * self.kappa_R * E)
        lam = minerbo_limiter(R) if self.kmode == "minerbo" else lp_limiter(R)
        return self.c * lam / (rho * self.kappa_R)

    # ---------------------------------------------------------------- assembly
    def assemble(self, level, dt, mode):
        """Matrix A (CSR over the level's leaves) and right-hand side b (eq. Er_imp1 with
        the interface rows of Sect. 3.2).  Returns (A, b, coupling) where coupling holds
        the terms needed for the temperature update, or None."""
        L = self.lev[level]
        w = {DIRICHLET: 1.0, NEUMANN: 0.0, ROBIN: self.alpha}[mode]
        K = self.cell_K(level)
        Kc = self.cell_K(level - 1) if level > self.base else None
        coef = dt / (L.dx * L.dx)
        leaves = L.leaf_slots
        nl = len(leaves)
        E = self.E[level]
        diag = np.ones(nl)
        b = E[leaves].copy()
        rows, cols, vals = [], [], []
        for d in range(6):
            t = L.ftype[leaves, d]
            nb = L.fnb[leaves, d]
            m = t == SAME
            C = harmonic_mean(K[leaves[m]], K[nb[m]]) * coef
            diag[m] += C
            rows.append(np.nonzero(m)[0])
            cols.append(L.leaf_of[nb[m]])
            vals.append(-C)
            m = t == C2F
            if m.any():
                C = harmonic_mean(K[leaves[m]], K[nb[m]]) * coef
                Fin = -self.reg[level][leaves[m], d] / L.vol
                diag[m] += w * C
                b[m] += w * C * E[nb[m]] + (1.0 - w) * Fin
            m = t == F2C
            if m.any():
                C = (2.0 / 3.0) * harmonic_mean(K[leaves[m]], Kc[nb[m]]) * coef
                diag[m] += C
                b[m] += C * self.E[level - 1][nb[m]]
            m = t == OUTER
            if d in self.outer and m.any():
                C = self._outer_C(K[leaves[m]], self.rho[level][leaves[m]], d, coef)
                diag[m] += C
                b[m] += C * self.outer[d]
        coupling = None
        if self.T.get(level) is not None:
            T = self.T[level][leaves]
            rho = self.rho[level][leaves]
            eta = self.kappa_P * rho * self.c * dt
            beta_T = 4.0 * self.a * T ** 3
            denom = rho * self.c_v + eta * beta_T
            f = eta * beta_T / denom
            diag += eta * (1.0 - f)
            b += eta * (1.0 - f) * self.a * T ** 4
            coupling = (eta, denom)
        rows.append(np.arange(nl))
        cols.append(np.arange(nl))
        vals.append(diag)
        A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nl, nl))
        A.sum_duplicates()
        A.sort_indices()
        return A, b, coupling

    # ------------------------------------------------------------------- solve
    def _outer_C(self, Ki, rho, d, coef):
        """Face held at a Dirichlet value dx / 2 from the cell centre: C = 2 K_f dt / dx^2,
        K_f the harmonic mean of the cell's and the boundary value's diffusivity."""
        Kb = self.K_of_value(self.outer[d], rho)
        return 2.0 * harmonic_mean(Ki, Kb) * coef

    def theta_scheme(self, A1, b1, En):
        """Theta-weighted form of a backward-Euler system (Crank-Nicolson for theta = 1/2,
        the remedy Sect. 3.3.6 names for the first-order time error): the face fluxes are
        taken theta at the new and 1 - theta at the old time, the ghost values being the
        same at both, so A = I + theta (A1 - I) and b = b1 - (1 - theta) (A1 - I) E^n."""
        I = sp.identity(A1.shape[0], format="csr")
        D = A1 - I
        return (I + self.theta * D).tocsr(), b1 - (1.0 - self.theta) * (D @ En)

    def solve_level(self, level, dt, mode=DIRICHLET, tol=1e-10, max_iter=None, solver="pcg"):
        """Advance one level by dt (Sect. 3.3.4).  Updates E (and T) in place, adds the
        fine-to-coarse fluxes to the parent register in Neumann / Robin mode, and
        clears this level's register."""
        L = self.lev[level]
        A, b, coupling = self.assemble(level, dt, mode)
        x0 = self.E[level][L.leaf_slots].copy()
        if self.theta != 1.0:
            A, b = self.theta_scheme(A, b, x0)
        if solver == "dense":
            x = dense_solve(A, b)
            st = {"iters": 0, "converged": True}
        else:
            x, st = pcg_jacobi(A, b, x0, tol, self.max_iter if max_iter is None else max_iter,
                               self.abs_floor, self.linf_test)
        r_true = b - A @ x
        st.update(level=level, dt=dt, n_leaf=len(x), true_res=float(np.linalg.norm(r_true)),
                  bnorm=float(np.linalg.norm(b)), min_E=float(x.min()) if len(x) else 0.0,
                  min_diag=float(A.diagonal().min()) if len(x) else 1.0)
        self._post_solve(level, dt, mode, x, coupling)
        self.history.append(st)
        return st

    def _post_solve(self, level, dt, mode, x, coupling):
        L = self.lev[level]
        if mode in (NEUMANN, ROBIN) and level > self.base:
            # energy gained by the fine leaves through each fine-to-coarse face (eq. mean_flux)
            K = self.cell_K(level)
            Kc = self.cell_K(level - 1)
            coef = dt / (L.dx * L.dx)
            leaves = L.leaf_slots
            for d in range(6):
                m = L.ftype[leaves, d] == F2C
                if not m.any():
                    continue
                s = leaves[m]
                c = L.fnb[s, d]
                C = (2.0 / 3.0) * harmonic_mean(K[s], Kc[c]) * coef
                gain = L.vol * C * (self.E[level - 1][c] - x[m])
                np.add.at(self.reg[level - 1][:, opposite(d)], c, gain)
        if coupling is not None:
            eta, denom = coupling
            T = self.T[level][L.leaf_slots]
            self.T[level][L.leaf_slots] = T + eta * (x - self.a * T ** 4) / denom
        self.E[level][L.leaf_slots] = x
        self.reg[level][:] = 0.0

    def restrict(self, fine_level):
        """Refined cells of the parent level take the mean of their eight children."""
        F = self.lev[fine_level]
        C = self.lev[fine_level - 1]
        parents = C.lookup(F.cells[0::8] >> 1)
        child_E = self.E[fine_level].reshape(-1, 8)
        self.E[fine_level - 1][parents] = child_E.mean(axis=1)

    def advance_subcycled(self, dt, mode=DIRICHLET, tol=1e-10, level=None):
        """One step of ``level`` (default: base) with the fine-first adaptive schedule."""
        level = self.base if level is None else level
        if level < self.max_level:
            ns = int(self.nsub.get(level + 1, 2))
            for _ in range(ns):
                self.advance_subcycled(dt / ns, mode, tol, level + 1)
            self.restrict(level + 1)
        return self.solve_level(level, dt, mode, tol)

    def total_energy(self):
        """Sum of V E over the leaves of every level."""
        return float(sum(L.vol * self.E[l][L.leaf_slots].sum() for l, L in self.lev.items()))

    # ------------------------------------------- unique time step (all levels coupled)
    def composite_numbering(self):
        """Offset of each level's leaves in the composite vector (levels base..max, leaves
        in slot order) and the total count."""
        off, n = {}, 0
        for l in range(self.base, self.max_level + 1):
            off[l] = n
            n += len(self.lev[l].leaf_slots)
        return off, n

    def _facing_children(self, level, nb, d):
        """Slots at level + 1 of the four children of the refined cells ``nb`` (level) that
        lie on the face reached by crossing direction d from a neighbouring cell: for a
        plus-side face (the refined cell lies at +axis) the children on its minus side."""
        F = self.lev[level + 1]
        axis, side = d >> 1, d & 1
        cell = self.lev[level].cells[nb]
        trans = [a for a in range(3) if a != axis]
        out = []
        for u in (0, 1):
            for v in (0, 1):
                off = np.zeros(3, dtype=np.int64)
                off[trans[0]], off[trans[1]] = u, v
                off[axis] = 0 if side == 1 else 1
                out.append(F.lookup(2 * cell + off))
        ch = np.stack(out, axis=1)
        if np.any(ch < 0) or np.any(F.refined[ch]):
            raise ValueError("a refined neighbour's facing children must be leaves (2:1 balance)")
        return ch

    def assemble_composite(self, dt):
        """One system over the leaves of every level, all advanced by the same dt (the
        unique-time-step method the paper compares with, Sect. 1; coefficients as in the
        remark closing Sect. 3.1).  Same-level faces: C = A = K_f dt / dx^2.  A cell's face
        towards a coarser leaf: C = (2/3) A (centres 3 dx / 2 apart).  A cell's face towards
        a refined neighbour: the 2^(ndim-1) = 4 finer cells on that face are not
        interpolated to the cell's level; each is coupled with C = 2^(3-ndim) A / 3 = A / 3
        (ndim = 3), K_f taken with that finer cell.  Every row is multiplied by its cell
        volume, which makes the matrix symmetric (V_f (2/3) A_f = V_c A_c / 3 for
        dx_c = 2 dx_f).  Returns (A, b, coupling per level, level offsets)."""
        off, n = self.composite_numbering()
        K = {l: self.cell_K(l) for l in self.lev}
        rows, cols, vals = [], [], []
        b = np.empty(n)
        couplings = {}
        for l, L in self.lev.items():
            leaves = L.leaf_slots
            nl = len(leaves)
            gi = off[l] + np.arange(nl)
            coef = dt / (L.dx * L.dx)
            diag = np.ones(nl)
            bl = self.E[l][leaves].copy()
            for d in range(6):
                t = L.ftype[leaves, d]
                nb = L.fnb[leaves, d]
                m = t == SAME
                C = harmonic_mean(K[l][leaves[m]], K[l][nb[m]]) * coef
                diag[m] += C
                rows.append(gi[m])
                cols.append(off[l] + L.leaf_of[nb[m]])
                vals.append(-L.vol * C)
                m = t == F2C
                if m.any():
                    C = (2.0 / 3.0) * harmonic_mean(K[l][leaves[m]], K[l - 1][nb[m]]) * coef
                    diag[m] += C
                    rows.append(gi[m])
                    cols.append(off[l - 1] + self.lev[l - 1].leaf_of[nb[m]])
                    vals.append(-L.vol * C)
                m = t == OUTER
                if d in self.outer and m.any():
                    C = self._outer_C(K[l][leaves[m]], self.rho[l][leaves[m]], d, coef)
                    diag[m] += C
                    bl[m] += C * self.outer[d]
                m = t == C2F
                if m.any():
                    ch = self._facing_children(l, nb[m], d)
                    for k in range(4):
                        f = ch[:, k]
                        C = harmonic_mean(K[l][leaves[m]], K[l + 1][f]) * coef / 3.0
                        diag[m] += C
                        rows.append(gi[m])
                        cols.append(off[l + 1] + self.lev[l + 1].leaf_of[f])
                        vals.append(-L.vol * C)
            if self.T.get(l) is not None:
                T = self.T[l][leaves]
                rho = self.rho[l][leaves]
                eta = self.kappa_P * rho * self.c * dt
                beta_T = 4.0 * self.a * T ** 3
                denom = rho * self.c_v + eta * beta_T
                f = eta * beta_T / denom
                diag += eta * (1.0 - f)
                bl += eta * (1.0 - f) * self.a * T ** 4
                couplings[l] = (eta, denom)
            rows.append(gi)
            cols.append(gi)
            vals.append(L.vol * diag)
            b[gi] = L.vol * bl
        A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
        A.sum_duplicates()
        A.sort_indices()
        return A, b, couplings, off

    def solve_composite(self, dt, tol=1e-10, max_iter=None, solver="pcg"):
        """Advance every level by dt in one composite solve; updates E (and T) of the
        leaves, then restricts each level into its parent's refined cells, finest first."""
        A, b, couplings, off = self.assemble_composite(dt)
        x0 = np.concatenate([self.E[l][self.lev[l].leaf_slots] for l in sorted(self.lev)])
        if solver == "dense":
            x = dense_solve(A, b)
            st = {"iters": 0, "converged": True}
        else:
            x, st = pcg_jacobi(A, b, x0, tol, self.max_iter if max_iter is None else max_iter,
                               self.abs_floor, self.linf_test)
        st.update(level=-1, dt=dt, n_leaf=len(x), true_res=float(np.linalg.norm(b - A @ x)),
                  bnorm=float(np.linalg.norm(b)), min_E=float(x.min()) if len(x) else 0.0)
        for l, L in self.lev.items():
            xl = x[off[l]:off[l] + len(L.leaf_slots)]
            if l in couplings:
                eta, denom = couplings[l]
                T = self.T[l][L.leaf_slots]
                self.T[l][L.leaf_slots] = T + eta * (xl - self.a * T ** 4) / denom
            self.E[l][L.leaf_slots] = xl
        for l in range(self.max_level, self.base, -1):
            self.restrict(l)
        self.history.append(st)
        return st

    def advance_unique(self, dt, tol=1e-10):
        """One coarse step dt with the unique time step of the finest level: as many
        composite solves as the adaptive schedule makes solves of the finest level."""
        n = 1
        for l in range(self.base + 1, self.max_level + 1):
            n *= int(self.nsub.get(l, 2))
        for _ in range(n):
            self.solve_composite(dt / n, tol)
        return n


def pcg_jacobi(A, b, x0, tol, max_iter, abs_floor=1e-14, linf_test=True):
    """Conjugate gradient with a diagonal preconditioner (Sect. 3.3.4).

    Stops after iteration j when ||r_j|| <= max(tol ||r_0||, abs_floor ||b||) and, with
    ``linf_test``, max_i |x_j - x_{j-1}| / |x_{j-1}| < tol (absolute change where the
    previous iterate is zero).  Returns (x, stats)."""
    d = A.diagonal()
    x = np.array(x0, dtype=np.float64)
    r = b - A @ x
    z = r / d
    rho = float(r @ z)
    r0 = float(np.sqrt(r @ r))
    bn = float(np.sqrt(b @ b))
    thresh = max(tol * r0, abs_floor * bn)
    st = {"iters": 0, "converged": True, "r0": r0, "rel_res": 0.0, "linf": 0.0}
    if r0 <= abs_floor * bn:
        return x, st
    p = z.copy()
    rn = r0
    linf = np.inf
    for j in range(1, max_iter + 1):
        q = A @ p
        alpha = rho / float(p @ q)
        dx = alpha * p
        ax = np.abs(x)
        rel = np.where(ax > 0.0, np.abs(dx) / np.where(ax > 0.0, ax, 1.0), np.abs(dx))
        linf = float(rel.max()) if len(rel) else 0.0
        x = x + dx
        r = r - alpha * q
        rn = float(np.sqrt(r @ r))
        if (rn <= thresh and (not linf_test or linf < tol)) or rn == 0.0:
            st.update(iters=j, converged=True, rel_res=rn / r0, linf=linf)
            return x, st
        z = r / d
        rho_new = float(r @ z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    st.update(iters=max_iter, converged=False, rel_res=rn / r0, linf=linf)
    return x, st


def dense_solve(A, b):
    """Direct solve of the SPD system by Cholesky factorisation (tiny systems only)."""
    M = A.toarray() if sp.issparse(A) else np.asarray(A)
    c, low = scipy.linalg.cho_factor(M)
    return scipy.linalg.cho_solve((c, low), b)
