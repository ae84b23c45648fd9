"""Convenience wrapper over the C ABI: one context per hierarchy, torch tensors for
device memory and the current torch stream for ordering."""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


class HierarchySolver:
    def __init__(self, base_level, octs, *, robin_alpha=0.5, max_iter=10000, precision=L.FP64,
                 linf_test=True, abs_floor=1e-14, a_rad=1.0, c_v=1.0, nsub=None, check_every=0,
                 true_residual=True, time_sweeps=0, inner_tol=3e-3, max_outer=30, max_blocks=0,
                 persistent=False, persistent_per_cu=0, theta=1.0, K_exp=0.0, outer=None, form_coefs=False,
                 graph=False, device="cuda:0", stream=None):
        L.load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        o = L.amrfld_default_opts()
        o.base_level = int(base_level)
        o.max_level = int(max(octs))
        o.robin_alpha = float(robin_alpha)
        o.max_iter = int(max_iter)
        o.precision = int(precision)
        o.linf_test = int(bool(linf_test))
        o.abs_floor = float(abs_floor)
        o.a_rad = float(a_rad)
        o.c_v = float(c_v)
        for lvl, v in (nsub or {}).items():
            o.nsub[int(lvl)] = int(v)
        o.check_every = int(check_every)
        o.true_residual = int(bool(true_residual))
        o.time_sweeps = int(time_sweeps)
        o.inner_tol = float(inner_tol)
        o.max_outer = int(max_outer)
        o.max_blocks = int(max_blocks)
        o.persistent = int(bool(persistent))
        o.persistent_per_cu = int(persistent_per_cu)
        o.theta = float(theta)
        o.K_exp = float(K_exp)
        o.form_coefs = int(bool(form_coefs))
        o.graph = int(bool(graph))
        for d, v in (outer or {}).items():  # box face direction -> Dirichlet energy held there
            o.outer_mode[int(d)] = 1
            o.outer_value[int(d)] = float(v)
        o.stream = self.stream.cuda_stream
        self.ctx = L.amrfld_create(o)
        self.levels = list(range(int(base_level), int(max(octs)) + 1))
        self._cells = {}
        for lvl in self.levels:
            st = L.amrfld_build_level(self.ctx, lvl, octs[lvl])
            if st != L.OK:
                msg = L.amrfld_last_error(self.ctx)
                self.close()
                raise L.AmrfldError(st, msg)
        self._fields = {}

    def close(self):
        if getattr(self, "ctx", None) is not None:
            L.amrfld_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != L.OK:
            raise L.AmrfldError(st, L.amrfld_last_error(self.ctx))
        return st

    def info(self, level):
        ns, nl, _ = L.amrfld_level_info(self.ctx, level, want_cells=False)
        return ns, nl

    def cells(self, level):
        if level not in self._cells:
            self._cells[level] = L.amrfld_level_info(self.ctx, level)[2]
        return self._cells[level]

    def _dev(self, a):
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=torch.float64)
        return t.to(self.device).contiguous()

    def set_fields(self, level, rho, E, T=None, *, kappa_R=1.0, kappa_P=1.0, c_light=1.0,
                   kmode=L.K_LP, K_const=1.0):
        r, e, t = self._dev(rho), self._dev(E), self._dev(T)
        self._fields[level] = (r, e, t)  # keep alive until the stream-ordered copy ran
        self._check(L.amrfld_set_coeffs(self.ctx, level, r, e, t, kappa_R, kappa_P, c_light,
                                        kmode, K_const))

    def solve_level(self, level, dt, bc_mode=L.BC_DIRICHLET, tol=1e-10, raise_on_error=True):
        st = L.amrfld_solve_level(self.ctx, level, dt, bc_mode, tol)
        if raise_on_error and st not in (L.OK,):
            self._check(st)
        return st

    def restrict(self, fine_level):
        """Restrict fine_level into its parent cells (as the driver does between levels)."""
        self._check(L.amrfld_restrict_level(self.ctx, fine_level))

    def advance(self, dt, bc_mode=L.BC_DIRICHLET, tol=1e-10, raise_on_error=True):
        st = L.amrfld_advance_subcycled(self.ctx, dt, bc_mode, tol)
        if raise_on_error and st != L.OK:
            self._check(st)
        return st

    def advance_unique(self, dt, tol=1e-10, raise_on_error=True):
        """One coarse step with the unique time step of the finest level (all levels in
        one composite system per fine step)."""
        st = L.amrfld_advance_unique(self.ctx, dt, tol)
        if raise_on_error and st != L.OK:
            self._check(st)
        return st

    def E(self, level, with_T=False):
        ns, _ = self.info(level)
        e = torch.empty(ns, dtype=torch.float64, device=self.device)
        t = torch.empty(ns, dtype=torch.float64, device=self.device) if with_T else None
        self._check(L.amrfld_get_E(self.ctx, level, e, t))
        return (e, t) if with_T else e

    def stats(self):
        return L.amrfld_last_stats(self.ctx)

    def last_error(self):
        return L.amrfld_last_error(self.ctx)

    def set_launch(self, max_blocks=0, persistent=False, persistent_per_cu=0, form_coefs=False):
        self._check(L.amrfld_set_launch(self.ctx, max_blocks, int(bool(persistent)), persistent_per_cu,
                                        int(bool(form_coefs))))

    def set_refinement(self, inner_tol, max_outer=30):
        self._check(L.amrfld_set_refinement(self.ctx, inner_tol, max_outer))


def sample_problem_fields(solver: HierarchySolver, problem):
    """Sample a problem's fields in the library's cell order and upload them."""
    kmode = {"const": L.K_CONST, "lp": L.K_LP, "minerbo": L.K_MINERBO, "power": L.K_POWER}[problem.kmode]
    for lvl in solver.levels:
        c = solver.cells(lvl)
        T = None if problem.T is None else problem.T(lvl, c)
        solver.set_fields(lvl, problem.rho(lvl, c), problem.E(lvl, c), T, kappa_R=problem.kappa_R,
                          kappa_P=problem.kappa_P, c_light=problem.c_light, kmode=kmode,
                          K_const=problem.K_const)


def solver_from_problem(problem, **over):
    kw = dict(robin_alpha=problem.robin_alpha, max_iter=problem.max_iter, linf_test=problem.linf_test,
              abs_floor=problem.abs_floor, a_rad=problem.a_rad, c_v=problem.c_v, nsub=problem.nsub,
              theta=getattr(problem, "theta", 1.0), K_exp=getattr(problem, "K_exp", 0.0),
              outer=getattr(problem, "outer", None))
    kw.update(over)
    s = HierarchySolver(problem.hierarchy.base_level, problem.hierarchy.octs, **kw)
    sample_problem_fields(s, problem)
    return s


def to_numpy(t):
    return t.detach().cpu().numpy() if isinstance(t, torch.Tensor) else np.asarray(t)


class BatchSolver:
    """Independent patches advanced together (amrfld_solve_batch)."""

    def __init__(self, *, robin_alpha=0.5, max_iter=10000, linf_test=True, abs_floor=1e-14,
                 inner_tol=3e-3, max_outer=30, max_blocks=0, time_sweeps=0, true_residual=True,
                 check_every=0, persistent=False, graph=False, persistent_per_cu=0, form_coefs=False,
                 device="cuda:0", stream=None):
        L.load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        o = L.amrfld_default_opts()
        o.base_level, o.max_level = 1, 1
        o.robin_alpha = float(robin_alpha)
        o.max_iter = int(max_iter)
        o.linf_test = int(bool(linf_test))
        o.abs_floor = float(abs_floor)
        o.inner_tol = float(inner_tol)
        o.max_outer = int(max_outer)
        o.max_blocks = int(max_blocks)
        o.time_sweeps = int(time_sweeps)
        o.true_residual = int(bool(true_residual))
        o.check_every = int(check_every)
        o.persistent = int(bool(persistent))
        o.graph = int(bool(graph))
        o.persistent_per_cu = int(persistent_per_cu)
        o.form_coefs = int(bool(form_coefs))
        o.stream = self.stream.cuda_stream
        self.ctx = L.amrfld_create(o)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            L.amrfld_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload(self, patches, kmode=L.K_LP, kappa_R=1.0, c_light=1.0, K_const=1.0):
        """Copy the patches' fields to the device once; returns a handle for run()."""
        keep, structs, offs = [], [], [0]
        for p in patches:
            n = int(p.n)
            rho = torch.as_tensor(np.ascontiguousarray(np.asarray(p.rho).transpose(2, 1, 0)).ravel(),
                                  dtype=torch.float64).to(self.device)
            E = torch.as_tensor(np.ascontiguousarray(np.asarray(p.E).transpose(2, 1, 0)).ravel(),
                                dtype=torch.float64).to(self.device)
            keep += [rho, E]
            st = L.amrfld_patch()
            st.n, st.dx, st.dt = n, float(p.dx), float(p.dt)
            st.rho, st.E = rho.data_ptr(), E.data_ptr()
            st.kmode, st.K_const, st.kappa_R, st.c_light = int(kmode), float(K_const), float(kappa_R), float(c_light)
            for d in range(6):
                st.face_mode[d] = int(p.face_mode[d])
                st.face_ghost[d] = float(p.face_ghost[d])
                st.face_flux[d] = float(p.face_flux[d])
            structs.append(st)
            offs.append(offs[-1] + n ** 3)
        out = torch.empty(offs[-1], dtype=torch.float64, device=self.device)
        return {"keep": keep, "structs": structs, "offs": offs, "out": out,
                "sizes": [int(p.n) for p in patches]}

    def run(self, h, n_steps, tol, precision=L.FP64, raise_on_error=True):
        status = L.amrfld_solve_batch(self.ctx, h["structs"], n_steps, tol, precision, h["out"])
        if raise_on_error and status != L.OK:
            raise L.AmrfldError(status, L.amrfld_last_error(self.ctx))
        return status

    def result(self, h):
        host = h["out"].cpu().numpy()
        res = []
        for q, n in enumerate(h["sizes"]):
            res.append(host[h["offs"][q]:h["offs"][q + 1]].reshape(n, n, n).transpose(2, 1, 0).copy())
        return res

    def solve(self, patches, n_steps, tol, precision=L.FP64, kmode=L.K_LP, kappa_R=1.0, c_light=1.0,
              K_const=1.0, raise_on_error=True):
        """patches: objects with n, dx, dt, rho, E ([i, j, k] arrays), face_mode, face_ghost,
        face_flux.  Returns the final energies as a list of (n, n, n) [i, j, k] arrays and the
        status."""
        h = self.upload(patches, kmode, kappa_R, c_light, K_const)
        status = self.run(h, n_steps, tol, precision, raise_on_error)
        return self.result(h), status

    def stats(self):
        return L.amrfld_last_stats(self.ctx)

    def last_error(self):
        return L.amrfld_last_error(self.ctx)

    def set_refinement(self, inner_tol, max_outer=30):
        st = L.amrfld_set_refinement(self.ctx, inner_tol, max_outer)
        if st != L.OK:
            raise L.AmrfldError(st, L.amrfld_last_error(self.ctx))

    def set_launch(self, max_blocks=0, persistent=False, persistent_per_cu=0, form_coefs=False):
        st = L.amrfld_set_launch(self.ctx, max_blocks, int(bool(persistent)), persistent_per_cu, int(bool(form_coefs)))
        if st != L.OK:
            raise L.AmrfldError(st, L.amrfld_last_error(self.ctx))
