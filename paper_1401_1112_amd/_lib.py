"""ctypes binding of libamrfld.so: the C ABI of include/amrfld.h, same names.

Argument marshalling only; every step of the solve runs in the library's HIP
kernels.  Device arrays are passed as torch CUDA tensors (float64, contiguous),
host arrays as numpy arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("AMRFLD_LIB") or os.path.join(_HERE, "libamrfld.so")

OK, E_INVALID, E_STATE, E_NOMEM, E_DEVICE, E_NOCONV, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_STATE", -3: "E_NOMEM", -4: "E_DEVICE",
                -5: "E_NOCONV", -6: "E_NONFINITE"}
BC_DIRICHLET, BC_NEUMANN, BC_ROBIN = 0, 1, 2
FP64, MIXED = 0, 1
K_CONST, K_LP, K_MINERBO, K_POWER = 0, 1, 2, 3


class amrfld_opts(ctypes.Structure):
    _fields_ = [
        ("base_level", ctypes.c_int), ("max_level", ctypes.c_int),
        ("robin_alpha", ctypes.c_double), ("max_iter", ctypes.c_int),
        ("precision", ctypes.c_int), ("linf_test", ctypes.c_int),
        ("abs_floor", ctypes.c_double), ("a_rad", ctypes.c_double), ("c_v", ctypes.c_double),
        ("nsub", ctypes.c_int * 32), ("check_every", ctypes.c_int),
        ("true_residual", ctypes.c_int), ("time_sweeps", ctypes.c_int),
        ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int), ("max_blocks", ctypes.c_int),
        ("persistent", ctypes.c_int), ("graph", ctypes.c_int), ("stream", ctypes.c_void_p),
        ("persistent_per_cu", ctypes.c_int), ("theta", ctypes.c_double),
        ("K_exp", ctypes.c_double), ("outer_mode", ctypes.c_int * 6), ("outer_value", ctypes.c_double * 6),
        ("form_coefs", ctypes.c_int),
    ]


class amrfld_stats(ctypes.Structure):
    _fields_ = [
        ("level", ctypes.c_int), ("iters", ctypes.c_int), ("converged", ctypes.c_int),
        ("status", ctypes.c_int), ("n_leaf", ctypes.c_int64),
        ("rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
        ("linf_change", ctypes.c_double), ("min_E", ctypes.c_double), ("ms", ctypes.c_double),
        ("pcg_ms", ctypes.c_double), ("dt", ctypes.c_double), ("outer_iters", ctypes.c_int),
        ("n_timed", ctypes.c_int), ("sweep_ms", ctypes.c_double), ("spare_ms", ctypes.c_double),
        ("launch_mode", ctypes.c_int), ("rnorm0", ctypes.c_double), ("bnorm", ctypes.c_double),
        ("sweep_blocks", ctypes.c_int), ("launch_blocks", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class amrfld_patch(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
        ("rho", ctypes.c_void_p), ("E", ctypes.c_void_p), ("kmode", ctypes.c_int),
        ("K_const", ctypes.c_double), ("kappa_R", ctypes.c_double), ("c_light", ctypes.c_double),
        ("face_mode", ctypes.c_int * 6), ("face_ghost", ctypes.c_double * 6),
        ("face_flux", ctypes.c_double * 6),
    ]


_lib = None

# (name, restype, argtypes) of every exported entry point of include/amrfld.h
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
SIGNATURES = [
    ("amrfld_default_opts", None, [ctypes.POINTER(amrfld_opts)]),
    ("amrfld_create", _I, [ctypes.POINTER(amrfld_opts), ctypes.POINTER(_P)]),
    ("amrfld_destroy", None, [_P]),
    ("amrfld_build_level", _I, [_P, _I, ctypes.c_int64, _P]),
    ("amrfld_level_info", _I, [_P, _I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), _P]),
    ("amrfld_set_coeffs", _I, [_P, _I, _P, _P, _P, _D, _D, _D, _I, _D]),
    ("amrfld_solve_level", _I, [_P, _I, _D, _I, _D]),
    ("amrfld_solve_level_noalloc", _I, [_P, _I, _D, _I, _D]),
    ("amrfld_restrict_level", _I, [_P, _I]),
    ("amrfld_advance_subcycled", _I, [_P, _D, _I, _D]),
    ("amrfld_advance_unique", _I, [_P, _D, _D]),
    ("amrfld_solve_batch", _I, [_P, _I, ctypes.POINTER(amrfld_patch), _I, _D, _I, _P]),
    ("amrfld_get_E", _I, [_P, _I, _P, _P]),
    ("amrfld_last_stats", _I, [_P, ctypes.POINTER(amrfld_stats), _I, ctypes.POINTER(_I)]),
    ("amrfld_set_launch", _I, [_P, _I, _I, _I, _I]),
    ("amrfld_set_refinement", _I, [_P, ctypes.c_double, _I]),
    ("amrfld_last_error", ctypes.c_char_p, [_P]),
    ("amrfld_create_error", ctypes.c_char_p, []),
]


def load(path: str = LIB_PATH):
    """Load the shared library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class AmrfldError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("device arrays must be contiguous CUDA tensors")
    return t.data_ptr()


# ------------------------------------------------------------- thin wrappers
def amrfld_default_opts():
    o = amrfld_opts()
    load().amrfld_default_opts(ctypes.byref(o))
    return o


def amrfld_create(opts):
    ctx = ctypes.c_void_p()
    st = load().amrfld_create(ctypes.byref(opts), ctypes.byref(ctx))
    if st != OK:
        raise AmrfldError(st, load().amrfld_create_error().decode())
    return ctx


def amrfld_destroy(ctx):
    load().amrfld_destroy(ctx)


def _err(ctx):
    return load().amrfld_last_error(ctx).decode()


def amrfld_build_level(ctx, level, oct_ijk):
    a = np.ascontiguousarray(oct_ijk, dtype=np.int32).reshape(-1, 3)
    return load().amrfld_build_level(ctx, int(level), len(a), a.ctypes.data)


def amrfld_level_info(ctx, level, want_cells=True):
    ns, nl = ctypes.c_int64(), ctypes.c_int64()
    st = load().amrfld_level_info(ctx, int(level), ctypes.byref(ns), ctypes.byref(nl), None)
    if st != OK:
        raise AmrfldError(st, _err(ctx))
    cells = None
    if want_cells:
        cells = np.zeros((ns.value, 3), dtype=np.int32)
        load().amrfld_level_info(ctx, int(level), None, None, cells.ctypes.data)
    return ns.value, nl.value, cells


def amrfld_set_coeffs(ctx, level, rho, E, T=None, kappa_R=1.0, kappa_P=1.0, c_light=1.0,
                      kmode=K_LP, K_const=1.0):
    return load().amrfld_set_coeffs(ctx, int(level), _ptr(rho), _ptr(E), _ptr(T), float(kappa_R),
                                    float(kappa_P), float(c_light), int(kmode), float(K_const))


def amrfld_solve_level(ctx, level, dt, bc_mode, tol):
    return load().amrfld_solve_level(ctx, int(level), float(dt), int(bc_mode), float(tol))


def amrfld_solve_level_noalloc(ctx, level, dt, bc_mode, tol):
    return load().amrfld_solve_level_noalloc(ctx, int(level), float(dt), int(bc_mode), float(tol))


def amrfld_restrict_level(ctx, fine_level):
    return load().amrfld_restrict_level(ctx, int(fine_level))


def amrfld_advance_subcycled(ctx, dt, bc_mode, tol):
    return load().amrfld_advance_subcycled(ctx, float(dt), int(bc_mode), float(tol))


def amrfld_advance_unique(ctx, dt, tol):
    return load().amrfld_advance_unique(ctx, float(dt), float(tol))


def amrfld_solve_batch(ctx, patches, n_steps, tol, precision, E_out):
    """patches: list of amrfld_patch (device pointers already filled in)."""
    arr = (amrfld_patch * len(patches))(*patches)
    return load().amrfld_solve_batch(ctx, len(patches), arr, int(n_steps), float(tol), int(precision),
                                     _ptr(E_out))


def amrfld_get_E(ctx, level, E_out, T_out=None):
    return load().amrfld_get_E(ctx, int(level), _ptr(E_out), _ptr(T_out))


def amrfld_last_stats(ctx, max_n=None):
    n = ctypes.c_int()
    load().amrfld_last_stats(ctx, None, 0, ctypes.byref(n))
    count = n.value if max_n is None else min(n.value, max_n)
    arr = (amrfld_stats * max(count, 1))()
    load().amrfld_last_stats(ctx, arr, count, ctypes.byref(n))
    return [arr[k].as_dict() for k in range(count)]


def amrfld_set_refinement(ctx, inner_tol, max_outer):
    return load().amrfld_set_refinement(ctx, float(inner_tol), int(max_outer))


def amrfld_set_launch(ctx, max_blocks, persistent, persistent_per_cu, form_coefs):
    return load().amrfld_set_launch(ctx, int(max_blocks), int(persistent), int(persistent_per_cu), int(form_coefs))


def amrfld_last_error(ctx):
    return _err(ctx)
