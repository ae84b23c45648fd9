"""The C ABI library loads and exports every entry point of include/amrfld.h
(CPU: no compute calls), plus argument checks that need no device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amrfld.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(amrfld_[a-z_]+)\s*\(", src)))


def _lib():
    from paper_1401_1112_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    return _lib


def test_header_declares_core_calls():
    names = _declared()
    for n in ("amrfld_build_level", "amrfld_set_coeffs", "amrfld_solve_level",
              "amrfld_advance_subcycled"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    bound = {name for name, _, _ in L.SIGNATURES}
    assert set(_declared()) <= bound


def test_default_opts_and_create_rejects_bad_levels():
    L = _lib()
    o = L.amrfld_default_opts()
    assert o.max_iter == 10000 and o.robin_alpha == 0.5 and o.abs_floor == 1e-14
    o.base_level, o.max_level = 5, 3
    ctx = ctypes.c_void_p()
    st = L.load().amrfld_create(ctypes.byref(o), ctypes.byref(ctx))
    assert st == L.E_INVALID
    assert b"levels" in L.load().amrfld_create_error()
