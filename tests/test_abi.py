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


def _c_layout(struct, fields):
    """sizeof and offsetof of a header struct, from a C program built with gcc."""
    import shutil
    import subprocess
    import tempfile
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    body = "".join(f'  printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src = (f'#include <stddef.h>\n#include <stdio.h>\n#include "amrfld.h"\n'
           f'int main(void) {{\n  printf("%zu\\n", sizeof({struct}));\n{body}  return 0;\n}}\n')
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return [int(x) for x in out]


@pytest.mark.parametrize("name", ["amrfld_opts", "amrfld_stats", "amrfld_patch"])
def test_binding_structs_match_header_layout(name):
    from paper_1401_1112_amd import _lib as L
    cls = getattr(L, name)
    fields = [f for f, _ in cls._fields_]
    got = _c_layout(name, fields)
    assert got[0] == ctypes.sizeof(cls), (name, got[0], ctypes.sizeof(cls))
    for f, off in zip(fields, got[1:]):
        assert getattr(cls, f).offset == off, (name, f)


@pytest.mark.parametrize("field,value", [("K_exp", float("inf")), ("outer_mode", 2), ("outer_value", float("nan"))])
def test_create_rejects_bad_power_law_and_box_faces(field, value):
    L = _lib()
    o = L.amrfld_default_opts()
    o.base_level, o.max_level = 3, 3
    if field == "K_exp":
        o.K_exp = value
    elif field == "outer_mode":
        o.outer_mode[1] = value
    else:
        o.outer_mode[0] = 1
        o.outer_value[0] = value
    ctx = ctypes.c_void_p()
    assert L.load().amrfld_create(ctypes.byref(o), ctypes.byref(ctx)) == L.E_INVALID
    assert b"K_exp" in L.load().amrfld_create_error() or b"outer" in L.load().amrfld_create_error()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no fallback: without the built HIP library every entry point of the package raises
    from paper_1401_1112_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        L.load(str(tmp_path / "libamrfld.so"))
