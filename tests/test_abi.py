"""The C-ABI library loads and exports every function include/vanka_mg.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vanka_mg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("vanka_mg_setup", "vanka_mg_solve", "paradiag_apply", "vanka_mg_destroy",
                 "vanka_mg_error_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2203_11154_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libvanka_mg.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTED) == declared_functions()


def test_error_strings_and_defaults_without_gpu():
    from paper_2203_11154_amd import _lib
    lib = _lib.load()
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert lib.vanka_mg_error_string(code)
    o = _lib.VmgOpts()
    assert lib.vanka_mg_default_opts(ctypes.byref(o)) == 0
    assert o.omega == pytest.approx(0.96) and (o.nu1, o.nu2, o.gamma) == (2, 2, 1)
    assert lib.vanka_mg_default_opts(None) == _lib.VMG_INVALID_ARG
    # null / invalid arguments are rejected before any device work
    h = ctypes.c_void_p()
    assert lib.vanka_mg_setup(None, 0, None, None, None, ctypes.byref(h)) == _lib.VMG_INVALID_ARG
    assert lib.paradiag_transform(0, 10, None, 0, None, None, None) == _lib.VMG_INVALID_ARG
    assert lib.vanka_mg_solve(None, None, None, 1e-10, 0, None, None, None, None) == _lib.VMG_INVALID_ARG
    assert lib.vanka_mg_destroy(None) == 0


def test_struct_layouts_match_header():
    from paper_2203_11154_amd import _lib
    assert ctypes.sizeof(_lib.VmgGrid) == 24
    assert ctypes.sizeof(_lib.VmgOpts) == 48
