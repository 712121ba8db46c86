"""The C ABI library loads without a GPU and exports every entry point that
include/jfft.h declares; the Python binding covers exactly those names.
No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jfft.h")
LIB = os.path.join(ROOT, "paper_2508_02613_amd", "libjfft.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jfft_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_entry_points():
    names = declared_functions()
    for core in ["jfft_create_cell", "jfft_set_material", "jfft_solve", "jfft_destroy_cell",
                 "jfft_workspace_bytes", "jfft_bind_workspace", "jfft_last_error"]:
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libjfft.so is not built (run python paper_2508_02613_amd/build.py)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.jfft_version is not None


def test_binding_matches_header():
    import paper_2508_02613_amd as pkg
    assert sorted(pkg.EXPORTED_SYMBOLS) == declared_functions()


def test_binding_loads_and_reports_errors_without_gpu():
    import paper_2508_02613_amd as pkg
    lib = pkg.load_library()
    assert b"gfx950" in lib.jfft_version()
    # argument validation happens on the host before any device call
    h = ctypes.c_void_p()
    n = (ctypes.c_int * 3)(5, 4, 1)
    st = lib.jfft_create_cell(2, n, None, 0, 3, None, ctypes.byref(h))
    assert st == 2  # odd grid
    assert b"even" in lib.jfft_last_error()
    n = (ctypes.c_int * 3)(14, 4, 1)  # 7 = n/2 is not a product of 2, 3, 5
    assert lib.jfft_create_cell(2, n, None, 0, 3, None, ctypes.byref(h)) == 1
    n = (ctypes.c_int * 3)(8, 8, 8)
    assert lib.jfft_create_cell(4, n, None, 0, 3, None, ctypes.byref(h)) == 1
