"""Host-side checks of the C ABI: the library loads and exports every symbol
that include/fjofc.h declares (no compute calls: there may be no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fjofc.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fjofc_[a-z0-9_]+)\s*\(", txt)))


def _lib_path():
    from paper_1502_03391_amd import fjofc
    return fjofc.LIB_PATH


def test_header_declares_the_paper_entry_points():
    names = _declared_functions()
    for must in ("fjofc_embed", "fjofc_oos", "fjofc_create", "fjofc_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    path = _lib_path()
    if not os.path.exists(path):
        pytest.skip("libfjofc.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_lists_every_declared_symbol():
    from paper_1502_03391_amd import fjofc
    assert sorted(fjofc.EXPORTS) == _declared_functions()


def test_strerror_is_host_only():
    path = _lib_path()
    if not os.path.exists(path):
        pytest.skip("libfjofc.so not built")
    lib = ctypes.CDLL(path)
    lib.fjofc_strerror.restype = ctypes.c_char_p
    assert lib.fjofc_strerror(0) == b"ok"
    assert lib.fjofc_strerror(1) == b"invalid argument"
