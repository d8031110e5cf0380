"""The C-ABI library loads and exports every symbol include/relnn.h
declares (CPU only: no compute call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "relnn.h")
LIB = os.path.join(ROOT, "paper_2605_24207_amd", "librelnn.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(relnn_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ["relnn_build_index", "relnn_layer_fwd", "relnn_layer_bwd", "relnn_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librelnn.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librelnn.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2605_24207_amd import _lib

    assert set(declared()) <= set(_lib.exported_symbols())


@pytest.mark.skipif(not os.path.exists(LIB), reason="librelnn.so not built")
def test_validation_errors_without_gpu():
    from paper_2605_24207_amd import _lib

    L = _lib.lib()
    out = ctypes.c_void_p()
    assert L.relnn_build_index(None, None, ctypes.byref(out)) == _lib.E_INVALID
    assert b"NULL" in L.relnn_last_error()
    d = _lib.JoinDesc()
    d.n_link, d.n_cols, d.n_atoms = 10, 0, 1
    assert L.relnn_build_index(ctypes.byref(d), None, ctypes.byref(out)) == _lib.E_INVALID
