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


@pytest.mark.skipif(not os.path.exists(LIB), reason="librelnn.so not built")
def test_more_validation_errors_without_gpu():
    from paper_2605_24207_amd import _lib

    L = _lib.lib()
    out = ctypes.c_void_p()
    # serving: NULL descriptor, then a descriptor with NULL relations
    assert L.relnn_serve_create(None, ctypes.byref(out)) == _lib.E_INVALID
    d = _lib.ServeDesc()
    d.n_user = d.n_item = d.n_cat = 10
    assert L.relnn_serve_create(ctypes.byref(d), ctypes.byref(out)) == _lib.E_INVALID
    # layer calls without an index
    ld = _lib.LayerDesc()
    assert L.relnn_layer_fwd(None, ctypes.byref(ld), None, None, None, None, None, None, None, 0, None) == \
        _lib.E_INVALID
    n = ctypes.c_size_t()
    assert L.relnn_workspace_size(None, ctypes.byref(ld), 0, ctypes.byref(n)) != _lib.OK
    assert L.relnn_serve_destroy(None) == _lib.OK
    # timing hooks are host-only
    assert L.relnn_timing_enable(0) == _lib.OK
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    assert L.relnn_timing_read(b"fwd_fused", ctypes.byref(ms), ctypes.byref(cnt)) == _lib.OK
    assert cnt.value == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="librelnn.so not built")
def test_static_variant_host_checks_without_gpu():
    from paper_2605_24207_amd import _lib

    L = _lib.lib()
    n = ctypes.c_size_t()
    assert L.relnn_static_scratch_bytes(ctypes.byref(n)) == _lib.OK and n.value == 32 << 20
    assert L.relnn_static_scratch_bytes(None) == _lib.E_INVALID
    ld = _lib.LayerDesc()
    assert L.relnn_layer_fwd_static(None, ctypes.byref(ld), None, None, None, None, None, None, None) == \
        _lib.E_INVALID
    ld.flags = _lib.PLAIN
    assert L.relnn_layer_fwd_static(None, ctypes.byref(ld), None, None, None, None, None, None, None) == \
        _lib.E_UNSUPPORTED


@pytest.mark.skipif(not os.path.exists(LIB), reason="librelnn.so not built")
def test_union_backward_and_dense_host_checks_without_gpu():
    from paper_2605_24207_amd import _lib

    L = _lib.lib()
    n = ctypes.c_size_t()
    # union calls without a union
    assert L.relnn_union_bwd_workspace_size(None, None, 0, 16, ctypes.byref(n)) == _lib.E_INVALID
    assert L.relnn_union_bwd(None, None, 0, 0, None, None, None, None, None, 16, None, None, None, None, None, None,
                             None, None, None, 0, None) == _lib.E_INVALID
    # dense layout: a non-positive width, then keys missing for a non-empty output
    assert L.relnn_out_dense(None, 0, None, 0, 10, None, None, None) == _lib.E_INVALID
    assert L.relnn_out_dense(None, 5, None, 16, 10, None, None, None) == _lib.E_INVALID
    assert b"required" in L.relnn_last_error()
