"""The C-ABI library loads and exports every symbol include/tucker_hip.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1804_09494_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1804_09494_amd import build
        build.build(force=False)
    return L.load(), L


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "tucker_hip.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tk_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib, L = _lib()
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(n for n, _, _ in L.SIGNATURES) == syms


def test_status_strings_and_default_options():
    lib, L = _lib()
    assert lib.tk_status_string(0) == b"ok"
    assert lib.tk_status_string(1) == b"invalid argument"
    o = L.tk_options()
    assert lib.tk_default_options(ctypes.byref(o)) == 0
    assert o.wg_nnz_target == 0 and o.refine == 1 and o.complete_rank_deficient == 1
    assert lib.tk_default_options(None) == 1


def test_null_context_is_rejected():
    lib, L = _lib()
    assert lib.tk_load_coo(None, 3, None, 0, None, None, 0, 0) == 1
    assert lib.tk_load_coo_begin(None, 3, None, 0, 0) == 1
    assert lib.tk_load_coo_append(None, 0, None, None, 0) == 1
    assert lib.tk_load_coo_end(None) == 1
    assert lib.tk_set_ranks(None, None) == 1
    assert lib.tk_hooi_iterate(None, 1, None) == 1
    assert lib.tk_ttm_chain(None, 0, None, None, 0) == 1
    assert lib.tk_create(0, None, None, None) == 1


def test_create_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib, L = _lib()
    h = ctypes.c_void_p()
    assert lib.tk_create(0, None, None, ctypes.byref(h)) == 4
    assert h.value is None


def test_product_path_has_no_fallback():
    """The binding must import nothing from the oracle and must fail loudly
    without the built library."""
    import paper_1804_09494_amd.api as api
    import paper_1804_09494_amd._lib as L
    src = open(api.__file__).read() + open(L.__file__).read()
    assert "oracle" not in src
    assert "raise ImportError" in open(L.__file__).read()
