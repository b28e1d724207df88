"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/hf.h declares, host-only calls agree with the oracle and
bad arguments are rejected before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hf():
    import paper_2508_21682_amd as hf

    if not os.path.exists(hf.LIB_PATH):
        pytest.skip("libhf.so not built")
    hf.lib()
    return hf


def _declared():
    src = open(os.path.join(ROOT, "include", "hf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hf_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(hf):
    names = _declared()
    assert len(names) >= 15
    L = C.CDLL(hf.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert sorted(hf.EXPORTS) == names


def test_status_strings(hf):
    L = hf.lib()
    assert L.hf_status_str(0) == b"ok"
    assert L.hf_status_str(6) == b"unsupported parameters"


@pytest.mark.parametrize("seed,T,d", [(0, 1, 2), (7, 5, 384), (123, 3, 33), (5, 2, 4096)])
def test_curves_match_oracle(hf, orc, seed, T, d):
    p, r = hf.curves(seed, T, d)
    po, ro = orc.curves(seed, T, d)
    assert (p == po).all() and (r == ro).all()


def test_invalid_arguments_rejected_on_host(hf):
    L = hf.lib()
    P = C.c_void_p
    dummy = P(16)
    # null pointers / bad sizes: HF_ERR_INVALID_ARG, detail in hf_last_error
    assert L.hf_hilbert_sort(None, 10, 4, 0, 0, dummy, None, None) == 1
    assert b"null" in L.hf_last_error()
    assert L.hf_hilbert_sort(dummy, 0, 4, 0, 0, dummy, None, None) == 1
    assert L.hf_hilbert_sort(dummy, 10, 5000, 0, 0, dummy, None, None) == 1
    assert L.hf_quantize(dummy, 0, 10, 40, dummy, None) == 1
    assert L.hf_quantize(dummy, 7, 10, 3, dummy, None) == 1
    p = hf.ForestParams(C.sizeof(hf.ForestParams) - 8, 4, 100, hf.HF_QUANT_AUTO, 1, 2, 0, 0, None)
    out = P()
    assert L.hf_build_forest(dummy, 0, 100, 8, C.byref(p), None, C.byref(out)) == 1
    assert b"struct_size" in L.hf_last_error()
    p = hf.ForestParams(C.sizeof(hf.ForestParams), 0, 100, hf.HF_QUANT_AUTO, 1, 2, 0, 0, None)
    assert L.hf_build_forest(dummy, 0, 100, 8, C.byref(p), None, C.byref(out)) == 1
    p = hf.ForestParams(C.sizeof(hf.ForestParams), 4097, 100, hf.HF_QUANT_AUTO, 1, 2, 0, 0, None)
    assert L.hf_build_forest(dummy, 0, 100, 8, C.byref(p), None, C.byref(out)) == 1
    assert b"n_trees" in L.hf_last_error()
    g = hf.GraphParams(C.sizeof(hf.GraphParams), 4, 60, 15, 0, hf.HF_QUANT_AUTO, 0, 1, 2, None)
    assert L.hf_knn_graph(dummy, 0, 100, 8, C.byref(g), dummy, dummy, None) == 1  # 2w >= N
    g = hf.GraphParams(C.sizeof(hf.GraphParams), 4, 8, 15, 3, hf.HF_QUANT_AUTO, 0, 1, 2, None)
    assert L.hf_knn_graph(dummy, 0, 100, 8, C.byref(g), dummy, dummy, None) == 1  # k2 < k


def test_allocator_registration_on_host(hf):
    """hf_set_allocator: NULL restores the default, an allocator needs both
    callbacks (no device work is involved in either)."""
    L = hf.lib()
    assert L.hf_set_allocator(None) == 0
    assert L.hf_set_allocator(C.byref(hf.Allocator())) == 1
    assert b"alloc and free" in L.hf_last_error()
    a = hf.Allocator(hf.ALLOC_FN(lambda n, c, s: None), hf.FREE_FN(lambda p, c, s: None), None)
    assert L.hf_set_allocator(C.byref(a)) == 0
    assert L.hf_set_allocator(None) == 0
    hf.use_torch_allocator(False)
    hf.restore_default_allocator()


def test_graph_arguments_rejected_on_host(hf):
    """Every graph argument check happens before any device work."""
    L = hf.lib()
    dummy = C.c_void_p(256)

    def gp(n=4, w=8, k=15, k2=0, sketch=0, lhash=None):
        return hf.GraphParams(C.sizeof(hf.GraphParams), n, w, k, k2, hf.HF_QUANT_AUTO, sketch, 1, 2, lhash)

    def call(g, X=dummy, dtype=0, N=1000, d=64):
        return L.hf_knn_graph(X, dtype, N, d, C.byref(g), dummy, dummy, None)

    assert call(gp(k2=257)) == 1                  # k2 above 256
    assert call(gp(w=513)) == 1                   # window above 512
    assert call(gp(k=33)) == 1                    # k above 32
    assert call(gp(n=0)) == 1                     # no orders
    assert call(gp(k2=20, sketch=7)) == 1         # unknown sketch kind
    assert call(gp(k2=20, sketch=1)) == 1         # learned sketches without a hash
    assert b"hash" in L.hf_last_error()
    assert call(gp(), X=C.c_void_p(258)) == 1     # rows not 16-byte aligned
    assert call(gp(), dtype=1) == 6               # fp32 rows: unsupported
    assert call(gp(), d=60) == 6                  # d not a multiple of 8
    g = gp()
    assert L.hf_knn_graph_debug(dummy, 0, 1000, 64, C.byref(g), dummy, dummy, dummy, None) == 1  # k2 = 0
    g = gp(k2=20)
    assert L.hf_knn_graph_debug(dummy, 0, 1000, 64, C.byref(g), dummy, dummy, None, None) == 1   # no C2 buffer


def test_invalid_handle(hf):
    L = hf.lib()
    info = hf.ForestInfo()
    assert L.hf_forest_get_info(None, C.byref(info)) == 5
    sp = hf.SearchParams(C.sizeof(hf.SearchParams), 10, 100, 50, 1, 0, 0, 0)
    assert L.hf_search(None, C.c_void_p(16), 0, 4, C.byref(sp), C.c_void_p(16), C.c_void_p(16), None) == 5
