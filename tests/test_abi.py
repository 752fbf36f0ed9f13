"""CPU checks of the C ABI boundary: the shared library loads (no GPU
needed to load it) and exports every function include/hss.h declares; the
Python binding keeps the C names; argument errors are rejected on the host
before any device work."""
import ctypes
import os
import re

import pytest

import paper_1503_05464_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hss.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(hss_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libhss.so not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(P.LIB_PATH)
    declared = _declared()
    assert "hss_compress" in declared and "hss_solve" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTED) == declared
    for name in declared:
        assert callable(getattr(P, name, None)) or name == "hss_last_error", name


def test_host_side_argument_errors():
    L = P.lib()
    out = ctypes.c_void_p()
    # NULL A / bad sizes: rejected before touching the device
    st = L.hss_compress(None, 0, 10, 10, None, None, None, ctypes.byref(out))
    assert st == P.HSS_ERR_ARG and out.value is None
    assert b"invalid" in L.hss_last_error()
    st = L.hss_compress(ctypes.c_void_p(16), 7, 10, 10, None, None, None, ctypes.byref(out))
    assert st == P.HSS_ERR_ARG
    o = P.hss_default_opts()
    assert (o.rtol, o.d0, o.dd, o.d_max, o.p_margin, o.leaf_size) == (1e-6, 64, 32, 4096, 10, 64)
    o.d0 = 0
    st = L.hss_compress(ctypes.c_void_p(16), 0, 10, 10, None, ctypes.byref(o), None, ctypes.byref(out))
    assert st == P.HSS_ERR_ARG
    assert L.hss_matvec(None, 1, None, 1, None, 1, None) == P.HSS_ERR_STATE
    assert L.hss_random_normal(0, 3, 10, 0, 1, 0, ctypes.c_void_p(16), 1, None) == P.HSS_ERR_ARG
    assert L.hss_random_normal(0, 0, 10, 0, 1, 5, ctypes.c_void_p(16), 1, None) == P.HSS_ERR_ARG
    # reduced-precision sampling needs FP32 storage; unknown modes are rejected
    o = P.hss_default_opts()
    o.sample_prec = P.HSS_SAMPLE_BF16X3
    st = L.hss_compress(ctypes.c_void_p(16), P.HSS_F64, 10, 10, None, ctypes.byref(o), None, ctypes.byref(out))
    assert st == P.HSS_ERR_ARG and b"FP32" in L.hss_last_error()
    o.sample_prec = 9
    st = L.hss_compress(ctypes.c_void_p(16), P.HSS_F32, 10, 10, None, ctypes.byref(o), None, ctypes.byref(out))
    assert st == P.HSS_ERR_ARG
    st = L.hss_sample(ctypes.c_void_p(16), P.HSS_F64, P.HSS_SAMPLE_F32, 10, 10, None, 1, ctypes.c_void_p(16),
                      None, 1, ctypes.c_void_p(16), None, 1, None)
    assert st == P.HSS_ERR_ARG
    assert L.hss_id_batched(-1, None, None, None, None, 0.1, None, None, None, None) == P.HSS_ERR_ARG


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", "/nonexistent/libhss.so")
    with pytest.raises(RuntimeError, match="no fallback"):
        P.lib()


@pytest.mark.parametrize("tree, n, msg", [
    (([0, 0, 5], [10, 5, 10], [1, -1, -1], [2, -1, -1]), 12, b"root interval"),
    (([0, 0, 6], [10, 5, 10], [1, -1, -1], [2, -1, -1]), 10, b"do not split"),
    (([0, 0, 5], [10, 5, 10], [1, -1, -1], [-1, -1, -1]), 10, b"one child"),
    (([0, 0, 5], [10, 5, 10], [1, -1, -1], [7, -1, -1]), 10, b"bad child"),
    (([0, 0, 5, 0], [10, 5, 10, 5], [1, -1, -1, -1], [2, -1, -1, -1]), 10, b"not reachable"),
    (([0, 0, 0], [10, 0, 10], [1, -1, -1], [2, -1, -1]), 10, b"empty"),
    (([0, 0, 5, 0, 5], [10, 5, 10, 5, 10], [1, 3, -1, -1, -1], [2, 4, -1, -1, -1]), 10, b"do not split"),
], ids=["root", "split", "one-child", "child-index", "unreachable", "empty", "grandchildren"])
def test_user_tree_errors(tree, n, msg):
    """A user tree that is not a binary partition of [0, n) is rejected on
    the host, before any device work, with a message naming the defect."""
    L = P.lib()
    out = ctypes.c_void_p()
    t, keep = P._tree_struct(tree)
    st = L.hss_compress(ctypes.c_void_p(16), P.HSS_F64, n, n, ctypes.byref(t), None, None, ctypes.byref(out))
    assert st == P.HSS_ERR_ARG and out.value is None
    assert msg in L.hss_last_error(), L.hss_last_error()


def test_set_allocator_arguments():
    """hss_set_allocator takes both callbacks or neither (checked on the host,
    no device needed); NULL/NULL restores the library's own pool."""
    L = P.lib()
    fa = P._ALLOC_FN(lambda nbytes, dev, stream, ctx: None)
    ff = P._FREE_FN(lambda p, nbytes, dev, stream, ctx: None)
    assert L.hss_set_allocator(fa, P._FREE_FN(), None) == P.HSS_ERR_ARG
    assert L.hss_set_allocator(P._ALLOC_FN(), ff, None) == P.HSS_ERR_ARG
    assert b"both" in L.hss_last_error()
    assert L.hss_set_allocator(P._ALLOC_FN(), P._FREE_FN(), None) == P.HSS_OK
    with pytest.raises(ValueError):
        P.hss_set_allocator(lambda *a: 0, None)
