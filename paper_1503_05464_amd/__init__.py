"""Python binding of the MI355X randomized HSS library (``include/hss.h``).

Argument marshalling only: every step runs in the HIP kernels of
``lib/libhss.so``.  PyTorch tensors provide device memory and streams.  The
functions keep the C names:

    hss_compress, hss_matvec, hss_factor, hss_solve, hss_stats, hss_ranks,
    hss_export_node, hss_import, hss_destroy, hss_release_cached_memory,
    hss_set_allocator, hss_random_normal, hss_sample, hss_id_batched,
    hss_default_opts

``use_torch_allocator()`` points hss_set_allocator at PyTorch's caching
allocator, so that the library and PyTorch share one device memory pool.

The library is loaded on first use; if it has not been built (see
``build.py``) every call raises ``RuntimeError`` -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libhss.so")

HSS_OK, HSS_NOT_CONVERGED = 0, 1
HSS_ERR_ARG, HSS_ERR_ALLOC, HSS_ERR_HIP, HSS_ERR_STATE, HSS_ERR_SINGULAR = -1, -2, -3, -4, -5
HSS_F64, HSS_F32 = 0, 1
HSS_SAMPLE_F64 = 0
HSS_SAMPLE_F32 = 1
HSS_SAMPLE_BF16X3 = 2
_PREC = {"f64": HSS_SAMPLE_F64, "f32": HSS_SAMPLE_F32, "bf16x3": HSS_SAMPLE_BF16X3}

EXPORTED = [
    "hss_default_opts", "hss_compress", "hss_compress_batched", "hss_matvec", "hss_matvec_batched",
    "hss_factor",
    "hss_solve", "hss_stats",
    "hss_ranks", "hss_export_node", "hss_import", "hss_destroy", "hss_release_cached_memory",
    "hss_set_allocator", "hss_last_error",
    "hss_random_normal", "hss_sample", "hss_sample_noalloc", "hss_id_batched", "hss_gemm_batched",
    "hss_gemm_variants",
    "hss_server_default_opts", "hss_server_create", "hss_server_submit", "hss_server_submit_request",
    "hss_server_wait", "hss_server_release", "hss_server_destroy",
]


class hss_server_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_longlong), ("max_batch", C.c_int), ("workers", C.c_int)]


class hss_request_info(C.Structure):
    _fields_ = [("status", C.c_int), ("batch_size", C.c_int), ("d_final", C.c_int), ("max_rank", C.c_int),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("handle", C.c_void_p)]


class hss_server_request(C.Structure):
    _fields_ = [("A", C.c_void_p), ("dtype", C.c_int), ("n", C.c_longlong), ("lda", C.c_longlong),
                ("opts", C.c_void_p), ("handle", C.c_void_p), ("nrhs", C.c_int), ("b", C.c_void_p),
                ("ldb", C.c_longlong), ("x", C.c_void_p), ("ldx", C.c_longlong), ("keep", C.c_int)]


class HSSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hss status {status}: {msg}")
        self.status = status


class hss_opts(C.Structure):
    _fields_ = [
        ("rtol", C.c_double), ("d0", C.c_int), ("dd", C.c_int), ("d_max", C.c_int),
        ("p_margin", C.c_int), ("seed", C.c_ulonglong), ("leaf_size", C.c_int),
        ("sample_prec", C.c_int), ("R_user_r", C.c_void_p), ("R_user_c", C.c_void_p),
        ("ld_R_user", C.c_longlong),
    ]


class hss_tree(C.Structure):
    _fields_ = [("n_nodes", C.c_int), ("lo", C.POINTER(C.c_int)), ("hi", C.POINTER(C.c_int)),
                ("left", C.POINTER(C.c_int)), ("right", C.POINTER(C.c_int))]


class hss_stats_t(C.Structure):
    _fields_ = [
        ("n", C.c_longlong), ("n_nodes", C.c_int), ("height", C.c_int), ("d_final", C.c_int),
        ("passes", C.c_int), ("converged", C.c_int), ("max_rank", C.c_int),
        ("generator_bytes", C.c_longlong), ("sample_flops", C.c_double),
        ("t_total_ms", C.c_double), ("t_sample_ms", C.c_double), ("t_levels_ms", C.c_double),
        ("t_id_ms", C.c_double), ("n_sample_launches", C.c_int), ("t_sample_gemm_ms", C.c_double),
        ("sample_gemm_flops", C.c_double), ("sample_gemm_bytes", C.c_double),
        ("id_flops", C.c_double), ("t_level_gemm_ms", C.c_double), ("level_gemm_bytes", C.c_double),
        ("t_gather_ms", C.c_double), ("gather_bytes", C.c_double),
    ]


class hss_node_generators(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("Jr", "Jc", "Er", "Ec", "Ir", "Ic", "D", "B12", "B21")]


# void* alloc(size_t bytes, int device, void* stream, void* ctx)
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p, C.c_void_p)
# void free(void* p, size_t bytes, int device, void* stream, void* ctx)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p, C.c_void_p)

_lib = None
_allocator_keep = None  # the ctypes callbacks in use must outlive their registration


def lib() -> C.CDLL:
    """The loaded shared library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1503_05464_amd/build.py "
                               "(there is no fallback implementation)")
        L = C.CDLL(LIB_PATH)
        vp, ll, i, d = C.c_void_p, C.c_longlong, C.c_int, C.c_double
        L.hss_last_error.restype = C.c_char_p
        L.hss_default_opts.argtypes = [C.POINTER(hss_opts)]
        L.hss_default_opts.restype = None
        L.hss_compress.argtypes = [vp, i, ll, ll, C.POINTER(hss_tree), C.POINTER(hss_opts), vp,
                                   C.POINTER(vp)]
        L.hss_compress_batched.argtypes = [i, vp, i, vp, vp, C.POINTER(hss_tree), C.POINTER(hss_opts),
                                           vp, vp, vp]
        L.hss_matvec.argtypes = [vp, i, vp, ll, vp, ll, vp]
        L.hss_matvec_batched.argtypes = [i, vp, i, vp, vp, vp, vp, vp]
        L.hss_server_default_opts.argtypes = [C.POINTER(hss_server_opts)]
        L.hss_server_default_opts.restype = None
        L.hss_server_create.argtypes = [C.POINTER(hss_server_opts), C.POINTER(vp)]
        L.hss_server_submit.argtypes = [vp, vp, i, ll, ll, C.POINTER(hss_opts), i, vp, ll, vp, ll, vp,
                                        C.POINTER(C.c_longlong)]
        L.hss_server_submit_request.argtypes = [vp, C.POINTER(hss_server_request), vp, C.POINTER(C.c_longlong)]
        L.hss_server_wait.argtypes = [vp, C.c_longlong, C.POINTER(hss_request_info)]
        L.hss_server_release.argtypes = [vp, vp]
        L.hss_server_destroy.argtypes = [vp]
        L.hss_server_destroy.restype = None
        L.hss_factor.argtypes = [vp, vp]
        L.hss_solve.argtypes = [vp, i, vp, ll, vp, ll, vp]
        L.hss_stats.argtypes = [vp, C.POINTER(hss_stats_t)]
        L.hss_ranks.argtypes = [vp, vp, vp, vp, vp]
        L.hss_export_node.argtypes = [vp, i, C.POINTER(hss_node_generators)]
        L.hss_import.argtypes = [ll, C.POINTER(hss_tree), vp, vp, vp, C.POINTER(vp)]
        L.hss_destroy.argtypes = [vp]
        L.hss_destroy.restype = None
        L.hss_release_cached_memory.argtypes = []
        L.hss_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
        L.hss_random_normal.argtypes = [C.c_ulonglong, i, ll, i, i, i, vp, ll, vp]
        L.hss_sample.argtypes = [vp, i, i, ll, ll, vp, i, vp, vp, ll, vp, vp, ll, vp]
        L.hss_sample_noalloc.argtypes = [vp, i, i, ll, ll, vp, i, vp, vp, ll, vp, vp, ll, vp]
        L.hss_id_batched.argtypes = [i, vp, vp, vp, vp, d, vp, vp, vp, vp]
        L.hss_gemm_batched.argtypes = [i, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, d, d, i, vp]
        L.hss_gemm_variants.argtypes = []
        for f in EXPORTED:
            if f not in ("hss_default_opts", "hss_destroy", "hss_last_error", "hss_server_default_opts",
                         "hss_server_destroy", "hss_gemm_variants"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(st: int, allow=(HSS_OK,)) -> int:
    if st not in allow:
        raise HSSError(st, lib().hss_last_error().decode(errors="replace"))
    return st


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _np_ptr(a: np.ndarray) -> C.c_void_p:
    return C.c_void_p(a.ctypes.data)


def _tree_struct(tree):
    """tree: None or (lo, hi, left, right) integer sequences."""
    if tree is None:
        return None, None
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.int32)) for a in tree]
    t = hss_tree(len(arrs[0]), *[a.ctypes.data_as(C.POINTER(C.c_int)) for a in arrs])
    return t, arrs


def hss_default_opts() -> hss_opts:
    o = hss_opts()
    lib().hss_default_opts(C.byref(o))
    return o


class HSSHandle:
    """Owns an hss_handle; destroyed with the object (or hss_destroy)."""

    def __init__(self, ptr: C.c_void_p, n: int, status: int, keep=None):
        self.ptr = ptr
        self.n = n
        self.status = status
        self._keep = keep

    @property
    def converged(self) -> bool:
        return self.status == HSS_OK

    def __del__(self):
        try:
            hss_destroy(self)
        except Exception:
            pass


def hss_compress(A, tree=None, *, rtol=1e-6, d0=64, dd=32, d_max=4096, p_margin=10, seed=0,
                 leaf_size=64, R_user=None, sample_prec="f64", stream=None) -> HSSHandle:
    """Compress the square CUDA tensor A (float32 or float64, row-major
    with unit column stride).  R_user: optional (R^r, R^c) CUDA float64
    tensors n x >= d_max (row-major) used instead of the Philox columns.
    sample_prec: "f64", or "f32" / "bf16x3" for a float32 A."""
    import torch

    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a square CUDA matrix with unit column stride")
    dt = {torch.float64: HSS_F64, torch.float32: HSS_F32}.get(A.dtype)
    if dt is None:
        raise ValueError("A must be float32 or float64")
    o = hss_default_opts()
    o.rtol, o.d0, o.dd, o.d_max, o.p_margin = float(rtol), int(d0), int(dd), int(d_max), int(p_margin)
    o.seed, o.leaf_size = int(seed), int(leaf_size)
    o.sample_prec = _PREC[sample_prec]
    keep = [A]
    if R_user is not None:
        rr, rc = R_user
        for r in (rr, rc):
            if r.dtype != torch.float64 or not r.is_cuda or r.stride(1) != 1 or r.shape[0] != A.shape[0] \
                    or r.shape[1] < d_max or r.stride(0) != rr.stride(0):
                raise ValueError("R_user tensors must be CUDA float64 n x >= d_max, same layout")
        o.R_user_r, o.R_user_c, o.ld_R_user = rr.data_ptr(), rc.data_ptr(), rr.stride(0)
        keep += [rr, rc]
    t, arrs = _tree_struct(tree)
    out = C.c_void_p()
    st = lib().hss_compress(_ptr(A), dt, A.shape[0], A.stride(0), C.byref(t) if t else None,
                            C.byref(o), _stream(stream), C.byref(out))
    _check(st, (HSS_OK, HSS_NOT_CONVERGED))
    return HSSHandle(out, A.shape[0], st)


def hss_compress_batched(As, trees=None, *, rtol=1e-6, d0=64, dd=32, d_max=4096, p_margin=10, seed=0,
                         leaf_size=64, sample_prec="f64", stream=None) -> list:
    """Compress the square CUDA tensors in As (all float32 or all float64)
    together: one adaptive pass schedule for all, each level of every
    unfinished matrix in one batched launch per phase.  trees: None or one
    (lo, hi, left, right) per matrix.  Returns one HSSHandle per matrix."""
    import torch

    if not As:
        return []
    dts = {A.dtype for A in As}
    if len(dts) != 1 or next(iter(dts)) not in (torch.float32, torch.float64):
        raise ValueError("the matrices must all be float32 or all float64")
    for A in As:
        if A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1 or not A.is_cuda:
            raise ValueError("each A must be a square CUDA matrix with unit column stride")
    dt = HSS_F32 if As[0].dtype == torch.float32 else HSS_F64
    nm = len(As)
    o = hss_default_opts()
    o.rtol, o.d0, o.dd, o.d_max, o.p_margin = float(rtol), int(d0), int(dd), int(d_max), int(p_margin)
    o.seed, o.leaf_size = int(seed), int(leaf_size)
    o.sample_prec = _PREC[sample_prec]
    ptrs = np.array([A.data_ptr() for A in As], dtype=np.uint64)
    ns = np.array([A.shape[0] for A in As], dtype=np.int64)
    lds = np.array([A.stride(0) for A in As], dtype=np.int64)
    keep = []
    tarr = None
    if trees is not None:
        tarr = (hss_tree * nm)()
        for q, tr in enumerate(trees):
            t, arrs = _tree_struct(tr)
            tarr[q] = t
            keep.append(arrs)
    outs = (C.c_void_p * nm)()
    status = np.zeros(nm, dtype=np.int32)
    st = lib().hss_compress_batched(nm, _np_ptr(ptrs), dt, _np_ptr(ns), _np_ptr(lds), tarr, C.byref(o),
                                    _stream(stream), outs, _np_ptr(status))
    _check(st, (HSS_OK, HSS_NOT_CONVERGED))
    return [HSSHandle(C.c_void_p(outs[q]), int(ns[q]), int(status[q])) for q in range(nm)]


def hss_matvec(h: HSSHandle, x, b=None, stream=None):
    """b = A_HSS x for a CUDA float64 tensor x (n or n x nrhs)."""
    import torch

    vec = x.dim() == 1
    x2 = x.reshape(-1, 1) if vec else x
    if x2.dtype != torch.float64 or x2.stride(1) != 1 or x2.shape[0] != h.n:
        raise ValueError("x must be float64, n x nrhs with unit column stride")
    if b is None:
        b = torch.empty_like(x2, memory_format=torch.contiguous_format)
    b2 = b.reshape(-1, 1) if b.dim() == 1 else b
    _check(lib().hss_matvec(h.ptr, x2.shape[1], _ptr(x2), x2.stride(0), _ptr(b2), b2.stride(0),
                            _stream(stream)))
    return b2.reshape(-1) if vec else b2


def hss_matvec_batched(hs, xs, bs=None, stream=None):
    """b[i] = A_HSS[i] x[i] for several handles in one call (every phase of
    the matvec is one launch over all of them).  xs: CUDA float64 tensors,
    n_i x nrhs (the same nrhs for all) with unit column stride."""
    import torch

    if len(hs) != len(xs):
        raise ValueError("one x per handle")
    if not hs:
        return []
    nrhs = xs[0].shape[1]
    for h, x in zip(hs, xs):
        if x.dim() != 2 or x.dtype != torch.float64 or x.stride(1) != 1 or x.shape[0] != h.n or x.shape[1] != nrhs:
            raise ValueError("each x must be float64, n_i x nrhs with unit column stride")
    if bs is None:
        bs = [torch.empty_like(x, memory_format=torch.contiguous_format) for x in xs]
    hp = np.array([h.ptr.value if hasattr(h.ptr, "value") else h.ptr for h in hs], dtype=np.uint64)
    xp = np.array([x.data_ptr() for x in xs], dtype=np.uint64)
    bp = np.array([b.data_ptr() for b in bs], dtype=np.uint64)
    ldx = np.array([x.stride(0) for x in xs], dtype=np.int64)
    ldb = np.array([b.stride(0) for b in bs], dtype=np.int64)
    _check(lib().hss_matvec_batched(len(hs), _np_ptr(hp), nrhs, _np_ptr(xp), _np_ptr(ldx), _np_ptr(bp),
                                    _np_ptr(ldb), _stream(stream)))
    return bs


def hss_factor(h: HSSHandle, stream=None) -> None:
    _check(lib().hss_factor(h.ptr, _stream(stream)))


def hss_solve(h: HSSHandle, b, x=None, stream=None):
    import torch

    vec = b.dim() == 1
    b2 = b.reshape(-1, 1) if vec else b
    if b2.dtype != torch.float64 or b2.stride(1) != 1 or b2.shape[0] != h.n:
        raise ValueError("b must be float64, n x nrhs with unit column stride")
    if x is None:
        x = torch.empty_like(b2, memory_format=torch.contiguous_format)
    x2 = x.reshape(-1, 1) if x.dim() == 1 else x
    _check(lib().hss_solve(h.ptr, b2.shape[1], _ptr(b2), b2.stride(0), _ptr(x2), x2.stride(0),
                           _stream(stream)))
    return x2.reshape(-1) if vec else x2


def hss_stats(h: HSSHandle) -> dict:
    s = hss_stats_t()
    _check(lib().hss_stats(h.ptr, C.byref(s)))
    return {f: getattr(s, f) for f, _ in hss_stats_t._fields_}


def _n_nodes(h: HSSHandle) -> int:
    return hss_stats(h)["n_nodes"]


def hss_ranks(h: HSSHandle):
    nn = _n_nodes(h)
    out = [np.zeros(nn, dtype=np.int32) for _ in range(4)]
    _check(lib().hss_ranks(h.ptr, *[_np_ptr(a) for a in out]))
    return tuple(out)


def hss_export_node(h: HSSHandle, node: int, tree_children=None) -> dict:
    """Host copies of one node's generators (numpy).  tree_children: the
    (left, right) child numbers of `node`, needed for B sizes."""
    kr, kc, mr, mc = hss_ranks(h)
    g = hss_node_generators()
    res = {}

    def buf(name, shape, dtype):
        a = np.zeros(shape, dtype=dtype)
        res[name] = a
        setattr(g, name, a.ctypes.data if a.size else None)

    if node != 0:
        buf("Jr", (kr[node],), np.int32)
        buf("Jc", (kc[node],), np.int32)
        buf("Er", (mr[node] - kr[node], kr[node]), np.float64)
        buf("Ec", (mc[node] - kc[node], kc[node]), np.float64)
        buf("Ir", (kr[node],), np.int32)
        buf("Ic", (kc[node],), np.int32)
    if tree_children is None or tree_children[0] < 0:
        buf("D", (mr[node], mr[node]), np.float64)
    else:
        a, b = tree_children
        buf("B12", (kr[a], kc[b]), np.float64)
        buf("B21", (kr[b], kc[a]), np.float64)
    _check(lib().hss_export_node(h.ptr, node, C.byref(g)))
    return res


def hss_import(n: int, tree, kr, kc, nodes) -> HSSHandle:
    """Handle from host generators: tree = (lo, hi, left, right); nodes[t] a
    dict with keys among Jr, Jc, Er, Ec, D, B12, B21 (numpy arrays)."""
    t, arrs = _tree_struct(tree)
    keep = [arrs]
    gens = (hss_node_generators * len(nodes))()
    for q, nd in enumerate(nodes):
        for f in ("Jr", "Jc", "Er", "Ec", "D", "B12", "B21"):
            if f in nd and nd[f] is not None:
                a = np.ascontiguousarray(nd[f], dtype=np.int32 if f in ("Jr", "Jc") else np.float64)
                keep.append(a)
                setattr(gens[q], f, a.ctypes.data if a.size else None)
    kr = np.ascontiguousarray(kr, dtype=np.int32)
    kc = np.ascontiguousarray(kc, dtype=np.int32)
    out = C.c_void_p()
    _check(lib().hss_import(int(n), C.byref(t), _np_ptr(kr), _np_ptr(kc), gens, C.byref(out)))
    return HSSHandle(out, n, HSS_OK)


def hss_destroy(h: HSSHandle) -> None:
    if h is not None and h.ptr:
        lib().hss_destroy(h.ptr)
        h.ptr = C.c_void_p()


def hss_release_cached_memory() -> None:
    """Returns the device and pinned host blocks the library keeps for
    reuse to the runtime (blocks of live handles are kept)."""
    _check(lib().hss_release_cached_memory())


def hss_set_allocator(alloc=None, free=None) -> None:
    """Device allocator of the library (hss_set_allocator): ``alloc(bytes,
    device, stream) -> int address`` (0 on failure) and ``free(address,
    bytes, device, stream)``, with stream the hipStream_t as an int (0: the
    default stream); both None restores the library's own pool."""
    global _allocator_keep
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        _check(lib().hss_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
        _allocator_keep = None
        return

    def _a(nbytes, dev, stream, ctx):
        try:
            return int(alloc(int(nbytes), int(dev), int(stream or 0))) or None
        except Exception:  # an exception must not cross into C: report failure
            return None

    def _f(p, nbytes, dev, stream, ctx):
        try:
            free(int(p), int(nbytes), int(dev), int(stream or 0))
        except Exception:
            pass

    fa, ff = _ALLOC_FN(_a), _FREE_FN(_f)
    _check(lib().hss_set_allocator(fa, ff, None))
    _allocator_keep = (fa, ff)


def use_torch_allocator(on: bool = True) -> None:
    """Let the library allocate its device memory from PyTorch's caching
    allocator (on=False: back to the library's own pool).  Blocks are taken
    for the stream the library uses them on and given back when it is done
    with them, with PyTorch's stream-ordered reuse."""
    import torch

    if not on:
        hss_set_allocator(None, None)
        return

    def alloc(nbytes, dev, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, dev, stream)

    def free(p, nbytes, dev, stream):
        torch.cuda.caching_allocator_delete(p)

    hss_set_allocator(alloc, free)


def hss_random_normal(seed: int, which: int, n: int, col0: int, col1: int, out=None, stream=None,
                      sample_prec: str = "f64"):
    import torch

    if out is None:
        out = torch.empty((n, col1 - col0), dtype=torch.float64, device="cuda")
    _check(lib().hss_random_normal(int(seed), int(which), int(n), int(col0), int(col1),
                                   _PREC[sample_prec], _ptr(out), out.stride(0), _stream(stream)))
    return out


def hss_sample(A, Rr=None, Rc=None, leaf_of=None, stream=None, sample_prec: str = "f64"):
    """(Sr, Sc) = ((A - M) Rr, (A - M)^T Rc); M = leaf diagonal blocks
    when leaf_of (CUDA int32, leaf ordinal of each index) is given.
    sample_prec "f32" / "bf16x3" need FP32 A and R from hss_random_normal
    with the same sample_prec."""
    import torch

    dt = {torch.float64: HSS_F64, torch.float32: HSS_F32}[A.dtype]
    R = Rr if Rr is not None else Rc
    ncols = R.shape[1]
    Sr = torch.empty((A.shape[0], ncols), dtype=torch.float64, device=A.device) if Rr is not None else None
    Sc = torch.empty((A.shape[0], ncols), dtype=torch.float64, device=A.device) if Rc is not None else None
    if Rr is not None and Rc is not None and Rr.stride(0) != Rc.stride(0):
        raise ValueError("Rr and Rc must share a leading dimension")
    S = Sr if Sr is not None else Sc
    _check(lib().hss_sample(_ptr(A), dt, _PREC[sample_prec], A.shape[0], A.stride(0),
                            _ptr(leaf_of) if leaf_of is not None else None, ncols,
                            _ptr(Rr) if Rr is not None else None, _ptr(Rc) if Rc is not None else None,
                            R.stride(0), _ptr(Sr) if Sr is not None else None,
                            _ptr(Sc) if Sc is not None else None, S.stride(0), _stream(stream)))
    return Sr, Sc


def hss_sample_noalloc(A, Rr, Rc, Sr, Sc, leaf_of=None, stream=None, sample_prec: str = "f64"):
    """hss_sample into caller-provided outputs Sr, Sc (CUDA float64, n x
    ncols, or None together with their R) with the library's fixed scratch
    as workspace: the call allocates no device memory.  Returns (Sr, Sc)."""
    import torch

    dt = {torch.float64: HSS_F64, torch.float32: HSS_F32}[A.dtype]
    R = Rr if Rr is not None else Rc
    S = Sr if Sr is not None else Sc
    if Rr is not None and Rc is not None and Rr.stride(0) != Rc.stride(0):
        raise ValueError("Rr and Rc must share a leading dimension")
    if Sr is not None and Sc is not None and Sr.stride(0) != Sc.stride(0):
        raise ValueError("Sr and Sc must share a leading dimension")
    _check(lib().hss_sample_noalloc(_ptr(A), dt, _PREC[sample_prec], A.shape[0], A.stride(0),
                                    _ptr(leaf_of) if leaf_of is not None else None, R.shape[1],
                                    _ptr(Rr) if Rr is not None else None,
                                    _ptr(Rc) if Rc is not None else None, R.stride(0),
                                    _ptr(Sr) if Sr is not None else None,
                                    _ptr(Sc) if Sc is not None else None, S.stride(0), _stream(stream)))
    return Sr, Sc


def hss_gemm_variants() -> int:
    return int(lib().hss_gemm_variants())


def hss_gemm_batched(As, Bs, Cs, transA=None, alpha=1.0, beta=0.0, variant=-1, stream=None):
    """C_p = alpha op(A_p) B_p + beta C_p for lists of CUDA float64 matrices
    (row-major, unit column stride), in one launch of the library's batched
    GEMM with tile shape `variant` (-1: the tuning table's choice).  Returns
    Cs."""
    nprob = len(As)
    if not (len(Bs) == len(Cs) == nprob):
        raise ValueError("one B and one C per A")
    tr = [bool(t) for t in (transA or [False] * nprob)]
    for a, b, c in zip(As, Bs, Cs):
        for x in (a, b, c):
            if x.dim() != 2 or not x.is_cuda or (x.numel() > 0 and x.stride(1) != 1):
                raise ValueError("matrices must be 2-D CUDA tensors with unit column stride")
    M = np.array([c.shape[0] for c in Cs], dtype=np.int32)
    N = np.array([c.shape[1] for c in Cs], dtype=np.int32)
    K = np.array([b.shape[0] for b in Bs], dtype=np.int32)
    for q, (a, t) in enumerate(zip(As, tr)):
        if (a.shape if not t else a.shape[::-1]) != (M[q], K[q]) or Bs[q].shape[1] != N[q]:
            raise ValueError(f"problem {q}: shapes do not match")
    ptr = lambda xs: np.array([x.data_ptr() for x in xs], dtype=np.uint64)
    ld = lambda xs: np.array([max(1, x.shape[1]) if x.numel() == 0 else max(1, x.stride(0)) for x in xs],
                            dtype=np.int64)
    ap, bp, cp = ptr(As), ptr(Bs), ptr(Cs)
    la, lb, lc = ld(As), ld(Bs), ld(Cs)
    ta = np.array(tr, dtype=np.int32)
    _check(lib().hss_gemm_batched(nprob, _np_ptr(M), _np_ptr(N), _np_ptr(K), _np_ptr(ap), _np_ptr(la),
                                  _np_ptr(ta), _np_ptr(bp), _np_ptr(lb), _np_ptr(cp), _np_ptr(lc),
                                  float(alpha), float(beta), int(variant), _stream(stream)))
    return Cs


def hss_id_batched(Ys, rtol: float, stream=None):
    """Interpolative decompositions of the d x m matrices whose columns are
    the rows of the CUDA float64 tensors in Ys (each m x d, unit column
    stride).  Returns a list of (k, perm, E) with perm = J then the rest."""
    import torch

    np_ = len(Ys)
    m = np.array([y.shape[0] for y in Ys], dtype=np.int32)
    d = np.array([y.shape[1] for y in Ys], dtype=np.int32)
    ldy = np.array([max(y.stride(0), y.shape[1]) for y in Ys], dtype=np.int64)
    perms = [torch.empty(int(mm), dtype=torch.int32, device="cuda") for mm in m]
    es = [torch.empty(int(mm) * int(mm) // 4 + 1, dtype=torch.float64, device="cuda") for mm in m]
    ys_p = np.array([y.data_ptr() for y in Ys], dtype=np.uint64)
    pp = np.array([p.data_ptr() for p in perms], dtype=np.uint64)
    ep = np.array([e.data_ptr() for e in es], dtype=np.uint64)
    k = np.zeros(np_, dtype=np.int32)
    _check(lib().hss_id_batched(np_, _np_ptr(ys_p), _np_ptr(m), _np_ptr(d), _np_ptr(ldy), float(rtol),
                                _np_ptr(pp), _np_ptr(ep), _np_ptr(k), _stream(stream)))
    out = []
    for q in range(np_):
        kk, mm = int(k[q]), int(m[q])
        out.append((kk, perms[q].cpu().numpy(), es[q][: (mm - kk) * kk].reshape(mm - kk, kk).cpu().numpy()))
    return out


class ResidentHandle:
    """A compressed and factored handle kept resident in a server (a
    compress request with keep=True); owned by the server until
    ``HSSServer.release``."""

    def __init__(self, ptr: int, n: int):
        self.ptr = C.c_void_p(ptr)
        self.n = n


class HSSServer:
    """The serving loop of the C ABI (hss_server_*): compress + ULV factor +
    solve requests and solve-only requests on resident handles, admitted by
    a device-memory budget and batched with the compatible requests waiting
    at the time, on several streams."""

    def __init__(self, hbm_budget: int = 0, max_batch: int = 32, workers: int = 2):
        o = hss_server_opts()
        lib().hss_server_default_opts(C.byref(o))
        o.hbm_budget, o.max_batch, o.workers = int(hbm_budget), int(max_batch), int(workers)
        self._ptr = C.c_void_p()
        _check(lib().hss_server_create(C.byref(o), C.byref(self._ptr)))
        self._keep = {}

    @staticmethod
    def _rhs(b, x, n):
        import torch

        b2 = b.reshape(-1, 1) if b.dim() == 1 else b
        if b2.dtype != torch.float64 or b2.stride(1) != 1 or b2.shape[0] != n or not b2.is_cuda:
            raise ValueError("b must be CUDA float64, n x nrhs with unit column stride")
        if x is None:
            x = torch.empty_like(b)
        x2 = x.reshape(-1, 1) if x.dim() == 1 else x
        return b2, x, x2

    def submit(self, A, b, x=None, *, keep=False, rtol=1e-6, d0=64, dd=32, d_max=4096, p_margin=10, seed=0,
               leaf_size=64, sample_prec="f64") -> int:
        """Queue a compress + factor + solve request: A (square CUDA
        float32/float64) and right-hand sides b (CUDA float64, n or n x
        nrhs); returns a ticket.  x (optional output, same shape as b) is
        allocated when not given.  keep=True keeps the factored handle
        resident: ``wait`` returns it as info["handle"] (a ResidentHandle)."""
        import torch

        dt = {torch.float64: HSS_F64, torch.float32: HSS_F32}.get(A.dtype)
        if dt is None or A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1 or not A.is_cuda:
            raise ValueError("A must be a square CUDA float32/float64 matrix with unit column stride")
        b2, x, x2 = self._rhs(b, x, A.shape[0])
        o = hss_default_opts()
        o.rtol, o.d0, o.dd, o.d_max, o.p_margin = float(rtol), int(d0), int(dd), int(d_max), int(p_margin)
        o.seed, o.leaf_size, o.sample_prec = int(seed), int(leaf_size), _PREC[sample_prec]
        q = hss_server_request(A=A.data_ptr(), dtype=dt, n=A.shape[0], lda=A.stride(0),
                               opts=C.addressof(o), handle=None, nrhs=b2.shape[1], b=b2.data_ptr(),
                               ldb=b2.stride(0), x=x2.data_ptr(), ldx=x2.stride(0), keep=1 if keep else 0)
        t = C.c_longlong()
        # the server reads A and b after the work queued so far on the current stream
        _check(lib().hss_server_submit_request(self._ptr, C.byref(q), _stream(None), C.byref(t)))
        self._keep[t.value] = (A, b, x, A.shape[0])
        return t.value

    def solve(self, handle: "ResidentHandle", b, x=None) -> int:
        """Queue a solve-only request A_HSS x = b on a resident handle;
        returns a ticket."""
        b2, x, x2 = self._rhs(b, x, handle.n)
        q = hss_server_request(A=None, dtype=0, n=handle.n, lda=0, opts=None, handle=handle.ptr,
                               nrhs=b2.shape[1], b=b2.data_ptr(), ldb=b2.stride(0), x=x2.data_ptr(),
                               ldx=x2.stride(0), keep=0)
        t = C.c_longlong()
        _check(lib().hss_server_submit_request(self._ptr, C.byref(q), _stream(None), C.byref(t)))
        self._keep[t.value] = (None, b, x, handle.n)
        return t.value

    def wait(self, ticket: int):
        """Blocks until the request is done; returns (x, info dict).  A
        request that failed is reported by info["status"] (x then holds no
        solution); an unknown ticket raises HSSError."""
        if ticket not in self._keep:
            _check(lib().hss_server_wait(self._ptr, int(ticket), None))
        info = hss_request_info()
        lib().hss_server_wait(self._ptr, int(ticket), C.byref(info))
        A, b, x, n = self._keep.pop(ticket)
        out = {f: getattr(info, f) for f, _ in hss_request_info._fields_}
        out["handle"] = ResidentHandle(info.handle, n) if info.handle else None
        return x, out

    def release(self, handle: "ResidentHandle") -> None:
        """Destroy a resident handle once the requests on it have finished."""
        _check(lib().hss_server_release(self._ptr, handle.ptr))
        handle.ptr = C.c_void_p()

    def close(self):
        if self._ptr:
            lib().hss_server_destroy(self._ptr)
            self._ptr = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hss_server_default_opts() -> hss_server_opts:
    o = hss_server_opts()
    lib().hss_server_default_opts(C.byref(o))
    return o


def hss_server_create(hbm_budget: int = 0, max_batch: int = 32, workers: int = 2) -> HSSServer:
    return HSSServer(hbm_budget, max_batch, workers)


def hss_server_submit(server: HSSServer, A, b, x=None, **kw) -> int:
    return server.submit(A, b, x, **kw)


def hss_server_wait(server: HSSServer, ticket: int):
    return server.wait(ticket)


def hss_server_submit_request(server: HSSServer, handle: ResidentHandle, b, x=None) -> int:
    """Solve-only request on a resident handle (compress requests: hss_server_submit)."""
    return server.solve(handle, b, x)


def hss_server_release(server: HSSServer, handle: ResidentHandle) -> None:
    server.release(handle)


def hss_server_destroy(server: HSSServer) -> None:
    server.close()
