"""Python binding of libhf (Hilbert forest on MI355X).

Argument marshalling only: every step runs in the HIP kernels of ``libhf.so``
behind the C ABI declared in ``include/hf.h``.  Device buffers are torch
tensors; the current torch stream is passed to the library.  Importing works
without a GPU (for host-only calls such as :func:`curves`); device calls need
the built library and a HIP device, and fail loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhf.so")

HF_OK = 0
HF_F16, HF_F32 = 0, 1
HF_PREC = {"fp32": 0, "bf16": 1, "fp8": 2, "c4": 3}
HF_SKETCH_SRP, HF_SKETCH_LEARNED, HF_SKETCH_SIGN = 0, 1, 2
HF_POS = {"leaf": 0, "exact": 1}
HF_QUANT_AUTO = -(2 ** 31)
STATUS = {0: "ok", 1: "invalid argument", 2: "invalid input", 3: "out of memory", 4: "device error",
          5: "invalid handle", 6: "unsupported"}

EXPORTS = ["hf_status_str", "hf_last_error", "hf_curves", "hf_quant_exp", "hf_quantize",
           "hf_hilbert_sort", "hf_srp_sketch", "hf_build_forest", "hf_forest_free",
           "hf_forest_get_info", "hf_forest_perm", "hf_forest_nodes", "hf_forest_pos2id",
           "hf_forest_sketches", "hf_search", "hf_search_debug", "hf_knn_graph",
           "hf_timing_enable", "hf_timing_read", "hf_timing_stage_name", "hf_forest_add_precision",
           "hf_search_lowprec_debug", "hf_audit_scores", "hf_lhash_create", "hf_lhash_free", "hf_lhash_get",
           "hf_lhash_encode", "hf_lhash_grad", "hf_lhash_train", "hf_forest_set_sketch",
           "hf_knn_graph_debug", "hf_set_allocator", "hf_search_noalloc", "hf_forest_node_splits"]
N_STAGES = 16


class HFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class ForestParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_trees", C.c_uint32), ("leaf_max", C.c_uint32),
                ("quant_exp", C.c_int32), ("seed", C.c_uint64), ("sketch_seed", C.c_uint64),
                ("sketch", C.c_uint32), ("reserved", C.c_uint32), ("lhash", C.c_void_p)]


class SearchParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("k", C.c_uint32), ("k1", C.c_uint32),
                ("k2", C.c_uint32), ("h", C.c_uint32), ("precision", C.c_uint32),
                ("survivors", C.c_uint32), ("trees", C.c_uint32), ("position", C.c_uint32),
                ("reserved", C.c_uint32)]


class GraphParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_orders", C.c_uint32), ("window", C.c_uint32),
                ("k", C.c_uint32), ("k2", C.c_uint32), ("quant_exp", C.c_int32),
                ("sketch", C.c_uint32), ("seed", C.c_uint64), ("sketch_seed", C.c_uint64),
                ("lhash", C.c_void_p)]


class LHashTrainParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("epochs", C.c_uint32), ("batch", C.c_uint32),
                ("lr", C.c_float), ("weight_decay", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("slope", C.c_float), ("tau", C.c_float), ("balance", C.c_float),
                ("keep_blocks", C.c_uint32), ("seed", C.c_uint64)]


def train_params(epochs=5, batch=1024, lr=1e-3, weight_decay=1e-2, slope=1.0, tau=0.1, balance=0.1, seed=7,
                 keep_blocks=False):
    return LHashTrainParams(C.sizeof(LHashTrainParams), epochs, batch, lr, weight_decay, 0.9, 0.999, 1e-8,
                            slope, tau, balance, int(keep_blocks), seed)


def hilbert_pairs(q_codes, nn_ids, seed: int, batch: int):
    """Pair order for training with spatial hard negatives: queries along a
    Hilbert order, one block per neighbour rank, so a block of `batch`
    consecutive pairs holds distinct, nearby queries.  Returns (query row,
    neighbour id) index arrays of the ordered pairs (host)."""
    order = hilbert_sort(q_codes, seed, 0).cpu().numpy().view(np.uint32).astype(np.int64)
    nq, kn = nn_ids.shape
    usable = (nq // batch) * batch
    order = order[:usable]
    qi = np.concatenate([order for _ in range(kn)])
    pi = np.concatenate([nn_ids[order, r] for r in range(kn)])
    return qi, pi


class ForestInfo(C.Structure):
    _fields_ = [("N", C.c_int64), ("d", C.c_int32), ("n_trees", C.c_int32), ("leaf_max", C.c_int32),
                ("quant_exp", C.c_int32), ("dtype", C.c_int32), ("device", C.c_int32),
                ("total_nodes", C.c_int64), ("device_bytes", C.c_int64)]


_lib = None


def lib():
    """The loaded libhf.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HFError(4, "libhf.so not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, u32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        sig = {
            "hf_status_str": (C.c_char_p, [C.c_int]),
            "hf_last_error": (C.c_char_p, []),
            "hf_curves": (C.c_int, [u64, i32, i32, P, P]),
            "hf_quant_exp": (C.c_int, [P, C.c_int, i64, P, P]),
            "hf_quantize": (C.c_int, [P, C.c_int, i64, i32, P, P]),
            "hf_hilbert_sort": (C.c_int, [P, i64, i32, u64, u32, P, P, P]),
            "hf_srp_sketch": (C.c_int, [P, C.c_int, i64, i32, i32, u64, P, P]),
            "hf_build_forest": (C.c_int, [P, C.c_int, i64, i32, P, P, P]),
            "hf_forest_free": (None, [P]),
            "hf_forest_get_info": (C.c_int, [P, P]),
            "hf_forest_perm": (C.c_int, [P, u32, P, P]),
            "hf_forest_nodes": (C.c_int, [P, u32, P, P, P]),
            "hf_forest_node_splits": (C.c_int, [P, u32, P, P, P]),
            "hf_forest_pos2id": (C.c_int, [P, P, P]),
            "hf_forest_sketches": (C.c_int, [P, P, P]),
            "hf_search": (C.c_int, [P, P, C.c_int, i64, P, P, P, P]),
            "hf_search_debug": (C.c_int, [P, P, C.c_int, i64, P, P, P, P, P, P, P, P]),
            "hf_search_noalloc": (C.c_int, [P, P, C.c_int, i64, P, P, P, P]),
            "hf_knn_graph": (C.c_int, [P, C.c_int, i64, i32, P, P, P, P]),
            "hf_timing_enable": (C.c_int, [i32]),
            "hf_timing_read": (C.c_int, [P, P]),
            "hf_timing_stage_name": (C.c_char_p, [i32]),
            "hf_forest_add_precision": (C.c_int, [P, C.c_int, P]),
            "hf_search_lowprec_debug": (C.c_int, [P, P, C.c_int, i64, P, P, P, P, P, P]),
            "hf_audit_scores": (C.c_int, [P, C.c_int, i64, i32, P, i64, P, i32, P, P]),
            "hf_lhash_create": (C.c_int, [i32, i32, P, P, P, P, P]),
            "hf_lhash_free": (None, [P]),
            "hf_lhash_get": (C.c_int, [P, P, P, P, P]),
            "hf_lhash_encode": (C.c_int, [P, P, C.c_int, i64, i32, P, P]),
            "hf_lhash_grad": (C.c_int, [P, P, P, P, C.c_int, i64, i32, P, P, P, P, P, P, P]),
            "hf_lhash_train": (C.c_int, [P, P, P, P, C.c_int, i64, i32, P, P, P]),
            "hf_forest_set_sketch": (C.c_int, [P, C.c_int, P, P]),
            "hf_knn_graph_debug": (C.c_int, [P, C.c_int, i64, i32, P, P, P, P, P]),
            "hf_set_allocator": (C.c_int, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        restore_default_allocator()
    return _lib


def _check(status):
    if status != HF_OK:
        raise HFError(status, lib().hf_last_error().decode())


def _torch():
    import torch

    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype(x):
    t = _torch()
    if x.dtype == t.float16:
        return HF_F16
    if x.dtype == t.float32:
        return HF_F32
    raise TypeError("fp16 or fp32 tensors only, got %s" % x.dtype)


def _dev(x):
    t = _torch()
    if not x.is_cuda:
        raise ValueError("expected a device tensor")
    return x.contiguous()


def _empty(shape, dtype, like):
    return _torch().empty(shape, dtype=dtype, device=like.device)


# ---------------------------------------------------------------- building blocks
def curves(seed: int, T: int, d: int):
    perm = np.empty((T, d), np.int32)
    refl = np.empty((T, d), np.uint8)
    _check(lib().hf_curves(seed, T, d, perm.ctypes.data_as(C.c_void_p), refl.ctypes.data_as(C.c_void_p)))
    return perm, refl


def quant_exp(x) -> int:
    x = _dev(x)
    e = C.c_int32()
    _check(lib().hf_quant_exp(_ptr(x), _dtype(x), x.numel(), C.byref(e), _stream()))
    return int(e.value)


def quantize(x, e: int):
    x = _dev(x)
    out = _empty(x.shape, _torch().uint8, x)
    _check(lib().hf_quantize(_ptr(x), _dtype(x), x.numel(), e, _ptr(out), _stream()))
    return out


def hilbert_sort(codes, seed: int, tree: int = 0, with_split: bool = False):
    """Ids in Hilbert order along curve `tree` (int32 tensor holding uint32 values)."""
    codes = _dev(codes)
    N, d = codes.shape
    t = _torch()
    order = _empty((N,), t.int32, codes)
    split = _empty((max(N - 1, 1),), t.int32, codes) if with_split else None
    _check(lib().hf_hilbert_sort(_ptr(codes), N, d, seed, tree, _ptr(order), _ptr(split), _stream()))
    return (order, split[:N - 1]) if with_split else order


def srp_sketch(x, e: int, sketch_seed: int):
    x = _dev(x)
    N, d = x.shape
    out = _empty((N, 8), _torch().int64, x)
    _check(lib().hf_srp_sketch(_ptr(x), _dtype(x), N, d, e, sketch_seed, _ptr(out), _stream()))
    return out


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    """hf_allocator: the library's per-call scratch goes through these callbacks."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


def _torch_alloc(nbytes, ctx, stream):
    try:
        return _torch().cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # reported by the library as HF_ERR_OOM
        return None


def _torch_free(ptr, ctx, stream):
    _torch().cuda.caching_allocator_delete(int(ptr))


_allocator = None  # keeps the registered callbacks alive


def restore_default_allocator():
    """The binding's default: per-call scratch from torch's caching allocator
    (a search at 23M x 384 takes about 2 GB of scratch per call, which the
    cache hands back without a new device mapping each time)."""
    use_torch_allocator(True)


def use_torch_allocator(on: bool = True):
    """Route the library's per-call scratch through torch's caching allocator
    (blocks are tied to the call's stream, so later work on it may reuse them
    in stream order), or back to hipMallocAsync.  Process-wide: switch only
    while no call is in flight."""
    global _allocator
    if on:
        a = Allocator(ALLOC_FN(_torch_alloc), FREE_FN(_torch_free), None)
        _check(lib().hf_set_allocator(C.byref(a)))
        _allocator = a
    else:
        _check(lib().hf_set_allocator(None))
        _allocator = None


def timing_enable(on: bool = True):
    _check(lib().hf_timing_enable(1 if on else 0))


def timing_read():
    """{stage: (total ms, launches)} of the kernels timed since the last read."""
    ms = (C.c_float * N_STAGES)()
    n = (C.c_int32 * N_STAGES)()
    _check(lib().hf_timing_read(ms, n))
    return {lib().hf_timing_stage_name(i).decode(): (float(ms[i]), int(n[i])) for i in range(N_STAGES)
            if n[i] > 0}


# ---------------------------------------------------------------- forest
class Forest:
    """Hilbert forest (Algorithm 1 preprocessing) owned by libhf on the current device."""

    def __init__(self, x, n_trees: int, leaf_max: int = 100, seed: int = 0, sketch_seed: int = 0,
                 quant_exp: int | None = None, sketch: str = "srp", lhash=None):
        x = _dev(x)
        kind = {"srp": HF_SKETCH_SRP, "learned": HF_SKETCH_LEARNED, "sign": HF_SKETCH_SIGN}[sketch]
        p = ForestParams(C.sizeof(ForestParams), n_trees, leaf_max,
                         HF_QUANT_AUTO if quant_exp is None else quant_exp, seed, sketch_seed,
                         kind, 0, None if lhash is None else lhash._h)
        self._lhash = lhash
        h = C.c_void_p()
        _check(lib().hf_build_forest(_ptr(x), _dtype(x), x.shape[0], x.shape[1], C.byref(p),
                                     _stream(), C.byref(h)))
        self._h = h
        self.device = x.device
        self.dtype = x.dtype
        inf = ForestInfo()
        _check(lib().hf_forest_get_info(self._h, C.byref(inf)))
        self.info = {f: getattr(inf, f) for f, _ in ForestInfo._fields_}

    def _like(self):
        return _torch().empty(1, device=self.device)

    def free(self):
        if getattr(self, "_h", None):
            lib().hf_forest_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def perm(self, t: int):
        out = _empty((self.info["N"],), _torch().int32, self._like())
        _check(lib().hf_forest_perm(self._h, t, _ptr(out), _stream()))
        return out

    def nodes(self, t: int):
        n = C.c_int64()
        _check(lib().hf_forest_nodes(self._h, t, None, C.byref(n), _stream()))
        out = _empty((n.value, 2), _torch().int32, self._like())
        _check(lib().hf_forest_nodes(self._h, t, _ptr(out), C.byref(n), _stream()))
        return out

    def node_splits(self, t: int):
        """Split records of tree t: internal {m, b}, leaf {lo, 0xFFFFFFFF}."""
        n = C.c_int64()
        _check(lib().hf_forest_node_splits(self._h, t, None, C.byref(n), _stream()))
        out = _empty((n.value, 2), _torch().int32, self._like())
        _check(lib().hf_forest_node_splits(self._h, t, _ptr(out), C.byref(n), _stream()))
        return out

    def pos2id(self):
        out = _empty((self.info["N"],), _torch().int32, self._like())
        _check(lib().hf_forest_pos2id(self._h, _ptr(out), _stream()))
        return out

    def sketches(self):
        out = _empty((self.info["N"], 8), _torch().int64, self._like())
        _check(lib().hf_forest_sketches(self._h, _ptr(out), _stream()))
        return out

    def _params(self, k, k1, k2, h, precision, survivors, trees=0, position="leaf"):
        return SearchParams(C.sizeof(SearchParams), k, k1, k2, h, HF_PREC[precision], survivors, trees,
                            HF_POS[position], 0)

    def search(self, q, k: int, k1: int, k2: int, h: int, precision: str = "fp32", survivors: int = 0,
               trees: int = 0, position: str = "leaf"):
        """hf_search; ``trees`` > 0 searches trees 0..trees-1 only; ``position``
        "leaf" (leaf midpoint) or "exact" (insertion rank) centres the windows."""
        q = _dev(q)
        t = _torch()
        ids = _empty((q.shape[0], k), t.int32, q)
        sc = _empty((q.shape[0], k), t.float32, q)
        p = self._params(k, k1, k2, h, precision, survivors, trees, position)
        _check(lib().hf_search(self._h, _ptr(q), _dtype(q), q.shape[0], C.byref(p), _ptr(ids), _ptr(sc),
                               _stream()))
        return ids, sc

    def search_noalloc(self, q, k: int, k1: int, k2: int, h: int, precision: str = "fp32", survivors: int = 0,
                       out=None, trees: int = 0):
        """hf_search_noalloc: the library allocates nothing (scratch from its fixed
        per-device array); ``out`` = (ids, scores) lets the caller bring the outputs too."""
        q = _dev(q)
        t = _torch()
        if out is None:
            out = (_empty((q.shape[0], k), t.int32, q), _empty((q.shape[0], k), t.float32, q))
        ids, sc = out
        p = self._params(k, k1, k2, h, precision, survivors, trees)
        _check(lib().hf_search_noalloc(self._h, _ptr(q), _dtype(q), q.shape[0], C.byref(p), _ptr(ids), _ptr(sc),
                                       _stream()))
        return ids, sc

    def set_sketch(self, kind: str, lhash=None):
        """'srp', 'learned' (lhash must outlive the forest's use of it) or 'sign'."""
        self._lhash = lhash
        _check(lib().hf_forest_set_sketch(self._h, {"srp": HF_SKETCH_SRP, "learned": HF_SKETCH_LEARNED, "sign": HF_SKETCH_SIGN}[kind],
                                          None if lhash is None else lhash._h, _stream()))

    def add_precision(self, precision: str):
        _check(lib().hf_forest_add_precision(self._h, HF_PREC[precision], _stream()))

    def search_lowprec_debug(self, q, k: int, k1: int, k2: int, h: int, precision: str, survivors: int = 0):
        q = _dev(q)
        t = _torch()
        nq = q.shape[0]
        S = survivors or 4 * k
        ids = _empty((nq, k), t.int32, q)
        sc = _empty((nq, k), t.float32, q)
        sp = _empty((nq, S), t.int32, q)
        ss = _empty((nq, S), t.float32, q)
        p = self._params(k, k1, k2, h, precision, survivors)
        _check(lib().hf_search_lowprec_debug(self._h, _ptr(q), _dtype(q), nq, C.byref(p), _ptr(ids), _ptr(sc),
                                             _ptr(sp), _ptr(ss), _stream()))
        return dict(ids=ids, scores=sc, surv_pos=sp, surv_score=ss)

    def search_debug(self, q, k: int, k1: int, k2: int, h: int, precision: str = "fp32",
                     survivors: int = 0, trees: int = 0, position: str = "leaf"):
        q = _dev(q)
        t = _torch()
        nq = q.shape[0]
        ids = _empty((nq, k), t.int32, q)
        sc = _empty((nq, k), t.float32, q)
        win = _empty((nq, trees or self.info["n_trees"]), t.int32, q)
        c2 = _empty((nq, k2), t.int32, q)
        c2n = _empty((nq,), t.int32, q)
        en = _empty((nq,), t.int32, q)
        p = self._params(k, k1, k2, h, precision, survivors, trees, position)
        _check(lib().hf_search_debug(self._h, _ptr(q), _dtype(q), nq, C.byref(p), _ptr(ids), _ptr(sc),
                                     _ptr(win), _ptr(c2), _ptr(c2n), _ptr(en), _stream()))
        return dict(ids=ids, scores=sc, winstart=win, c2=c2, c2n=c2n, en=en)


def audit_scores(x, q, ids):
    """FP64 inner products of each query with the rows its ids name (GPU audit kernel)."""
    x, q, ids = _dev(x), _dev(q), _dev(ids)
    out = _empty(tuple(ids.shape), _torch().float64, x)
    _check(lib().hf_audit_scores(_ptr(x), _dtype(x), x.shape[0], x.shape[1], _ptr(q), q.shape[0], _ptr(ids),
                                 ids.shape[1], _ptr(out), _stream()))
    return out


class LHash:
    """Learned MLP hash d -> hidden -> 512 sign bits, weights trained by libhf's kernels."""

    def __init__(self, W1, b1, W2, b2):
        f = lambda a: np.ascontiguousarray(a, np.float32)
        W1, b1, W2, b2 = f(W1), f(b1), f(W2), f(b2)
        self.hidden, self.d = W1.shape
        h = C.c_void_p()
        _check(lib().hf_lhash_create(self.d, self.hidden, *[a.ctypes.data_as(C.c_void_p) for a in (W1, b1, W2, b2)],
                                     C.byref(h)))
        self._h = h

    @staticmethod
    def init(d: int, hidden: int, seed: int):
        """He-style random initialisation drawn on the host (seeded numpy)."""
        rng = np.random.Generator(np.random.PCG64(seed))
        W1 = rng.standard_normal((hidden, d)) * np.sqrt(2.0 / d)
        W2 = rng.standard_normal((512, hidden)) * np.sqrt(1.0 / hidden)
        return LHash(W1, np.zeros(hidden), W2, np.zeros(512))

    def free(self):
        if getattr(self, "_h", None):
            lib().hf_lhash_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def weights(self):
        out = [np.empty((self.hidden, self.d), np.float32), np.empty(self.hidden, np.float32),
               np.empty((512, self.hidden), np.float32), np.empty(512, np.float32)]
        _check(lib().hf_lhash_get(self._h, *[a.ctypes.data_as(C.c_void_p) for a in out]))
        return out

    def encode(self, x):
        x = _dev(x)
        out = _empty((x.shape[0], 8), _torch().int64, x)
        _check(lib().hf_lhash_encode(self._h, _ptr(x), _dtype(x), x.shape[0], x.shape[1], _ptr(out), _stream()))
        return out

    def grad(self, A, B, params, N=None):
        """Loss and gradients on pairs (A[i], B[i]), with hard negatives N[i] if given."""
        A, B = _dev(A), _dev(B)
        N = None if N is None else _dev(N)
        t = _torch()
        g = [t.empty((self.hidden, self.d), dtype=t.float32, device=A.device),
             t.empty(self.hidden, dtype=t.float32, device=A.device),
             t.empty((512, self.hidden), dtype=t.float32, device=A.device),
             t.empty(512, dtype=t.float32, device=A.device)]
        loss = C.c_float()
        _check(lib().hf_lhash_grad(self._h, _ptr(A), _ptr(B), _ptr(N), _dtype(A), A.shape[0], A.shape[1],
                                   C.byref(params),
                                   C.byref(loss), *[_ptr(v) for v in g], _stream()))
        return float(loss.value), g

    def train(self, A, B, params, N=None):
        """AdamW on pairs (A[i], B[i]) (hard negatives N[i] if given); loss per epoch."""
        A, B = _dev(A), _dev(B)
        N = None if N is None else _dev(N)
        curve = np.zeros(max(1, params.epochs), np.float32)
        _check(lib().hf_lhash_train(self._h, _ptr(A), _ptr(B), _ptr(N), _dtype(A), A.shape[0], A.shape[1],
                                    C.byref(params), curve.ctypes.data_as(C.c_void_p), _stream()))
        return curve


# ---------------------------------------------------------------- graph
def _graph_params(n_orders, window, k, seed, k2, sketch, sketch_seed, lhash, quant_exp):
    kind = {"srp": HF_SKETCH_SRP, "learned": HF_SKETCH_LEARNED, "sign": HF_SKETCH_SIGN}[sketch]
    return GraphParams(C.sizeof(GraphParams), n_orders, window, k, k2,
                       HF_QUANT_AUTO if quant_exp is None else quant_exp, kind, seed, sketch_seed,
                       None if lhash is None else lhash._h.value)


def knn_graph(x, n_orders: int, window: int, k: int, seed: int, k2: int = 0, sketch_seed: int = 0,
              quant_exp: int | None = None, sketch: str = "srp", lhash=None):
    """Algorithm 2 graph: (ids N x k int32, cosines N x k float32); k2 > 0 adds the sketch stage."""
    x = _dev(x)
    N, d = x.shape
    t = _torch()
    ids = _empty((N, k), t.int32, x)
    sc = _empty((N, k), t.float32, x)
    p = _graph_params(n_orders, window, k, seed, k2, sketch, sketch_seed, lhash, quant_exp)
    _check(lib().hf_knn_graph(_ptr(x), _dtype(x), N, d, C.byref(p), _ptr(ids), _ptr(sc), _stream()))
    return ids, sc


def knn_graph_debug(x, n_orders: int, window: int, k: int, seed: int, k2: int, sketch_seed: int = 0,
                    quant_exp: int | None = None, sketch: str = "srp", lhash=None):
    """knn_graph with the sketch stage, also returning every point's C2 (N x k2 ids, -1 padded)."""
    x = _dev(x)
    N, d = x.shape
    t = _torch()
    ids = _empty((N, k), t.int32, x)
    sc = _empty((N, k), t.float32, x)
    c2 = _empty((N, k2), t.int32, x)
    p = _graph_params(n_orders, window, k, seed, k2, sketch, sketch_seed, lhash, quant_exp)
    _check(lib().hf_knn_graph_debug(_ptr(x), _dtype(x), N, d, C.byref(p), _ptr(ids), _ptr(sc), _ptr(c2),
                                    _stream()))
    return ids, sc, c2
