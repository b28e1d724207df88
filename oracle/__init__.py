"""Hilbert-forest ORACLE (test infrastructure only).

Plain CPU implementation of the method of arXiv 2508.21682 (Hilbert forest),
used by the tests, the package smoke check and the benchmark's CPU-baseline
leg -- never by the library.  The arithmetic lives in ``hf_oracle.c`` (plain
C, FP64 for floating point); this module compiles it with gcc, loads it with
ctypes and composes its steps in the order of Algorithms 1 and 2.  Exact
brute-force k-NN, used for recall and for the reductions that pin the
oracle, is a numpy FP64 matrix product plus a stable sort.

Parity status: every function is pinned by tests under ``tests/`` except the
recall values themselves (the paper's datasets are absent), which are
"parity unpinned" context.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hf_oracle.c")
_LIB = os.path.join(_HERE, "libhf_oracle.so")
_lib = None

SKETCH_WORDS = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i32, i64, u64 = C.c_int32, C.c_int64, C.c_uint64
        sig = {
            "hfo_splitmix64": (u64, [u64, i64]),
            "hfo_curves": (None, [u64, i32, i32, P, P]),
            "hfo_f16_to_f64": (C.c_double, [C.c_uint16]),
            "hfo_quant_exp": (i32, [P, i32, i64]),
            "hfo_quantize": (None, [P, i32, i64, i32, P]),
            "hfo_key": (None, [P, i32, i32, P]),
            "hfo_tree_keys": (None, [P, i64, i32, P, P, P]),
            "hfo_sort": (None, [P, i64, i32, P]),
            "hfo_trie": (i64, [P, P, i64, i32, i32, P, P, P, P, i64, P]),
            "hfo_window_starts": (None, [P, P, i64, i32, i64, i32, P, i64]),
            "hfo_exact_ranks": (None, [P, P, i64, i32, P, i64, P, P, i32, P, P]),
            "hfo_c4_encode": (None, [P, i32, i64, i32, P, P, P]),
            "hfo_search_c4": (None, [i64, i32, P, P, i32, P, P, P, P, P, i32, i64, i32, i32, i32, i32, P, P, P, P,
                                     P]),
            "hfo_srp": (None, [P, i32, i64, i32, u64, P]),
            "hfo_search_stage2": (None, [P, i32, i64, i32, P, P, i32, P, P, P, P, i64,
                                         i32, i32, i32, i32, P, P, P, P, P, P]),
            "hfo_graph_rows": (None, [P, i32, i64, i32, P, i32, i32, P, i64, i32, i32, P, P, P, P, P]),
            "hfo_bf16": (C.c_double, [C.c_double]),
            "hfo_e4m3_decode": (C.c_double, [C.c_uint8]),
            "hfo_e4m3_encode": (C.c_uint8, [C.c_float]),
            "hfo_fp8_scale": (C.c_float, [P, i32, i64, i32]),
            "hfo_mlp_forward": (None, [P, i32, i64, i32, i32, P, P, P, P, i32, P, P, P, P]),
            "hfo_lhash_grad": (C.c_double, [P, P, P, i32, i64, i32, i32, P, P, P, P, C.c_double, C.c_double,
                                            C.c_double, i32, P, P, P, P]),
            "hfo_search_lowprec": (None, [P, i32, i64, i32, P, P, P, i32, P, i64, i32, i32, i32, i32,
                                          P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def set_num_threads(n: int) -> int:
    """OpenMP threads the oracle's parallel loops use from now on (libgomp is
    loaded with the oracle); returns the previous setting."""
    lib()
    g = C.CDLL("libgomp.so.1")
    g.omp_get_max_threads.restype = C.c_int
    old = int(g.omp_get_max_threads())
    g.omp_set_num_threads(C.c_int(int(n)))
    return old


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dtype_code(x):
    if x.dtype == np.float16:
        return 0
    if x.dtype == np.float32:
        return 1
    raise TypeError("oracle takes float16 or float32 values, got %s" % x.dtype)


# --------------------------------------------------------------------------- steps
def splitmix64(seed: int, index: int) -> int:
    return int(lib().hfo_splitmix64(seed, index))


def curves(seed: int, T: int, d: int):
    """(perm[T,d] int32, refl[T,d] uint8): tree axis i reads data axis perm[t,i]."""
    perm = np.empty((T, d), np.int32)
    refl = np.empty((T, d), np.uint8)
    lib().hfo_curves(seed, T, d, _p(perm), _p(refl))
    return perm, refl


def quant_exp(x: np.ndarray) -> int:
    x = np.ascontiguousarray(x)
    return int(lib().hfo_quant_exp(_p(x), _dtype_code(x), x.size))


def quantize(x: np.ndarray, e: int) -> np.ndarray:
    x = np.ascontiguousarray(x)
    out = np.empty(x.shape, np.uint8)
    lib().hfo_quantize(_p(x), _dtype_code(x), x.size, e, _p(out))
    return out


def key_words(d: int, B: int = 8) -> int:
    return (d * B + 63) // 64


def hilbert_key(v, B: int) -> np.ndarray:
    """Skilling Hilbert index of one B-bit point, as big-endian uint64 words."""
    v = np.ascontiguousarray(np.asarray(v, dtype=np.uint8))
    out = np.empty(key_words(v.size, B), np.uint64)
    lib().hfo_key(_p(v), v.size, B, _p(out))
    return out


def hilbert_index_int(v, B: int) -> int:
    """The key as a Python integer (d*B bits)."""
    w = hilbert_key(v, B)
    d = len(v)
    val = 0
    for x in w:
        val = (val << 64) | int(x)
    return val >> (64 * len(w) - d * B)


def tree_keys(codes: np.ndarray, perm_t: np.ndarray, refl_t: np.ndarray) -> np.ndarray:
    codes = np.ascontiguousarray(codes)
    N, d = codes.shape
    keys = np.empty((N, key_words(d)), np.uint64)
    lib().hfo_tree_keys(_p(codes), N, d, _p(np.ascontiguousarray(perm_t, np.int32)),
                        _p(np.ascontiguousarray(refl_t, np.uint8)), _p(keys))
    return keys


def sort_keys(keys: np.ndarray) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    order = np.empty(keys.shape[0], np.uint32)
    lib().hfo_sort(_p(keys), keys.shape[0], keys.shape[1], _p(order))
    return order


def trie(keys, order, codes, perm_t, refl_t, M: int, with_splits: bool = False):
    """Leaf-compressed Hilbert trie in pre-order; (n_nodes, 2) uint32 records,
    and with ``with_splits`` also the split records (internal {m, b}, leaf {lo, ~0})."""
    N, d = codes.shape
    cap = 2 * N + 8  # a binary tree over N points has at most 2N-1 nodes
    nodes = np.zeros((cap, 2), np.uint32)
    aux = np.zeros((cap, 2), np.uint32)
    n = lib().hfo_trie(_p(np.ascontiguousarray(keys)), _p(np.ascontiguousarray(order)), N, d, M,
                       _p(np.ascontiguousarray(codes)), _p(np.ascontiguousarray(perm_t, np.int32)),
                       _p(np.ascontiguousarray(refl_t, np.uint8)), _p(nodes), cap, _p(aux))
    if n < 0:
        raise RuntimeError("oracle trie failed (%d)" % n)
    if with_splits:
        return nodes[:n].copy(), aux[:n].copy()
    return nodes[:n].copy()


def window_starts(nodes: np.ndarray, qcodes: np.ndarray, N: int, k1: int) -> np.ndarray:
    qcodes = np.ascontiguousarray(qcodes)
    out = np.empty(qcodes.shape[0], np.uint32)
    lib().hfo_window_starts(_p(np.ascontiguousarray(nodes)), _p(qcodes), qcodes.shape[0],
                            qcodes.shape[1], N, k1, _p(out), 1)
    return out


def exact_ranks(keys, order, qcodes, perm_t, refl_t, k1: int):
    """Exact insertion rank of each query along one tree's curve (before equal
    keys) and the window start centred on it: (rank[nq], start[nq])."""
    qcodes = np.ascontiguousarray(qcodes)
    nq, d = qcodes.shape
    rank = np.empty(nq, np.uint32)
    start = np.empty(nq, np.uint32)
    lib().hfo_exact_ranks(_p(np.ascontiguousarray(keys)), _p(np.ascontiguousarray(order)), keys.shape[0], d,
                          _p(qcodes), nq, _p(np.ascontiguousarray(perm_t, np.int32)),
                          _p(np.ascontiguousarray(refl_t, np.uint8)), k1, _p(rank), _p(start))
    return rank, start


def srp(x: np.ndarray, e: int, sketch_seed: int) -> np.ndarray:
    x = np.ascontiguousarray(x)
    out = np.empty((x.shape[0], SKETCH_WORDS), np.uint64)
    lib().hfo_srp(_p(x), _dtype_code(x), x.shape[0], x.shape[1], e, sketch_seed, _p(out))
    return out


def hamming(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    x = np.bitwise_xor(a, b)
    return np.unpackbits(x.view(np.uint8), axis=-1).sum(axis=-1)


# --------------------------------------------------------------------------- Alg. 1
def build_forest(x: np.ndarray, T: int, M: int, seed: int, sketch_seed: int, quant_e=None,
                 with_nodes: bool = True, trees=None):
    """Preprocessing of Alg. 1: codes, sketches, master order, n trees.

    ``trees`` restricts the trees built (their curves still come from the one
    seeded stream, so tree t is the same tree as in the full forest); tree 0
    (the master order) is always built.
    """
    N, d = x.shape
    e = quant_exp(x) if quant_e is None else int(quant_e)
    codes = quantize(x, e)
    perm, refl = curves(seed, T, d)
    want = sorted(set([0] + (list(range(T)) if trees is None else list(trees))))
    orders, keys_t = {}, {}
    for t in want:
        k = tree_keys(codes, perm[t], refl[t])
        orders[t] = sort_keys(k)
        keys_t[t] = k
    pos2id = orders[0].copy()
    pos = np.empty(N, np.uint32)
    pos[pos2id] = np.arange(N, dtype=np.uint32)
    tree_perm = {t: pos[orders[t]] for t in want}
    nodes, splits = {}, {}
    if with_nodes:
        for t in want:
            nodes[t], splits[t] = trie(keys_t[t], orders[t], codes, perm[t], refl[t], M, with_splits=True)
    sk = srp(x, e, sketch_seed)
    return dict(N=N, d=d, T=T, M=M, e=e, codes=codes, perm=perm, refl=refl, orders=orders,
                pos2id=pos2id, pos=pos, tree_perm=tree_perm, nodes=nodes, trees=want,
                sk_pos=sk[pos2id].copy(), x=x, sketch_seed=sketch_seed, keys=keys_t, splits=splits)


def search(F, q: np.ndarray, k1: int, k2: int, h: int, k: int, position: str = "leaf"):
    """Alg. 1 search for queries q over the trees of forest F (FP64 scores).

    position: where a query sits along a tree's curve: "leaf" = the midpoint
    of the leaf its descent reaches, "exact" = its insertion rank among the
    tree's sorted keys."""
    N, d = F["N"], F["d"]
    trees = F["trees"]
    T = len(trees)
    qcodes = quantize(q, F["e"])
    nq = q.shape[0]
    win = np.empty((nq, T), np.uint32)
    for j, t in enumerate(trees):
        if position == "exact":
            win[:, j] = exact_ranks(F["keys"][t], F["orders"][t], qcodes, F["perm"][t], F["refl"][t], k1)[1]
        else:
            win[:, j] = window_starts(F["nodes"][t], qcodes, N, k1)
    tp = np.ascontiguousarray(np.stack([F["tree_perm"][t] for t in trees]))
    qsk = srp(q, F["e"], F["sketch_seed"])
    ids = np.empty((nq, k), np.int32)
    scores = np.empty((nq, k), np.float64)
    c2 = np.empty((nq, k2), np.uint32)
    c2n = np.empty(nq, np.int32)
    c1n = np.empty(nq, np.int32)
    en = np.empty(nq, np.int32)
    x = np.ascontiguousarray(F["x"])
    qq = np.ascontiguousarray(q.astype(x.dtype))
    lib().hfo_search_stage2(_p(x), _dtype_code(x), N, d, _p(F["pos2id"]), _p(tp), T, _p(win),
                            _p(F["sk_pos"]), _p(qq), _p(qsk), nq, k1, k2, h, k, _p(ids),
                            _p(scores), _p(c2), _p(c2n), _p(c1n), _p(en))
    return dict(ids=ids, scores=scores, winstart=win, c2=c2, c2n=c2n, c1n=c1n, en=en, qcodes=qcodes,
                qsk=qsk)


def c4_encode(x: np.ndarray):
    """The compressed layout of rows x: (sign sketches [N, ceil(d/64)] uint64,
    magnitudes [N, d] uint8 in 0..7, scales [N] float64 = max|x| / 8)."""
    x = np.ascontiguousarray(x)
    N, d = x.shape
    sg = np.empty((N, (d + 63) // 64), np.uint64)
    mag = np.empty((N, d), np.uint8)
    sc = np.empty(N, np.float64)
    lib().hfo_c4_encode(_p(x), _dtype_code(x), N, d, _p(sg), _p(mag), _p(sc))
    return sg, mag, sc


def search_c4(F, q: np.ndarray, k1: int, k2: int, h: int, k: int, position: str = "leaf"):
    """Alg. 1 in the compressed layout: sign-sketch Hamming filter, rerank
    from the 4-bit codes with the stored (unquantized) query values."""
    N, d = F["N"], F["d"]
    trees = F["trees"]
    T = len(trees)
    qcodes = quantize(q, F["e"])
    nq = q.shape[0]
    win = np.empty((nq, T), np.uint32)
    for j, t in enumerate(trees):
        if position == "exact":
            win[:, j] = exact_ranks(F["keys"][t], F["orders"][t], qcodes, F["perm"][t], F["refl"][t], k1)[1]
        else:
            win[:, j] = window_starts(F["nodes"][t], qcodes, N, k1)
    tp = np.ascontiguousarray(np.stack([F["tree_perm"][t] for t in trees]))
    if "c4" not in F:
        sg, mag, sc = c4_encode(F["x"])
        p2i = F["pos2id"]
        F["c4"] = (sg[p2i].copy(), mag[p2i].copy(), sc[p2i].copy())
    sg, mag, sc = F["c4"]
    ids = np.empty((nq, k), np.int32)
    scores = np.empty((nq, k), np.float64)
    c2 = np.empty((nq, k2), np.uint32)
    c2n = np.empty(nq, np.int32)
    en = np.empty(nq, np.int32)
    qq = np.ascontiguousarray(q.astype(F["x"].dtype))
    lib().hfo_search_c4(N, d, _p(F["pos2id"]), _p(tp), T, _p(win), _p(sg), _p(mag), _p(sc), _p(qq),
                        _dtype_code(qq), nq, k1, k2, h, k, _p(ids), _p(scores), _p(c2), _p(c2n), _p(en))
    return dict(ids=ids, scores=scores, winstart=win, c2=c2, c2n=c2n, en=en)


def search_lowprec(F, q: np.ndarray, c2: np.ndarray, c2n: np.ndarray, h: int, k: int, prec: str, S: int):
    """Precision form of the final selection from given C2 lists (emulated BF16/FP8)."""
    code = {"bf16": 1, "fp8": 2}[prec]
    x = np.ascontiguousarray(F["x"])
    qq = np.ascontiguousarray(q.astype(x.dtype))
    nq = q.shape[0]
    k2 = c2.shape[1]
    ids = np.empty((nq, k), np.int32)
    sc = np.empty((nq, k), np.float64)
    sp = np.empty((nq, S), np.uint32)
    ss = np.empty((nq, S), np.float64)
    lib().hfo_search_lowprec(_p(x), _dtype_code(x), F["N"], F["d"], _p(F["pos2id"]),
                             _p(np.ascontiguousarray(c2, np.uint32)), _p(np.ascontiguousarray(c2n, np.int32)),
                             k2, _p(qq), nq, h, k, code, S, _p(ids), _p(sc), _p(sp), _p(ss))
    return dict(ids=ids, scores=sc, surv_pos=sp, surv_score=ss)


def bf16(x: float) -> float:
    return float(lib().hfo_bf16(x))


def e4m3_decode(c: int) -> float:
    return float(lib().hfo_e4m3_decode(c))


def e4m3_encode(y: float) -> int:
    return int(lib().hfo_e4m3_encode(y))


def mlp_forward(x, W1, b1, W2, b2, rounded=True):
    """Learned-hash forward in FP64: (z1, a, z2, band) with band = fragile margin of z2."""
    x = np.ascontiguousarray(x)
    n, d = x.shape
    hid = W1.shape[0]
    f = lambda a: np.ascontiguousarray(a, np.float32)
    W1, b1, W2, b2 = f(W1), f(b1), f(W2), f(b2)
    z1 = np.empty((n, hid)); a = np.empty((n, hid)); z2 = np.empty((n, 512)); band = np.empty((n, 512))
    lib().hfo_mlp_forward(_p(x), _dtype_code(x), n, d, hid, _p(W1), _p(b1), _p(W2), _p(b2), int(rounded),
                          _p(z1), _p(a), _p(z2), _p(band))
    return z1, a, z2, band


def lhash_grad(A, B, W1, b1, W2, b2, slope, tau, lam, rounded=True, Neg=None):
    """Loss and FP64 gradients of the learned-hash training objective on one
    batch of pairs (A[i], B[i]), with one hard negative Neg[i] per query if given."""
    A = np.ascontiguousarray(A)
    Bm = np.ascontiguousarray(B.astype(A.dtype))
    Ng = None if Neg is None else np.ascontiguousarray(Neg.astype(A.dtype))
    n, d = A.shape
    hid = W1.shape[0]
    f = lambda a: np.ascontiguousarray(a, np.float32)
    W1, b1, W2, b2 = f(W1), f(b1), f(W2), f(b2)
    g = [np.empty((hid, d)), np.empty(hid), np.empty((512, hid)), np.empty(512)]
    loss = lib().hfo_lhash_grad(_p(A), _p(Bm), _p(Ng), _dtype_code(A), n, d, hid, _p(W1), _p(b1), _p(W2), _p(b2),
                                slope, tau, lam, int(rounded), *[_p(v) for v in g])
    return float(loss), g


# --------------------------------------------------------------------------- Alg. 2
def graph_orders(x: np.ndarray, n: int, seed: int, quant_e=None):
    """The n Hilbert orders of Alg. 2 (ids sorted along each seeded curve)."""
    N, d = x.shape
    e = quant_exp(x) if quant_e is None else int(quant_e)
    codes = quantize(x, e)
    perm, refl = curves(seed, n, d)
    orders = np.empty((n, N), np.uint32)
    for t in range(n):
        orders[t] = sort_keys(tree_keys(codes, perm[t], refl[t]))
    return orders, e


def graph_rows(x, orders, w: int, k: int, rows, k2: int = 0, sk=None, with_c2: bool = False):
    """Rows of the Alg. 2 graph: (ids[nrows,k], cos[nrows,k], |C1|[nrows]) and, with
    ``with_c2`` (k2 > 0), C2[nrows,k2] in (Hamming, id) order, -1 padded."""
    x = np.ascontiguousarray(x)
    N, d = x.shape
    rows = np.ascontiguousarray(np.asarray(rows, np.int64))
    ids = np.empty((rows.size, k), np.int32)
    sc = np.empty((rows.size, k), np.float64)
    c1n = np.empty(rows.size, np.int32)
    c2 = np.empty((rows.size, k2), np.int32) if (with_c2 and k2 > 0) else None
    orders = np.ascontiguousarray(orders, np.uint32)
    lib().hfo_graph_rows(_p(x), _dtype_code(x), N, d, _p(orders), orders.shape[0], w, _p(rows),
                         rows.size, k, k2, _p(None if sk is None else np.ascontiguousarray(sk)),
                         _p(ids), _p(sc), _p(c1n), _p(c2))
    if with_c2:
        return ids, sc, c1n, c2
    return ids, sc, c1n


# --------------------------------------------------------------------------- brute force
def brute_force_ip(x: np.ndarray, q: np.ndarray, k: int, block: int = 4096):
    """Exact top-k by inner product (FP64), ties by smaller id."""
    X = x.astype(np.float64)
    out_i = np.empty((q.shape[0], k), np.int64)
    out_s = np.empty((q.shape[0], k), np.float64)
    for s in range(0, q.shape[0], block):
        S = q[s:s + block].astype(np.float64) @ X.T
        o = np.argsort(-S, axis=1, kind="stable")[:, :k]
        out_i[s:s + block] = o
        out_s[s:s + block] = np.take_along_axis(S, o, axis=1)
    return out_i, out_s


def brute_force_graph(x: np.ndarray, rows, k: int, block: int = 1024):
    """Exact k-NN graph rows by cosine (FP64), self excluded, ties by smaller id."""
    X = x.astype(np.float64)
    nrm = np.linalg.norm(X, axis=1)
    rows = np.asarray(rows, np.int64)
    out_i = np.empty((rows.size, k), np.int64)
    out_s = np.empty((rows.size, k), np.float64)
    for s in range(0, rows.size, block):
        r = rows[s:s + block]
        S = (X[r] @ X.T) / (nrm[r, None] * nrm[None, :])
        S[np.arange(r.size), r] = -np.inf
        o = np.argsort(-S, axis=1, kind="stable")[:, :k]
        out_i[s:s + block] = o
        out_s[s:s + block] = np.take_along_axis(S, o, axis=1)
    return out_i, out_s


def recall(found: np.ndarray, truth: np.ndarray) -> float:
    k = truth.shape[1]
    hits = sum(len(set(map(int, f[:k])) & set(map(int, t))) for f, t in zip(found, truth))
    return hits / float(truth.shape[0] * k)
