"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types an oracle formula: each checks a property, a closed
form, a special case that reduces to a textbook object, a hand-drawn table or
brute force on tiny inputs.
"""
import itertools
import os

import numpy as np
import pytest

import datagen

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


# ----------------------------------------------------------------- SplitMix64
def test_splitmix64_published_outputs(orc):
    want = [int(v, 16) for v in _read_golden("splitmix64_seed0.txt")]
    assert [orc.splitmix64(0, i) for i in range(3)] == want


def test_curves_are_permutations_and_seeded(orc):
    perm, refl = orc.curves(7, 5, 384)
    for t in range(5):
        assert sorted(perm[t].tolist()) == list(range(384))
    assert set(np.unique(refl).tolist()) <= {0, 1}
    assert 100 < refl.sum() / 5 < 284  # about half the axes reflected
    p2, r2 = orc.curves(7, 5, 384)
    assert (p2 == perm).all() and (r2 == refl).all()
    p3, _ = orc.curves(8, 5, 384)
    assert (p3 != perm).any()
    # tree t of a longer forest equals tree t of a shorter one (one stream, tree order)
    p4, r4 = orc.curves(7, 3, 384)
    assert (p4 == perm[:3]).all() and (r4 == refl[:3]).all()


def test_curves_fisher_yates_first_draw(orc):
    """d=2: the single Fisher-Yates draw j = next mod 2 decides the swap."""
    perm, refl = orc.curves(0, 1, 2)
    j = orc.splitmix64(0, 0) % 2
    assert perm[0].tolist() == ([1, 0] if j == 0 else [0, 1])
    bits = orc.splitmix64(0, 1)
    assert refl[0].tolist() == [bits & 1, (bits >> 1) & 1]


# ----------------------------------------------------------------- stored values
def test_f16_to_f64_all_codes(orc):
    lib = orc.lib()
    codes = np.arange(65536, dtype=np.uint16)
    ref = codes.view(np.float16).astype(np.float64)
    got = np.array([lib.hfo_f16_to_f64(int(c)) for c in codes])
    fin = np.isfinite(ref)
    assert (got[fin] == ref[fin]).all()
    assert (np.isnan(got) == np.isnan(ref)).all()
    assert (got[np.isinf(ref)] == ref[np.isinf(ref)]).all()


# ----------------------------------------------------------------- quantiser
def test_quant_exp_defining_inequalities(orc):
    rng = np.random.default_rng(1)
    for scale in [1e-3, 0.05, 0.3, 1.0, 7.0, 100.0, 3e4]:
        x = (rng.standard_normal((50, 17)) * scale).astype(np.float32)
        e = orc.quant_exp(x)
        assert -8 <= e <= 24
        ok = lambda ee: (2.0 ** ee) * x.max() < 128 and (2.0 ** ee) * x.min() >= -128
        if ok(-8):
            assert ok(e)
            assert e == 24 or not ok(e + 1)
        else:  # no exponent fits: the coarsest one, codes clamp
            assert e == -8


def test_quant_exp_nonfinite(orc):
    x = np.ones((4, 4), np.float32)
    x[2, 1] = np.inf
    assert orc.quant_exp(x) == np.iinfo(np.int32).min


def test_quantize_hand_values(orc):
    x = np.array([0.0, -0.0, 0.5, -0.5, 0.49609375, -0.001, 1e9, -1e9], np.float32)
    # e = 8: 0 -> 128, -0 -> 128, 0.5*256=128 -> 256 -> clamp 255, -128 -> 0,
    # 0.49609375*256 = 127 -> 255, -0.256 -> floor -1 -> 127, huge -> 255, tiny -> 0
    got = orc.quantize(x, 8)
    assert got.tolist() == [128, 128, 255, 0, 255, 127, 255, 0]
    # floor, not round: 0.9/256 below one step stays in the same cell
    assert orc.quantize(np.array([0.9 / 256], np.float32), 8).tolist() == [128]


# ----------------------------------------------------------------- Skilling keys
@pytest.mark.parametrize("d,B", [(1, 1), (1, 4), (2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2),
                                 (3, 3), (4, 2), (4, 3), (5, 2)])
def test_hilbert_bijection_adjacency_subcubes(orc, d, B):
    side = 1 << B
    cells = list(itertools.product(range(side), repeat=d))
    idx = {c: orc.hilbert_index_int(c, B) for c in cells}
    # bijection onto [0, 2^(dB))
    assert sorted(idx.values()) == list(range(side ** d))
    inv = {v: c for c, v in idx.items()}
    # starts at the origin
    assert inv[0] == (0,) * d
    # unit steps: consecutive indices are grid neighbours
    for h in range(side ** d - 1):
        a, b = inv[h], inv[h + 1]
        assert sum(abs(x - y) for x, y in zip(a, b)) == 1, (h, a, b)
    # every aligned sub-cube of side 2^l is one contiguous index interval
    for lev in range(1, B):
        s = 1 << lev
        groups = {}
        for c, v in idx.items():
            groups.setdefault(tuple(x // s for x in c), []).append(v)
        for vs in groups.values():
            vs.sort()
            assert vs[-1] - vs[0] == len(vs) - 1


def test_hilbert_2d_order2_hand_table(orc):
    cells = [tuple(int(t) for t in r.split()) for r in _read_golden("hilbert_2d_order2.txt")]
    order = sorted(itertools.product(range(4), repeat=2), key=lambda c: orc.hilbert_index_int(c, 2))
    assert order == cells


def test_hilbert_order1_2d_u_shape(orc):
    order = sorted(itertools.product(range(2), repeat=2), key=lambda c: orc.hilbert_index_int(c, 1))
    assert order == [(0, 0), (0, 1), (1, 1), (1, 0)]


@pytest.mark.parametrize("d", [1, 2, 3, 5, 10])
def test_hilbert_B1_is_gray_code(orc, d):
    """B=1: the curve visits the cube corners in binary-reflected Gray-code order, axis 0 MSB."""
    for h in range(1 << d):
        g = h ^ (h >> 1)
        corner = [(g >> (d - 1 - j)) & 1 for j in range(d)]
        assert orc.hilbert_index_int(corner, 1) == h


def test_hilbert_B1_gray_code_d384(orc):
    rng = np.random.default_rng(3)
    for _ in range(20):
        h = int.from_bytes(rng.bytes(48), "big")
        g = h ^ (h >> 1)
        corner = [(g >> (383 - j)) & 1 for j in range(384)]
        assert orc.hilbert_index_int(corner, 1) == h


def test_hilbert_d1_identity(orc):
    for B in [1, 3, 8]:
        assert [orc.hilbert_index_int((v,), B) for v in range(1 << B)] == list(range(1 << B))


def test_hilbert_top_level_is_gray_of_msbs(orc):
    """Level B-1 of the key depends only on the coordinates' top bits (a sub-cube fact)."""
    rng = np.random.default_rng(4)
    d = 40
    for _ in range(10):
        v = rng.integers(0, 256, d, dtype=np.uint8)
        w = v.copy()
        w ^= rng.integers(0, 128, d, dtype=np.uint8)  # change only lower bits
        kv, kw = orc.hilbert_index_int(v, 8), orc.hilbert_index_int(w, 8)
        assert kv >> (7 * d) == kw >> (7 * d)
        # and it is the Gray decode of the top bits (the B=1 curve of the top bits)
        assert kv >> (7 * d) == orc.hilbert_index_int(list(v >> 7), 1)


# ----------------------------------------------------------------- sort
def test_sort_by_key_then_id(orc):
    rng = np.random.default_rng(5)
    codes = rng.integers(120, 136, (300, 6), dtype=np.uint8)
    codes[50] = codes[7]  # exact duplicates
    codes[200] = codes[7]
    perm, refl = orc.curves(11, 1, 6)
    keys = orc.tree_keys(codes, perm[0], refl[0])
    order = orc.sort_keys(keys)
    ref = sorted(range(300), key=lambda i: (tuple(int(w) for w in keys[i]), i))
    assert order.tolist() == ref
    # and the keys are the Skilling keys of the permuted/reflected codes
    for p in [0, 7, 123]:
        v = codes[p][perm[0]] ^ np.where(refl[0] == 1, 255, 0).astype(np.uint8)
        assert (keys[p] == orc.hilbert_key(v, 8)).all()


# ----------------------------------------------------------------- trie
def _check_trie(orc, nodes, keys, order, codes, perm_t, refl_t, M):
    N, d = codes.shape
    W = keys.shape[1]
    kint = [int("".join("%016x" % int(w) for w in keys[p]), 16) for p in range(N)]
    nbits = 64 * W
    leaves = []

    def walk(idx, lo, hi, depth):
        w0, w1 = int(nodes[idx, 0]), int(nodes[idx, 1])
        if w1 >> 31:
            assert w0 == lo and (w1 & 0x7FFFFFFF) == hi - lo
            allsame = kint[order[lo]] == kint[order[hi - 1]]
            assert hi - lo <= M or allsame
            leaves.append((lo, hi))
            return idx + 1
        assert hi - lo > M
        a, L, flip = w1 & 0xFFFF, (w1 >> 16) & 7, (w1 >> 19) & 1
        bits = [(((codes[order[i], a] >> L) & 1) ^ flip) for i in range(lo, hi)]
        # node test equals key bit b for every point of the range, and splits 0* 1+
        x = kint[order[lo]] ^ kint[order[hi - 1]]
        b = nbits - x.bit_length()
        kb = [(kint[order[i]] >> (nbits - 1 - b)) & 1 for i in range(lo, hi)]
        assert bits == kb
        assert kb[0] == 0 and kb[-1] == 1 and kb == sorted(kb)
        assert L == 7 - b // d
        m = lo + kb.index(1)
        nxt = walk(idx + 1, lo, m, depth + 1)
        assert w0 == nxt  # right child follows the left subtree (pre-order)
        return walk(w0, m, hi, depth + 1)

    end = walk(0, 0, N, 0)
    assert end == nodes.shape[0]
    # leaves partition [0, N) in order
    assert leaves[0][0] == 0 and leaves[-1][1] == N
    assert all(a[1] == b[0] for a, b in zip(leaves, leaves[1:]))
    return leaves


@pytest.mark.parametrize("N,d,M,seed", [(500, 8, 10, 1), (700, 32, 25, 2), (300, 70, 7, 3),
                                        (64, 5, 100, 4)])
def test_trie_invariants_and_self_descent(orc, N, d, M, seed):
    rng = np.random.default_rng(seed)
    x = datagen.draw(datagen.centres(d, 4, seed, False), N, 0.1, seed + 9, np.float32)
    e = orc.quant_exp(x)
    codes = orc.quantize(x, e)
    codes[N // 3] = codes[N // 2]  # a duplicate pair
    perm, refl = orc.curves(seed, 2, d)
    for t in range(2):
        keys = orc.tree_keys(codes, perm[t], refl[t])
        order = orc.sort_keys(keys)
        nodes = orc.trie(keys, order, codes, perm[t], refl[t], M)
        leaves = _check_trie(orc, nodes, keys, order, codes, perm[t], refl[t], M)
        # every data point, used as a query, lands in the leaf that holds it
        k1 = 2
        ws = orc.window_starts(nodes, codes, N, k1)
        rank = np.empty(N, np.int64)
        rank[order] = np.arange(N)
        for p in rng.choice(N, 60, replace=False):
            lo, hi = next(l for l in leaves if l[0] <= rank[p] < l[1])
            mid = (lo + hi) // 2
            assert ws[p] == min(max(mid - k1 // 2, 0), max(0, N - k1))


def test_trie_all_equal_is_one_leaf(orc):
    codes = np.full((250, 6), 131, np.uint8)
    perm, refl = orc.curves(1, 1, 6)
    keys = orc.tree_keys(codes, perm[0], refl[0])
    order = orc.sort_keys(keys)
    nodes = orc.trie(keys, order, codes, perm[0], refl[0], 10)
    assert nodes.tolist() == [[0, 0x80000000 | 250]]
    assert order.tolist() == list(range(250))


def test_window_start_clamping(orc):
    nodes = np.array([[0, 0x80000000 | 10]], np.uint32)  # one leaf [0, 10)
    q = np.zeros((1, 3), np.uint8)
    assert orc.window_starts(nodes, q, 10, 4).tolist() == [3]  # mid 5 - 2
    assert orc.window_starts(nodes, q, 10, 20).tolist() == [0]  # k1 > N
    nodes = np.array([[5, 0x80000000 | 5]], np.uint32)  # leaf [5, 10), mid 7
    assert orc.window_starts(nodes, q, 10, 8).tolist() == [2]  # 7-4=3 > N-k1=2 -> 2


# ----------------------------------------------------------------- sketches
def _splitmix_words(orc, seed, n):
    # independent: drive the published generator through Python integers
    M64 = (1 << 64) - 1
    s, out = seed, []
    for _ in range(n):
        s = (s + 0x9E3779B97F4A7C15) & M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    assert out[0] == orc.splitmix64(seed, 0)
    return out


def test_srp_against_matmul(orc):
    d, n = 24, 40
    x = datagen.mixture(n, d, 3, 0.2, 5, dtype=np.float16)
    e = orc.quant_exp(x)
    sk = orc.srp(x, e, 99)
    words = _splitmix_words(orc, 99, (512 * d + 63) // 64)
    bits = np.array([(words[b // 64] >> (b % 64)) & 1 for b in range(512 * d)], np.int64)
    R = (2 * bits - 1).reshape(512, d)
    xq = np.clip(np.rint(x.astype(np.float64) * 2.0 ** (e + 5)), -8191, 8191).astype(np.int64)
    z = xq @ R.T
    want_bits = (z >= 0).astype(np.uint8)
    got_bits = np.unpackbits(sk.view(np.uint8), axis=1, bitorder="little")
    assert (got_bits == want_bits).all()


def test_srp_sign_symmetry_and_hamming(orc):
    x = datagen.mixture(200, 64, 5, 0.1, 6, dtype=np.float32)
    e = orc.quant_exp(np.concatenate([x, -x]))
    a, b = orc.srp(x, e, 3), orc.srp(-x, e, 3)
    # sketch(-x) is the complement except where a projection is exactly 0
    ham = orc.hamming(a, b)
    assert (ham >= 505).all() and (ham <= 512).mean() == 1.0
    assert (orc.hamming(a, a) == 0).all()
    h1 = orc.hamming(a[:50], a[50:100])
    h2 = orc.hamming(a[50:100], a[:50])
    assert (h1 == h2).all()


# ----------------------------------------------------------------- Alg. 1 reductions
def test_search_reduces_to_brute_force(orc):
    """T=1, k1 >= N, k2 >= N, h=0: every point is a candidate, so S is the exact top-k."""
    x, q = datagen.mixture(400, 16, 4, 0.1, 7, unit=False, dtype=np.float32, nq=30)
    F = orc.build_forest(x, T=1, M=20, seed=1, sketch_seed=2)
    r = orc.search(F, q, k1=400, k2=400, h=0, k=10)
    bi, bs = orc.brute_force_ip(x, q, 10)
    assert (r["c1n"] == 400).all()
    assert (r["ids"] == bi).all()
    assert np.allclose(r["scores"], bs, rtol=0, atol=1e-12)


def test_search_set_algebra_tiny(orc):
    """C1, C2 and E rebuilt with Python sets from the trees' windows."""
    x, q = datagen.mixture(300, 12, 3, 0.1, 8, unit=False, dtype=np.float32, nq=12)
    F = orc.build_forest(x, T=3, M=15, seed=3, sketch_seed=4)
    k1, k2, h, k = 40, 25, 2, 5
    r = orc.search(F, q, k1, k2, h, k)
    N = 300
    for i in range(q.shape[0]):
        C1 = set()
        for j, t in enumerate(F["trees"]):
            s = int(r["winstart"][i, j])
            C1 |= set(int(v) for v in F["tree_perm"][t][s:s + k1])
        assert len(C1) == r["c1n"][i]
        hm = {c: int(orc.hamming(r["qsk"][i], F["sk_pos"][c])) for c in C1}
        C2 = sorted(C1, key=lambda c: (hm[c], c))[:k2]
        assert r["c2"][i, :r["c2n"][i]].tolist() == C2
        E = set()
        for c in C2:
            E |= set(range(max(0, c - h), min(N - 1, c + h) + 1))
        assert len(E) == r["en"][i]
        sc = {c: float(np.dot(q[i].astype(np.float64), x[F["pos2id"][c]].astype(np.float64)))
              for c in E}
        best = sorted(E, key=lambda c: (-sc[c], c))[:k]
        assert r["ids"][i].tolist() == [int(F["pos2id"][c]) for c in best]


def test_master_order_and_tree_positions(orc):
    x = datagen.mixture(200, 8, 2, 0.2, 9, unit=False, dtype=np.float32)
    F = orc.build_forest(x, T=2, M=10, seed=5, sketch_seed=6)
    assert (F["tree_perm"][0] == np.arange(200)).all()  # tree 0 is the master order
    assert (F["pos2id"][F["pos"]] == np.arange(200)).all()
    assert sorted(F["tree_perm"][1].tolist()) == list(range(200))


# ----------------------------------------------------------------- Alg. 2 reductions
def test_graph_reduces_to_brute_force(orc):
    x = datagen.mixture(300, 16, 4, 0.1, 10, dtype=np.float16)
    orders, _ = orc.graph_orders(x, 2, 7)
    rows = np.arange(300)
    ids, sc, c1n = orc.graph_rows(x, orders, w=300, k=7, rows=rows)
    bi, bs = orc.brute_force_graph(x, rows, 7)
    assert (c1n == 299).all()
    assert (ids == bi).all()
    assert np.allclose(sc, bs, rtol=0, atol=1e-12)


def test_graph_window_sets_tiny(orc):
    x = datagen.mixture(120, 8, 3, 0.2, 11, dtype=np.float32)
    orders, _ = orc.graph_orders(x, 3, 5)
    w, k = 4, 3
    rows = np.arange(0, 120, 7)
    ids, sc, c1n = orc.graph_rows(x, orders, w, k, rows)
    X = x.astype(np.float64)
    for ri, p in enumerate(rows):
        C1 = set()
        for t in range(3):
            i = int(np.where(orders[t] == p)[0][0])
            C1 |= set(int(v) for v in orders[t][max(0, i - w):i + w + 1])
        C1.discard(int(p))
        assert len(C1) == c1n[ri]
        cos = {c: X[p] @ X[c] / (np.linalg.norm(X[p]) * np.linalg.norm(X[c])) for c in C1}
        assert ids[ri].tolist() == sorted(C1, key=lambda c: (-cos[c], c))[:k]


@pytest.mark.parametrize("w,k,k2", [(6, 4, 9), (3, 4, 40)])
def test_graph_prefilter_by_hamming(orc, w, k, k2):
    """C2 = the k2 smallest (Hamming, id) of the window union, -1 padded when
    the union is smaller; the result is the cosine top-k of C2 (Python sets,
    popcounts of Python integers)."""
    x = datagen.mixture(150, 16, 3, 0.2, 12, dtype=np.float16)
    orders, e = orc.graph_orders(x, 2, 5)
    sk = orc.srp(x, e, 13)
    rows = np.arange(0, 150, 5)
    ids, sc, c1n, c2 = orc.graph_rows(x, orders, w, k, rows, k2=k2, sk=sk, with_c2=True)
    X = x.astype(np.float64)
    for ri, p in enumerate(rows):
        C1 = set()
        for t in range(2):
            i = int(np.where(orders[t] == p)[0][0])
            C1 |= set(int(v) for v in orders[t][max(0, i - w):i + w + 1])
        C1.discard(int(p))
        hm = {c: sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(sk[p], sk[c])) for c in C1}
        C2 = sorted(C1, key=lambda c: (hm[c], c))[:k2]
        assert c2[ri].tolist() == C2 + [-1] * (k2 - len(C2))
        cos = {c: X[p] @ X[c] / (np.linalg.norm(X[p]) * np.linalg.norm(X[c])) for c in C2}
        want = sorted(C2, key=lambda c: (-cos[c], c))[:k]
        assert ids[ri].tolist() == want + [-1] * (k - len(want))


# ----------------------------------------------------------------- precision emulation
def test_e4m3_codes_roundtrip_and_extremes(orc):
    vals = [orc.e4m3_decode(c) for c in range(0x7F)]
    assert vals[0x7E] == 448.0 and vals[1] == 2.0 ** -9 and vals[8] == 2.0 ** -6
    assert all(b > a for a, b in zip(vals, vals[1:]))  # positive codes are increasing
    for c in range(0x7F):
        assert orc.e4m3_encode(vals[c]) == c
        assert orc.e4m3_encode(-vals[c]) == (c | 0x80 if c else 0x80)
    # midpoints go to the even code, beyond 448 saturates
    for c in range(0x7E):
        mid = (vals[c] + vals[c + 1]) / 2
        assert orc.e4m3_encode(mid) == (c if c % 2 == 0 else c + 1)
    assert orc.e4m3_encode(1e6) == 0x7E and orc.e4m3_encode(-500.0) == 0xFE


def test_bf16_rounding_against_bit_arithmetic(orc):
    import struct

    rng = np.random.default_rng(9)
    xs = np.concatenate([rng.standard_normal(2000), [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -1.5, 2.0 ** -20]])
    for x in xs.astype(np.float16).astype(np.float64):
        u = struct.unpack("<I", struct.pack("<f", x))[0]
        lo = u & 0xFFFF
        hi = u >> 16
        if lo > 0x8000 or (lo == 0x8000 and (hi & 1)):
            hi += 1
        want = struct.unpack("<f", struct.pack("<I", hi << 16))[0]
        assert orc.bf16(float(x)) == want


# ----------------------------------------------------------------- learned hash
def _small_net(seed, d=24, hid=16):
    rng = np.random.default_rng(seed)
    W1 = (rng.standard_normal((hid, d)) / np.sqrt(d)).astype(np.float32)
    b1 = (0.1 * rng.standard_normal(hid)).astype(np.float32)
    W2 = (rng.standard_normal((512, hid)) / np.sqrt(hid)).astype(np.float32)
    b2 = (0.1 * rng.standard_normal(512)).astype(np.float32)
    return W1, b1, W2, b2


def test_lhash_forward_is_a_plain_mlp(orc):
    W1, b1, W2, b2 = _small_net(1)
    x = np.random.default_rng(2).standard_normal((5, 24)).astype(np.float32)
    z1, a, z2, _ = orc.mlp_forward(x, W1, b1, W2, b2, rounded=False)
    X = x.astype(np.float64)
    ref1 = X @ W1.astype(np.float64).T + b1
    ref2 = np.maximum(ref1, 0) @ W2.astype(np.float64).T + b2
    assert np.allclose(z1, ref1, atol=1e-12) and np.allclose(z2, ref2, atol=1e-12)


def test_lhash_gradients_match_finite_differences(orc):
    W1, b1, W2, b2 = _small_net(3)
    rng = np.random.default_rng(4)
    A = rng.standard_normal((6, 24)).astype(np.float32)
    B = (A + 0.3 * rng.standard_normal((6, 24))).astype(np.float32)
    args = dict(slope=2.0, tau=0.2, lam=0.05, rounded=False)
    loss, g = orc.lhash_grad(A, B, W1, b1, W2, b2, **args)
    params = [W1, b1, W2, b2]
    for pi, P in enumerate(params):
        flat = P.reshape(-1)
        for idx in rng.choice(flat.size, 6, replace=False):
            h = 1e-3
            old = flat[idx]
            vals = []
            for sgn in (+1, -1):
                flat[idx] = old + sgn * h
                vals.append(orc.lhash_grad(A, B, *params, **args)[0])
            flat[idx] = old
            # the float32 parameter holds old+-h exactly only approximately: use the stored step
            num = (vals[0] - vals[1]) / (np.float64(np.float32(old + h)) - np.float64(np.float32(old - h)))
            ana = g[pi].reshape(-1)[idx]
            assert abs(num - ana) <= 1e-5 * max(1.0, abs(ana)) + 1e-7, (pi, idx, num, ana)


# ----------------------------------------------------------------- pins added for the precision and learned forms
def _bf16_bits(x):
    """bf16 rounding of binary64 values by integer arithmetic on their bits:
    keep the sign, the exponent and the top 7 fraction bits, rounding the 45
    dropped bits to nearest with ties to an even kept part."""
    u = np.asarray(x, np.float64).view(np.uint64)
    lo = u & np.uint64((1 << 45) - 1)
    hi = u >> np.uint64(45)
    up = (lo > np.uint64(1 << 44)) | ((lo == np.uint64(1 << 44)) & ((hi & np.uint64(1)) == 1))
    hi = hi + up.astype(np.uint64)
    return (hi << np.uint64(45)).view(np.float64)


def test_bf16_bit_helper_against_float32_path():
    """The test's own binary64 helper agrees with the float32 bit recipe on values
    that are exact in binary32 (no double rounding there)."""
    import struct

    rng = np.random.default_rng(21)
    xs = rng.standard_normal(500).astype(np.float32).astype(np.float64)
    for x in xs:
        u = struct.unpack("<I", struct.pack("<f", x))[0]
        hi, lo = u >> 16, u & 0xFFFF
        if lo > 0x8000 or (lo == 0x8000 and (hi & 1)):
            hi += 1
        assert _bf16_bits(x) == struct.unpack("<f", struct.pack("<I", hi << 16))[0]


def test_lhash_rounded_forward_against_bit_arithmetic(orc):
    """The deployed (bf16-rounded) forward equals a numpy MLP whose roundings are
    done on the bits of binary64 values."""
    W1, b1, W2, b2 = _small_net(11, d=40, hid=24)
    x = np.random.default_rng(12).standard_normal((9, 40)).astype(np.float32)
    z1, a, z2, band = orc.mlp_forward(x, W1, b1, W2, b2, rounded=True)
    X = _bf16_bits(x.astype(np.float64))
    ref1 = X @ _bf16_bits(W1.astype(np.float64)).T + b1.astype(np.float64)
    refa = _bf16_bits(np.maximum(ref1, 0.0))
    ref2 = refa @ _bf16_bits(W2.astype(np.float64)).T + b2.astype(np.float64)
    assert np.allclose(z1, ref1, rtol=0, atol=1e-12)
    assert (a == refa).all()
    assert np.allclose(z2, ref2, rtol=0, atol=1e-12)
    assert (band >= 0).all()


@pytest.mark.parametrize("a_val,below", [(1.5, True), (1.5, False), (1.0, True), (1.0, False),
                                          (0.75, True), (3.25, False)])
def test_lhash_band_flags_rounding_midpoints(orc, a_val, below):
    """A hidden pre-activation next to either rounding midpoint of its bf16 value
    (the lower one of a non-power-of-two value lies a half spacing 2^(e-9) below
    it, the lower one of a power of two 2^(e-10)) must put every output bit that
    depends on it in the fragile band, with a margin of at least one bf16 step of
    the activation times the weight."""
    e = int(np.frexp(a_val)[1])  # a_val in [2^(e-1), 2^e)
    up = 2.0 ** (e - 8)
    down = 2.0 ** (e - 9) if a_val == 2.0 ** (e - 1) else up
    mid = a_val - down / 2 if below else a_val + up / 2
    # z1 = W1 * bf16(x) + b1 with W1 = 1, x = 1 (exact in bf16); b1 carries the value
    eps = 2.0 ** -20
    z1_target = mid + (eps if below else -eps)  # on a_val's side of the midpoint
    b1 = np.array([z1_target - 1.0], np.float32)
    assert float(b1[0]) + 1.0 == z1_target
    W1 = np.ones((1, 1), np.float32)
    W2 = np.full((512, 1), 0.5, np.float32)
    b2 = np.zeros(512, np.float32)
    z1, a, z2, band = orc.mlp_forward(np.ones((1, 1), np.float32), W1, b1, W2, b2, rounded=True)
    assert z1[0, 0] == z1_target and a[0, 0] == a_val
    assert (band[0] >= 0.5 * min(up, down)).all(), (band[0, 0], up, down)
    # the other side of the midpoint really does round to the neighbour value
    other = _bf16_bits(np.array([mid - (eps if below else -eps)]))[0]
    assert other != a_val and abs(other - a_val) <= max(up, down)


def test_lhash_band_quiet_away_from_midpoints(orc):
    """Far from every midpoint and from the relu kink the band is only the
    summation term (2^-16 of the magnitudes)."""
    W1 = np.ones((1, 1), np.float32)
    b1 = np.array([0.25 + 2.0 ** -12], np.float32)  # z1 = 1.25 + 2^-12, far inside the cell of 1.25
    W2 = np.full((512, 1), 0.5, np.float32)
    b2 = np.zeros(512, np.float32)
    _, a, z2, band = orc.mlp_forward(np.ones((1, 1), np.float32), W1, b1, W2, b2, rounded=True)
    assert a[0, 0] == 1.25
    assert np.allclose(band[0], 2.0 ** -16 * np.abs(z2[0]), rtol=1e-12)


# e4m3 values from the format's definition (bias 7, 3 fraction bits, subnormals
# below 2^-6, no infinities, 0x7F/0xFF NaN), independent of the oracle's codec
E4M3_POS = np.array([(m / 8.0) * 2.0 ** -6 if E == 0 else (1 + m / 8.0) * 2.0 ** (E - 7)
                     for E in range(16) for m in range(8)][:0x7F])


def test_fp8_scale_rule(orc):
    rng = np.random.default_rng(31)
    x = (rng.standard_normal((40, 24)) * rng.uniform(1e-3, 10, (40, 1))).astype(np.float32)
    x[5] = 0.0
    for r in range(x.shape[0]):
        s = orc.lib().hfo_fp8_scale(x.ctypes.data, 1, r, x.shape[1])
        m = float(np.abs(x[r]).max())
        if m == 0.0:
            assert s == 1.0
            continue
        # s is max|x| / 448 to binary32 precision ...
        assert abs(s * 448.0 - m) <= 2.0 ** -23 * m
        # ... so the largest element encodes to the largest finite code and none saturates beyond it
        codes = [orc.e4m3_encode(float(np.float32(v) / np.float32(s))) for v in x[r]]
        assert orc.e4m3_encode(float(np.float32(m) / np.float32(s))) == 0x7E
        assert all((c & 0x7F) <= 0x7E for c in codes)


def _lowprec_case(orc, x, q, c2_sets, h, k, prec, S):
    N, d = x.shape
    F = dict(x=x, N=N, d=d, pos2id=np.arange(N, dtype=np.uint32))
    k2 = max(len(c) for c in c2_sets)
    c2 = np.full((len(c2_sets), k2), 0xFFFFFFFF, np.uint32)
    c2n = np.array([len(c) for c in c2_sets], np.int32)
    for i, c in enumerate(c2_sets):
        c2[i, :len(c)] = c
    return orc.search_lowprec(F, q, c2, c2n, h, k, prec, S), c2, c2n


def _expansion(c2_set, h, N):
    return sorted({p for r in c2_set for p in range(max(0, r - h), min(N - 1, r + h) + 1)})


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_lowprec_exact_when_values_are_representable(orc, prec):
    """Rows and queries made of values the format holds exactly (for FP8: e4m3
    values times a power of two, with an element at 448 times it, so the
    scale is that power of two): the low-precision scores are then the exact
    inner products, the survivors are the first S of E by (exact score desc,
    position asc), built here with Python sets and sorting, and the result is
    the FP64 top-k of the survivors.  Duplicate rows make ties at the cut."""
    rng = np.random.default_rng(41 if prec == "bf16" else 42)
    N, d, nq, h, k, S = 90, 16, 6, 1, 5, 12
    if prec == "bf16":
        vals = _bf16_bits(rng.standard_normal((N + nq, d)))
    else:
        pick = rng.integers(0, 0x7F, (N + nq, d))
        vals = E4M3_POS[pick] * rng.choice([-1.0, 1.0], (N + nq, d))
        vals[:, 0] = 448.0 * rng.choice([-1.0, 1.0], N + nq)
        vals *= (2.0 ** -rng.integers(3, 12, (N + nq, 1)))
    vals = vals.astype(np.float32)
    x, q = vals[:N].copy(), vals[N:].copy()
    x[31] = x[30]  # tied rows
    x[61] = x[60]
    c2_sets = [sorted(rng.choice(N, size=rng.integers(3, 15), replace=False).tolist()) for _ in range(nq)]
    c2_sets[0] = [30, 31, 60, 61, 0, 89]
    res, _, _ = _lowprec_case(orc, x, q, c2_sets, h, k, prec, S)
    X, Q = x.astype(np.float64), q.astype(np.float64)
    for i in range(nq):
        E = _expansion(c2_sets[i], h, N)
        exact = {p: float(Q[i] @ X[p]) for p in E}
        surv = sorted(E, key=lambda p: (-exact[p], p))[:S]
        ns = len(surv)
        assert res["surv_pos"][i][:ns].tolist() == surv
        assert (res["surv_pos"][i][ns:] == 0xFFFFFFFF).all()
        assert res["surv_score"][i][:ns].tolist() == [exact[p] for p in surv]
        top = sorted(surv, key=lambda p: (-exact[p], p))[:k]
        assert res["ids"][i][:len(top)].tolist() == top
        assert (res["ids"][i][len(top):] == -1).all()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_lowprec_scores_within_format_error(orc, prec):
    """On general values every survivor's low-precision score lies within the
    rounding error of the format of the exact inner product (bf16: relative
    2^-9 per operand; e4m3: relative 2^-4 per normal operand, absolute half the
    smallest subnormal 2^-10 times the scale below 2^-6), the survivors are
    positions of E (Python sets) in non-increasing score order, and the
    result is the FP64 top-k over them."""
    rng = np.random.default_rng(43)
    N, d, nq, h, k, S = 200, 24, 8, 2, 6, 15
    x = rng.standard_normal((N, d)).astype(np.float32)
    q = rng.standard_normal((nq, d)).astype(np.float32)
    c2_sets = [sorted(rng.choice(N, size=10, replace=False).tolist()) for _ in range(nq)]
    res, _, _ = _lowprec_case(orc, x, q, c2_sets, h, k, prec, S)
    X, Q = x.astype(np.float64), q.astype(np.float64)

    def op_err(v):
        if prec == "bf16":
            return 2.0 ** -9 * np.abs(v)
        s = np.abs(v).max() / 448.0
        return np.maximum(2.0 ** -4 * np.abs(v), 2.0 ** -10 * s) * (1 + 2.0 ** -20)

    for i in range(nq):
        E = set(_expansion(c2_sets[i], h, N))
        sp = res["surv_pos"][i]
        ns = min(S, len(E))
        got = sp[:ns].tolist()
        assert len(set(got)) == ns and set(got) <= E
        sc = res["surv_score"][i][:ns]
        assert (np.diff(sc) <= 0).all()
        eq = op_err(Q[i])
        for p, s in zip(got, sc):
            ex = op_err(X[p])
            bound = np.sum(np.abs(Q[i]) * ex + np.abs(X[p]) * eq + eq * ex) + 1e-12
            assert abs(s - Q[i] @ X[p]) <= bound
        exact = {p: float(Q[i] @ X[p]) for p in got}
        top = sorted(got, key=lambda p: (-exact[p], p))[:k]
        assert res["ids"][i].tolist() == top


# ----------------------------------------------------------------- exact position of a query (Section 2)
def test_exact_rank_counts_smaller_keys(orc):
    """The exact rank of a query is the number of data points with a strictly
    smaller Hilbert key (Python integers of every key), and the window start
    centres k1 on it, shifted into [0, N)."""
    rng = np.random.default_rng(61)
    N, d, k1 = 300, 5, 40
    codes = rng.integers(0, 256, (N, d), dtype=np.uint8)
    codes[10] = codes[3]  # equal keys
    perm, refl = orc.curves(9, 1, d)
    keys = orc.tree_keys(codes, perm[0], refl[0])
    order = orc.sort_keys(keys)
    q = rng.integers(0, 256, (60, d), dtype=np.uint8)
    q[0] = codes[3]  # equal to two data keys: ranks before both
    q[1] = 0
    q[2] = 255
    rank, start = orc.exact_ranks(keys, order, q, perm[0], refl[0], k1)
    tc = lambda c: [int(c[perm[0][i]]) ^ (255 if refl[0][i] else 0) for i in range(d)]
    dk = [orc.hilbert_index_int(tc(c), 8) for c in codes]
    for i in range(q.shape[0]):
        qk = orc.hilbert_index_int(tc(q[i]), 8)
        want = sum(1 for v in dk if v < qk)
        assert rank[i] == want
        assert start[i] == min(max(want - k1 // 2, 0), N - k1)


def test_exact_rank_of_a_data_point_is_its_place(orc):
    """A data point whose key is unique, used as a query, ranks at its own
    position in the tree's order; with repeats, at the first of them."""
    rng = np.random.default_rng(62)
    N, d = 500, 12
    codes = rng.integers(100, 156, (N, d), dtype=np.uint8)
    codes[7] = codes[400]
    perm, refl = orc.curves(4, 3, d)
    for t in range(3):
        keys = orc.tree_keys(codes, perm[t], refl[t])
        order = orc.sort_keys(keys)
        place = np.empty(N, np.int64)
        place[order] = np.arange(N)
        rank, _ = orc.exact_ranks(keys, order, codes, perm[t], refl[t], 1)
        for p in range(N):
            same = np.where((keys == keys[p]).all(axis=1))[0]
            assert rank[p] == min(place[same])


def test_exact_position_search_reduces_to_brute_force(orc):
    """With one tree, k1 >= N, k2 >= N and h = 0 the search with exact
    positions is the exact k-NN too (the window is every point)."""
    x, q = datagen.mixture(400, 16, 4, 0.1, 63, unit=False, dtype=np.float32, query_seed=64, nq=20)
    F = orc.build_forest(x, T=1, M=20, seed=3, sketch_seed=4)
    r = orc.search(F, q, 400, 400, 0, 7, position="exact")
    bi, bs = orc.brute_force_ip(x, q, 7)
    assert (r["ids"] == bi).all()
    assert np.allclose(r["scores"], bs, rtol=0, atol=1e-12)


# ----------------------------------------------------------------- the paper's compressed layout (Section 3.1)
def test_c4_codes_against_exact_rationals(orc):
    """Magnitude levels by exact rational arithmetic (m = #{k in 1..7 : 8|x| >=
    k max|x|}), signs by Python bit packing, scale = max|x| / 8, and every
    value within half a level of the stored one (the largest element at 7.5 s)."""
    from fractions import Fraction

    rng = np.random.default_rng(71)
    x = (rng.standard_normal((40, 70)) * rng.uniform(0.01, 3, (40, 1))).astype(np.float32)
    x[3] = 0.0
    x[4, :5] = -0.0
    x[5] = np.abs(x[5])
    sg, mag, sc = orc.c4_encode(x)
    for p in range(x.shape[0]):
        mx = max(Fraction(abs(float(v))) for v in x[p])
        assert sc[p] == float(mx / 8)
        bits = 0
        for i, v in enumerate(x[p]):
            a = Fraction(abs(float(v)))
            assert mag[p, i] == sum(1 for kk in range(1, 8) if 8 * a >= kk * mx)
            if float(v) >= 0.0:
                bits |= 1 << i
            val = (float(mag[p, i]) + 0.5) * sc[p] * (1 if float(v) >= 0 else -1)
            assert abs(val - float(v)) <= sc[p] / 2 + 1e-300
        words = [(bits >> (64 * w)) & ((1 << 64) - 1) for w in range(sg.shape[1])]
        assert [int(w) for w in sg[p]] == words


def test_c4_search_reduces_to_brute_force_on_decoded_rows(orc):
    """One tree, k1 >= N, k2 >= N, h = 0: the compressed-layout search is the
    exact top-k of the inner products with the decoded rows (decoded here from
    the definition, numpy FP64)."""
    x, q = datagen.mixture(600, 24, 6, 0.1, 72, unit=False, dtype=np.float32, query_seed=73, nq=25)
    F = orc.build_forest(x, T=1, M=30, seed=3, sketch_seed=4)
    r = orc.search_c4(F, q, 600, 600, 0, 9)
    mx = np.abs(x.astype(np.float64)).max(axis=1, keepdims=True)
    m = np.zeros(x.shape)
    for kk in range(1, 8):
        m += (8 * np.abs(x.astype(np.float64)) >= kk * mx)
    dec = np.where(x >= 0, 1.0, -1.0) * (m + 0.5) * mx / 8
    S = q.astype(np.float64) @ dec.T
    o = np.argsort(-S, axis=1, kind="stable")[:, :9]
    assert (r["ids"] == o).all()
    assert np.allclose(r["scores"], np.take_along_axis(S, o, 1), rtol=0, atol=1e-12)


def test_c4_search_c2_by_sign_hamming(orc):
    """C2 is the first k2 of the windows' union by (Hamming distance of the
    coordinate-sign sketches, position), rebuilt with Python sets and integers."""
    x, q = datagen.mixture(500, 20, 5, 0.1, 74, unit=False, dtype=np.float32, query_seed=75, nq=8)
    F = orc.build_forest(x, T=3, M=10, seed=5, sketch_seed=6)
    k1, k2, h, k = 30, 25, 1, 5
    r = orc.search_c4(F, q, k1, k2, h, k)
    X = x[F["pos2id"]]  # rows in master order
    sgn = lambda v: sum(1 << i for i, a in enumerate(v) if float(a) >= 0)
    for i in range(q.shape[0]):
        C1 = set()
        for j, t in enumerate(F["trees"]):
            s0 = int(r["winstart"][i, j])
            C1 |= set(int(v) for v in F["tree_perm"][t][s0:s0 + k1])
        qs = sgn(q[i])
        want = sorted(C1, key=lambda p: (bin(qs ^ sgn(X[p])).count("1"), p))[:k2]
        assert r["c2"][i][:len(want)].tolist() == want


def test_lhash_gradients_with_hard_negatives_match_finite_differences(orc):
    """The objective with one hard negative per query (an extra logit in each
    query's softmax) has the gradients the central finite differences give."""
    W1, b1, W2, b2 = _small_net(13)
    rng = np.random.default_rng(14)
    A = rng.standard_normal((5, 24)).astype(np.float32)
    B = (A + 0.3 * rng.standard_normal((5, 24))).astype(np.float32)
    N = (A + 0.6 * rng.standard_normal((5, 24))).astype(np.float32)
    args = dict(slope=2.0, tau=0.2, lam=0.05, rounded=False, Neg=N)
    loss, g = orc.lhash_grad(A, B, W1, b1, W2, b2, **args)
    loss0, _ = orc.lhash_grad(A, B, W1, b1, W2, b2, slope=2.0, tau=0.2, lam=0.05, rounded=False)
    assert loss != loss0  # the negative enters the loss
    params = [W1, b1, W2, b2]
    for pi, P in enumerate(params):
        flat = P.reshape(-1)
        for idx in rng.choice(flat.size, 5, replace=False):
            h = 1e-4  # well inside the relu kinks of this batch (the nearest pre-activation is 3e-4 from 0)
            old = flat[idx]
            vals = []
            for sgn in (+1, -1):
                flat[idx] = old + sgn * h
                vals.append(orc.lhash_grad(A, B, *params, **args)[0])
            flat[idx] = old
            num = (vals[0] - vals[1]) / (np.float64(np.float32(old + h)) - np.float64(np.float32(old - h)))
            ana = g[pi].reshape(-1)[idx]
            assert abs(num - ana) <= 1e-5 * max(1.0, abs(ana)) + 1e-7, (pi, idx, num, ana)


def test_lhash_loss_with_negatives_closed_form(orc):
    """With all weights zero every code is 0: every logit is 0, so the loss is
    log(B + 1) with a negative per query (log B without) and all gradients of
    W1 and W2 vanish."""
    d, hid, Bn = 6, 4, 5
    W1, b1 = np.zeros((hid, d), np.float32), np.zeros(hid, np.float32)
    W2, b2 = np.zeros((512, hid), np.float32), np.zeros(512, np.float32)
    A = np.random.default_rng(15).standard_normal((Bn, d)).astype(np.float32)
    loss, g = orc.lhash_grad(A, A, W1, b1, W2, b2, 1.0, 0.5, 0.1, rounded=False, Neg=A)
    assert abs(loss - np.log(Bn + 1)) < 1e-12
    loss2, _ = orc.lhash_grad(A, A, W1, b1, W2, b2, 1.0, 0.5, 0.1, rounded=False)
    assert abs(loss2 - np.log(Bn)) < 1e-12
    assert np.abs(g[0]).max() == 0 and np.abs(g[2]).max() == 0
