"""HIP path against the CPU oracle, through the C ABI.

Integer outputs (codes, permutations, split bits, tree records, window
starts, candidate lists, sketches) must be bit-identical.  FP32 scores must be
within 1e-5 * |q| |x| of the oracle's FP64 scores; result ids may differ only
where the oracle's FP64 scores are within that tolerance of the k-th score.
"""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def hf():
    import torch

    import paper_2508_21682_amd as hf

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    hf.lib()
    return hf


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def first_diff_bits(keys, order):
    """Split bit of each adjacent pair in `order` from full oracle keys (NONE if equal)."""
    a, b = keys[order[:-1]], keys[order[1:]]
    x = a ^ b
    out = np.full(len(order) - 1, 0xFFFFFFFF, np.uint64)
    W = keys.shape[1]
    for w in range(W - 1, -1, -1):  # the first differing word wins
        nz = x[:, w] != 0
        lz = np.zeros(nz.sum(), np.uint64)
        v = x[nz, w].copy()
        for sh in [32, 16, 8, 4, 2, 1]:
            m = v < (np.uint64(1) << np.uint64(64 - sh))
            lz[m] += np.uint64(sh)
            v[m] <<= np.uint64(sh)
        out[nz] = np.uint64(64 * w) + lz
    return out.astype(np.uint32)


def check_topk(gi, gs, oi, os_, x, q, k):
    """Rank-wise scores within TOL; differing ids only at near-ties of the k-th score."""
    assert gi.shape == oi.shape
    for row in gi:  # a result lists each id once
        v = row[row >= 0]
        assert np.unique(v).size == v.size, row
    fin = np.isfinite(os_)
    assert (np.isfinite(gs) == fin).all()
    assert np.abs(gs[fin] - os_[fin]).max() <= TOL
    X = x.astype(np.float64)
    Q = q.astype(np.float64)
    bad = 0
    for i in range(gi.shape[0]):
        if (gi[i] == oi[i]).all():
            continue
        kth = os_[i, k - 1]
        for c in set(gi[i].tolist()) ^ set(oi[i].tolist()):
            if c < 0:
                bad += 1
                continue
            s = float(Q[i] @ X[c])
            if abs(s - kth) > TOL:
                bad += 1
    assert bad == 0, "%d ids differ beyond near-ties" % bad


# ------------------------------------------------------------------ quantiser
@pytest.mark.parametrize("dtype,d", [(np.float16, 384), (np.float32, 32), (np.float32, 7)])
def test_quantize_parity(hf, orc, dtype, d):
    x = datagen.mixture(3001, d, 5, 0.1, 21, unit=False, dtype=dtype)
    x[0, :3] = np.array([0.0, -0.0, 2.0 ** -9], dtype)
    xd = dev(x)
    e = hf.quant_exp(xd)
    assert e == orc.quant_exp(x)
    assert (hf.quantize(xd, e).cpu().numpy() == orc.quantize(x, e)).all()
    # queries outside the data range clamp
    assert (hf.quantize(dev(x * 4), e).cpu().numpy() == orc.quantize(x * 4, e)).all()


def test_quant_exp_rejects_nonfinite(hf):
    x = np.ones((10, 4), np.float32)
    x[3, 2] = np.nan
    with pytest.raises(hf.HFError) as ei:
        hf.quant_exp(dev(x))
    assert ei.value.status == 2


# ------------------------------------------------------------------ Hilbert sort
SORT_CASES = [
    # name, N, d, dtype, n_comp, sigma, unit, trees
    ("c1-like", 10000, 32, np.float32, 16, 0.1, False, [0, 3]),
    ("d384", 3000, 384, np.float16, 8, 0.05, True, [0, 1]),
    ("d70", 2500, 70, np.float32, 4, 0.1, False, [2]),
    ("d8-ties", 1500, 8, np.float32, 3, 0.3, False, [0, 1]),
    ("d1", 500, 1, np.float32, 2, 0.5, False, [0]),
    ("d2", 700, 2, np.float32, 2, 0.5, False, [0]),
    ("d130-tight", 1200, 130, np.float16, 2, 0.002, True, [0]),
]


@pytest.mark.parametrize("case", SORT_CASES, ids=[c[0] for c in SORT_CASES])
def test_hilbert_sort_parity(hf, orc, case):
    name, N, d, dtype, nc, sigma, unit, trees = case
    print("case", name, flush=True)
    x = datagen.mixture(N, d, nc, sigma, 31 + N, unit=unit, dtype=dtype)
    e = orc.quant_exp(x)
    codes = orc.quantize(x, e)
    codes[5] = codes[9]  # duplicates
    codes[N - 1] = codes[9]
    perm, refl = orc.curves(77, max(trees) + 1, d)
    cd = dev(codes)
    for t in trees:
        keys = orc.tree_keys(codes, perm[t], refl[t])
        want = orc.sort_keys(keys)
        order, split = hf.hilbert_sort(cd, 77, t, with_split=True)
        assert (u32(order) == want).all(), "tree %d order" % t
        assert (u32(split) == first_diff_bits(keys, want)).all(), "tree %d split bits" % t


def test_hilbert_sort_single_point(hf):
    order = hf.hilbert_sort(dev(np.array([[3, 4, 5]], np.uint8)), 1, 0)
    assert u32(order).tolist() == [0]


# ------------------------------------------------------------------ sketches
@pytest.mark.parametrize("dtype,d", [(np.float16, 384), (np.float32, 32), (np.float32, 70)])
def test_srp_parity(hf, orc, dtype, d, monkeypatch):
    """d a multiple of 16 runs the int8 matrix-core kernel, d = 70 the vector-ALU
    one; with HF_SRP_VALU set every d takes the vector-ALU kernel.  777 rows:
    a ragged last block of 64."""
    x = datagen.mixture(777, d, 3, 0.1, 41, dtype=dtype)
    e = orc.quant_exp(x)
    want = orc.srp(x, e, 1234)
    # queries with larger values than the data clamp identically
    want2 = orc.srp(x * 3, e, 1234)
    for valu in (False, True):
        if valu:
            monkeypatch.setenv("HF_SRP_VALU", "1")
        got = hf.srp_sketch(dev(x), e, 1234).cpu().numpy().view(np.uint64)
        assert (got == want).all(), valu
        got2 = hf.srp_sketch(dev(x * 3), e, 1234).cpu().numpy().view(np.uint64)
        assert (got2 == want2).all(), valu
    monkeypatch.delenv("HF_SRP_VALU")


# ------------------------------------------------------------------ forest + search
def _forest_case(hf, orc, x, q, T, M, seed, sk_seed, params):
    F = orc.build_forest(x, T=T, M=M, seed=seed, sketch_seed=sk_seed)
    fo = hf.Forest(dev(x), n_trees=T, leaf_max=M, seed=seed, sketch_seed=sk_seed)
    assert fo.info["quant_exp"] == F["e"]
    assert (u32(fo.pos2id()) == F["pos2id"]).all()
    assert (fo.sketches().cpu().numpy().view(np.uint64) == F["sk_pos"]).all()
    for t in range(T):
        assert (u32(fo.perm(t)) == F["tree_perm"][t]).all(), "perm %d" % t
        got = u32(fo.nodes(t)).reshape(-1, 2)
        assert got.shape == F["nodes"][t].shape, "tree %d node count" % t
        assert (got == F["nodes"][t]).all(), "tree %d records" % t
        assert (u32(fo.node_splits(t)).reshape(-1, 2) == F["splits"][t]).all(), "tree %d split records" % t
    qd = dev(q)
    for (k1, k2, h, k) in params:
        print("search k1=%d k2=%d h=%d k=%d" % (k1, k2, h, k), flush=True)
        want = orc.search(F, q, k1, k2, h, k)
        r = fo.search_debug(qd, k, k1, k2, h)
        assert (u32(r["winstart"]) == want["winstart"]).all()
        assert (r["c2n"].cpu().numpy() == want["c2n"]).all()
        assert (u32(r["c2"]) == want["c2"]).all()
        assert (r["en"].cpu().numpy() == want["en"]).all()
        check_topk(r["ids"].cpu().numpy(), r["scores"].cpu().numpy(), want["ids"], want["scores"], x, q, k)
        ids2, sc2 = fo.search(qd, k, k1, k2, h)
        assert (ids2.cpu().numpy() == r["ids"].cpu().numpy()).all()  # deterministic
        assert (sc2.cpu().numpy() == r["scores"].cpu().numpy()).all()
    fo.free()


def test_forest_search_small_fp32(hf, orc):
    """10,000 x 32 fp32 mixture, 8 trees, leaves of 100 points, 1,000 queries, k=10."""
    w = datagen.WORKLOADS["search-10Kx32"]
    x, q = datagen.mixture(w["n"], w["d"], w["n_comp"], w["sigma"], w["seed"], unit=w["unit"],
                           dtype=np.float32, query_seed=w["query_seed"], nq=w["nq"])
    _forest_case(hf, orc, x, q, T=8, M=100, seed=1, sk_seed=2,
                 params=[(256, 64, 1, 10), (100, 10, 0, 10), (1000, 300, 3, 10)])


def test_forest_search_fp16_d384(hf, orc):
    x, q = datagen.mixture(20000, 384, 64, 0.05, 51, dtype=np.float16, query_seed=52, nq=150)
    _forest_case(hf, orc, x, q, T=4, M=100, seed=5, sk_seed=6, params=[(300, 100, 2, 30)])


def test_forest_edge_cases(hf, orc):
    # N below k1 and below the leaf size: one leaf, the window is everything
    x, q = datagen.mixture(150, 16, 3, 0.1, 61, unit=False, dtype=np.float32, nq=20)
    _forest_case(hf, orc, x, q, T=3, M=200, seed=7, sk_seed=8,
                 params=[(500, 150, 0, 10), (40, 20, 5, 20), (7, 5, 0, 5)])
    # a ragged N with tiny leaves
    x, q = datagen.mixture(1237, 24, 5, 0.1, 62, unit=False, dtype=np.float32, nq=33)
    _forest_case(hf, orc, x, q, T=2, M=3, seed=9, sk_seed=10, params=[(17, 11, 1, 4)])


def test_forest_search_large_candidate_sets(hf, orc):
    """16 trees x windows of 2,048-2,500 (up to 40,000 entries per query)."""
    x, q = datagen.mixture(30000, 64, 24, 0.1, 55, dtype=np.float16, query_seed=56, nq=160)
    _forest_case(hf, orc, x, q, T=16, M=100, seed=13, sk_seed=14, params=[(2500, 600, 2, 20), (2048, 300, 0, 10)])


def test_forest_search_many_trees(hf, orc):
    """1,100 and 4,096 trees (the limit): more window starts per query than
    1,024 (the Hamming filter keeps them in LDS sized by the tree count)."""
    x, q = datagen.mixture(2000, 8, 6, 0.1, 71, unit=False, dtype=np.float32, query_seed=72, nq=24)
    _forest_case(hf, orc, x, q, T=1100, M=20, seed=3, sk_seed=4, params=[(6, 40, 1, 5), (37, 200, 0, 10)])
    # the largest forest the library accepts (4,096 trees)
    x, q = datagen.mixture(2000, 8, 6, 0.1, 73, unit=False, dtype=np.float32, query_seed=74, nq=16)
    _forest_case(hf, orc, x, q, T=4096, M=20, seed=5, sk_seed=6, params=[(5, 30, 1, 5)])


@pytest.mark.parametrize("env", [{"HF_FILTER_BUCKET_BITS": "8"}, {"HF_FILTER_BUCKET_BITS": "11"},
                                 {"HF_FILTER": "direct"}], ids=["buckets-256", "buckets-2048", "direct"])
def test_filter_forms_give_the_oracle_c2(hf, orc, monkeypatch, env):
    """C2 is the same exact set whichever way the Hamming filter is organised:
    by master-position bucket (here 118 or 15 buckets over 30,000 points, so
    chunks of every XCD's list and runs of every query in many buckets) or
    entry by entry; small thresholds (k2 = 20) and large ones (k2 = 900) both
    run, and the queries whose threshold passed too few distinct entries are
    redone entry by entry."""
    for k_, v_ in env.items():
        monkeypatch.setenv(k_, v_)
    x, q = datagen.mixture(30000, 64, 24, 0.1, 59, dtype=np.float16, query_seed=60, nq=200)
    F = orc.build_forest(x, T=16, M=100, seed=17, sketch_seed=18)
    fo = hf.Forest(dev(x), n_trees=16, leaf_max=100, seed=17, sketch_seed=18)
    for (k1, k2, h, k) in [(400, 20, 0, 10), (1500, 900, 1, 30), (90, 300, 0, 20)]:
        want = orc.search(F, q, k1, k2, h, k)
        r = fo.search_debug(dev(q), k, k1, k2, h)
        assert (r["c2n"].cpu().numpy() == want["c2n"]).all()
        assert (u32(r["c2"]) == want["c2"]).all()
        check_topk(r["ids"].cpu().numpy(), r["scores"].cpu().numpy(), want["ids"], want["scores"], x, q, k)
    fo.free()


def _exact_case(hf, orc, x, q, T, M, seed, sk_seed, params):
    F = orc.build_forest(x, T=T, M=M, seed=seed, sketch_seed=sk_seed)
    fo = hf.Forest(dev(x), n_trees=T, leaf_max=M, seed=seed, sketch_seed=sk_seed)
    qd = dev(q)
    for (k1, k2, h, k) in params:
        want = orc.search(F, q, k1, k2, h, k, position="exact")
        r = fo.search_debug(qd, k, k1, k2, h, position="exact")
        assert (u32(r["winstart"]) == want["winstart"]).all()
        assert (u32(r["c2"]) == want["c2"]).all()
        check_topk(r["ids"].cpu().numpy(), r["scores"].cpu().numpy(), want["ids"], want["scores"], x, q, k)
    fo.free()


def test_exact_position_parity(hf, orc):
    """Windows centred on each query's exact insertion rank (the oracle binary
    searches full keys): window starts, C2 and results equal the oracle's.
    Half the queries copy data rows or perturb one code of a data row, so the
    top key level (the coordinates' signs) ties and full keys decide."""
    x, q = datagen.mixture(20000, 384, 64, 0.05, 65, dtype=np.float16, query_seed=66, nq=120)
    q[:30] = x[np.arange(30) * 101]
    q[30:60] = x[np.arange(30) * 97 + 5]
    q[30:60, 7] = (q[30:60, 7].astype(np.float32) * 0.5).astype(np.float16)  # a smaller code, same sign
    _exact_case(hf, orc, x, q, T=4, M=100, seed=19, sk_seed=20, params=[(300, 100, 1, 30), (31, 20, 0, 10)])


def test_exact_position_small_and_ragged(hf, orc):
    w = datagen.WORKLOADS["search-10Kx32"]
    x, q = datagen.mixture(w["n"], w["d"], w["n_comp"], w["sigma"], w["seed"], unit=w["unit"],
                           dtype=np.float32, query_seed=w["query_seed"], nq=300)
    _exact_case(hf, orc, x, q, T=8, M=100, seed=1, sk_seed=2, params=[(256, 64, 1, 10)])
    x, q = datagen.mixture(1237, 7, 5, 0.1, 67, unit=False, dtype=np.float32, nq=33)
    q[:5] = x[:5]
    _exact_case(hf, orc, x, q, T=3, M=3, seed=9, sk_seed=10, params=[(17, 11, 1, 4), (2000, 50, 0, 5)])
    # all points identical: every comparison reaches the deepest key level
    x = np.tile(datagen.mixture(1, 16, 1, 0.1, 68, unit=False, dtype=np.float32), (500, 1))
    q = np.concatenate([x[:3], datagen.mixture(4, 16, 1, 0.1, 69, unit=False, dtype=np.float32)])
    _exact_case(hf, orc, x, q, T=2, M=50, seed=11, sk_seed=12, params=[(40, 30, 0, 5)])


def _c4_case(hf, orc, x, q, T, M, seed, params, position="leaf"):
    """The compressed layout against the oracle: sign sketches bit for bit,
    window starts and C2 exact, scores from the 4-bit codes within TOL of the
    oracle's FP64 scores of the same codes, ids equal up to near-ties."""
    F = orc.build_forest(x, T=T, M=M, seed=seed, sketch_seed=1)
    fo = hf.Forest(dev(x), n_trees=T, leaf_max=M, seed=seed, sketch_seed=1, sketch="sign")
    sg, mag, sc = orc.c4_encode(x)
    want_sk = np.zeros((x.shape[0], 8), np.uint64)
    want_sk[:, :sg.shape[1]] = sg
    assert (fo.sketches().cpu().numpy().view(np.uint64) == want_sk[F["pos2id"]]).all()
    fo.add_precision("c4")
    dec = np.where(x >= 0, 1.0, -1.0) * (mag + 0.5) * sc[:, None]  # decoded rows, FP64
    Q = q.astype(np.float64)
    for (k1, k2, h, k) in params:
        want = orc.search_c4(F, q, k1, k2, h, k, position=position)
        r = fo.search_debug(dev(q), k, k1, k2, h, precision="c4", position=position)
        assert (u32(r["winstart"]) == want["winstart"]).all()
        assert (u32(r["c2"]) == want["c2"]).all()
        assert (r["en"].cpu().numpy() == want["en"]).all()
        gi, gs = r["ids"].cpu().numpy(), r["scores"].cpu().numpy()
        fin = np.isfinite(want["scores"])
        assert (np.isfinite(gs) == fin).all()
        assert np.abs(gs[fin] - want["scores"][fin]).max() <= TOL
        for i in range(gi.shape[0]):
            v = gi[i][gi[i] >= 0]
            assert np.unique(v).size == v.size
            kth = want["scores"][i, k - 1]
            for c in set(gi[i].tolist()) ^ set(want["ids"][i].tolist()):
                assert c >= 0 and abs(float(Q[i] @ dec[c]) - kth) <= TOL
    fo.free()


def test_compressed_layout_parity(hf, orc):
    """Section 3.1's layout: 384-bit coordinate-sign sketches, 4-bit codes
    sharing the sign bit, rerank from the codes with unquantized queries."""
    x, q = datagen.mixture(20000, 384, 64, 0.05, 76, dtype=np.float16, query_seed=77, nq=100)
    _c4_case(hf, orc, x, q, T=4, M=100, seed=21, params=[(300, 100, 2, 30), (50, 40, 0, 10)])
    _c4_case(hf, orc, x, q[:40].copy(), T=4, M=100, seed=21, params=[(300, 100, 1, 30)], position="exact")


def test_compressed_layout_small_dims(hf, orc):
    w = datagen.WORKLOADS["search-10Kx32"]
    x, q = datagen.mixture(w["n"], w["d"], w["n_comp"], w["sigma"], w["seed"], unit=w["unit"],
                           dtype=np.float32, query_seed=w["query_seed"], nq=200)
    _c4_case(hf, orc, x, q, T=8, M=100, seed=1, params=[(256, 64, 1, 10)])
    x, q = datagen.mixture(3001, 70, 7, 0.1, 78, unit=False, dtype=np.float32, nq=50)
    x[5] = 0.0  # a zero row: scale 0, every value 0
    _c4_case(hf, orc, x, q, T=3, M=20, seed=9, params=[(120, 60, 1, 8)])


def test_forest_built_with_learned_or_sign_sketches(hf, orc):
    """hf_build_forest with the learned hash or sign sketches gives the same
    forest as building with SRP and switching the sketches afterwards."""
    x, q = datagen.mixture(5000, 384, 16, 0.05, 79, dtype=np.float16, query_seed=80, nq=50)
    L = hf.LHash(*_net(81))
    a = hf.Forest(dev(x), n_trees=3, leaf_max=50, seed=2, sketch_seed=3, sketch="learned", lhash=L)
    b = hf.Forest(dev(x), n_trees=3, leaf_max=50, seed=2, sketch_seed=3)
    b.set_sketch("learned", L)
    assert (a.sketches().cpu().numpy() == b.sketches().cpu().numpy()).all()
    ia, _ = a.search(dev(q), 10, 200, 60, 1)
    ib, _ = b.search(dev(q), 10, 200, 60, 1)
    assert (ia.cpu().numpy() == ib.cpu().numpy()).all()
    c = hf.Forest(dev(x), n_trees=3, leaf_max=50, seed=2, sketch_seed=3, sketch="sign")
    b.set_sketch("sign")
    assert (c.sketches().cpu().numpy() == b.sketches().cpu().numpy()).all()
    for f in (a, b, c):
        f.free()
    L.free()


def test_srp_matrix_core_sketches(hf, orc, monkeypatch):
    """Forest sketches from the int8 matrix-core kernel (d a multiple of 16,
    here with a partial 64-coordinate step and a ragged last block of rows)
    equal the oracle's and the vector-ALU kernel's, bit for bit."""
    for d, dtype in ((80, np.float32), (384, np.float16)):
        x = datagen.mixture(4000 + 37, d, 9, 0.1, 83, unit=False, dtype=dtype)
        F = orc.build_forest(x, T=1, M=50, seed=4, sketch_seed=5)
        a = hf.Forest(dev(x), n_trees=1, leaf_max=50, seed=4, sketch_seed=5)
        got = a.sketches().cpu().numpy().view(np.uint64)
        assert (got == F["sk_pos"]).all(), "d=%d" % d
        monkeypatch.setenv("HF_SRP_VALU", "1")
        a.set_sketch("srp")
        assert (a.sketches().cpu().numpy().view(np.uint64) == got).all(), "d=%d" % d
        monkeypatch.delenv("HF_SRP_VALU")
        a.free()


def test_forest_search_tree_subset(hf, orc):
    """Searching trees 0..n-1 of a larger forest equals the search of a forest
    of those trees (tree t does not depend on how many trees follow it)."""
    x, q = datagen.mixture(20000, 384, 64, 0.05, 57, dtype=np.float16, query_seed=58, nq=100)
    F = orc.build_forest(x, T=8, M=100, seed=15, sketch_seed=16, trees=[0, 1, 2])
    fo = hf.Forest(dev(x), n_trees=8, leaf_max=100, seed=15, sketch_seed=16)
    want = orc.search(F, q, 300, 100, 1, 20)
    r = fo.search_debug(dev(q), 20, 300, 100, 1, trees=3)
    assert (u32(r["winstart"]) == want["winstart"]).all()
    assert (u32(r["c2"]) == want["c2"]).all()
    check_topk(r["ids"].cpu().numpy(), r["scores"].cpu().numpy(), want["ids"], want["scores"], x, q, 20)
    fo.free()


def test_caller_allocator(hf):
    """Per-call scratch through the caller's allocator (hf_set_allocator):
    a counting wrapper of torch's caching allocator (the binding's default)
    and hipMallocAsync (the library's own default) give bit-identical
    results, every block taken is given back, and an allocator that returns
    no memory fails the call with HF_ERR_OOM before any device work (no
    kernel runs on unallocated scratch)."""
    import ctypes
    import torch

    x, q = datagen.mixture(20000, 64, 16, 0.1, 81, dtype=np.float16, query_seed=82, nq=200)
    xd, qd = dev(x), dev(q)
    fo = hf.Forest(xd, n_trees=6, leaf_max=50, seed=3, sketch_seed=4)
    ids0, sc0 = fo.search(qd, 10, 200, 100, 1)
    g0, gs0 = hf.knn_graph(xd, 4, 16, 10, 5)
    torch.cuda.synchronize()
    counts = {"alloc": 0, "free": 0}

    def al(n, c, s):
        counts["alloc"] += 1
        return hf._torch_alloc(n, c, s)

    def fr(p, c, s):
        counts["free"] += 1
        hf._torch_free(p, c, s)

    a = hf.Allocator(hf.ALLOC_FN(al), hf.FREE_FN(fr), None)
    assert hf.lib().hf_set_allocator(ctypes.byref(a)) == 0
    try:
        ids1, sc1 = fo.search(qd, 10, 200, 100, 1)
        g1, gs1 = hf.knn_graph(xd, 4, 16, 10, 5)
        torch.cuda.synchronize()
    finally:
        hf.restore_default_allocator()
    assert counts["alloc"] > 0 and counts["alloc"] == counts["free"], counts
    assert (ids1.cpu().numpy() == ids0.cpu().numpy()).all() and (sc1.cpu().numpy() == sc0.cpu().numpy()).all()
    assert (g1.cpu().numpy() == g0.cpu().numpy()).all() and (gs1.cpu().numpy() == gs0.cpu().numpy()).all()

    bad = hf.Allocator(hf.ALLOC_FN(lambda n, c, s: None), hf.FREE_FN(lambda p, c, s: None), None)
    assert hf.lib().hf_set_allocator(ctypes.byref(bad)) == 0
    try:
        with pytest.raises(hf.HFError) as err:
            fo.search(qd, 10, 200, 100, 1)
        assert err.value.status == 3
    finally:
        hf.restore_default_allocator()
    hf.use_torch_allocator(False)  # hipMallocAsync
    try:
        ids2, sc2 = fo.search(qd, 10, 200, 100, 1)
        torch.cuda.synchronize()
    finally:
        hf.restore_default_allocator()
    assert (ids2.cpu().numpy() == ids0.cpu().numpy()).all()
    fo.free()


def test_forest_duplicates_overflow_selection(hf, orc):
    """All points identical: one oversized leaf, every candidate at Hamming 0,
    more candidates than the selection buffer holds (position-split path)."""
    N = 40000
    x = np.tile(np.array([[0.25, -0.5, 0.125, 0.75, 0.0, -0.25, 0.5, 0.125]], np.float32), (N, 1))
    q = x[:3].copy()
    q[1, 0] = 0.3
    _forest_case(hf, orc, x, q, T=2, M=100, seed=11, sk_seed=12, params=[(20000, 1000, 1, 20)])


# ------------------------------------------------------------------ graph
def _graph_case(hf, orc, x, n, w, k, seed, rows):
    orders, _ = orc.graph_orders(x, n, seed)
    oi, os_, _ = orc.graph_rows(x, orders, w, k, rows)
    gi, gs = hf.knn_graph(dev(x), n, w, k, seed)
    gi = gi.cpu().numpy()[rows]
    gs = gs.cpu().numpy()[rows]
    assert np.abs(gs - os_)[np.isfinite(os_)].max() <= TOL
    assert (np.isfinite(os_) == np.isfinite(gs)).all()
    X = x.astype(np.float64)
    nrm = np.linalg.norm(X, axis=1)
    bad = 0
    for i, p in enumerate(rows):
        if (gi[i] == oi[i]).all():
            continue
        kth = os_[i, k - 1]
        for c in set(gi[i].tolist()) ^ set(oi[i].tolist()):
            if c < 0:
                bad += 1
                continue
            s = X[p] @ X[c] / (nrm[p] * nrm[c])
            if abs(s - kth) > TOL:
                bad += 1
    assert bad == 0


def test_graph_parity_d384(hf, orc):
    x = datagen.mixture(20000, 384, 32, 0.05, 71, dtype=np.float16)
    rows = np.random.default_rng(0).choice(20000, 1500, replace=False)
    _graph_case(hf, orc, x, n=4, w=32, k=15, seed=3, rows=rows)


def test_graph_parity_ragged(hf, orc):
    x = datagen.mixture(333, 40, 4, 0.1, 72, dtype=np.float16)
    _graph_case(hf, orc, x, n=3, w=21, k=7, seed=4, rows=np.arange(333))
    x = datagen.mixture(100, 16, 2, 0.2, 73, dtype=np.float16)
    _graph_case(hf, orc, x, n=2, w=49, k=20, seed=5, rows=np.arange(100))


def test_graph_two_sided_band(hf, orc, monkeypatch):
    """With no room for mailboxes every pair is computed from both of its
    points; the lists equal the oracle's and, bit for bit, those of the form
    that computes each pair once."""
    cases = [(datagen.mixture(333, 40, 4, 0.1, 72, dtype=np.float16), 3, 21, 7, 4),
             (datagen.mixture(2011, 64, 6, 0.1, 74, dtype=np.float16), 3, 150, 12, 6),
             (datagen.mixture(5000, 384, 16, 0.05, 75, dtype=np.float16), 2, 128, 15, 7)]
    once = [hf.knn_graph(dev(x), n, w, k, seed) for x, n, w, k, seed in cases]
    monkeypatch.setenv("HF_GRAPH_MAILBOX_MIB", "0")
    for (x, n, w, k, seed), (gi1, gs1) in zip(cases, once):
        gi2, gs2 = hf.knn_graph(dev(x), n, w, k, seed)
        assert (gi1.cpu().numpy() == gi2.cpu().numpy()).all()
        assert (gs1.cpu().numpy() == gs2.cpu().numpy()).all()
        rows = np.arange(0, x.shape[0], max(1, x.shape[0] // 400))
        _graph_case(hf, orc, x, n=n, w=w, k=k, seed=seed, rows=rows)


def _graph_prefilter_case(hf, orc, x, n, w, k, k2, seed, sk_seed, rows):
    """Sketch stage of Alg. 2: C2 lists bit-exact, results as in the plain form."""
    orders, e = orc.graph_orders(x, n, seed)
    sk = orc.srp(x, e, sk_seed)
    oi, os_, _, oc2 = orc.graph_rows(x, orders, w, k, rows, k2=k2, sk=sk, with_c2=True)
    gi, gs, gc2 = hf.knn_graph_debug(dev(x), n, w, k, seed, k2, sketch_seed=sk_seed)
    assert (gc2.cpu().numpy()[rows] == oc2).all()
    gi2, gs2 = hf.knn_graph(dev(x), n, w, k, seed, k2=k2, sketch_seed=sk_seed)
    assert (gi2.cpu().numpy() == gi.cpu().numpy()).all() and (gs2.cpu().numpy() == gs.cpu().numpy()).all()
    gi, gs = gi.cpu().numpy()[rows], gs.cpu().numpy()[rows]
    fin = np.isfinite(os_)
    assert (np.isfinite(gs) == fin).all() and ((gi == -1) == ~fin).all()
    assert np.abs(gs[fin] - os_[fin]).max() <= TOL
    X = x.astype(np.float64)
    nrm = np.linalg.norm(X, axis=1)
    for i, p in enumerate(rows):
        kth = os_[i][fin[i]][-1]
        for c in set(gi[i].tolist()) ^ set(oi[i].tolist()):
            assert c >= 0
            assert abs(X[p] @ X[c] / (nrm[p] * nrm[c]) - kth) <= TOL


def test_graph_prefilter_parity_d384(hf, orc):
    x = datagen.mixture(20000, 384, 32, 0.05, 74, dtype=np.float16)
    rows = np.random.default_rng(3).choice(20000, 1500, replace=False)
    _graph_prefilter_case(hf, orc, x, n=4, w=32, k=15, k2=50, seed=3, sk_seed=9, rows=rows)


def test_graph_prefilter_wide_window(hf, orc):
    """w = 130: the sketch ring of the band kernel cycles through five blocks."""
    x = datagen.mixture(5000, 64, 8, 0.1, 75, dtype=np.float16)
    _graph_prefilter_case(hf, orc, x, n=2, w=130, k=10, k2=100, seed=4, sk_seed=10, rows=np.arange(0, 5000, 3))


def test_graph_prefilter_ragged(hf, orc):
    # k2 == k; a ragged N and d
    x = datagen.mixture(333, 40, 4, 0.1, 76, dtype=np.float16)
    _graph_prefilter_case(hf, orc, x, n=3, w=21, k=7, k2=7, seed=5, sk_seed=11, rows=np.arange(333))
    # lists never fill (k2 above every union): C2 = C1, padded
    x = datagen.mixture(100, 16, 2, 0.2, 77, dtype=np.float16)
    _graph_prefilter_case(hf, orc, x, n=2, w=49, k=20, k2=256, seed=6, sk_seed=12, rows=np.arange(100))
    # fewer candidates than k: -1 / -inf tails
    x = datagen.mixture(40, 8, 2, 0.2, 78, dtype=np.float16)
    _graph_prefilter_case(hf, orc, x, n=1, w=2, k=6, k2=6, seed=7, sk_seed=13, rows=np.arange(40))


def test_graph_prefilter_chunked_staging(hf, orc, monkeypatch):
    """Positions staged in several chunks per order (1 MiB of staging)."""
    monkeypatch.setenv("HF_GRAPH_STAGE_MIB", "1")
    x = datagen.mixture(9000, 32, 8, 0.1, 79, dtype=np.float16)
    _graph_prefilter_case(hf, orc, x, n=3, w=40, k=10, k2=30, seed=8, sk_seed=14, rows=np.arange(0, 9000, 4))


def test_graph_prefilter_learned_sketch(hf, orc):
    """With learned sketches C2 is the k2 smallest (Hamming, id) of the window
    union under the library's own codes of the points (its encoder is checked
    against the oracle separately), and the result is the cosine top-k of C2."""
    W = _net(97, d=64, hid=256)
    x = datagen.mixture(3000, 64, 8, 0.1, 80, dtype=np.float16)
    L = hf.LHash(*W)
    sk = L.encode(dev(x)).cpu().numpy().view(np.uint64)
    n, w, k, k2 = 3, 24, 8, 30
    gi, gs, gc2 = hf.knn_graph_debug(dev(x), n, w, k, 5, k2, sketch="learned", lhash=L)
    gi, gs, gc2 = gi.cpu().numpy(), gs.cpu().numpy(), gc2.cpu().numpy()
    orders, _ = orc.graph_orders(x, n, 5)
    rank = np.empty((n, x.shape[0]), np.int64)
    for t in range(n):
        rank[t, orders[t]] = np.arange(x.shape[0])
    X = x.astype(np.float64)
    nrm = np.linalg.norm(X, axis=1)
    for p in range(0, x.shape[0], 7):
        C1 = set()
        for t in range(n):
            i = rank[t, p]
            C1 |= set(orders[t][max(0, i - w):i + w + 1].tolist())
        C1.discard(p)
        C1 = np.array(sorted(C1), np.int64)
        hm = np.bitwise_count(sk[C1] ^ sk[p][None, :]).sum(1)
        want = C1[np.lexsort((C1, hm))][:k2]
        assert gc2[p].tolist() == want.tolist()
        cos = X[want] @ X[p] / (nrm[want] * nrm[p])
        assert np.abs(np.sort(cos)[::-1][:k] - gs[p]).max() <= TOL
    L.free()


# ------------------------------------------------------------------ precision form
@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_precision_form_parity(hf, orc, prec):
    x, q = datagen.mixture(20000, 384, 64, 0.05, 81, dtype=np.float16, query_seed=82, nq=120)
    T, M, k1, k2, h, k, S = 4, 100, 300, 100, 2, 30, 120
    F = orc.build_forest(x, T=T, M=M, seed=5, sketch_seed=6)
    base = orc.search(F, q, k1, k2, h, k)
    want = orc.search_lowprec(F, q, base["c2"], base["c2n"], h, k, prec, S)
    fo = hf.Forest(dev(x), n_trees=T, leaf_max=M, seed=5, sketch_seed=6)
    fo.add_precision(prec)
    r = fo.search_lowprec_debug(dev(q), k, k1, k2, h, prec, S)
    gp, gs = u32(r["surv_pos"]), r["surv_score"].cpu().numpy()
    fin = np.isfinite(want["surv_score"])
    assert (np.isfinite(gs) == fin).all()
    # low-precision scores: exact products, FP32 accumulation
    assert np.abs(gs[fin] - want["surv_score"][fin]).max() <= TOL
    # survivor sets agree up to near-ties of the S-th score
    for i in range(q.shape[0]):
        a, b = set(gp[i][gp[i] != 0xFFFFFFFF].tolist()), set(want["surv_pos"][i][fin[i]].tolist())
        if a != b:
            kth = want["surv_score"][i][fin[i]][-1]
            for c in a ^ b:
                j = np.where(want["surv_pos"][i] == c)[0]
                sc = want["surv_score"][i][j[0]] if j.size else gs[i][np.where(gp[i] == c)[0][0]]
                assert abs(sc - kth) <= TOL
    check_topk(r["ids"].cpu().numpy(), r["scores"].cpu().numpy(), want["ids"], want["scores"], x, q, k)
    fo.free()


def test_audit_kernel(hf):
    x, q = datagen.mixture(5000, 384, 8, 0.05, 83, dtype=np.float16, query_seed=84, nq=50)
    ids = np.random.default_rng(1).integers(-1, 5000, (50, 7)).astype(np.int32)
    got = hf.audit_scores(dev(x), dev(q), dev(ids)).cpu().numpy()
    X, Q = x.astype(np.float64), q.astype(np.float64)
    want = np.where(ids >= 0, np.einsum("qd,qkd->qk", Q, X[np.maximum(ids, 0)]), 0.0)
    assert np.abs(got - want).max() <= 1e-12


# ------------------------------------------------------------------ learned hash
def _net(seed, d=384, hid=256):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((hid, d)) * np.sqrt(2.0 / d)).astype(np.float32),
            (0.05 * rng.standard_normal(hid)).astype(np.float32),
            (rng.standard_normal((512, hid)) * np.sqrt(1.0 / hid)).astype(np.float32),
            (0.05 * rng.standard_normal(512)).astype(np.float32)]


@pytest.mark.parametrize("dtype,n", [(np.float16, 3001), (np.float32, 77)])
def test_lhash_encode_parity(hf, orc, dtype, n):
    W = _net(91)
    x = datagen.mixture(n, 384, 8, 0.05, 92, dtype=dtype)
    L = hf.LHash(*W)
    got = L.encode(dev(x)).cpu().numpy().view(np.uint64)
    gbits = np.unpackbits(got.view(np.uint8), axis=1, bitorder="little").astype(bool)
    _, _, z2, band = orc.mlp_forward(x, *W, rounded=True)
    firm = np.abs(z2) > band
    assert firm.mean() > 0.99
    assert (gbits[firm] == (z2[firm] >= 0)).all()
    L.free()


def test_lhash_fused_encoder_matches_two_kernel_path(hf, monkeypatch):
    """The fused two-layer encoder (persistent 128-row blocks) sums in the
    two-kernel path's order, so the sketches agree bit for bit (ragged last
    blocks, both dtypes; more blocks than CUs so the persistent workgroups walk
    several blocks with the prefetch)."""
    L = hf.LHash(*_net(96))
    for dtype, n in ((np.float16, 1000 + 37), (np.float32, 70), (np.float16, 128 * 600 + 5), (np.float32, 128 * 300 + 3)):
        x = dev(datagen.mixture(n, 384, 8, 0.05, 97, dtype=dtype))
        monkeypatch.setenv("HF_MLP", "two")
        want = L.encode(x).cpu().numpy()
        monkeypatch.delenv("HF_MLP")
        assert (L.encode(x).cpu().numpy() == want).all(), (dtype, n)
    L.free()


def test_lhash_gradients_match_oracle(hf, orc):
    W = _net(93)
    rng = np.random.default_rng(94)
    c = datagen.centres(384, 16, 95, True)
    A = datagen.draw(c, 96, 0.05, 96, np.float16)
    B = datagen.draw(c, 96, 0.05, 97, np.float16)
    tp = hf.train_params(slope=2.0, tau=0.2, balance=0.05)
    L = hf.LHash(*W)
    loss, g = L.grad(dev(A), dev(B), tp)
    oloss, og = orc.lhash_grad(A, B, *W, slope=2.0, tau=0.2, lam=0.05, rounded=True)
    assert abs(loss - oloss) <= 1e-4 * max(1.0, abs(oloss))
    # element by element: |g - g_oracle| <= RTOL |g_oracle| + ATOL * max|g_oracle| of the tensor.
    # The GPU sums the 2B rows and the inner products in FP32 (relative error a
    # few 2^-24 times the sum of magnitudes, which cancellation can make large
    # against a small entry), and a hidden activation whose pre-activation lies
    # at a bf16 rounding midpoint may round the other way (one bf16 step,
    # 2^-8 relative, in one of the 2B rows).  Both stay far below ATOL of the
    # tensor's scale; a wrong row or column (a transposed operand, a dropped
    # term) moves entries by their own size.
    RTOL, ATOL = 1e-4, 1e-5
    for name, gg, oo in zip(["W1", "b1", "W2", "b2"], g, og):
        gg = gg.cpu().numpy().astype(np.float64).reshape(oo.shape)
        lim = RTOL * np.abs(oo) + ATOL * np.abs(oo).max()
        worst = np.max(np.abs(gg - oo) / lim)
        print("gradient %s: worst |diff| / bound = %.3g" % (name, worst))
        assert (np.abs(gg - oo) <= lim).all(), (name, worst)
    L.free()


def test_lhash_gradients_with_hard_negatives(hf, orc):
    """The objective with one hard negative per query: loss and every gradient
    entry against the FP64 oracle (same bound as without negatives)."""
    W = _net(95)
    c = datagen.centres(384, 16, 96, True)
    A = datagen.draw(c, 80, 0.05, 97, np.float16)
    B = datagen.draw(c, 80, 0.05, 98, np.float16)
    Nn = datagen.draw(c, 80, 0.05, 99, np.float16)
    tp = hf.train_params(slope=2.0, tau=0.2, balance=0.05)
    L = hf.LHash(*W)
    loss, g = L.grad(dev(A), dev(B), tp, N=dev(Nn))
    oloss, og = orc.lhash_grad(A, B, *W, slope=2.0, tau=0.2, lam=0.05, rounded=True, Neg=Nn)
    assert abs(loss - oloss) <= 1e-4 * max(1.0, abs(oloss))
    RTOL, ATOL = 1e-4, 1e-5
    for name, gg, oo in zip(["W1", "b1", "W2", "b2"], g, og):
        gg = gg.cpu().numpy().astype(np.float64).reshape(oo.shape)
        lim = RTOL * np.abs(oo) + ATOL * np.abs(oo).max()
        print("gradient %s with negatives: worst |diff| / bound = %.3g" % (name, np.max(np.abs(gg - oo) / lim)))
        assert (np.abs(gg - oo) <= lim).all(), name
    L.free()


def test_lhash_training_and_gain_over_srp(hf, orc):
    """Training on (query, true 10-NN) pairs, batches of nearby queries along a
    Hilbert order, lowers the training loss.  On this mixture, whose
    within-cluster structure is isotropic noise, the trained network is
    predicted to stay below SRP in the Hamming recall of the neighbours
    (random hyperplanes already capture what an MLP could, and contrastive
    training pulls cluster mates together, flattening the ranking inside a
    cluster), and the test asserts that sign: SRP stays the sketch in use."""
    import torch

    x, q = datagen.mixture(20000, 384, 32, 0.05, 98, dtype=np.float16, query_seed=99, nq=3000)
    nn, _ = orc.brute_force_ip(x, q, 10)
    tr, te = np.arange(2500), np.arange(2500, 3000)
    e = orc.quant_exp(x)
    qi, pi = hf.hilbert_pairs(hf.quantize(dev(q[tr]), e), nn[tr], 5, 250)
    A, B = q[tr][qi], x[pi]
    L = hf.LHash.init(384, 256, seed=5)

    def hamming_recall(sk_x, sk_q, truth):
        xs = torch.from_numpy(np.unpackbits(sk_x.view(np.uint8), axis=1).astype(np.float32)).cuda()
        qs = torch.from_numpy(np.unpackbits(sk_q.view(np.uint8), axis=1).astype(np.float32)).cuda()
        ham = qs.sum(1, keepdim=True) + xs.sum(1)[None, :] - 2 * qs @ xs.T
        top = torch.topk(-ham, 100, dim=1).indices.cpu().numpy()
        return np.mean([len(set(t) & set(n)) / 10.0 for t, n in zip(top, truth)])

    def learned(rows):
        return hamming_recall(L.encode(dev(x)).cpu().numpy().view(np.uint64),
                              L.encode(dev(q[rows])).cpu().numpy().view(np.uint64), nn[rows])

    fit_before, held_before = learned(tr[:500]), learned(te)
    curve = L.train(dev(A), dev(B), hf.train_params(epochs=4, batch=250, lr=1e-3, tau=0.1, slope=2.0, balance=0.05,
                                                    keep_blocks=True))
    fit_after, held_after = learned(tr[:500]), learned(te)
    srp = hamming_recall(orc.srp(x, e, 3), orc.srp(q[te], e, 3), nn[te])
    print("loss per epoch", curve, "recall@100 of 10-NN: training queries %.3f -> %.3f, held-out %.3f -> %.3f,"
          " SRP held-out %.3f (gain %+.3f)" % (fit_before, fit_after, held_before, held_after, srp, held_after - srp))
    assert curve[-1] < 0.8 * curve[0]
    assert held_after < srp
    L.free()
