"""Checks at the benchmark's full sizes, in the configuration bench.py times.

The oracle cannot rebuild 1,280 trees over 23M points inside a test, so the
23M x 384 search is checked on sampled outputs the oracle computes one by one
and on properties that hold at any size:

* the code exponent, sampled sketches (oracle SRP of the data rows) bit-exact;
* sampled adjacent tree positions in (Skilling key, id) order, keys computed
  by the oracle from the data rows;
* sampled data points descend to the leaf that holds them;
* for sampled queries: each tree's window start is the one the descent of the
  oracle's query codes gives; C2 is exactly the k2 smallest (Hamming, position)
  pairs of the union of the windows, with query sketches from the oracle;
  |E| is the size of the +-h expansion of C2; the returned ids are the top-k
  of E by FP64 inner product (near-ties of the k-th score aside).

The 1M x 384 plain graph (16 orders, window +-32) is small enough for the
oracle to sort in full: its sampled rows are compared exactly.  The 3M x 384
graph in the benchmark's configuration (228 orders, +-160, k=15) is checked
on sampled rows: cosines equal FP64 recomputations, sorted, distinct
neighbours other than the row itself.
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


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _rows(x, ids):
    import torch

    return x[torch.from_numpy(np.asarray(ids, np.int64)).to(x.device)].cpu().numpy()


def _descend(nodes, u):
    """Leaf (lo, size) reached by codes u through pre-order trie records."""
    idx = 0
    while not nodes[idx, 1] >> 31:
        w1 = int(nodes[idx, 1])
        bit = ((int(u[w1 & 0xFFFF]) >> ((w1 >> 16) & 7)) & 1) ^ ((w1 >> 19) & 1)
        idx = int(nodes[idx, 0]) if bit else idx + 1
    return int(nodes[idx, 0]), int(nodes[idx, 1] & 0x7FFFFFFF)


def test_search_23M_sampled(hf, orc):
    import torch

    w = datagen.WORKLOADS["search-23Mx384"]
    N, d = w["n"], w["d"]
    T, M, k, k1, k2, h = 1280, 100, 30, 70, 1000, 0
    print("drawing %d x %d" % (N, d), flush=True)
    x = datagen.mixture_device(N, d, w["n_comp"], w["sigma"], w["seed"], w["unit"])
    q = datagen.mixture_device(2000, d, w["n_comp"], w["sigma"], w["seed"], w["unit"],
                               draw_seed=w["query_seed"])
    print("building %d trees" % T, flush=True)
    fo = hf.Forest(x, n_trees=T, leaf_max=M, seed=5, sketch_seed=6)
    rng = np.random.default_rng(0)
    e = orc.quant_exp(np.array([x.min().item(), x.max().item()], np.float32))
    assert fo.info["quant_exp"] == e
    pos2id = _u32(fo.pos2id())
    assert np.bincount(pos2id, minlength=N).max() == 1
    sk_all = fo.sketches()
    pos = rng.choice(N, 3000, replace=False)
    assert (sk_all[torch.from_numpy(pos).cuda()].cpu().numpy().view(np.uint64)
            == orc.srp(_rows(x, pos2id[pos]), e, 6)).all()

    print("key order and self descent", flush=True)
    perm, refl = orc.curves(5, T, d)
    for t in [0, 1, 640, 1279]:
        tp = _u32(fo.perm(t))
        i = rng.choice(N - 1, 300, replace=False)
        a, b = pos2id[tp[i]], pos2id[tp[i + 1]]
        ka = orc.tree_keys(orc.quantize(_rows(x, a), e), perm[t], refl[t])
        kb = orc.tree_keys(orc.quantize(_rows(x, b), e), perm[t], refl[t])
        for j in range(len(i)):
            ta, tb = tuple(ka[j].tolist()), tuple(kb[j].tolist())
            assert ta < tb or (ta == tb and a[j] < b[j]), (t, int(i[j]))
        nodes = _u32(fo.nodes(t)).reshape(-1, 2)
        rank = np.empty(N, np.int64)
        rank[tp] = np.arange(N)
        p = rng.choice(N, 200, replace=False)
        codes = orc.quantize(_rows(x, pos2id[p]), e)
        for j in range(len(p)):
            lo, size = _descend(nodes, codes[j])
            assert 1 <= size and lo <= rank[p[j]] < lo + size, (t, int(p[j]))

    print("search", flush=True)
    r = fo.search_debug(q, k, k1, k2, h)
    ids2, sc2 = fo.search(q, k, k1, k2, h)
    assert (ids2.cpu().numpy() == r["ids"].cpu().numpy()).all()
    assert (sc2.cpu().numpy() == r["scores"].cpu().numpy()).all()
    qs = rng.choice(q.shape[0], 12, replace=False)
    Q = q.cpu().numpy()[qs]
    qcodes = orc.quantize(Q, e)
    qsk = orc.srp(Q, e, 6)
    win = _u32(r["winstart"])[qs]
    c2, c2n, en = _u32(r["c2"])[qs], r["c2n"].cpu().numpy()[qs], r["en"].cpu().numpy()[qs]
    ids, sc = r["ids"].cpu().numpy()[qs], r["scores"].cpu().numpy()[qs]
    c1 = [[] for _ in qs]
    for t in range(T):
        tp = fo.perm(t)
        s = torch.from_numpy(win[:, t].astype(np.int64))[:, None] + torch.arange(k1)[None, :]
        got = tp[s.cuda()].cpu().numpy().view(np.uint32)
        if t % 160 == 0:
            nodes = _u32(fo.nodes(t)).reshape(-1, 2)
            for j in range(len(qs)):
                lo, size = _descend(nodes, qcodes[j])
                want = min(max(lo + size // 2 - k1 // 2, 0), max(N - k1, 0))
                assert win[j, t] == want, (t, j)
        for j in range(len(qs)):
            c1[j].append(got[j])
    for j in range(len(qs)):
        C1 = np.unique(np.concatenate(c1[j])).astype(np.int64)
        ham = np.bitwise_count(sk_all[torch.from_numpy(C1).cuda()].cpu().numpy().view(np.uint64)
                               ^ qsk[j][None, :]).sum(1)
        order = np.lexsort((C1, ham))
        assert c2n[j] == min(k2, C1.size)
        assert set(c2[j, :c2n[j]].tolist()) == set(C1[order[:c2n[j]]].tolist()), j
        E = np.unique((c2[j, :c2n[j]].astype(np.int64)[:, None] + np.arange(-h, h + 1)[None, :]).ravel())
        E = E[(E >= 0) & (E < N)]
        assert en[j] == E.size
        s = _rows(x, pos2id[E]).astype(np.float64) @ Q[j].astype(np.float64)
        top = np.argsort(-s, kind="stable")[:k]
        want_ids, want_sc = pos2id[E][top], s[top]
        assert np.abs(sc[j] - want_sc).max() <= TOL
        kth = want_sc[-1]
        for c in set(ids[j].tolist()) ^ set(want_ids.tolist()):
            sc_c = _rows(x, [c])[0].astype(np.float64) @ Q[j].astype(np.float64)
            assert abs(sc_c - kth) <= TOL, (j, c)
    fo.free()


def test_graph_1M_against_oracle(hf, orc):
    """The 1M x 384 plain graph (16 orders, window +-32, k=15), 1,000 sampled rows exact."""
    import torch

    w = datagen.WORKLOADS["graph-1Mx384"]
    print("drawing 1M x 384 on the host", flush=True)
    x = datagen.mixture(w["n"], w["d"], w["n_comp"], w["sigma"], w["seed"], dtype=np.float16)
    gi, gs = hf.knn_graph(torch.from_numpy(x).cuda(), 16, 32, 15, 3)
    print("oracle orders", flush=True)
    orders, _ = orc.graph_orders(x, 16, 3)
    rows = np.random.default_rng(1).choice(w["n"], 1000, replace=False)
    oi, os_, _ = orc.graph_rows(x, orders, 32, 15, rows)
    gi, gs = gi.cpu().numpy()[rows], gs.cpu().numpy()[rows]
    assert np.abs(gs - os_).max() <= TOL
    X = x.astype(np.float64)
    nrm = np.linalg.norm(X, axis=1)
    for r, p in enumerate(rows):
        kth = os_[r, -1]
        for c in set(gi[r].tolist()) ^ set(oi[r].tolist()):
            s = X[p] @ X[c] / (nrm[p] * nrm[c])
            assert abs(s - kth) <= TOL, (int(p), c)


def test_graph_3M_bench_config_sampled(hf):
    w = datagen.WORKLOADS["graph-3Mx384"]
    print("drawing 3M x 384", flush=True)
    x = datagen.mixture_device(w["n"], w["d"], w["n_comp"], w["sigma"], w["seed"], w["unit"])
    gi, gs = hf.knn_graph(x, 228, 160, 15, 3)
    rows = np.random.default_rng(2).choice(w["n"], 2000, replace=False)
    gi, gs = gi.cpu().numpy()[rows], gs.cpu().numpy()[rows]
    X = _rows(x, rows).astype(np.float64)
    for r, p in enumerate(rows):
        assert len(set(gi[r].tolist())) == 15 and p not in gi[r] and gi[r].min() >= 0
        Y = _rows(x, gi[r]).astype(np.float64)
        cos = Y @ X[r] / (np.linalg.norm(Y, axis=1) * np.linalg.norm(X[r]))
        assert np.abs(cos - gs[r]).max() <= TOL
        assert (np.diff(gs[r]) <= 0).all()
