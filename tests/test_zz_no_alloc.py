"""hf_search_noalloc (no device allocation, scratch in the library's fixed
per-device array) against hf_search, through the C ABI.  Both run the same
kernels on the same inputs, so ids and scores must agree bit for bit; the
second call of each pair is smaller than the first, so stale contents of the
shared array would show."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hf():
    import torch

    import paper_2508_21682_amd as hf

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    hf.lib()
    return hf


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _same(hf, fo, q, args):
    import torch

    a_ids, a_sc = fo.search(q, *args)
    b_ids, b_sc = fo.search_noalloc(q, *args)
    torch.cuda.synchronize()
    assert torch.equal(a_ids, b_ids)
    assert torch.equal(a_sc.view(torch.int32), b_sc.view(torch.int32))


def test_noalloc_matches_search_two_calls(hf):
    x, q = datagen.mixture(20000, 384, 64, 0.05, 301, dtype=np.float16, query_seed=302, nq=300)
    fo = hf.Forest(_dev(x), n_trees=4, leaf_max=100, seed=5, sketch_seed=6)
    qd = _dev(q)
    args = (10, 300, 100, 1)
    _same(hf, fo, qd, args)
    _same(hf, fo, qd[:37].contiguous(), args)
    fo.free()


def test_noalloc_chunks_queries(hf):
    """64 trees x windows of 2,000: about 0.27 MB of scratch a query, so 600
    queries run as three chunks of the fixed array."""
    x, q = datagen.mixture(20000, 384, 64, 0.05, 303, dtype=np.float16, query_seed=304, nq=600)
    fo = hf.Forest(_dev(x), n_trees=64, leaf_max=100, seed=7, sketch_seed=8)
    qd = _dev(q)
    args = (30, 2000, 400, 2)
    _same(hf, fo, qd, args)
    _same(hf, fo, qd[:250].contiguous(), args)
    fo.free()


def test_noalloc_learned_sketch(hf):
    W = [np.random.default_rng(s).standard_normal(sh).astype(np.float32) * sc
         for s, sh, sc in [(1, (256, 384), 0.07), (2, (256,), 0.05), (3, (512, 256), 0.06), (4, (512,), 0.05)]]
    x, q = datagen.mixture(20000, 384, 64, 0.05, 305, dtype=np.float16, query_seed=306, nq=200)
    fo = hf.Forest(_dev(x), n_trees=4, leaf_max=100, seed=9, sketch_seed=10)
    L = hf.LHash(*W)
    fo.set_sketch("learned", L)
    qd = _dev(q)
    _same(hf, fo, qd, (10, 300, 100, 0))
    _same(hf, fo, qd[:20].contiguous(), (10, 300, 100, 0))
    fo.free()
    L.free()


def test_noalloc_rejects_what_does_not_fit(hf):
    """One query of 1,700 trees x windows of 20,000 needs 68 MB of distances:
    more than the array holds, refused before any launch."""
    x, q = datagen.mixture(20000, 32, 16, 0.1, 307, unit=False, dtype=np.float32, query_seed=308, nq=4)
    fo = hf.Forest(_dev(x), n_trees=1700, leaf_max=100, seed=11, sketch_seed=12)
    with pytest.raises(hf.HFError) as ei:
        fo.search_noalloc(_dev(q), 10, 20000, 100, 0)
    assert ei.value.status == 6 and "scratch" in str(ei.value)
    fo.free()
