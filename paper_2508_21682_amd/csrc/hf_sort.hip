// Hilbert sort of N points along one curve (Section 2), exact on full keys.
//
// Round 0 computes the first 64-bit chunk of every key and radix-sorts
// (chunk, id) stably.  Points whose chunks tie form segments; round c
// computes chunk c for the tied points only and sorts them by (segment,
// chunk) with the same stable radix sort, which refines every segment in
// place.  Rounds stop when no ties remain, when the remaining ties are
// points with identical codes (equal keys at every depth) or when the key is
// exhausted.  Equal keys stay in id order because every pass is stable.
// While refining, the first differing key bit of every adjacent pair is
// recorded: it is the split bit the trie needs.
#include "hf_internal.h"

namespace hf {
namespace {

__global__ void k_iota(uint32_t* a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    a[i] = (uint32_t)i;
}

__global__ void k_fill(uint32_t* a, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    a[i] = v;
}

__global__ void k_gather_pts(const uint32_t* __restrict__ A, const uint32_t* __restrict__ order,
                             int64_t n, uint32_t* __restrict__ pts) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
    pts[j] = order[A[j]];
}

__global__ void k_init_kv(const uint64_t* __restrict__ kc, int64_t n, uint64_t* __restrict__ keys,
                          uint32_t* __restrict__ vals) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    keys[j] = kc[j];
    vals[j] = (uint32_t)j;
  }
}

__global__ void k_seg_keys(const uint32_t* __restrict__ seg, const uint32_t* __restrict__ vals,
                           int64_t n, uint64_t* __restrict__ keys) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
    keys[j] = seg[vals[j]];
}

__global__ void k_apply(const uint32_t* __restrict__ o, const uint32_t* __restrict__ pts,
                        const uint64_t* __restrict__ kc, const uint32_t* __restrict__ seg,
                        const uint32_t* __restrict__ A, int64_t n, uint32_t* __restrict__ order,
                        uint32_t* __restrict__ npts, uint64_t* __restrict__ nkc,
                        uint32_t* __restrict__ nseg) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    uint32_t s = o[j];
    uint32_t p = pts[s];
    npts[j] = p;
    nkc[j] = kc[s];
    nseg[j] = seg[s];
    order[A[j]] = p;
  }
}

// Round 0: every point is active, in id order, in one segment (A and pts
// are the identity, seg is 0), so the sorted chunks and ids are the new
// state as they stand.
__global__ void k_apply0(const uint32_t* __restrict__ o, const uint64_t* __restrict__ skeys, int64_t n,
                         uint32_t* __restrict__ order, uint32_t* __restrict__ npts,
                         uint64_t* __restrict__ nkc, uint32_t* __restrict__ nseg) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    const uint32_t s = o[j];
    order[j] = s;
    npts[j] = s;
    nkc[j] = skeys[j];
    nseg[j] = 0;
  }
}

// tied[j] for the pair (j, j+1): 0 = split (or different segments),
// 1 = equal chunk, different codes, 2 = equal chunk, identical codes.
__global__ void k_ties(const uint32_t* __restrict__ npts, const uint64_t* __restrict__ nkc,
                       const uint32_t* __restrict__ nseg, const uint32_t* __restrict__ A, int64_t n,
                       int chunk, const uint8_t* __restrict__ codes, int d,
                       uint32_t* __restrict__ split, uint32_t* __restrict__ tied) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    uint32_t t = 0;
    if (j + 1 < n && nseg[j] == nseg[j + 1]) {
      uint64_t x = nkc[j] ^ nkc[j + 1];
      if (x) {
        split[A[j]] = (uint32_t)chunk * 64u + (uint32_t)__clzll((long long)x);
      } else {
        const uint8_t* a = codes + (int64_t)npts[j] * d;
        const uint8_t* b = codes + (int64_t)npts[j + 1] * d;
        int i = 0;
        while (i < d && a[i] == b[i]) ++i;
        t = (i == d) ? 2u : 1u;
      }
    }
    tied[j] = t;
  }
}

__global__ void k_heads(const uint32_t* __restrict__ tied, int64_t n, uint32_t* __restrict__ head) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
    head[j] = (j == 0 || tied[j - 1] == 0) ? 1u : 0u;
}

// segrank = inclusive scan of heads - 1; mark segments holding a pair that
// still differs somewhere deeper.
__global__ void k_segrank(const uint32_t* __restrict__ head, const uint32_t* __restrict__ excl,
                          const uint32_t* __restrict__ tied, int64_t n, uint32_t* __restrict__ srank,
                          uint32_t* __restrict__ nonident) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    uint32_t r = excl[j] + head[j] - 1u;
    srank[j] = r;
    if (tied[j] == 1u) nonident[r] = 1u;
  }
}

__global__ void k_active(const uint32_t* __restrict__ tied, const uint32_t* __restrict__ srank,
                         const uint32_t* __restrict__ nonident, int64_t n,
                         uint32_t* __restrict__ active) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    bool t = tied[j] != 0u || (j > 0 && tied[j - 1] != 0u);
    active[j] = (t && nonident[srank[j]]) ? 1u : 0u;
  }
}

__global__ void k_compact(const uint32_t* __restrict__ active, const uint32_t* __restrict__ pos,
                          const uint32_t* __restrict__ A, const uint32_t* __restrict__ srank,
                          int64_t n, uint32_t* __restrict__ A2, uint32_t* __restrict__ seg2) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
    if (active[j]) {
      A2[pos[j]] = A[j];
      seg2[pos[j]] = srank[j];
    }
}

inline unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, ceil_div(n, 256)));
}

}  // namespace

hf_status hilbert_sort_dev(const uint8_t* codes, const uint32_t* msb, int64_t N, int d,
                           const int32_t* perm, const uint8_t* refl, uint32_t* order, uint32_t* split,
                           Workspace& ws) {
  hipStream_t s = ws.stream;
  const int W = (int)ceil_div((int64_t)d * 8, 64);
  uint32_t *A, *A2, *seg, *seg2, *pts, *npts, *nseg, *vals, *avals, *tied, *head, *excl, *srank,
      *nonident, *active, *pos, *tot;
  uint64_t *kc, *nkc, *keys, *akeys;
  HF_TRY(ws.alloc(&A, N));
  HF_TRY(ws.alloc(&A2, N));
  HF_TRY(ws.alloc(&seg, N));
  HF_TRY(ws.alloc(&seg2, N));
  HF_TRY(ws.alloc(&pts, N));
  HF_TRY(ws.alloc(&npts, N));
  HF_TRY(ws.alloc(&nseg, N));
  HF_TRY(ws.alloc(&vals, N));
  HF_TRY(ws.alloc(&avals, N));
  HF_TRY(ws.alloc(&tied, N));
  HF_TRY(ws.alloc(&head, N));
  HF_TRY(ws.alloc(&excl, N));
  HF_TRY(ws.alloc(&srank, N));
  HF_TRY(ws.alloc(&nonident, N));
  HF_TRY(ws.alloc(&active, N));
  HF_TRY(ws.alloc(&pos, N));
  HF_TRY(ws.alloc(&tot, 2));
  HF_TRY(ws.alloc(&kc, N));
  HF_TRY(ws.alloc(&nkc, N));
  HF_TRY(ws.alloc(&keys, N));
  HF_TRY(ws.alloc(&akeys, N));

  k_iota<<<grid_for(N), 256, 0, s>>>(order, N);
  k_iota<<<grid_for(N), 256, 0, s>>>(A, N);
  k_fill<<<grid_for(N), 256, 0, s>>>(seg, N, 0u);
  if (split && N > 1) k_fill<<<grid_for(N - 1), 256, 0, s>>>(split, N - 1, NONE32);
  HF_LAUNCH_CHECK();
  uint32_t* scratch_split = split;
  if (!scratch_split) HF_TRY(ws.alloc(&scratch_split, N));

  int64_t na = N;
  int segbits = 0;
  for (int c = 0; c < W && na > 1; ++c) {
    k_gather_pts<<<grid_for(na), 256, 0, s>>>(A, order, na, pts);
    HF_LAUNCH_CHECK();
    HF_TRY(key_chunks(codes, msb, d, perm, refl, pts, na, c, kc, s));
    k_init_kv<<<grid_for(na), 256, 0, s>>>(kc, na, keys, vals);
    HF_LAUNCH_CHECK();
    uint64_t *k1 = keys, *k2 = akeys;
    uint32_t *v1 = vals, *v2 = avals;
    HF_TRY(radix_sort_pairs(&k1, &v1, &k2, &v2, na, 0, 64, ws));
    if (segbits > 0) {
      k_seg_keys<<<grid_for(na), 256, 0, s>>>(seg, v1, na, k1);
      HF_LAUNCH_CHECK();
      HF_TRY(radix_sort_pairs(&k1, &v1, &k2, &v2, na, 0, (segbits + 7) / 8 * 8, ws));
    }
    if (c == 0)
      k_apply0<<<grid_for(na), 256, 0, s>>>(v1, k1, na, order, npts, nkc, nseg);
    else
      k_apply<<<grid_for(na), 256, 0, s>>>(v1, pts, kc, seg, A, na, order, npts, nkc, nseg);
    k_ties<<<grid_for(na), 256, 0, s>>>(npts, nkc, nseg, A, na, c, codes, d, scratch_split, tied);
    k_heads<<<grid_for(na), 256, 0, s>>>(tied, na, head);
    HF_LAUNCH_CHECK();
    HF_TRY(excl_scan_u32(head, excl, na, tot, ws));
    HIP_TRY(hipMemsetAsync(nonident, 0, sizeof(uint32_t) * na, s));
    k_segrank<<<grid_for(na), 256, 0, s>>>(head, excl, tied, na, srank, nonident);
    k_active<<<grid_for(na), 256, 0, s>>>(tied, srank, nonident, na, active);
    HF_LAUNCH_CHECK();
    HF_TRY(excl_scan_u32(active, pos, na, tot + 1, ws));
    k_compact<<<grid_for(na), 256, 0, s>>>(active, pos, A, srank, na, A2, seg2);
    HF_LAUNCH_CHECK();
    uint32_t h_tot[2];
    HIP_TRY(hipMemcpyAsync(h_tot, tot, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    na = h_tot[1];
    segbits = bits_for(h_tot[0] > 0 ? h_tot[0] - 1 : 0);
    std::swap(A, A2);
    std::swap(seg, seg2);
  }
  return HF_OK;
}

}  // namespace hf
