// Leaf-compressed Hilbert tree (Section 2 "Hilbert tree"; Section 3.1: subtrees
// of about M points become leaves), built as a binary trie over the sorted
// Hilbert keys.
//
// For sorted keys the first bit where the two ends of a range differ is the
// smallest split bit of the adjacent pairs inside it, and the pair holding it
// is where that bit turns from 0 to 1.  So every node is a range-minimum
// query over the split bits the sort recorded.  The tree is built top-down,
// one level per launch (a wavefront per node, with a two-level table of block
// minima so a query touches at most ~3000 entries), then laid out in
// pre-order (left subtree first) from subtree sizes.  Node tests come from
// the lazy key machinery: for the first point of a node's range, which data
// axis and polarity decide the split bit.
#include "hf_internal.h"

namespace hf {
namespace {

constexpr int BLK = 256;

__device__ __forceinline__ uint64_t pack(uint32_t b, int64_t g) {
  return ((uint64_t)b << 32) | (uint64_t)(uint32_t)g;
}

__global__ __launch_bounds__(256) void k_block_min0(const uint32_t* __restrict__ split,
                                                    int64_t ngaps, int64_t nblk,
                                                    uint64_t* __restrict__ bm1) {
  int64_t k = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (k >= nblk) return;
  uint64_t best = ~0ull;
  for (int64_t g = k * BLK + __lane_id(); g < (k + 1) * BLK && g < ngaps; g += 64)
    best = min(best, pack(split[g], g));
  best = wave_min_u64(best);
  if (__lane_id() == 0) bm1[k] = best;
}

__global__ __launch_bounds__(256) void k_block_min1(const uint64_t* __restrict__ in, int64_t nin,
                                                    int64_t nout, uint64_t* __restrict__ out) {
  int64_t k = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (k >= nout) return;
  uint64_t best = ~0ull;
  for (int64_t g = k * BLK + __lane_id(); g < (k + 1) * BLK && g < nin; g += 64)
    best = min(best, in[g]);
  best = wave_min_u64(best);
  if (__lane_id() == 0) out[k] = best;
}

__device__ uint64_t range_min(const uint32_t* __restrict__ split, const uint64_t* __restrict__ bm1,
                              const uint64_t* __restrict__ bm2, int64_t s, int64_t e) {
  const int l = __lane_id();
  uint64_t best = ~0ull;
  if (e - s <= 4 * BLK) {
    for (int64_t g = s + l; g < e; g += 64) best = min(best, pack(split[g], g));
  } else {
    int64_t s1 = (s + BLK - 1) / BLK, e1 = e / BLK;
    for (int64_t g = s + l; g < s1 * BLK; g += 64) best = min(best, pack(split[g], g));
    for (int64_t g = e1 * BLK + l; g < e; g += 64) best = min(best, pack(split[g], g));
    if (e1 - s1 <= 4 * BLK) {
      for (int64_t k = s1 + l; k < e1; k += 64) best = min(best, bm1[k]);
    } else {
      int64_t s2 = (s1 + BLK - 1) / BLK, e2 = e1 / BLK;
      for (int64_t k = s1 + l; k < s2 * BLK; k += 64) best = min(best, bm1[k]);
      for (int64_t k = e2 * BLK + l; k < e1; k += 64) best = min(best, bm1[k]);
      for (int64_t k = s2 + l; k < e2; k += 64) best = min(best, bm2[k]);
    }
  }
  return wave_min_u64(best);
}

// Classify the nodes of one level: leaf (split = NONE) or internal with split
// bit b at position m; internal[i] = 1 for the child-offset scan.
__global__ __launch_bounds__(256) void k_classify(const uint32_t* __restrict__ lo,
                                                  const uint32_t* __restrict__ hi, int64_t n,
                                                  int M, const uint32_t* __restrict__ split,
                                                  const uint64_t* __restrict__ bm1,
                                                  const uint64_t* __restrict__ bm2,
                                                  uint32_t* __restrict__ bsplit,
                                                  uint32_t* __restrict__ mpos,
                                                  uint32_t* __restrict__ internal) {
  int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (i >= n) return;
  uint32_t a = lo[i], z = hi[i];
  uint32_t b = NONE32, m = 0;
  if (z - a > (uint32_t)M) {
    uint64_t r = range_min(split, bm1, bm2, a, (int64_t)z - 1);
    if ((uint32_t)(r >> 32) != NONE32) {
      b = (uint32_t)(r >> 32);
      m = (uint32_t)r + 1u;
    }
  }
  if (__lane_id() == 0) {
    bsplit[i] = b;
    mpos[i] = m;
    internal[i] = b != NONE32 ? 1u : 0u;
  }
}

__global__ void k_children(const uint32_t* __restrict__ lo, const uint32_t* __restrict__ hi,
                           const uint32_t* __restrict__ bsplit, const uint32_t* __restrict__ mpos,
                           const uint32_t* __restrict__ cidx, int64_t n, uint32_t* __restrict__ nlo,
                           uint32_t* __restrict__ nhi, const uint32_t* __restrict__ order,
                           uint32_t* __restrict__ tpt) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    tpt[i] = order[lo[i]];
    if (bsplit[i] != NONE32) {
      uint32_t c = 2u * cidx[i];
      nlo[c] = lo[i];
      nhi[c] = mpos[i];
      nlo[c + 1] = mpos[i];
      nhi[c + 1] = hi[i];
    }
  }
}

__global__ void k_sizes(const uint32_t* __restrict__ bsplit, const uint32_t* __restrict__ cidx,
                        const uint32_t* __restrict__ csize, int64_t n, uint32_t* __restrict__ size) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (bsplit[i] == NONE32) {
      size[i] = 1u;
    } else {
      uint32_t c = 2u * cidx[i];
      size[i] = 1u + csize[c] + csize[c + 1];
    }
  }
}

// Pre-order indices of the children, and the records of this level.
// aux (2 words per node): internal {split position m, split bit b}, leaf
// {lo, NONE}.
__global__ void k_emit(const uint32_t* __restrict__ lo, const uint32_t* __restrict__ hi,
                       const uint32_t* __restrict__ bsplit, const uint32_t* __restrict__ mpos,
                       const uint32_t* __restrict__ cidx,
                       const uint32_t* __restrict__ w1, const uint32_t* __restrict__ idx,
                       const uint32_t* __restrict__ csize, int64_t n, uint32_t* __restrict__ cix,
                       uint32_t* __restrict__ out, uint32_t* __restrict__ aux) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint32_t me = idx[i];
    aux[2 * (int64_t)me] = bsplit[i] == NONE32 ? lo[i] : mpos[i];
    aux[2 * (int64_t)me + 1] = bsplit[i];
    if (bsplit[i] == NONE32) {
      out[2 * (int64_t)me] = lo[i];
      out[2 * (int64_t)me + 1] = 0x80000000u | (hi[i] - lo[i]);
    } else {
      uint32_t c = 2u * cidx[i];
      uint32_t left = me + 1u, right = me + 1u + csize[c];
      cix[c] = left;
      cix[c + 1] = right;
      out[2 * (int64_t)me] = right;
      out[2 * (int64_t)me + 1] = w1[i];
    }
  }
}

__global__ void k_bits_or_zero(const uint32_t* __restrict__ b, int64_t n, uint32_t* __restrict__ o) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    o[i] = b[i] == NONE32 ? 0u : b[i];
}

inline unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, ceil_div(n, 256)));
}

struct Level {
  int64_t n;
  uint32_t *lo, *hi, *b, *m, *internal, *cidx, *w1, *pt, *size, *idx;
};

}  // namespace

hf_status build_trie(const uint8_t* codes, int64_t N, int d, int M, const int32_t* perm,
                     const uint8_t* refl, const uint32_t* order, const uint32_t* split,
                     uint32_t** nodes_out, uint32_t** aux_out, int64_t* n_nodes, Workspace& ws) {
  hipStream_t s = ws.stream;
  int64_t ngaps = N - 1;
  int64_t nb1 = std::max<int64_t>(1, ceil_div(ngaps, BLK));
  int64_t nb2 = std::max<int64_t>(1, ceil_div(nb1, BLK));
  uint64_t *bm1, *bm2;
  HF_TRY(ws.alloc(&bm1, nb1));
  HF_TRY(ws.alloc(&bm2, nb2));
  if (ngaps > 0) {
    k_block_min0<<<(unsigned)ceil_div(nb1, 4), 256, 0, s>>>(split, ngaps, nb1, bm1);
    k_block_min1<<<(unsigned)ceil_div(nb2, 4), 256, 0, s>>>(bm1, nb1, nb2, bm2);
    HF_LAUNCH_CHECK();
  }
  uint32_t* tot;
  HF_TRY(ws.alloc(&tot, 1));
  std::vector<Level> lv;
  {
    Level L0{};
    L0.n = 1;
    HF_TRY(ws.alloc(&L0.lo, 1));
    HF_TRY(ws.alloc(&L0.hi, 1));
    uint32_t init[2] = {0u, (uint32_t)N};
    HIP_TRY(hipMemcpyAsync(L0.lo, &init[0], 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(L0.hi, &init[1], 4, hipMemcpyHostToDevice, s));
    lv.push_back(L0);
  }
  // top-down: classify each level, place the children of internal nodes
  for (size_t li = 0; li < lv.size(); ++li) {
    if (li > (size_t)(8 * d + 2)) {
      set_error("trie deeper than the key length (internal error)");
      return HF_ERR_DEVICE;
    }
    Level& L = lv[li];
    HF_TRY(ws.alloc(&L.b, L.n));
    HF_TRY(ws.alloc(&L.m, L.n));
    HF_TRY(ws.alloc(&L.internal, L.n));
    HF_TRY(ws.alloc(&L.cidx, L.n));
    HF_TRY(ws.alloc(&L.pt, L.n));
    k_classify<<<(unsigned)ceil_div(L.n, 4), 256, 0, s>>>(L.lo, L.hi, L.n, M, split, bm1, bm2, L.b,
                                                           L.m, L.internal);
    HF_LAUNCH_CHECK();
    HF_TRY(excl_scan_u32(L.internal, L.cidx, L.n, tot, ws));
    uint32_t h_int = 0;
    HIP_TRY(hipMemcpyAsync(&h_int, tot, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    Level C{};
    C.n = 2 * (int64_t)h_int;
    uint32_t *nlo = nullptr, *nhi = nullptr;
    if (C.n > 0) {
      HF_TRY(ws.alloc(&nlo, C.n));
      HF_TRY(ws.alloc(&nhi, C.n));
    }
    k_children<<<grid_for(L.n), 256, 0, s>>>(L.lo, L.hi, L.b, L.m, L.cidx, L.n, nlo, nhi, order,
                                             L.pt);
    HF_LAUNCH_CHECK();
    // node tests of this level (computed for every node; leaves ignore theirs)
    HF_TRY(ws.alloc(&L.w1, L.n));
    {
      uint32_t* bits;
      HF_TRY(ws.alloc(&bits, L.n));
      // leaves carry NONE as split: test bit 0 instead (result unused)
      k_bits_or_zero<<<grid_for(L.n), 256, 0, s>>>(L.b, L.n, bits);
      HF_LAUNCH_CHECK();
      HF_TRY(node_tests(codes, d, perm, refl, L.pt, bits, L.n, L.w1, s));
    }
    if (C.n > 0) {
      C.lo = nlo;
      C.hi = nhi;
      lv.push_back(C);
    }
  }
  // bottom-up subtree sizes
  for (size_t li = lv.size(); li-- > 0;) {
    Level& L = lv[li];
    HF_TRY(ws.alloc(&L.size, L.n));
    const uint32_t* csize = (li + 1 < lv.size()) ? lv[li + 1].size : nullptr;
    k_sizes<<<grid_for(L.n), 256, 0, s>>>(L.b, L.cidx, csize, L.n, L.size);
    HF_LAUNCH_CHECK();
  }
  uint32_t total = 0;
  HIP_TRY(hipMemcpyAsync(&total, lv[0].size, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  uint32_t *out, *aux;
  HIP_TRY(hipMalloc(&out, sizeof(uint32_t) * 2 * (size_t)total));
  if (hipMalloc(&aux, sizeof(uint32_t) * 2 * (size_t)total) != hipSuccess) {
    (void)hipFree(out);
    set_error("device allocation of %zu bytes of split records failed", sizeof(uint32_t) * 2 * (size_t)total);
    return HF_ERR_OOM;
  }
  // top-down pre-order indices and records
  HF_TRY(ws.alloc(&lv[0].idx, 1));
  HIP_TRY(hipMemsetAsync(lv[0].idx, 0, 4, s));
  for (size_t li = 0; li < lv.size(); ++li) {
    Level& L = lv[li];
    uint32_t* cix = nullptr;
    const uint32_t* csize = nullptr;
    if (li + 1 < lv.size()) {
      HF_TRY(ws.alloc(&lv[li + 1].idx, lv[li + 1].n));
      cix = lv[li + 1].idx;
      csize = lv[li + 1].size;
    }
    k_emit<<<grid_for(L.n), 256, 0, s>>>(L.lo, L.hi, L.b, L.m, L.cidx, L.w1, L.idx, csize, L.n, cix,
                                         out, aux);
    HF_LAUNCH_CHECK();
  }
  *nodes_out = out;
  *aux_out = aux;
  *n_nodes = total;
  return HF_OK;
}

}  // namespace hf
