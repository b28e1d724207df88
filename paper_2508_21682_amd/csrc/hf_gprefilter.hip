// Sketch prefilter of the k-NN graph (Algorithm 2, second-stage filtering).
//
// Every point p keeps a list of the k2 smallest keys (Hamming(sk_p, sk_c) << 32
// | c) over the distinct candidates c seen so far, sorted ascending, in HBM
// (N x k2 u64, empty slots all-ones).  Per Hilbert order:
//
//  k_hband   one lane per position i of the order (a wavefront owns 64
//            consecutive positions).  The sketches of positions i-w..i+w
//            stream through a two-block LDS ring (64 rows per block), each
//            lane XOR-popcounts them against its own sketch and keeps the
//            keys below its point's current k2-th key in a staging area.
//  k_hmerge  16 lanes per point merge the staged keys into the point's list:
//            keys already present are dropped (a key fixes its candidate), the
//            rest are ranked against the list and the list is rewritten in
//            place, truncated to k2.  A candidate evicted earlier is above
//            the k2-th key for good, so the list is always the k2 smallest
//            keys of the union of all windows seen (C2 of the paper).
//
// After the last order, k_hfinal scores each point's list by FP32 cosine and
// returns the top-k by (cosine desc, id asc).
#include <math.h>

#include "hf_internal.h"
#include "hf_select.h"

namespace hf {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));

constexpr int HB_RS = 20;          // LDS row stride in words: 64-byte sketch + 16-byte pad
constexpr uint64_t EMPTY = ~0ull;  // empty list slot

__global__ void k_fill_u64(uint64_t* __restrict__ a, int64_t n, uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a[i] = v;
}

__global__ void k_list_ids(const uint64_t* __restrict__ lists, int64_t n, int32_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint64_t v = lists[i];
    out[i] = v == EMPTY ? -1 : (int32_t)(uint32_t)v;
  }
}

// Positions [p0, p0 + np) of one order.  stage is column-major: entry j of
// position p0 + q at stage[j * np + q], j < 2w.
__global__ __launch_bounds__(256) void k_hband(const uint64_t* __restrict__ sk,
                                               const uint32_t* __restrict__ order, int64_t N, int w,
                                               int k2, const uint64_t* __restrict__ lists, int64_t p0,
                                               int64_t np, uint64_t* __restrict__ stage,
                                               uint32_t* __restrict__ cnt) {
  __shared__ uint32_t ring[4][128 * HB_RS];
  __shared__ uint32_t rid[4][128];
  const int wv = threadIdx.x / 64, l = __lane_id();
  const int64_t i0 = p0 + ((int64_t)blockIdx.x * 4 + wv) * 64;
  const int64_t pend = p0 + np;  // <= N
  if (i0 >= pend) return;  // waves are independent: no block barriers below
  const int64_t i = i0 + l;
  const bool own = i < pend;
  uint32_t s[16];
  uint64_t thr = 0;  // nothing passes for a lane without a position
  if (own) {
    const uint32_t id = order[i];
    const uint4* src = (const uint4*)(sk + (int64_t)id * 8);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint4 t = src[v];
      s[4 * v] = t.x;
      s[4 * v + 1] = t.y;
      s[4 * v + 2] = t.z;
      s[4 * v + 3] = t.w;
    }
    thr = lists[(int64_t)id * k2 + (k2 - 1)];
  }
  uint32_t* R = ring[wv];
  uint32_t* RI = rid[wv];
  // block b holds positions i0 - w + 64b .. +63 in ring slot b & 1
  auto load_block = [&](int b) {
    const int64_t r = i0 - w + 64 * (int64_t)b + l;
    uint32_t* dst = R + ((b & 1) * 64 + l) * HB_RS;
    uint4 t0 = make_uint4(0, 0, 0, 0), t1 = t0, t2 = t0, t3 = t0;
    uint32_t cid = 0xFFFFFFFFu;
    if (r >= 0 && r < N) {
      cid = order[r];
      const uint4* src = (const uint4*)(sk + (int64_t)cid * 8);
      t0 = src[0];
      t1 = src[1];
      t2 = src[2];
      t3 = src[3];
    }
    ((uint4*)dst)[0] = t0;
    ((uint4*)dst)[1] = t1;
    ((uint4*)dst)[2] = t2;
    ((uint4*)dst)[3] = t3;
    RI[(b & 1) * 64 + l] = cid;
  };
  load_block(0);
  load_block(1);
  wave_lds_sync();
  uint32_t c = 0;
  const int64_t q = i - p0;
  for (int jj = 0; jj <= 2 * w; ++jj) {
    if (jj > 0 && (jj & 63) == 0) {
      // every lane is past block (jj >> 6) - 1: its slot takes block (jj >> 6) + 1
      wave_lds_sync();
      load_block((jj >> 6) + 1);
      wave_lds_sync();
    }
    const int r = jj + l;
    const int slot = ((r >> 6) & 1) * 64 + (r & 63);
    const uint4* row = (const uint4*)(R + slot * HB_RS);
    uint32_t h = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint4 t = row[v];
      h += __popc(t.x ^ s[4 * v]) + __popc(t.y ^ s[4 * v + 1]) + __popc(t.z ^ s[4 * v + 2]) +
           __popc(t.w ^ s[4 * v + 3]);
    }
    const int64_t pos = i0 - w + jj + l;
    const uint64_t key = ((uint64_t)h << 32) | RI[slot];
    if (own && jj != w && pos >= 0 && pos < N && key < thr) {
      stage[(int64_t)c * np + q] = key;
      ++c;
    }
  }
  if (own) cnt[q] = c;
}

__device__ __forceinline__ int lower_bound_u64(const uint64_t* a, int n, uint64_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int group16_sum(int v) {
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m);
  return v;
}

// 16 lanes per position; a block covers 16 positions.
__global__ __launch_bounds__(256) void k_hmerge(const uint32_t* __restrict__ order, int64_t p0, int64_t np,
                                                int k2, const uint64_t* __restrict__ stage,
                                                const uint32_t* __restrict__ cnt,
                                                uint64_t* __restrict__ lists) {
  __shared__ uint64_t sL[16][GRAPH_K2_MAX];
  __shared__ uint64_t sB[16][64];
  const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15;
  const int64_t q = (int64_t)blockIdx.x * 16 + grp;
  const uint32_t c = q < np ? cnt[q] : 0u;
  uint32_t cmax = c;
  cmax = max(cmax, (uint32_t)__shfl_xor((int)cmax, 16));
  cmax = max(cmax, (uint32_t)__shfl_xor((int)cmax, 32));
  if (cmax == 0) return;  // the wave's four positions took nothing
  uint64_t* sl = sL[grp];
  uint64_t* sb = sB[grp];
  uint64_t* Lg = nullptr;
  int nL = 0;
  if (c > 0) {
    Lg = lists + (int64_t)order[p0 + q] * k2;
    for (int i = gl; i < k2; i += 16) {
      const uint64_t v = Lg[i];
      sl[i] = v;
      nL += v != EMPTY;
    }
  }
  nL = group16_sum(nL);
  wave_lds_sync();
  constexpr int LPL = GRAPH_K2_MAX / 16;  // list entries per lane
  for (uint32_t base = 0; base < cmax; base += 64) {
    const int cc = c > base ? (int)min(64u, c - base) : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = gl + 16 * j;
      if (t < cc) sb[t] = stage[(int64_t)(base + t) * np + q];
    }
    wave_lds_sync();
    uint64_t bv[4];
    int bl[4];
    int nnew = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = gl + 16 * j;
      bv[j] = EMPTY;
      bl[j] = 0;
      if (t < cc) {
        const uint64_t b = sb[t];
        const int p = lower_bound_u64(sl, nL, b);
        if (!(p < nL && sl[p] == b)) {
          bv[j] = b;
          bl[j] = p;
          ++nnew;
        }
      }
    }
    wave_lds_sync();
    // drop keys already listed: EMPTY sorts after every key
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = gl + 16 * j;
      if (t < cc && bv[j] == EMPTY) sb[t] = EMPTY;
    }
    wave_lds_sync();
    uint64_t lv[LPL];
    int lessL[LPL], lessB[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < LPL; ++j) {
      const int i = gl + 16 * j;
      lv[j] = i < nL ? sl[i] : EMPTY;
      lessL[j] = 0;
    }
    for (int u = 0; u < cc; ++u) {
      const uint64_t v = sb[u];
#pragma unroll
      for (int j = 0; j < 4; ++j) lessB[j] += v < bv[j];
#pragma unroll
      for (int j = 0; j < LPL; ++j) lessL[j] += v < lv[j];
    }
    nnew = group16_sum(nnew);
    wave_lds_sync();  // every read of sl precedes the rewrite
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (bv[j] == EMPTY) continue;
      const int r = bl[j] + lessB[j];
      if (r < k2) {
        sl[r] = bv[j];
        Lg[r] = bv[j];
      }
    }
#pragma unroll
    for (int j = 0; j < LPL; ++j) {
      const int i = gl + 16 * j;
      if (i >= nL) continue;
      const int r = i + lessL[j];
      if (r != i && r < k2) {
        sl[r] = lv[j];
        Lg[r] = lv[j];
      }
    }
    nL = min(k2, nL + nnew);
    wave_lds_sync();
  }
}

__device__ __forceinline__ void wave_bitonic_u64(uint64_t* a, int n2) {
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = __lane_id(); i < n2; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t x = a[i], y = a[ixj];
          if ((x > y) == ((i & k) == 0)) {
            a[i] = y;
            a[ixj] = x;
          }
        }
      }
      wave_lds_sync();
    }
}

// One wavefront per point: FP32 cosines of its listed candidates (16 lanes
// per candidate), then the top-k by (cosine desc, id asc).
__global__ __launch_bounds__(256) void k_hfinal(const __half* __restrict__ X, const float* __restrict__ nrm,
                                                int64_t N, int d, const uint64_t* __restrict__ lists,
                                                int k2, int k, int32_t* __restrict__ ids,
                                                float* __restrict__ sc) {
  __shared__ uint64_t key[4][GRAPH_K2_MAX];
  const int wv = threadIdx.x / 64, l = __lane_id();
  const int64_t p = (int64_t)blockIdx.x * 4 + wv;
  if (p >= N) return;
  const int g = l >> 4, gl = l & 15;
  const uint64_t* Lp = lists + p * k2;
  int nv = 0;
  for (int i = l; i < k2; i += 64) nv += Lp[i] != EMPTY;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) nv += __shfl_xor(nv, m);
  const __half* xp = X + p * d;
  const float np_ = nrm[p];
  uint64_t* K = key[wv];
  for (int c0 = 0; c0 < nv; c0 += 4) {
    const int ci = c0 + g;
    const bool ok = ci < nv;
    const uint32_t cid = ok ? (uint32_t)Lp[ci] : 0u;
    float acc = 0.f;
    if (ok) {
      const __half* xc = X + (int64_t)cid * d;
      for (int k0 = 8 * gl; k0 < d; k0 += 128) {
        const half8 a = __builtin_bit_cast(half8, *(const uint4*)(xp + k0));
        const half8 b = __builtin_bit_cast(half8, *(const uint4*)(xc + k0));
#pragma unroll
        for (int e = 0; e < 8; ++e) acc = fmaf((float)a[e], (float)b[e], acc);
      }
    }
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) acc += __shfl_xor(acc, m);
    if (ok && gl == 0) {
      const float cs = acc / (np_ * nrm[cid]);
      K[ci] = ((uint64_t)(~float_to_ordered(cs)) << 32) | cid;
    }
  }
  int n2 = 1;
  while (n2 < nv) n2 <<= 1;
  for (int i = nv + l; i < n2; i += 64) K[i] = EMPTY;
  wave_lds_sync();
  wave_bitonic_u64(K, n2);
  for (int r = l; r < k; r += 64) {
    if (r < nv) {
      const uint64_t v = K[r];
      ids[p * k + r] = (int32_t)(uint32_t)v;
      sc[p * k + r] = ordered_to_float(~(uint32_t)(v >> 32));
    } else {
      ids[p * k + r] = -1;
      sc[p * k + r] = -INFINITY;
    }
  }
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, ceil_div(n, 256)));
}

}  // namespace

hf_status gpf_init_lists(uint64_t* lists, int64_t n, hipStream_t s) {
  k_fill_u64<<<grid_for(n), 256, 0, s>>>(lists, n, EMPTY);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

hf_status gpf_order(const uint64_t* sk, const uint32_t* order, int64_t N, int w, int k2, uint64_t* lists,
                    int64_t chunk, uint64_t* stage, uint32_t* cnt, hipStream_t s) {
  for (int64_t p0 = 0; p0 < N; p0 += chunk) {
    const int64_t np = std::min(chunk, N - p0);
    {
      StageTimer tm(ST_GHAM, s);
      k_hband<<<(unsigned)ceil_div(np, 256), 256, 0, s>>>(sk, order, N, w, k2, lists, p0, np, stage, cnt);
      HF_LAUNCH_CHECK();
    }
    StageTimer tm(ST_GMERGE, s);
    k_hmerge<<<(unsigned)ceil_div(np, 16), 256, 0, s>>>(order, p0, np, k2, stage, cnt, lists);
    HF_LAUNCH_CHECK();
  }
  return HF_OK;
}

hf_status gpf_final(const void* X, const float* nrm, int64_t N, int d, const uint64_t* lists, int k2, int k,
                    int32_t* ids, float* sc, int32_t* c2_ids, hipStream_t s) {
  StageTimer tm(ST_GFINAL, s);
  k_hfinal<<<(unsigned)ceil_div(N, 4), 256, 0, s>>>((const __half*)X, nrm, N, d, lists, k2, k, ids, sc);
  HF_LAUNCH_CHECK();
  if (c2_ids) {
    k_list_ids<<<grid_for(N * k2), 256, 0, s>>>(lists, N * k2, c2_ids);
    HF_LAUNCH_CHECK();
  }
  return HF_OK;
}

}  // namespace hf
