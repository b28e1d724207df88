// Hilbert keys computed lazily, 64 bits at a time, one wavefront per point.
//
// The Hilbert index of a point (Skilling's transform on 8-bit coordinates)
// is read level-major: key bit b sits at level 7 - b/d, axis b%d.  The bits
// of one level only need the coordinates after the "inverse undo" sweeps of
// the levels above it, and each such sweep is a left-to-right pass over the
// axes that carries the low bits of axis 0: a set level bit inverts the
// carrier, a clear one swaps it with the axis' low bits.  Those per-axis
// maps (constant or xor) compose associatively, so a wavefront does one
// level as a 64-lane prefix scan: lane l owns G consecutive axes, composes
// them locally, scans across lanes and replays its axes with the incoming
// carrier.  The Gray-code step of the transform becomes a prefix parity over
// the axes of a level (ballot + popcount) XOR the parities of the levels
// above.
//
// For node tests the carrier also tracks where the low bits came from (the
// tree axis and whether they were inverted), which gives the data axis and
// polarity that decide a key bit for every point sharing the key prefix.
#include "hf_internal.h"

namespace hf {
namespace {

// Carrier / label format: bits 0..7 low-bit value, bit 8 inverted, bits 9..21
// origin tree axis.  A map is that plus bit 31 = constant (else xor).
constexpr uint32_t F_CONST = 0x80000000u;
constexpr uint32_t F_XORBITS = 0x1FFu;
constexpr uint32_t F_ORIGIN = 0x1FFFu << 9;

__device__ __forceinline__ uint32_t compose(uint32_t first, uint32_t then) {
  if (then & F_CONST) return then;
  return (first & (F_CONST | F_ORIGIN)) | ((first ^ then) & F_XORBITS);
}

__device__ __forceinline__ uint32_t apply(uint32_t f, uint32_t c) {
  return (f & F_CONST) ? (f & ~F_CONST) : (c ^ (f & F_XORBITS));
}

template <int G>
struct Lane {
  uint8_t x[G];
  uint32_t lab[G];  // bit 8 inverted, bits 9..21 origin; value bits unused
};

template <int G>
__device__ __forceinline__ void load_lane(Lane<G>& s, const uint8_t* __restrict__ row, int dl,
                                          const int32_t* __restrict__ perm,
                                          const uint8_t* __restrict__ refl) {
  int l = __lane_id();
#pragma unroll
  for (int g = 0; g < G; ++g) {
    int i = l * G + g;
    if (i < dl) {
      s.x[g] = (uint8_t)(row[perm[i]] ^ (refl[i] ? 0xFFu : 0u));
      s.lab[g] = (uint32_t)i << 9;
    } else {
      s.x[g] = 0;
      s.lab[g] = 0;
    }
  }
}

// One "inverse undo" sweep at level L >= 1 over axes [0, dl).
template <int G>
__device__ __forceinline__ void undo_level(Lane<G>& s, int L, int dl) {
  const int l = __lane_id();
  const uint32_t P = (1u << L) - 1u;
  uint32_t F = 0;  // identity
#pragma unroll
  for (int g = 0; g < G; ++g) {
    int i = l * G + g;
    if (i < dl) {
      uint32_t fi;
      if ((s.x[g] >> L) & 1u)
        fi = P | 0x100u;
      else if (i == 0)
        fi = 0;
      else
        fi = F_CONST | (s.x[g] & P) | s.lab[g];
      F = compose(F, fi);
    }
  }
  uint32_t inc = F;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_up(inc, off);
    if (l >= off) inc = compose(o, inc);
  }
  uint32_t ex = __shfl_up(inc, 1);
  if (l == 0) ex = 0;
  uint32_t c0 = __shfl((uint32_t)(s.x[0] & P) | s.lab[0], 0);
  uint32_t cd = apply(__shfl(inc, 63), c0);
  uint32_t c = apply(ex, c0);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    int i = l * G + g;
    if (i < dl) {
      if ((s.x[g] >> L) & 1u) {
        c ^= P | 0x100u;
      } else if (i != 0) {
        uint32_t nc = (uint32_t)(s.x[g] & P) | s.lab[g];
        s.x[g] = (uint8_t)((s.x[g] & ~P) | (c & P));
        s.lab[g] = c & ~0xFFu;
        c = nc;
      }
    }
  }
  if (l == 0) {
    s.x[0] = (uint8_t)((s.x[0] & ~P) | (cd & P));
    s.lab[0] = cd & ~0xFFu;
  }
}

// Gray-coded bits of level L: key bit of axis i = prefix parity ^ tau.
// Returns per-axis bits in `kb`, and the level's total parity.
template <int G>
__device__ __forceinline__ uint32_t level_bits(const Lane<G>& s, int L, int dl, uint32_t tau,
                                               uint32_t* kb) {
  const int l = __lane_id();
  uint32_t pre = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    int i = l * G + g;
    uint32_t b = (i < dl) ? ((s.x[g] >> L) & 1u) : 0u;
    pre ^= b;
    kb[g] = pre;
  }
  uint64_t m = __ballot(pre);
  uint32_t ex = (uint32_t)__popcll(m & lanemask_lt()) & 1u;
  uint32_t tot = (uint32_t)__popcll(m) & 1u;
#pragma unroll
  for (int g = 0; g < G; ++g) kb[g] ^= ex ^ tau;
  return tot;
}

template <int G>
__global__ __launch_bounds__(256) void chunk_kernel(const uint8_t* __restrict__ codes, int d,
                                                    const int32_t* __restrict__ perm,
                                                    const uint8_t* __restrict__ refl,
                                                    const uint32_t* __restrict__ items,
                                                    int64_t n, int chunk,
                                                    uint64_t* __restrict__ out) {
  int64_t it = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (it >= n) return;
  const int l = __lane_id();
  uint32_t p = items ? items[it] : (uint32_t)it;
  const int64_t b0 = (int64_t)chunk * 64;
  const int li_lo = (int)(b0 / d);
  int li_hi = (int)((b0 + 63) / d);
  if (li_hi > 7) li_hi = 7;
  const int dl = (li_hi == 0) ? (int)min<int64_t>(d, b0 + 64) : d;
  Lane<G> s;
  load_lane<G>(s, codes + (int64_t)p * d, dl, perm, refl);
  uint32_t tau = 0;
  uint64_t part = 0;
  for (int li = 0; li <= li_hi; ++li) {
    int L = 7 - li;
    uint32_t kb[G];
    uint32_t tot = level_bits<G>(s, L, dl, tau, kb);
    if (li >= li_lo) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        int i = l * G + g;
        int64_t b = (int64_t)li * d + i;
        if (i < dl && b >= b0 && b < b0 + 64 && kb[g]) part |= 1ull << (63 - (b - b0));
      }
    }
    tau ^= tot;
    if (li < li_hi) undo_level<G>(s, L, dl);
  }
  part = wave_or_u64(part);
  if (l == 0) out[it] = part;
}

template <int G>
__global__ __launch_bounds__(256) void node_test_kernel(const uint8_t* __restrict__ codes, int d,
                                                        const int32_t* __restrict__ perm,
                                                        const uint8_t* __restrict__ refl,
                                                        const uint32_t* __restrict__ points,
                                                        const uint32_t* __restrict__ bits,
                                                        int64_t n, uint32_t* __restrict__ out) {
  int64_t it = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (it >= n) return;
  const int l = __lane_id();
  uint32_t p = points[it], b = bits[it];
  int li = (int)(b / (uint32_t)d), j = (int)(b % (uint32_t)d), L = 7 - li;
  const uint8_t* row = codes + (int64_t)p * d;
  Lane<G> s;
  load_lane<G>(s, row, d, perm, refl);
  uint32_t tau = 0;
  for (int lv = 0; lv < li; ++lv) {
    uint32_t kb[G];
    tau ^= level_bits<G>(s, 7 - lv, d, tau, kb);
    undo_level<G>(s, 7 - lv, d);
  }
  uint32_t kb[G];
  level_bits<G>(s, L, d, tau, kb);
  int owner = j / G, gj = j % G;
  uint32_t mybit = 0, mylab = 0;
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (g == gj) {
      mybit = kb[g];
      mylab = s.lab[g];
    }
  uint32_t keybit = __shfl(mybit, owner);
  uint32_t lab = __shfl(mylab, owner);
  if (l == 0) {
    uint32_t origin = (lab >> 9) & 0x1FFFu;
    uint32_t a = (uint32_t)perm[origin];
    uint32_t flip = keybit ^ ((row[a] >> L) & 1u);
    out[it] = a | ((uint32_t)L << 16) | (flip << 19);
  }
}

// Top bit of every code, 32 axes per word (bit i%32 of word i/32).
__global__ void k_msb_plane(const uint8_t* __restrict__ codes, int64_t N, int d, int nw,
                            uint32_t* __restrict__ msb) {
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < N * nw;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t p = idx / nw;
    const int w = (int)(idx - p * nw);
    const uint8_t* row = codes + p * d;
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) {
      const int i = 32 * w + b;
      if (i < d) v |= (uint32_t)(row[i] >> 7) << b;
    }
    msb[idx] = v;
  }
}

// Chunks that lie inside the top level need no undo sweep: key bit j is the
// parity of the (reflected) top bits of tree axes 0..j.  One thread per point,
// the point's top bits in registers, tree axes read as uniform indices.
template <int NW>
__global__ __launch_bounds__(256) void chunk_top_kernel(const uint32_t* __restrict__ msb,
                                                        const int32_t* __restrict__ perm,
                                                        const uint8_t* __restrict__ refl,
                                                        const uint32_t* __restrict__ items,
                                                        int64_t n, int chunk,
                                                        uint64_t* __restrict__ out) {
  const int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (it >= n) return;
  const uint32_t p = items ? items[it] : (uint32_t)it;
  uint32_t m[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) m[w] = msb[(int64_t)p * NW + w];
  uint32_t run = 0;
  uint64_t key = 0;
  const int i0 = 64 * chunk;
  for (int i = 0; i < i0; ++i) {
    const int a = perm[i];
    run ^= ((m[a >> 5] >> (a & 31)) & 1u) ^ (uint32_t)refl[i];
  }
#pragma unroll 8
  for (int j = 0; j < 64; ++j) {
    const int a = perm[i0 + j];
    run ^= ((m[a >> 5] >> (a & 31)) & 1u) ^ (uint32_t)refl[i0 + j];
    key |= (uint64_t)run << (63 - j);
  }
  out[it] = key;
}

// Exact position of a (query, tree) pair with full keys: a wavefront per
// pair, every lane walking the same path; two keys are compared level by
// level (the undo sweep of each level done as in chunk_kernel for both
// points), the first differing key bit found by a ballot.
// A data point's codes are recomputed from its stored row (the quantiser
// is exact).
template <int G>
__device__ __forceinline__ void load_lane_x(Lane<G>& s, const void* X, hf_dtype dt, int64_t row, int d, int e,
                                            const int32_t* __restrict__ perm, const uint8_t* __restrict__ refl) {
  const int l = __lane_id();
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int i = l * G + g;
    if (i < d) {
      const int64_t at = row * d + perm[i];
      const float v = dt == HF_F16 ? __half2float(((const __half*)X)[at]) : ((const float*)X)[at];
      float f = floorf(ldexpf(v, e)) + 128.0f;
      f = f < 0.0f ? 0.0f : (f > 255.0f ? 255.0f : f);
      s.x[g] = (uint8_t)((uint32_t)f ^ (refl[i] ? 0xFFu : 0u));
      s.lab[g] = (uint32_t)i << 9;
    } else {
      s.x[g] = 0;
      s.lab[g] = 0;
    }
  }
}

// Sign of key(a) - key(b); *jstar = the first differing key bit (INT32_MAX
// when equal).  Both lanes' states are consumed.
template <int G>
__device__ __forceinline__ int cmp_full(Lane<G>& a, Lane<G>& b, int d, int* jstar) {
  const int l = __lane_id();
  uint32_t ta = 0, tb = 0;
  for (int li = 0; li < 8; ++li) {
    const int L = 7 - li;
    uint32_t ka[G], kb[G];
    const uint32_t sa = level_bits<G>(a, L, d, ta, ka);
    const uint32_t sb = level_bits<G>(b, L, d, tb, kb);
    int first = G;
    uint32_t bit = 0;
#pragma unroll
    for (int g = G - 1; g >= 0; --g)
      if (l * G + g < d && ka[g] != kb[g]) {
        first = g;
        bit = ka[g];
      }
    const uint64_t m = __ballot(first < G);
    if (m) {
      const int owner = __ffsll((unsigned long long)m) - 1;
      const int g0 = __shfl(first, owner);
      const uint32_t qb = (uint32_t)__shfl((int)bit, owner);
      *jstar = li * d + owner * G + g0;
      return qb ? 1 : -1;
    }
    ta ^= sa;
    tb ^= sb;
    if (li < 7) {
      undo_level<G>(a, L, d);
      undo_level<G>(b, L, d);
    }
  }
  *jstar = 0x7FFFFFFF;
  return 0;
}

template <int G>
__global__ __launch_bounds__(256) void k_rank_deep(const uint64_t* __restrict__ deep, const uint32_t* __restrict__ ndeep,
                                                   const uint32_t* __restrict__ nodes,
                                                   const uint32_t* __restrict__ aux,
                                                   const int64_t* __restrict__ node_off,
                                                   const uint8_t* __restrict__ qcodes, const void* X, hf_dtype dt,
                                                   int e, const uint32_t* __restrict__ tree_perm,
                                                   const int32_t* __restrict__ cperm,
                                                   const uint8_t* __restrict__ crefl, int d, int T, int64_t N,
                                                   int k1, int max_steps, uint32_t* __restrict__ win) {
  const uint32_t n = *ndeep;
  const uint32_t stride = gridDim.x * 4;
  for (uint32_t it = blockIdx.x * 4 + threadIdx.x / 64; it < n; it += stride) {
    const uint64_t v = deep[it];
    const int64_t q = (int64_t)(v >> 32);
    const int t = (int)(uint32_t)v;
    const int32_t* pt = cperm + (int64_t)t * d;
    const uint8_t* rt = crefl + (int64_t)t * d;
    const uint32_t* nd = nodes + 2 * node_off[t];
    const uint32_t* au = aux + 2 * node_off[t];
    const uint32_t* tp = tree_perm + (int64_t)t * N;
    const uint8_t* u = qcodes + q * d;
    auto test = [&](uint32_t w1) -> uint32_t {
      const uint32_t a = w1 & 0xFFFFu, L = (w1 >> 16) & 7u, flip = (w1 >> 19) & 1u;
      return ((u[a] >> L) & 1u) ^ flip;
    };
    auto cmp = [&](uint32_t p, int* js) -> int {
      Lane<G> a, b;
      load_lane<G>(a, u, d, pt, rt);
      load_lane_x<G>(b, X, dt, (int64_t)p, d, e, pt, rt);
      return cmp_full<G>(a, b, d, js);
    };
    uint32_t idx = 0, leaf_lo = 0;
    for (int step = 0; step < max_steps; ++step) {
      const uint2 r = *(const uint2*)(nd + 2 * (int64_t)idx);
      if (r.y >> 31) {
        leaf_lo = r.x;
        break;
      }
      idx = test(r.y) ? r.x : idx + 1u;
    }
    int jstar;
    const int c = cmp(tp[leaf_lo], &jstar);
    int64_t lo = 0, hi = N, rank = -1;
    idx = 0;
    for (int step = 0; step < max_steps; ++step) {
      const uint2 r = *(const uint2*)(nd + 2 * (int64_t)idx);
      if (r.y >> 31) break;
      const uint2 sb = *(const uint2*)(au + 2 * (int64_t)idx);
      if ((int64_t)sb.y > (int64_t)jstar && c != 0) {
        rank = c > 0 ? hi : lo;
        break;
      }
      if (test(r.y)) {
        lo = sb.x;
        idx = r.x;
      } else {
        hi = sb.x;
        idx = idx + 1u;
      }
    }
    if (rank < 0) {
      int64_t a = lo, b = hi;
      while (a < b) {
        const int64_t mid = (a + b) >> 1;
        int j2;
        if (cmp(tp[mid], &j2) > 0)
          a = mid + 1;
        else
          b = mid;
      }
      rank = a;
    }
    int64_t s = rank - k1 / 2, smax = N - k1 > 0 ? N - k1 : 0;
    s = s < 0 ? 0 : (s > smax ? smax : s);
    if (__lane_id() == 0) win[q * T + t] = (uint32_t)s;
  }
}

int pick_g(int d) {
  int g = (d + 63) / 64;
  int G = 1;
  while (G < g) G <<= 1;
  return G;
}

}  // namespace

#define HF_DISPATCH_G(G, KERNEL, ...)                                                \
  switch (G) {                                                                       \
    case 1: KERNEL<1><<<grid, 256, 0, s>>>(__VA_ARGS__); break;                      \
    case 2: KERNEL<2><<<grid, 256, 0, s>>>(__VA_ARGS__); break;                      \
    case 4: KERNEL<4><<<grid, 256, 0, s>>>(__VA_ARGS__); break;                      \
    case 8: KERNEL<8><<<grid, 256, 0, s>>>(__VA_ARGS__); break;                      \
    case 16: KERNEL<16><<<grid, 256, 0, s>>>(__VA_ARGS__); break;                    \
    case 32: KERNEL<32><<<grid, 256, 0, s>>>(__VA_ARGS__); break;                    \
    default: KERNEL<64><<<grid, 256, 0, s>>>(__VA_ARGS__); break;                    \
  }

int msb_words(int d) {
  const int nw = (d + 31) / 32;
  return nw <= 1 ? 1 : nw <= 2 ? 2 : nw <= 4 ? 4 : nw <= 8 ? 8 : nw <= 12 ? 12 : nw <= 16 ? 16 : 0;
}

hf_status msb_plane(const uint8_t* codes, int64_t N, int d, uint32_t* msb, hipStream_t s) {
  const int nw = msb_words(d);
  if (nw == 0 || N <= 0) return HF_OK;
  k_msb_plane<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, ceil_div(N * nw, 256))), 256, 0, s>>>(
      codes, N, d, nw, msb);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

hf_status key_chunks(const uint8_t* codes, const uint32_t* msb, int d, const int32_t* perm,
                     const uint8_t* refl, const uint32_t* items, int64_t n_items, int chunk,
                     uint64_t* out, hipStream_t s) {
  if (n_items <= 0) return HF_OK;
  const int nw = msb_words(d);
  if (msb && nw > 0 && (int64_t)chunk * 64 + 64 <= d) {
    dim3 grid((unsigned)ceil_div(n_items, 256));
    switch (nw) {
#define HF_NW(n) \
  case n: chunk_top_kernel<n><<<grid, 256, 0, s>>>(msb, perm, refl, items, n_items, chunk, out); break;
      HF_NW(1) HF_NW(2) HF_NW(4) HF_NW(8) HF_NW(12) HF_NW(16)
#undef HF_NW
    }
    HF_LAUNCH_CHECK();
    return HF_OK;
  }
  dim3 grid((unsigned)ceil_div(n_items, 4));
  int G = pick_g(d);
  HF_DISPATCH_G(G, chunk_kernel, codes, d, perm, refl, items, n_items, chunk, out);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

hf_status rank_deep(const hf_forest* f, const uint8_t* qcodes, int64_t nq, int T, int k1, const uint64_t* deep,
                    const uint32_t* ndeep, uint32_t* win, hipStream_t s) {
  (void)nq;
  const int d = f->d;
  dim3 grid(1024);
  int G = pick_g(d);
  HF_DISPATCH_G(G, k_rank_deep, deep, ndeep, f->nodes, f->node_aux, f->node_off_dev, qcodes, f->X_pos, f->dtype,
                f->e, f->tree_perm, f->curve_perm, f->curve_refl, d, T, f->N, k1, 8 * d + 2, win);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

hf_status node_tests(const uint8_t* codes, int d, const int32_t* perm, const uint8_t* refl,
                     const uint32_t* points, const uint32_t* bits, int64_t n, uint32_t* out_w1,
                     hipStream_t s) {
  if (n <= 0) return HF_OK;
  dim3 grid((unsigned)ceil_div(n, 4));
  int G = pick_g(d);
  HF_DISPATCH_G(G, node_test_kernel, codes, d, perm, refl, points, bits, n, out_w1);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

}  // namespace hf
