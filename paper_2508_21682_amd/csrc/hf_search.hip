// Search path of Algorithm 1 on the GPU:
//   descend   - every (query, tree) pair walks its tree: the whole batch
//               located along every curve at once (first stage);
//   ham       - streams each query's n*k1 window entries (duplicates
//               included, as the paper counts them), gathers 64-byte
//               sketches 16 bytes per lane and writes Hamming distances plus
//               a per-query histogram;
//   select    - the k2 smallest distinct (Hamming, master position) pairs:
//               histogram -> largest bin range that fits in LDS -> collect,
//               bitonic sort, drop duplicates; repeats on the next range
//               (splitting a bin by position when it alone overflows);
//   rerank    - C2 sorted by position, expanded by +-h into merged
//               intervals (the expansion set E in increasing master order),
//               FP32 inner products by 16-lane groups, radix select of the
//               k best (score desc, position asc) and a final small sort.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "hf_internal.h"
#include "hf_select.h"

namespace hf {
namespace {

// ------------------------------------------------------------------ descend
__global__ __launch_bounds__(256) void k_descend(const uint32_t* __restrict__ nodes,
                                                 const int64_t* __restrict__ node_off,
                                                 const uint8_t* __restrict__ qcodes, int64_t nq,
                                                 int d, int T, int64_t N, int k1, int max_steps,
                                                 uint32_t* __restrict__ win) {
  int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int t = blockIdx.y;
  if (q >= nq) return;
  const uint32_t* nd = nodes + 2 * node_off[t];
  const uint8_t* u = qcodes + q * d;
  uint32_t idx = 0;
  int64_t mid = 0;
  for (int step = 0; step < max_steps; ++step) {
    uint2 r = *(const uint2*)(nd + 2 * (int64_t)idx);
    if (r.y >> 31) {
      mid = (int64_t)r.x + (int64_t)((r.y & 0x7FFFFFFFu) >> 1);
      break;
    }
    uint32_t a = r.y & 0xFFFFu, L = (r.y >> 16) & 7u, flip = (r.y >> 19) & 1u;
    uint32_t bit = ((u[a] >> L) & 1u) ^ flip;
    idx = bit ? r.x : idx + 1u;
  }
  int64_t s = mid - k1 / 2, smax = N - k1 > 0 ? N - k1 : 0;
  s = s < 0 ? 0 : (s > smax ? smax : s);
  win[q * T + t] = (uint32_t)s;
}

// The same walk with the codes of the block's 64 queries staged in LDS: a
// wavefront per tree, a lane per query, so each level waits for one global
// load (the node) instead of two (the node, then the code byte it tests).
// WPB wavefronts (trees) share one copy of the codes.  Rows of d bytes, d a
// multiple of 16 and at most DS_MAXD.
constexpr int DS_Q = 64, DS_MAXD = 512;
template <int WPB>
__global__ __launch_bounds__(64 * WPB) void k_descend_lds(const uint32_t* __restrict__ nodes,
                                                          const int64_t* __restrict__ node_off,
                                                          const uint8_t* __restrict__ qcodes, int64_t nq,
                                                          int d, int T, int64_t N, int k1, int max_steps,
                                                          uint32_t* __restrict__ win) {
  extern __shared__ __align__(16) uint8_t sc[];  // DS_Q x d code bytes (dynamic LDS)
  const int64_t q0 = (int64_t)blockIdx.x * DS_Q;
  const int nqb = (int)min<int64_t>(DS_Q, nq - q0);
  const int c16 = d / 16;
  for (int i = threadIdx.x; i < nqb * c16; i += 64 * WPB)
    ((uint4*)sc)[i] = ((const uint4*)(qcodes + q0 * d))[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.y * WPB + (threadIdx.x >> 6);
  if (lane >= nqb || t >= T) return;
  const uint32_t* nd = nodes + 2 * node_off[t];
  const uint8_t* u = sc + lane * d;
  uint32_t idx = 0;
  int64_t mid = 0;
  for (int step = 0; step < max_steps; ++step) {
    uint2 r = *(const uint2*)(nd + 2 * (int64_t)idx);
    if (r.y >> 31) {
      mid = (int64_t)r.x + (int64_t)((r.y & 0x7FFFFFFFu) >> 1);
      break;
    }
    uint32_t a = r.y & 0xFFFFu, L = (r.y >> 16) & 7u, flip = (r.y >> 19) & 1u;
    uint32_t bit = ((u[a] >> L) & 1u) ^ flip;
    idx = bit ? r.x : idx + 1u;
  }
  int64_t s = mid - k1 / 2, smax = N - k1 > 0 ? N - k1 : 0;
  s = s < 0 ? 0 : (s > smax ? smax : s);
  win[(q0 + lane) * T + t] = (uint32_t)s;
}

// ------------------------------------------------------- exact query position
// A query's exact place along tree t's curve (its insertion rank among the
// tree's sorted keys, before equal keys), found as in a Patricia trie: the
// descent by node tests reaches a leaf; z, the leaf's first point, shares
// with the query every key bit before the first bit j* where they differ, so
// the descent agreed with the query's own key on every node whose split bit
// is below j*.  The first node on the path whose split bit lies beyond j* is
// the subtree the query leaves: its rank is that node's lo (query bit 0 at
// j*) or hi (bit 1).  If no such node exists the query falls inside the leaf,
// and a binary search over the leaf's keys places it.
//
// Key comparisons here use only the top level of the keys, which depends on
// the coordinates' signs alone: with a the tree's axis order and r its
// reflections, top-level key bit i is the parity of sign[a_0] ^ r_0, ...,
// sign[a_i] ^ r_i, so two keys first differ at the first tree axis whose
// sign differs, and the one whose parity is 1 there is larger.  Points with
// equal sign rows need the deeper levels: such (query, tree) pairs are
// listed for the wavefront-per-pair kernel that computes full keys.
constexpr int RK_T = 256;
// Compares the query's and a point's top key levels from tree position
// `start` on, `par` being the query's prefix parity before it (both agree
// before `start`).  *par_at (if c_at >= start) receives the parity before
// position c_at.
__device__ __forceinline__ int cmp_top(const uint32_t* sq, const uint32_t* sp, const uint16_t* ax, int d, int start,
                                       uint32_t par, int* jstar, int c_at, uint32_t* par_at) {
  for (int i = start; i < d; ++i) {
    if (i == c_at) *par_at = par;
    const uint32_t v = ax[i];
    const uint32_t a = v & 0x7FFFu, w = a >> 5, sh = a & 31u;
    const uint32_t qb = (sq[w * RK_T] >> sh) & 1u, pb = (sp[w * RK_T] >> sh) & 1u;
    par ^= qb ^ (v >> 15);
    if (qb != pb) {
      *jstar = i;
      return par ? 1 : -1;
    }
  }
  return 0;
}

template <int NW>
__global__ __launch_bounds__(RK_T) void k_rank_top(const uint32_t* __restrict__ nodes,
                                                   const uint32_t* __restrict__ aux,
                                                   const int64_t* __restrict__ node_off,
                                                   const uint8_t* __restrict__ qcodes,
                                                   const uint32_t* __restrict__ qsgn,
                                                   const uint32_t* __restrict__ sgn,
                                                   const uint32_t* __restrict__ tree_perm,
                                                   const int32_t* __restrict__ cperm,
                                                   const uint8_t* __restrict__ crefl, int64_t nq, int d, int T,
                                                   int64_t N, int k1, int max_steps, uint32_t* __restrict__ win,
                                                   uint64_t* __restrict__ deep, uint32_t* __restrict__ ndeep) {
  __shared__ uint32_t s_q[NW * RK_T], s_p[NW * RK_T];  // sign rows, word-major
  __shared__ uint16_t s_ax[4][512];                    // each wavefront's tree: axis | reflected << 15
  // the 64 queries' codes (d bytes each, dynamic LDS): a node test then waits
  // for the node record only, not for a code byte behind it
  extern __shared__ __align__(16) uint8_t s_code[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = blockIdx.y * 4 + wv;
  const int64_t qb = (int64_t)blockIdx.x * 64, q = qb + lane;
  {
    const int nqb = (int)min<int64_t>(64, nq - qb);
    if (d % 16 == 0)
      for (int i = threadIdx.x; i < nqb * (d / 16); i += RK_T)
        ((uint4*)s_code)[i] = ((const uint4*)(qcodes + qb * d))[i];
    else
      for (int i = threadIdx.x; i < nqb * d; i += RK_T) s_code[i] = qcodes[qb * d + i];
  }
  if (t < T)
    for (int i = lane; i < d; i += 64)
      s_ax[wv][i] = (uint16_t)(cperm[(int64_t)t * d + i] | ((uint32_t)crefl[(int64_t)t * d + i] << 15));
  if (q < nq)
#pragma unroll
    for (int w = 0; w < NW; ++w) s_q[w * RK_T + threadIdx.x] = qsgn[q * NW + w];
  __syncthreads();  // the codes are shared by the four wavefronts
  if (q >= nq || t >= T) return;
  const uint32_t* sq = s_q + threadIdx.x;
  uint32_t* sp = s_p + threadIdx.x;
  const uint16_t* ax = s_ax[wv];
  const uint32_t* nd = nodes + 2 * node_off[t];
  const uint32_t* au = aux + 2 * node_off[t];
  const uint32_t* tp = tree_perm + (int64_t)t * N;
  const uint8_t* u = s_code + lane * d;
  auto test = [&](uint32_t w1) -> uint32_t {
    const uint32_t a = w1 & 0xFFFFu, L = (w1 >> 16) & 7u, flip = (w1 >> 19) & 1u;
    return ((u[a] >> L) & 1u) ^ flip;
  };
  auto load_row = [&](uint32_t p) {
#pragma unroll
    for (int w = 0; w < NW; ++w) sp[w * RK_T] = sgn[(int64_t)p * NW + w];
  };
  // descent by node tests to a leaf [lo, hi); b_last = split bit of its parent
  uint32_t idx = 0;
  int64_t lo = 0, hi = N;
  int b_last = -1;
  for (int step = 0; step < max_steps; ++step) {
    const uint2 r = *(const uint2*)(nd + 2 * (int64_t)idx);
    const uint2 sb = *(const uint2*)(au + 2 * (int64_t)idx);  // {m, b} or {lo, NONE}
    if (r.y >> 31) break;
    b_last = (int)sb.y;
    if (test(r.y)) {
      lo = sb.x;
      idx = r.x;
    } else {
      hi = sb.x;
      idx = idx + 1u;
    }
  }
  // the leaf's first point z: the query agrees with it before key bit j*
  load_row(tp[lo]);
  int jstar = 0;
  uint32_t par0 = 0;
  const int c0 = b_last + 1;  // every key of the leaf agrees with z before c0
  const int c = cmp_top(sq, sp, ax, d, 0, 0u, &jstar, c0, &par0);
  bool need_deep = c == 0;
  int64_t rank = -1;
  if (!need_deep && jstar < b_last) {
    // the query leaves the path above the leaf: the first node whose split
    // bit lies beyond j* holds it entirely before (bit 0) or after (bit 1)
    int64_t l2 = 0, h2 = N;
    idx = 0;
    for (int step = 0; step < max_steps; ++step) {
      const uint2 r = *(const uint2*)(nd + 2 * (int64_t)idx);
      const uint2 sb = *(const uint2*)(au + 2 * (int64_t)idx);
      if ((int)sb.y > jstar) {
        rank = c > 0 ? h2 : l2;
        break;
      }
      if (test(r.y)) {
        l2 = sb.x;
        idx = r.x;
      } else {
        h2 = sb.x;
        idx = idx + 1u;
      }
    }
  } else if (!need_deep) {
    // inside the leaf: the query and every key of the leaf agree before c0,
    // so comparisons start there from the query's parity before c0
    int64_t a = lo, b = hi;
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      load_row(tp[mid]);
      int j2;
      uint32_t unused;
      const int c2 = cmp_top(sq, sp, ax, d, c0, par0, &j2, -1, &unused);
      if (c2 == 0) {
        need_deep = true;
        break;
      }
      if (c2 > 0)
        a = mid + 1;
      else
        b = mid;
    }
    rank = a;
  }
  if (need_deep) {
    const uint32_t slot = atomicAdd(ndeep, 1u);
    deep[slot] = ((uint64_t)q << 32) | (uint32_t)t;
    win[q * T + t] = 0u;  // written by the full-key kernel
    return;
  }
  int64_t s = rank - k1 / 2, smax = N - k1 > 0 ? N - k1 : 0;
  s = s < 0 ? 0 : (s > smax ? smax : s);
  win[q * T + t] = (uint32_t)s;
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------- ham + hist
constexpr int HB = 513;  // Hamming values 0..512

// The n*len window entries of one query form one list, entry e = t*len + i
// (tree t, offset i in its window), taken 256 at a time: the group of four
// lanes grp reads the sketches of entries e0 + 4 grp + u, u < 4, 16 bytes a
// lane.  Lane qd of the group loads the position of entry e0 + 4 grp + qd
// (the group shares them by quad broadcasts) and ends with that entry's
// distance, so a wave stores 64 consecutive distances at once.  Positions of
// the next 256 entries are loaded while the current sketches are in flight.
// No load or store is conditional (entries past the list read its last
// position and write into the row's padding, which is a multiple of 256
// entries; their histogram count goes to a spare bin): a memory operation
// that some paths skip makes the compiler wait for every one before it.
// mlen = ceil(2^32 / len): t = (e * mlen) >> 32 is floor(e / len) or one
// more, since e < 2^30.

template <int KT>
__global__ __launch_bounds__(KT) void k_ham(const uint32_t* __restrict__ tree_perm, int64_t N,
                                             int T, int len, uint64_t mlen, int64_t qstride,
                                             const uint32_t* __restrict__ win,
                                             const uint64_t* __restrict__ sk,
                                             const uint64_t* __restrict__ qsk,
                                             uint16_t* __restrict__ ham,
                                             uint32_t* __restrict__ hist,
                                             const uint32_t* __restrict__ only) {
  constexpr int NWV = KT / 64;
  __shared__ uint32_t h[NWV][HB + 1];
  extern __shared__ uint32_t s_win[];  // T window starts (dynamic LDS)
  const int64_t q = blockIdx.x;
  if (only && !only[q]) return;  // the query's C2 came from the bucketed filter
  for (int i = threadIdx.x; i < NWV * (HB + 1); i += KT) (&h[0][0])[i] = 0;
  for (int t = threadIdx.x; t < T; t += KT) s_win[t] = win[q * T + t];
  __syncthreads();
  const int w = threadIdx.x / 64, grp = threadIdx.x / 4, qd = threadIdx.x & 3;
  const uint64_t q0 = qsk[q * 8 + 2 * qd], q1 = qsk[q * 8 + 2 * qd + 1];
  uint16_t* out = ham + q * qstride;
  const uint32_t total = (uint32_t)T * (uint32_t)len, ulen = (uint32_t)len;
  auto pos_of = [&](uint32_t e) -> uint32_t {
    e = e < total ? e : total - 1u;
    uint32_t t = (uint32_t)(((uint64_t)e * mlen) >> 32);
    t -= t * ulen > e ? 1u : 0u;
    return tree_perm[(int64_t)t * N + s_win[t] + (e - t * ulen)];
  };
  const uint32_t mine = (uint32_t)(4 * grp + qd);
  const bool b0 = qd & 1, b1 = qd & 2;
  uint32_t pc = pos_of(mine);
  __builtin_amdgcn_sched_barrier(0);
  // a store behind the first position load, as every iteration has one behind
  // its position load (the first iteration overwrites it): the wait for the
  // position then never has to include the store
  out[mine] = 0;
  uint32_t e0 = 0;
  do {  // total >= 1
    ulonglong2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = *(const ulonglong2*)(sk + (int64_t)quad_bcast(pc, u) * 8 + 2 * qd);
    pc = pos_of(e0 + (uint32_t)KT + mine);
    // issue the next position load before any use of the sketches
    __builtin_amdgcn_sched_barrier(0);
    uint32_t a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = (uint32_t)(__popcll(v[u].x ^ q0) + __popcll(v[u].y ^ q1));
    // reduce-scatter over the quad: lane qd ends with the sum for entry u = qd
    const uint32_t k0 = (b0 ? a[1] : a[0]) + quad_perm<QP_XOR1>(b0 ? a[0] : a[1]);  // u = b0
    const uint32_t k1 = (b0 ? a[3] : a[2]) + quad_perm<QP_XOR1>(b0 ? a[2] : a[3]);  // u = 2 + b0
    const uint32_t c = (b1 ? k1 : k0) + quad_perm<QP_XOR2>(b1 ? k0 : k1);
    const uint32_t e = e0 + mine;
    out[e] = (uint16_t)c;
    atomicAdd(&h[w][e < total ? c : (uint32_t)HB], 1u);
    e0 += KT;
  } while (e0 < total);
  __syncthreads();
  for (int i = threadIdx.x; i < HB; i += KT) {
    uint32_t c = 0;
#pragma unroll
    for (int v = 0; v < NWV; ++v) c += h[v][i];
    hist[q * HB + i] = c;
  }
}

// The queries the bucketed filter flags, spread over many workgroups: their
// histogram rows are zeroed and their indices listed (k_ham_flagged, one
// wavefront a query; ctr[0] counts them, zeroed by k_ham_ctr_zero), then
// k_ham_split's persistent workgroups take (flagged query, slice) items,
// each slice a run of whole KT-entry steps of the query's entries, and add
// their histograms to the query's row.  Per entry the same work as k_ham.
__global__ void k_ham_ctr_zero(uint32_t* __restrict__ ctr) { ctr[0] = 0u; }

__global__ __launch_bounds__(256) void k_ham_flagged(const uint32_t* __restrict__ flag, int64_t nb,
                                                     uint32_t* __restrict__ hist, uint32_t* __restrict__ list,
                                                     uint32_t* __restrict__ ctr) {
  const int64_t q = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (q >= nb || !flag[q]) return;
  for (int i = __lane_id(); i < HB; i += 64) hist[q * HB + i] = 0u;
  if (__lane_id() == 0) list[atomicAdd(ctr, 1u)] = (uint32_t)q;
}

template <int KT>
__global__ __launch_bounds__(KT) void k_ham_split(const uint32_t* __restrict__ tree_perm, int64_t N, int T, int len,
                                                  uint64_t mlen, int64_t qstride, const uint32_t* __restrict__ win,
                                                  const uint64_t* __restrict__ sk,
                                                  const uint64_t* __restrict__ qsk, uint16_t* __restrict__ ham,
                                                  uint32_t* __restrict__ hist, const uint32_t* __restrict__ list,
                                                  const uint32_t* __restrict__ ctr, int S) {
  constexpr int NWV = KT / 64;
  __shared__ uint32_t h[NWV][HB + 1];
  extern __shared__ uint32_t s_win[];  // T window starts (dynamic LDS)
  const uint32_t total = (uint32_t)T * (uint32_t)len, ulen = (uint32_t)len;
  const uint32_t per = ((total + (uint32_t)S - 1) / (uint32_t)S + KT - 1) / KT * KT;  // entries a slice
  const uint32_t nitems = ctr[0] * (uint32_t)S;
  const int w = threadIdx.x / 64, grp = threadIdx.x / 4, qd = threadIdx.x & 3;
  const uint32_t mine = (uint32_t)(4 * grp + qd);
  const bool b0 = qd & 1, b1 = qd & 2;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int64_t q = list[it / (uint32_t)S];
    const uint32_t s0 = (it % (uint32_t)S) * per;
    if (s0 >= total) continue;  // the same for the whole workgroup
    const uint32_t s1 = min(total, s0 + per);
    for (int i = threadIdx.x; i < NWV * (HB + 1); i += KT) (&h[0][0])[i] = 0;
    for (int t = threadIdx.x; t < T; t += KT) s_win[t] = win[q * T + t];
    __syncthreads();
    const uint64_t q0 = qsk[q * 8 + 2 * qd], q1 = qsk[q * 8 + 2 * qd + 1];
    uint16_t* out = ham + q * qstride;
    auto pos_of = [&](uint32_t e) -> uint32_t {
      e = e < total ? e : total - 1u;
      uint32_t t = (uint32_t)(((uint64_t)e * mlen) >> 32);
      t -= t * ulen > e ? 1u : 0u;
      return tree_perm[(int64_t)t * N + s_win[t] + (e - t * ulen)];
    };
    uint32_t pc = pos_of(s0 + mine);
    __builtin_amdgcn_sched_barrier(0);
    out[s0 + mine] = 0;  // (as in k_ham: a store behind the first position load)
    uint32_t e0 = s0;
    do {  // s0 < s1
      ulonglong2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = *(const ulonglong2*)(sk + (int64_t)quad_bcast(pc, u) * 8 + 2 * qd);
      pc = pos_of(e0 + (uint32_t)KT + mine);
      __builtin_amdgcn_sched_barrier(0);
      uint32_t a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = (uint32_t)(__popcll(v[u].x ^ q0) + __popcll(v[u].y ^ q1));
      const uint32_t k0 = (b0 ? a[1] : a[0]) + quad_perm<QP_XOR1>(b0 ? a[0] : a[1]);
      const uint32_t k1 = (b0 ? a[3] : a[2]) + quad_perm<QP_XOR1>(b0 ? a[2] : a[3]);
      const uint32_t c = (b1 ? k1 : k0) + quad_perm<QP_XOR2>(b1 ? k0 : k1);
      const uint32_t e = e0 + mine;
      out[e] = (uint16_t)c;
      atomicAdd(&h[w][e < s1 ? c : (uint32_t)HB], 1u);
      e0 += KT;
    } while (e0 < s1);
    __syncthreads();
    for (int i = threadIdx.x; i < HB; i += KT) {
      uint32_t c = 0;
#pragma unroll
      for (int v = 0; v < NWV; ++v) c += h[v][i];
      if (c) atomicAdd(&hist[q * HB + i], c);
    }
    __syncthreads();  // h and s_win are rewritten for the next item
  }
}

// ------------------------------------------------------------------ select
constexpr int SEL_T = 512;
constexpr int CAP = 8192;
constexpr int NBK = 1024;

// Visits every window entry of one query: the Hamming values are read 8 at a
// time (16-byte loads of the query's padded row), the tree position of an
// entry is read only when `want(ham)` holds.  f(ham, pos) runs per wanted entry.
template <class W, class F>
__device__ __forceinline__ void scan_entries(const uint16_t* __restrict__ hq,
                                             const uint32_t* __restrict__ tree_perm, int64_t N,
                                             const uint32_t* __restrict__ wq, int len, int64_t total,
                                             W want, F f) {
  const int64_t n8 = (total + 7) / 8;
  for (int64_t j0 = threadIdx.x; j0 < n8; j0 += 2 * SEL_T) {
    uint4 v[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t j = j0 + (int64_t)u * SEL_T;
      v[u] = j < n8 ? *(const uint4*)(hq + 8 * j) : make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t j = j0 + (int64_t)u * SEL_T;
      const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int hv = (int)((w[s >> 1] >> (16 * (s & 1))) & 0xFFFFu);
        const int64_t e = 8 * j + s;
        if (e < total && want(hv)) {
          const uint32_t t = (uint32_t)(e / len), i = (uint32_t)(e - (int64_t)t * len);
          f(hv, tree_perm[(int64_t)t * N + wq[t] + i]);
        }
      }
    }
  }
}

// Keys of every entry whose distance lies in [hf, hb], when no position bound
// applies (all of them are wanted), in two phases: the row is scanned with
// four 16-byte loads in flight per thread and the wanted entry indices are
// appended to keys[] (one LDS atomic per wavefront and step); then each
// thread takes wanted entries and loads their positions and distances, all
// of these loads in flight together (a position load under the scan's branch
// would be waited for entry by entry).  The caller's histogram bounds the
// count by CAP.
__device__ __forceinline__ void collect_bins(const uint16_t* __restrict__ hq,
                                             const uint32_t* __restrict__ tree_perm, int64_t N,
                                             const uint32_t* __restrict__ wq, int len, int64_t total,
                                             int hf, int hb, int pos_bits, uint32_t* keys,
                                             uint32_t* s_cnt) {
  const int64_t n8 = (total + 7) / 8;
  const int lane = threadIdx.x & 63;
  for (int64_t j0 = 0; j0 < n8; j0 += 4 * SEL_T) {
    uint4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = j0 + u * SEL_T + threadIdx.x;
      v[u] = *(const uint4*)(hq + 8 * (j < n8 ? j : n8 - 1));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = j0 + u * SEL_T + threadIdx.x;
      const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int hv = (int)((w[s >> 1] >> (16 * (s & 1))) & 0xFFFFu);
        const int64_t e = 8 * j + s;
        const bool want = e < total && hv >= hf && hv <= hb;
        const uint64_t m = __ballot(want);
        if (m) {
          const int leader = __ffsll((unsigned long long)m) - 1;
          uint32_t base = 0;
          if (lane == leader) base = atomicAdd(s_cnt, (uint32_t)__popcll(m));
          base = (uint32_t)__shfl((int)base, leader);
          const uint32_t slot = base + (uint32_t)__popcll(m & lanemask_lt());
          if (want && slot < (uint32_t)CAP) keys[slot] = (uint32_t)e;
        }
      }
    }
  }
  __syncthreads();
  const int cnt = (int)min(*s_cnt, (uint32_t)CAP);
  __syncthreads();
  if (threadIdx.x == 0) *s_cnt = (uint32_t)cnt;
  for (int i = threadIdx.x; i < cnt; i += SEL_T) {
    const uint32_t e = keys[i];
    const uint32_t t = e / (uint32_t)len, off = e - t * (uint32_t)len;
    const uint32_t p = tree_perm[(int64_t)t * N + wq[t] + off];
    const int hv = (int)hq[e];
    keys[i] = ((uint32_t)(hv - hf) << pos_bits) | p;
  }
}

__global__ __launch_bounds__(SEL_T) void k_select(const uint32_t* __restrict__ tree_perm,
                                                  int64_t N, int T, int len, int64_t qstride,
                                                  const uint32_t* __restrict__ win,
                                                  const uint16_t* __restrict__ ham,
                                                  const uint32_t* __restrict__ hist0, int k2,
                                                  int pos_bits, uint32_t* __restrict__ c2,
                                                  int32_t* __restrict__ c2n,
                                                  const uint32_t* __restrict__ only) {
  __shared__ uint32_t keys[CAP];
  __shared__ uint32_t hist[HB];
  __shared__ uint32_t bk[NBK];
  __shared__ uint32_t scan_tmp[SEL_T / 64 + 1];
  __shared__ uint32_t s_cnt;
  __shared__ int s_mode, s_hf, s_hb;
  __shared__ uint32_t s_plo, s_pend, s_phi;

  const int64_t q = blockIdx.x;
  if (only && !only[q]) return;
  const uint16_t* hq = ham + q * qstride;
  const uint32_t* wq = win + q * T;
  const int HM = (int)((1ull << (32 - pos_bits)) - 1ull);
  const uint32_t pmask = (uint32_t)((1ull << pos_bits) - 1ull);
  int need = k2, outn = 0;
  int lo_ham = 0;
  uint32_t lo_pos = 0;
  bool first = true;
  const int64_t total = (int64_t)T * len;

  while (need > 0) {
    // histogram of the entries not yet consumed: (ham, pos) >= (lo_ham, lo_pos)
    if (first) {
      for (int i = threadIdx.x; i < HB; i += SEL_T) hist[i] = hist0[q * HB + i];
      __syncthreads();
    } else {
      for (int i = threadIdx.x; i < HB; i += SEL_T) hist[i] = 0;
      __syncthreads();
      const int lh = lo_ham;
      const uint32_t lp = lo_pos;
      scan_entries(hq, tree_perm, N, wq, len, total, [&](int hv) { return hv >= lh; },
                   [&](int hv, uint32_t p) {
                     if (hv > lh || p >= lp) atomicAdd(&hist[hv], 1u);
                   });
      __syncthreads();
    }
    first = false;
    if (threadIdx.x == 0) {
      int hf = -1;
      for (int h = lo_ham; h < HB; ++h)
        if (hist[h]) {
          hf = h;
          break;
        }
      // bins from hf on until they hold `enough` entries, or CAP.  The
      // entries of smallest distance are the query's near neighbours, which
      // sit in the windows of many trees, so duplicates are common there and
      // a round short of `need` distinct entries would cost two more scans
      // of the query's row: at least 1.5 need + 64, and up to 64 below the
      // power of two that the bitonic sort pads that to (the sort costs the
      // same for any count up to it)
      int hb = -1;
      if (hf >= 0) {
        uint32_t cum = 0;
        const uint32_t lo = (uint32_t)need + (uint32_t)need / 2u + 64u;
        uint32_t p2 = 1;
        while (p2 < lo) p2 <<= 1;
        const uint32_t enough = max(lo, p2 - 64u);
        for (int h = hf; h < HB && h - hf < HM; ++h) {
          if (cum + hist[h] > (uint32_t)CAP) break;
          cum += hist[h];
          hb = h;
          if (cum >= enough) break;
        }
      }
      s_hf = hf;
      s_hb = hb;
      s_mode = hf < 0 ? 0 : (hb >= hf ? 1 : 2);
      s_cnt = 0;
      s_plo = (hf == lo_ham) ? lo_pos : 0u;
      s_phi = (uint32_t)N;
    }
    __syncthreads();
    const int mode = s_mode, hf = s_hf, hb = s_hb;
    if (mode == 0) break;
    if (mode == 2) {
      // a single Hamming value overflows: narrow a position range until the
      // first bucket prefix fits (a bucket of width 1 holds at most T entries)
      for (;;) {
        const uint32_t plo = s_plo, phi = s_phi;
        const uint32_t width = (uint32_t)ceil_div((int64_t)(phi - plo), NBK);
        for (int i = threadIdx.x; i < NBK; i += SEL_T) bk[i] = 0;
        __syncthreads();
        scan_entries(hq, tree_perm, N, wq, len, total, [&](int hv) { return hv == hf; },
                     [&](int, uint32_t p) {
                       if (p >= plo && p < phi) atomicAdd(&bk[(p - plo) / width], 1u);
                     });
        __syncthreads();
        if (threadIdx.x == 0) {
          uint32_t cum = 0;
          int kb = -1;
          for (int b = 0; b < NBK; ++b) {
            if (cum + bk[b] > (uint32_t)CAP) break;
            cum += bk[b];
            kb = b;
          }
          if (kb >= 0) {
            uint64_t e = (uint64_t)plo + (uint64_t)(kb + 1) * width;
            s_pend = (uint32_t)(e < phi ? e : phi);
            s_mode = 3;
          } else {
            s_phi = plo + width;
          }
        }
        __syncthreads();
        if (s_mode == 3) break;
      }
    }
    // collect the chunk
    {
      const uint32_t plo = s_plo, pend = s_pend;
      const int lh = lo_ham;
      const uint32_t lp = lo_pos;
      if (mode == 1 && lp == 0) {
        collect_bins(hq, tree_perm, N, wq, len, total, hf, hb, pos_bits, keys, &s_cnt);
      } else if (mode == 1) {
        scan_entries(hq, tree_perm, N, wq, len, total, [&](int hv) { return hv >= hf && hv <= hb; },
                     [&](int hv, uint32_t p) {
                       if (hv > lh || p >= lp) keys[atomicAdd(&s_cnt, 1u)] = ((uint32_t)(hv - hf) << pos_bits) | p;
                     });
      } else {
        scan_entries(hq, tree_perm, N, wq, len, total, [&](int hv) { return hv == hf; },
                     [&](int, uint32_t p) {
                       if (p >= plo && p < pend) keys[atomicAdd(&s_cnt, 1u)] = p;
                     });
      }
    }
    __syncthreads();
    const int cnt = (int)s_cnt;
    int n2 = 1;
    while (n2 < cnt) n2 <<= 1;
    for (int i = cnt + threadIdx.x; i < n2; i += SEL_T) keys[i] = NONE32;
    __syncthreads();
    bitonic_u32(keys, n2);
    // distinct keys in order: each thread takes a contiguous run
    const int per = (cnt + SEL_T - 1) / SEL_T;
    const int a0 = threadIdx.x * per, a1 = min(cnt, a0 + per);
    uint32_t mine = 0;
    for (int i = a0; i < a1; ++i)
      if (i == 0 || keys[i] != keys[i - 1]) ++mine;
    uint32_t tot;
    uint32_t r = block_excl_scan<SEL_T>(mine, scan_tmp, &tot);
    for (int i = a0; i < a1; ++i)
      if (i == 0 || keys[i] != keys[i - 1]) {
        if ((int)r < need) {
          uint32_t k = keys[i];
          c2[q * k2 + outn + r] = mode == 1 ? (k & pmask) : k;
        }
        ++r;
      }
    int took = min(need, (int)tot);
    need -= took;
    outn += took;
    if (mode == 1) {
      lo_ham = hb + 1;
      lo_pos = 0;
      if (lo_ham >= HB) break;
    } else {
      lo_ham = hf;
      lo_pos = s_pend;
    }
    __syncthreads();
  }
  for (int i = outn + threadIdx.x; i < k2; i += SEL_T) c2[q * k2 + i] = NONE32;
  if (threadIdx.x == 0) c2n[q] = outn;
}

// ------------------------------------------------------------------ rerank
constexpr int RR_T = 256;  // six workgroups a CU: their sort, row and select phases overlap

constexpr int RROWS = 4;

// MCH > 0: rows read as 16-byte chunks, MCH chunks per lane; MCH == 0: scalar reads.
template <class T, int MCH>
__global__ __launch_bounds__(RR_T) void k_rerank(const T* __restrict__ Xp, int64_t N, int d,
                                                 const T* __restrict__ Q,
                                                 const uint32_t* __restrict__ c2,
                                                 const int32_t* __restrict__ c2n, int k2, int h,
                                                 int k, int k2p, int emax, int kp,
                                                 const uint32_t* __restrict__ pos2id,
                                                 int32_t* __restrict__ ids,
                                                 float* __restrict__ scores,
                                                 int32_t* __restrict__ en_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* sq = (float*)smem;                                  // d
  uint32_t* sc = (uint32_t*)(sq + ((d + 3) & ~3));           // k2p
  uint32_t* st = sc + k2p;                                   // k2p
  uint32_t* off = st + k2p;                                  // k2p + 1
  uint32_t* ekey = off + k2p + 4;                            // emax
  uint64_t* sel = (uint64_t*)(((uintptr_t)(ekey + emax) + 7) & ~(uintptr_t)7);  // kp
  __shared__ uint32_t hist[256];
  __shared__ uint32_t scan_tmp[RR_T / 64 + 1];
  __shared__ uint32_t s_E, s_lt, s_eq_need, s_nsel;
  __shared__ uint32_t s_prefix;

  const int64_t q = blockIdx.x;
  const int n2 = c2n[q];
  for (int i = threadIdx.x; i < d; i += RR_T) {
    if constexpr (sizeof(T) == 2)
      sq[i] = __half2float(Q[q * d + i]);
    else
      sq[i] = Q[q * d + i];
  }
  for (int i = threadIdx.x; i < k2p; i += RR_T) sc[i] = i < n2 ? c2[q * k2 + i] : NONE32;
  __syncthreads();
  bitonic_u32(sc, k2p);
  expansion_intervals<RR_T>(sc, n2, h, N, st, off, scan_tmp, &s_E);
  const uint32_t E = s_E;
  // scores: a 16-lane group per row, RROWS consecutive expansion rows in
  // flight per group (mostly adjacent master positions: contiguous reads)
  {
    const int g = threadIdx.x / 16, gl = threadIdx.x % 16;
    constexpr int NG = RR_T / 16;
    constexpr int EPC = 16 / sizeof(T);  // elements per 16-byte chunk
    const int nch = d / EPC;
    for (uint32_t e0 = (uint32_t)g * RROWS; e0 < E; e0 += NG * RROWS) {
      float acc[RROWS];
      if constexpr (MCH > 0) {
        uint4 raw[RROWS][MCH];
#pragma unroll
        for (int u = 0; u < RROWS; ++u) {
          const uint32_t e = e0 + u;
          const T* row = Xp + (int64_t)(e < E ? epos(st, off, n2, e) : 0u) * d;
#pragma unroll
          for (int m = 0; m < MCH; ++m) {
            const int c = gl + 16 * m;
            // unconditional (past E the row is row 0, its score never stored)
            raw[u][m] = *(const uint4*)(row + (c < nch ? c : 0) * EPC);
          }
        }
#pragma unroll
        for (int u = 0; u < RROWS; ++u) {
          float a = 0.f;
#pragma unroll
          for (int m = 0; m < MCH; ++m) {
            const int c = gl + 16 * m;
            if (c < nch) {
              const float* qq = sq + c * EPC;
              if constexpr (sizeof(T) == 2) {
                const __half2* hv = (const __half2*)&raw[u][m];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  float2 f2 = __half22float2(hv[j]);
                  a = fmaf(f2.x, qq[2 * j], a);
                  a = fmaf(f2.y, qq[2 * j + 1], a);
                }
              } else {
                const float* fv = (const float*)&raw[u][m];
#pragma unroll
                for (int j = 0; j < 4; ++j) a = fmaf(fv[j], qq[j], a);
              }
            }
          }
          acc[u] = a;
        }
      } else {
#pragma unroll
        for (int u = 0; u < RROWS; ++u) {
          const uint32_t e = e0 + u;
          float a = 0.f;
          if (e < E) {
            const T* row = Xp + (int64_t)epos(st, off, n2, e) * d;
            for (int c = gl; c < d; c += 16) {
              float xv;
              if constexpr (sizeof(T) == 2)
                xv = __half2float(row[c]);
              else
                xv = row[c];
              a = fmaf(xv, sq[c], a);
            }
          }
          acc[u] = a;
        }
      }
#pragma unroll
      for (int u = 0; u < RROWS; ++u) {
        float a = acc[u];
        a += __shfl_xor(a, 8);
        a += __shfl_xor(a, 4);
        a += __shfl_xor(a, 2);
        a += __shfl_xor(a, 1);
        if (gl == 0 && e0 + u < E) ekey[e0 + u] = ~float_to_ordered(a);  // ascending key = descending score
      }
    }
  }
  __syncthreads();
  const uint32_t kk = (uint32_t)min<int64_t>(k, E);
  select_smallest<RR_T>(ekey, E, kk, sel, hist, scan_tmp, &s_prefix, &s_lt, &s_eq_need, &s_nsel);
  __syncthreads();
  for (int i = (int)kk + threadIdx.x; i < kp; i += RR_T) sel[i] = ~0ull;
  __syncthreads();
  bitonic_u64(sel, kp);
  for (int i = threadIdx.x; i < k; i += RR_T) {
    if (i < (int)kk) {
      uint64_t v = sel[i];
      uint32_t e = (uint32_t)v;
      uint32_t p = epos(st, off, n2, e);
      ids[q * k + i] = (int32_t)pos2id[p];
      scores[q * k + i] = ordered_to_float(~(uint32_t)(v >> 32));
    } else {
      ids[q * k + i] = -1;
      scores[q * k + i] = -INFINITY;
    }
  }
  if (threadIdx.x == 0 && en_out) en_out[q] = (int32_t)E;
}

}  // namespace

// ------------------------------------------------------------------ host side
// Entries of one query's row of distances: T windows of len, padded to 256.
// rows padded to a multiple of 1,024 entries: the tail of a row takes the
// last step's stores of a 1,024-thread workgroup
int64_t ham_row_entries(int T, int len) { return ((int64_t)T * len + 1023) / 1024 * 1024; }

// Queries per filter batch: rows of distances of a batch stay under 2 GB.
int64_t filter_batch(int64_t nq, int64_t per_q) {
  int64_t batch = std::max<int64_t>(1, std::min<int64_t>(nq, (int64_t)(1ll << 31) / (per_q * 2 + 1)));
  return ceil_div(nq, ceil_div(nq, batch));  // equal batches
}

size_t search_scratch_bytes(const hf_forest* f, int64_t nq, const hf_search_params& p) {
  const int T = p.trees ? (int)p.trees : f->T;
  const int len = (int)std::min<int64_t>(p.k1, f->N);
  const int64_t per_q = ham_row_entries(T, len);
  const int64_t batch = filter_batch(nq, per_q);
  auto A = [](size_t b) { return Workspace::arena_bytes(b); };
  size_t total = A((size_t)nq * f->d) + A((size_t)nq * 64) + A((size_t)nq * T * 4) +
                 A((size_t)batch * per_q * 2) + A((size_t)batch * HB * 4) + A((size_t)nq * p.k2 * 4) +
                 A((size_t)nq * 4);
  if (f->sketch_kind == HF_SKETCH_LEARNED)
    total += A((size_t)std::min<int64_t>(nq, 1 << 20) * lhash_hidden(f->lhash) * 2);  // bf16 hidden layer
  if (p.position == HF_POS_EXACT)
    total += A((size_t)nq * f->sgn_words * 4) + A(4) + A((size_t)nq * T * 8);
  return total;
}

hf_status search_launch(const hf_forest* f, const void* Q, int64_t nq, const hf_search_params& p,
                        int32_t* ids, float* scores, uint32_t* win_out, uint32_t* c2_out,
                        int32_t* c2n_out, int32_t* en_out, uint32_t* surv_pos, float* surv_score,
                        hipStream_t s, Workspace* ext) {
  Workspace own(s);
  Workspace& ws = ext ? *ext : own;
  const int64_t N = f->N;
  const int d = f->d, T = p.trees ? (int)p.trees : f->T;  // trees 0..T-1
  const int len = (int)std::min<int64_t>(p.k1, N);
  const int k2 = (int)p.k2;
  // query codes and sketches
  uint8_t* qcodes;
  uint64_t* qsk;
  HF_TRY(ws.alloc(&qcodes, (size_t)(nq * d)));
  HF_TRY(ws.alloc(&qsk, (size_t)(nq * 8)));
  {
    StageTimer tm(ST_QCODES, s);
    HF_TRY(quantize(Q, f->dtype, nq * d, f->e, qcodes, s));
  }
  {
    StageTimer tm(ST_QSKETCH, s);
    if (f->sketch_kind == HF_SKETCH_LEARNED)
      HF_TRY(lhash_encode_dev(f->lhash, Q, f->dtype, nq, qsk, s, &ws));
    else if (f->sketch_kind == HF_SKETCH_SIGN)
      HF_TRY(sign_sketch(Q, f->dtype, nq, d, qsk, s));
    else if (f->srp_Rb && getenv("HF_SRP_VALU") == nullptr)
      HF_TRY(srp_sketch_mfma(Q, f->dtype, nq, d, f->e, f->srp_Rb, qsk, s));
    else
      HF_TRY(srp_sketch(Q, f->dtype, nq, d, f->e, f->sketch_seed, qsk, ws, f->srp_R));
  }
  uint32_t* win = win_out;
  if (!win) HF_TRY(ws.alloc(&win, (size_t)(nq * T)));
  const int64_t* doff = f->node_off_dev;
  if (p.position == HF_POS_EXACT) {
    StageTimer tm(ST_DESCEND, s);
    const int nw = f->sgn_words;
    uint32_t *qsgn, *ndeep;
    uint64_t* deep;
    HF_TRY(ws.alloc(&qsgn, (size_t)nq * nw));
    HF_TRY(ws.alloc(&ndeep, 1));
    HF_TRY(ws.alloc(&deep, (size_t)nq * T));
    HF_TRY(msb_plane(qcodes, nq, d, qsgn, s));
    k_zero_u32<<<1, 64, 0, s>>>(ndeep, 1);
    dim3 grid((unsigned)ceil_div(nq, 64), (unsigned)ceil_div(T, 4));
    const size_t rk_lds = 64 * (size_t)d;  // dynamic: the codes; static: 2 NW RK_T words + 4 KB
#define HF_RK(n)                                                                                                    \
  case n:                                                                                                           \
    if (rk_lds + 8 * (size_t)n * RK_T + 4096 > 64 * 1024)                                                          \
      HIP_TRY(hipFuncSetAttribute((const void*)k_rank_top<n>, hipFuncAttributeMaxDynamicSharedMemorySize,          \
                                  (int)rk_lds));                                                                    \
    k_rank_top<n><<<grid, RK_T, rk_lds, s>>>(f->nodes, f->node_aux, doff, qcodes, qsgn, f->sgn_pos, f->tree_perm,  \
                                             f->curve_perm, f->curve_refl, nq, d, T, N, (int)p.k1, 8 * d + 2, win, \
                                             deep, ndeep);                                                          \
    break;
    switch (nw) { HF_RK(1) HF_RK(2) HF_RK(4) HF_RK(8) HF_RK(12) HF_RK(16) }
#undef HF_RK
    HF_LAUNCH_CHECK();
    HF_TRY(rank_deep(f, qcodes, nq, T, (int)p.k1, deep, ndeep, win, s));
  } else {
    StageTimer tm(ST_DESCEND, s);
    if (d % 16 == 0 && d <= DS_MAXD) {
      // sixteen trees a workgroup share one copy of the codes (four: 1.54
      // against 1.49 ms per 10,000 queries at 1,280 trees; eight: 1.60)
      dim3 grid((unsigned)ceil_div(nq, DS_Q), (unsigned)ceil_div(T, 16));
      k_descend_lds<16><<<grid, 1024, (size_t)DS_Q * d, s>>>(f->nodes, doff, qcodes, nq, d, T, N, (int)p.k1,
                                                              8 * d + 2, win);
    } else {
      dim3 grid((unsigned)ceil_div(nq, 256), (unsigned)T);
      k_descend<<<grid, 256, 0, s>>>(f->nodes, doff, qcodes, nq, d, T, N, (int)p.k1, 8 * d + 2, win);
    }
    HF_LAUNCH_CHECK();
  }
  // the second stage runs in batches of queries sized to bound scratch memory
  const int64_t per_q = ham_row_entries(T, len);
  // the bucketed filter (not with a fixed scratch arena: its records take
  // 4 bytes per window entry)
  const bool bucketed = !ws.arena && bfilter_usable(N, T, k2);
  int64_t batch = filter_batch(nq, per_q);
  if (bucketed) batch = std::min(batch, bfilter_max_batch(N));
  uint16_t* ham;
  uint32_t *hist, *c2 = c2_out;
  int32_t* c2n = c2n_out;
  HF_TRY(ws.alloc(&ham, (size_t)(batch * per_q)));
  HF_TRY(ws.alloc(&hist, (size_t)(batch * HB)));
  uint32_t *flist = nullptr, *fctr = nullptr;  // the bucketed filter's flagged queries
  int ncu = 256;
  if (bucketed) {
    HF_TRY(ws.alloc(&flist, (size_t)batch));
    HF_TRY(ws.alloc(&fctr, 1));
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  }
  if (!c2) HF_TRY(ws.alloc(&c2, (size_t)(nq * k2)));
  if (!c2n) HF_TRY(ws.alloc(&c2n, (size_t)nq));
  const int pos_bits = std::max(1, bits_for((uint64_t)(N - 1)));
  const int k2p = [&] { int v = 1; while (v < k2) v <<= 1; return v; }();
  const int kp = [&] { int v = 1; while (v < (int)p.k) v <<= 1; return v; }();
  const int64_t emax = std::min<int64_t>((int64_t)k2 * (2 * p.h + 1), N);
  size_t smem = sizeof(float) * (((size_t)d + 3) & ~(size_t)3) + sizeof(uint32_t) * (3 * (size_t)k2p + 4) +
                sizeof(uint32_t) * (size_t)emax + 8 + sizeof(uint64_t) * (size_t)kp;
  if (smem > 160 * 1024) {
    set_error("rerank needs %zu bytes of LDS (k2*(2h+1) too large)", smem);
    return HF_ERR_UNSUPPORTED;
  }
  const size_t esz = f->dtype == HF_F16 ? 2 : 4;
  // chunks of 16 bytes per lane when rows are 16-byte multiples and short enough
  int mch = 0;
  if (((size_t)d * esz) % 16 == 0) {
    const int per_lane = (int)ceil_div((int64_t)d * esz / 16, 16);
    mch = per_lane <= 1 ? 1 : per_lane <= 2 ? 2 : per_lane <= 3 ? 3 : per_lane <= 4 ? 4 : per_lane <= 6 ? 6 : per_lane <= 8 ? 8 : 0;
  }
  auto rerank = [&](int64_t q0, int64_t nb) -> hf_status {
    const void* Qb = (const char*)Q + q0 * d * esz;
    const void* kern = nullptr;
#define HF_RR(TY, M) if (mch == M) kern = (const void*)k_rerank<TY, M>;
    if (f->dtype == HF_F16) {
      HF_RR(__half, 0) HF_RR(__half, 1) HF_RR(__half, 2) HF_RR(__half, 3) HF_RR(__half, 4) HF_RR(__half, 6) HF_RR(__half, 8)
    } else {
      HF_RR(float, 0) HF_RR(float, 1) HF_RR(float, 2) HF_RR(float, 3) HF_RR(float, 4) HF_RR(float, 6) HF_RR(float, 8)
    }
#undef HF_RR
    if (smem > 64 * 1024)
      HIP_TRY(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    const void* Xp = f->X_pos;
    const uint32_t* c2b = c2 + q0 * k2;
    const int32_t* c2nb = c2n + q0;
    int h_ = (int)p.h, k_ = (int)p.k, emax_ = (int)emax;
    const uint32_t* p2i = f->pos2id;
    int32_t* idsb = ids + q0 * p.k;
    float* scb = scores + q0 * p.k;
    int32_t* enb = en_out ? en_out + q0 : nullptr;
    int64_t N_ = N;
    int d_ = d, k2_ = k2, k2p_ = k2p, kp_ = kp;
    void* args[] = {(void*)&Xp, &N_, &d_, (void*)&Qb, (void*)&c2b, (void*)&c2nb, &k2_, &h_, &k_, &k2p_,
                    &emax_, &kp_, (void*)&p2i, (void*)&idsb, (void*)&scb, (void*)&enb};
    HIP_TRY(hipLaunchKernel(kern, dim3((unsigned)nb), dim3(RR_T), args, smem, s));
    return HF_OK;
  };
  uint32_t* flag = nullptr;
  if (bucketed) HF_TRY(ws.alloc(&flag, (size_t)batch));
  for (int64_t q0 = 0; q0 < nq; q0 += batch) {
    const int64_t nb = std::min(batch, nq - q0);
    if (bucketed) {
      {
        StageTimer tm(ST_HAM, s);
        HF_TRY(bfilter_run(f, T, len, nb, win + q0 * T, qsk + q0 * 8, k2, c2 + q0 * k2, c2n + q0, flag, ws));
      }
      if (getenv("HF_FILTER_STATS")) {  // diagnostic: how many queries the exact fallback redoes
        std::vector<uint32_t> fl((size_t)nb);
        HIP_TRY(hipMemcpyAsync(fl.data(), flag, 4 * (size_t)nb, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        int64_t redo = 0;
        for (uint32_t v : fl) redo += v != 0;
        fprintf(stderr, "hf filter: %lld of %lld queries redone entry by entry\n", (long long)redo, (long long)nb);
      }
    }
    {
      // the entry-by-entry filter: every query, or the queries the bucketed
      // filter flagged (the others' workgroups return at once)
      StageTimer tm(bucketed ? ST_SELECT : ST_HAM, s);
      const uint64_t mlen = ((1ull << 32) + (uint64_t)len - 1) / (uint64_t)len;
      // the few queries the bucketed filter flags are spread over many
      // workgroups: 64 slices each (one 1,024-thread workgroup a query took
      // 0.23 ms for 9 flagged queries of 10,000)
      if (bucketed) {
        k_ham_ctr_zero<<<1, 1, 0, s>>>(fctr);
        k_ham_flagged<<<(unsigned)ceil_div(nb, 4), 256, 0, s>>>(flag, nb, hist, flist, fctr);
        k_ham_split<1024><<<(unsigned)(2 * ncu), 1024, sizeof(uint32_t) * (size_t)T, s>>>(
            f->tree_perm, N, T, len, mlen, per_q, win + q0 * T, f->sk_pos, qsk + q0 * 8, ham, hist, flist, fctr,
            64);
      } else
        k_ham<256><<<(unsigned)nb, 256, sizeof(uint32_t) * (size_t)T, s>>>(
            f->tree_perm, N, T, len, mlen, per_q, win + q0 * T, f->sk_pos, qsk + q0 * 8, ham, hist, flag);
      HF_LAUNCH_CHECK();
    }
    {
      StageTimer tm(ST_SELECT, s);
      k_select<<<(unsigned)nb, SEL_T, 0, s>>>(f->tree_perm, N, T, len, per_q, win + q0 * T, ham, hist, k2,
                                              pos_bits, c2 + q0 * k2, c2n + q0, flag);
      HF_LAUNCH_CHECK();
    }
    if (p.precision == HF_PREC_FP32) {
      StageTimer tm(ST_RERANK, s);
      HF_TRY(rerank(q0, nb));
    } else if (p.precision == HF_PREC_C4) {
      StageTimer tm(ST_RERANK, s);
      HF_TRY(rerank_c4_launch(f, (const char*)Q + q0 * d * esz, nb, c2 + q0 * k2, c2n + q0, k2, (int)p.h,
                              (int)p.k, ids + q0 * p.k, scores + q0 * p.k, en_out ? en_out + q0 : nullptr, s));
    } else {
      StageTimer tm(ST_LOWPREC, s);
      const int S = (int)(p.survivors ? p.survivors : 4 * p.k);
      HF_TRY(rerank_lp_launch(f, (hf_precision)p.precision, (const char*)Q + q0 * d * esz, nb, c2 + q0 * k2,
                              c2n + q0, k2, (int)p.h, (int)p.k, S, ids + q0 * p.k, scores + q0 * p.k,
                              surv_pos ? surv_pos + q0 * S : nullptr, surv_score ? surv_score + q0 * S : nullptr,
                              en_out ? en_out + q0 : nullptr, s));
    }
  }
  return HF_OK;
}

}  // namespace hf
