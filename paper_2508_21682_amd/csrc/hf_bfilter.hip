// Hamming filter of Algorithm 1's second stage, organised by master-position
// bucket so that each sketch line read from HBM serves every window entry of
// the query batch that names it.
//
// A batch of nb queries holds nb * n * k1 window entries (one per query, tree
// and window offset), each naming a master position whose 64-byte sketch is
// compared with the query's.  Read entry by entry, each comparison is a
// random 64-byte read (a whole 128-byte line) and the batch reads every sketch
// line about n * k1 * nb / N times.  Here the entries are first regrouped by
// bucket (2^bb consecutive master positions, whose sketches fit one XCD's L2),
// then each bucket's entries are scored while its sketches sit in L2:
//
//   tau     per query, the Hamming distances of a sample of its trees give a
//           threshold tau_q expected to pass a few times k2 entries;
//   count   per query, its entries per bucket (bucket-major counts);
//   scan    bucket-major exclusive scan: every (bucket, query) run of entries
//           gets its place in one array of 4-byte records (query, offset in
//           bucket), query-major within a bucket;
//   scatter per query, its entries written to their runs;
//   score   persistent workgroups take chunks of one bucket at a time, each
//           XCD its own share of buckets; an entry whose distance is at most
//           tau_q appends (distance << 32 | position) to its query's list;
//   select  per query, the list sorted; the first k2 distinct keys are C2
//           when at least k2 distinct keys passed (C2's k2 smallest keys all
//           have distance <= tau_q then) or when tau_q let every entry pass.
//           Otherwise, or when the list overflowed, the query is flagged and
//           the caller runs the entry-by-entry filter for it, so C2 is
//           always the exact first k2 of the union by (Hamming, position).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "hf_internal.h"
#include "hf_select.h"

namespace hf {
namespace {

constexpr int BF_T = 256;        // threads of the count, scatter, tau and score workgroups
constexpr int BF_XCD = 8;        // XCDs of an MI355X: workgroup i runs on XCD i mod 8
constexpr int BF_SEL_T = 512;
constexpr int HBINS = 513;       // Hamming distances 0..512

struct EntryMap {
  const uint32_t* tree_perm;
  int64_t N;
  int len;
  uint64_t mlen;  // ceil(2^32 / len): t = (e * mlen) >> 32 is floor(e / len) or one more
  __device__ __forceinline__ uint32_t pos(const uint32_t* s_win, uint32_t e) const {
    uint32_t t = (uint32_t)(((uint64_t)e * mlen) >> 32);
    t -= t * (uint32_t)len > e ? 1u : 0u;
    return tree_perm[(int64_t)t * N + s_win[t] + (e - t * (uint32_t)len)];
  }
};

// Threshold per query from the trees t = j * tstride, j < Ts: the smallest h
// whose sampled count reaches need_s + 3 sqrt(need_s) + 1 (need_s = the wanted
// count scaled to the sample), 512 (every entry passes) if none does.
__global__ __launch_bounds__(BF_T) void k_tau(const uint32_t* __restrict__ tree_perm, int64_t N, int T, int len,
                                              int tstride, int Ts, const uint32_t* __restrict__ win,
                                              const uint64_t* __restrict__ sk, const uint64_t* __restrict__ qsk,
                                              float need_s, uint32_t* __restrict__ tau) {
  __shared__ uint32_t h[HBINS + 1];
  const int64_t q = blockIdx.x;
  for (int i = threadIdx.x; i <= HBINS; i += BF_T) h[i] = 0;
  const uint32_t total = (uint32_t)Ts * (uint32_t)len;
  // four lanes per entry, each on 16 bytes of its sketch (one 64-byte run)
  constexpr int R = 8;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, qd = lane >> 2, part = lane & 3;
  const uint4 qp = ((const uint4*)(qsk + q * 8))[part];
  __syncthreads();
  for (uint32_t e0 = 16u * R * wv; e0 < total; e0 += 16u * R * (BF_T / 64)) {
    uint4 sv[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      uint32_t e = e0 + 16u * u + qd;
      e = e < total ? e : total - 1u;
      const uint32_t j = e / (uint32_t)len, i = e - j * (uint32_t)len;
      const int64_t t = (int64_t)j * tstride;
      const uint32_t p = tree_perm[t * N + win[q * T + t] + i];
      sv[u] = ((const uint4*)(sk + (int64_t)p * 8))[part];
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      uint32_t hv = __popc(sv[u].x ^ qp.x) + __popc(sv[u].y ^ qp.y) + __popc(sv[u].z ^ qp.z) + __popc(sv[u].w ^ qp.w);
      hv += (uint32_t)__shfl_xor((int)hv, 1);
      hv += (uint32_t)__shfl_xor((int)hv, 2);
      if (part == 0 && e0 + 16u * u + qd < total) atomicAdd(&h[hv], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float want = need_s + 3.0f * sqrtf(need_s) + 1.0f;
    uint32_t cum = 0, t = HBINS - 1;
    for (int i = 0; i < HBINS; ++i) {
      cum += h[i];
      if ((float)cum >= want) {
        t = (uint32_t)i;
        break;
      }
    }
    tau[q] = t;
  }
}

// Entries of query q per bucket, written bucket-major: cnt[b * nb + q].  Also
// clears the query's candidate count.
__global__ __launch_bounds__(BF_T) void k_bcount(EntryMap em, int T, const uint32_t* __restrict__ win, int bb,
                                                 int nbk, int64_t nb, uint32_t* __restrict__ cnt,
                                                 uint32_t* __restrict__ ccnt) {
  extern __shared__ uint32_t lds[];  // nbk counters, then T window starts
  uint32_t* c = lds;
  uint32_t* s_win = lds + nbk;
  const int64_t q = blockIdx.x;
  for (int i = threadIdx.x; i < nbk; i += BF_T) c[i] = 0;
  for (int t = threadIdx.x; t < T; t += BF_T) s_win[t] = win[q * T + t];
  if (threadIdx.x == 0) ccnt[q] = 0;
  __syncthreads();
  const uint32_t total = (uint32_t)T * (uint32_t)em.len;
  constexpr int U = 16;  // position loads in flight per thread
  for (uint32_t e0 = threadIdx.x; e0 < total; e0 += BF_T * U) {
    uint32_t p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t e = e0 + u * BF_T;
      p[u] = em.pos(s_win, e < total ? e : total - 1u);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * BF_T < total) atomicAdd(&c[p[u] >> bb], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbk; b += BF_T) cnt[(int64_t)b * nb + q] = c[b];
}

// Exclusive scan of one bucket's row cnt[b][0..nb) in place; tot[b] = its sum.
constexpr int BS_T = 1024;
__global__ __launch_bounds__(BS_T) void k_brow_scan(uint32_t* __restrict__ cnt, int64_t nb,
                                                   uint32_t* __restrict__ tot) {
  __shared__ uint32_t tmp[BS_T / 64 + 1];
  uint32_t* row = cnt + (int64_t)blockIdx.x * nb;
  const int64_t per = (nb + BS_T - 1) / BS_T;
  const int64_t a0 = (int64_t)threadIdx.x * per, a1 = min<int64_t>(nb, a0 + per);
  uint32_t mine = 0;
  for (int64_t i = a0; i < a1; ++i) mine += row[i];
  uint32_t total;
  uint32_t run = block_excl_scan<BS_T>(mine, tmp, &total);
  for (int64_t i = a0; i < a1; ++i) {
    const uint32_t v = row[i];
    row[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// Bucket bases (exclusive scan of tot) and each XCD's chunk list: XCD x takes
// the buckets b = x, x + 8, ...; cumx[x * (nbx + 1) + i] = chunks of its first
// i buckets.  Clears the XCDs' work counters.
__global__ __launch_bounds__(BS_T) void k_bplan(const uint32_t* __restrict__ tot, int nbk, int nbx, uint32_t chunk,
                                               uint32_t* __restrict__ base, uint32_t* __restrict__ cumx,
                                               uint32_t* __restrict__ next) {
  __shared__ uint32_t tmp[BS_T / 64 + 1];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  if (threadIdx.x < BF_XCD) next[threadIdx.x] = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nbk; b0 += BS_T) {
    const int b = b0 + threadIdx.x;
    const uint32_t v = b < nbk ? tot[b] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan<BS_T>(v, tmp, &total);
    if (b < nbk) base[b] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
  for (int x = 0; x < BF_XCD; ++x) {
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int i0 = 0; i0 < nbx; i0 += BS_T) {
      const int i = i0 + threadIdx.x, b = i * BF_XCD + x;
      const uint32_t v = (i < nbx && b < nbk) ? (tot[b] + chunk - 1) / chunk : 0u;
      uint32_t total;
      const uint32_t ex = block_excl_scan<BS_T>(v, tmp, &total);
      if (i < nbx) cumx[x * (nbx + 1) + i] = carry + ex;
      __syncthreads();
      if (threadIdx.x == 0) carry += total;
      __syncthreads();
    }
    if (threadIdx.x == 0) cumx[x * (nbx + 1) + nbx] = carry;
    __syncthreads();
  }
}

// Records (q << bb | position within bucket) of query q written to its runs.
// The query's entries go through LDS SC_CH at a time, counting-sorted by
// bucket, so that consecutive lanes store consecutive records of one run
// instead of one scattered 4-byte store per entry.
template <int SC_T, int SC_PER>
__global__ __launch_bounds__(SC_T) __attribute__((amdgpu_waves_per_eu(4))) void k_bscatter(EntryMap em, int T, const uint32_t* __restrict__ win, int bb,
                                                   int nbk, int64_t nb, const uint32_t* __restrict__ cnt,
                                                   const uint32_t* __restrict__ base,
                                                   uint32_t* __restrict__ rec) {
  // nbk next global slots, nbk chunk counts, nbk chunk offsets, T window
  // starts, SC_CH master positions (4 bytes an entry: the bucket and the
  // record both follow from the position)
  constexpr int SC_CH = SC_T * SC_PER;
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t scan_tmp[SC_T / 64 + 1];
  uint32_t* gslot = lds;
  uint32_t* lc = gslot + nbk;
  uint32_t* offs = lc + nbk;
  uint32_t* s_win = offs + nbk;
  uint32_t* spos = s_win + T;
  const int64_t q = blockIdx.x;
  for (int b = threadIdx.x; b < nbk; b += SC_T) gslot[b] = base[b] + cnt[(int64_t)b * nb + q];
  for (int t = threadIdx.x; t < T; t += SC_T) s_win[t] = win[q * T + t];
  const uint32_t total = (uint32_t)T * (uint32_t)em.len;
  const uint32_t qtag = (uint32_t)q << bb, pmask = (1u << bb) - 1u;
  const int per = (nbk + SC_T - 1) / SC_T;
  const int a0 = threadIdx.x * per, a1 = min(nbk, a0 + per);
  for (uint32_t c0 = 0; c0 < total; c0 += SC_CH) {
    const uint32_t n = min((uint32_t)SC_CH, total - c0);
    for (int b = threadIdx.x; b < nbk; b += SC_T) lc[b] = 0;
    __syncthreads();
    uint32_t p[SC_PER], r[SC_PER];
#pragma unroll
    for (int u = 0; u < SC_PER; ++u) {
      const uint32_t e = c0 + u * SC_T + threadIdx.x;
      p[u] = em.pos(s_win, e < total ? e : total - 1u);
    }
#pragma unroll
    for (int u = 0; u < SC_PER; ++u)
      r[u] = (u * SC_T + threadIdx.x < n) ? atomicAdd(&lc[p[u] >> bb], 1u) : 0u;
    __syncthreads();
    uint32_t mine = 0;
    for (int i = a0; i < a1; ++i) mine += lc[i];
    uint32_t tot;
    uint32_t run = block_excl_scan<SC_T>(mine, scan_tmp, &tot);
    for (int i = a0; i < a1; ++i) {
      offs[i] = run;
      run += lc[i];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SC_PER; ++u)
      if (u * SC_T + threadIdx.x < n) spos[offs[p[u] >> bb] + r[u]] = p[u];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += SC_T) {
      const uint32_t pp = spos[i], b = pp >> bb;
      rec[gslot[b] + (i - offs[b])] = qtag | (pp & pmask);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbk; b += SC_T) gslot[b] += lc[b];
  }
}

// LDS staging of a chunk's passing entries: appended with LDS atomics while
// scoring, then flushed with one global atomic per query of the chunk.
constexpr int QS_MAX = 128;  // queries of a chunk staged in LDS
constexpr int CB = 1024;     // passing entries a chunk stages in LDS
struct ChunkLds {
  uint4 qs[QS_MAX][4];   // sketches of the chunk's queries
  uint32_t tau[QS_MAX];  // their thresholds
  uint32_t qc[QS_MAX];   // passing entries per query (then: fill counters)
  uint32_t qbase[QS_MAX];
  uint64_t key[CB];
  uint16_t ql[CB];
  uint32_t nc;
};

// Appends (hv, p) to query q's global list directly: one returning atomic per
// query among the wavefront's passing lanes.
__device__ __forceinline__ void append_global(bool pass, uint32_t q, uint64_t key, uint64_t* __restrict__ cand,
                                              uint32_t* __restrict__ ccnt, int capc) {
  const int lane = threadIdx.x & 63;
  uint64_t m = __ballot(pass);
  while (m) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    const uint32_t ql = (uint32_t)__shfl((int)q, leader);
    const uint64_t mq = __ballot(pass && q == ql);
    uint32_t slot = 0;
    if (lane == leader) slot = atomicAdd(&ccnt[ql], (uint32_t)__popcll(mq));
    slot = (uint32_t)__shfl((int)slot, leader) + (uint32_t)__popcll(mq & lanemask_lt());
    if (pass && q == ql && slot < (uint32_t)capc) cand[(int64_t)q * capc + slot] = key;
    m &= ~mq;
  }
}

// Scores records [r0, r1) of one bucket.  Four lanes share a record: lane
// part j reads bytes 16 j .. 16 j + 15 of the entry's sketch, so the four
// lanes' loads fall on one 64-byte run (one cache-line access for the
// record, not one per 16 bytes), and a DPP quad sum gives the distance.  A
// wavefront takes R rounds of 16 records at a time, every record and sketch
// load of the R rounds in flight together; no load or store is conditional
// (past r1 the last record is re-read and its entry cannot pass), so the
// loads never wait on a branch.  STAGED: the chunk's queries
// q0 .. q0 + QS_MAX - 1 have their sketches and thresholds in LDS, and the
// passing entries of a batch are appended to the chunk's LDS list with one
// atomic per wavefront (the global lists directly once CB are staged).
template <bool STAGED, int SB>
__device__ __forceinline__ void score_chunk(const uint32_t* __restrict__ rec, uint32_t r0, uint32_t r1, uint32_t btag,
                                            int bb, const uint64_t* __restrict__ sk,
                                            const uint64_t* __restrict__ qsk, const uint32_t* __restrict__ tau,
                                            ChunkLds& L, uint32_t q0, uint64_t* __restrict__ cand,
                                            uint32_t* __restrict__ ccnt, int capc) {
  const uint32_t pmask = (1u << bb) - 1u;
  constexpr int NW = BF_T / 64, R = 4 * SB;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, qd = lane >> 2, part = lane & 3;
  for (uint32_t rb = r0 + 16u * R * wv; rb < r1; rb += 16u * R * NW) {
    uint32_t v[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const uint32_t r = rb + 16u * u + qd;
      v[u] = rec[r < r1 ? r : r1 - 1u];
    }
    uint4 sv[R];
#pragma unroll
    for (int u = 0; u < R; ++u) sv[u] = ((const uint4*)(sk + (int64_t)(btag | (v[u] & pmask)) * 8))[part];
    bool pass[R];
    uint32_t hvs[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const uint32_t q = v[u] >> bb;
      uint4 qs;
      uint32_t tq;
      if constexpr (STAGED) {
        qs = L.qs[q - q0][part];
        tq = L.tau[q - q0];
      } else {
        qs = ((const uint4*)(qsk + (int64_t)q * 8))[part];
        tq = tau[q];
      }
      uint32_t hv = __popc(sv[u].x ^ qs.x) + __popc(sv[u].y ^ qs.y) + __popc(sv[u].z ^ qs.z) + __popc(sv[u].w ^ qs.w);
      hv += quad_perm<QP_XOR1>(hv);
      hv += quad_perm<QP_XOR2>(hv);
      hvs[u] = hv;
      pass[u] = part == 0 && rb + 16u * u + qd < r1 && hv <= tq;
    }
    if constexpr (STAGED) {
      // slots of the batch's passing entries: one LDS atomic per wavefront
      uint64_t m[R];
      uint32_t tot = 0;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        m[u] = __ballot(pass[u]);
        tot += (uint32_t)__popcll(m[u]);
      }
      if (tot == 0) continue;
      uint32_t at = 0;
      if (lane == 0) at = atomicAdd(&L.nc, tot);
      at = (uint32_t)__shfl((int)at, 0);
      bool direct[R];
      bool any_direct = false;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const uint32_t slot = at + (uint32_t)__popcll(m[u] & lanemask_lt());
        at += (uint32_t)__popcll(m[u]);
        const uint32_t q = v[u] >> bb;
        direct[u] = pass[u] && slot >= (uint32_t)CB;
        any_direct |= direct[u];
        if (pass[u] && slot < (uint32_t)CB) {
          L.key[slot] = ((uint64_t)hvs[u] << 32) | (btag | (v[u] & pmask));
          L.ql[slot] = (uint16_t)(q - q0);
          atomicAdd(&L.qc[q - q0], 1u);
        }
      }
      if (__ballot(any_direct)) {
#pragma unroll
        for (int u = 0; u < R; ++u)
          append_global(direct[u], v[u] >> bb, ((uint64_t)hvs[u] << 32) | (btag | (v[u] & pmask)), cand, ccnt,
                        capc);
      }
    } else {
#pragma unroll
      for (int u = 0; u < R; ++u)
        append_global(pass[u], v[u] >> bb, ((uint64_t)hvs[u] << 32) | (btag | (v[u] & pmask)), cand, ccnt, capc);
    }
  }
}

// Persistent scoring: workgroup i starts on XCD i mod 8's chunk list and
// moves on to the other XCDs' lists once its own is used up; every list is
// finite, so every workgroup exits.  Records of a bucket are query-major, so
// a chunk usually spans few queries: their sketches and thresholds are staged
// in LDS when at most QS_MAX of them.
template <int SB>
__global__ __launch_bounds__(BF_T) void k_bscore(const uint32_t* __restrict__ rec, const uint32_t* __restrict__ base,
                                                 const uint32_t* __restrict__ tot,
                                                 const uint32_t* __restrict__ cumx, int nbx, int bb, uint32_t chunk,
                                                 uint32_t* __restrict__ next, const uint64_t* __restrict__ sk,
                                                 const uint64_t* __restrict__ qsk,
                                                 const uint32_t* __restrict__ tau, uint64_t* __restrict__ cand,
                                                 uint32_t* __restrict__ ccnt, int capc) {
  __shared__ ChunkLds L;
  __shared__ int s_j, s_b;
  __shared__ uint32_t s_r0, s_r1, s_q0, s_qn;
  const int x0 = blockIdx.x % BF_XCD;
  for (int xi = 0; xi < BF_XCD; ++xi) {
    const int x = (x0 + xi) % BF_XCD;
    const uint32_t* cx = cumx + x * (nbx + 1);
    const uint32_t nch = cx[nbx];
    for (;;) {
      if (threadIdx.x == 0) {
        const uint32_t j = atomicAdd(&next[x], 1u);
        s_j = (int)min(j, nch);
        if (j < nch) {
          int lo = 0, hi = nbx - 1;  // last i with cx[i] <= j
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cx[mid] <= j)
              lo = mid;
            else
              hi = mid - 1;
          }
          const int b = lo * BF_XCD + x;
          const uint32_t r0 = base[b] + (j - cx[lo]) * chunk;
          const uint32_t r1 = min(base[b] + tot[b], r0 + chunk);
          s_b = b;
          s_r0 = r0;
          s_r1 = r1;
          s_q0 = rec[r0] >> bb;
          s_qn = (rec[r1 - 1u] >> bb) - s_q0 + 1u;
        }
        L.nc = 0;
      }
      __syncthreads();
      const uint32_t j = (uint32_t)s_j;
      const int b = s_b;
      const uint32_t r0 = s_r0, r1 = s_r1, q0 = s_q0, qn = s_qn;
      if (j >= nch) {
        __syncthreads();
        break;
      }
      const uint32_t btag = (uint32_t)b << bb;
      if (qn <= (uint32_t)QS_MAX) {
        for (uint32_t i = threadIdx.x; i < qn * 4u; i += BF_T)
          L.qs[i >> 2][i & 3] = ((const uint4*)(qsk + (int64_t)(q0 + (i >> 2)) * 8))[i & 3];
        for (uint32_t i = threadIdx.x; i < qn; i += BF_T) {
          L.tau[i] = tau[q0 + i];
          L.qc[i] = 0;
        }
        __syncthreads();
        score_chunk<true, SB>(rec, r0, r1, btag, bb, sk, qsk, tau, L, q0, cand, ccnt, capc);
        __syncthreads();
        // one global atomic per query of the chunk reserves its entries' slots
        for (uint32_t i = threadIdx.x; i < qn; i += BF_T) {
          const uint32_t c = L.qc[i];
          L.qbase[i] = c ? atomicAdd(&ccnt[q0 + i], c) : 0u;
          L.qc[i] = 0;
        }
        __syncthreads();
        const uint32_t nc = min(L.nc, (uint32_t)CB);
        for (uint32_t i = threadIdx.x; i < nc; i += BF_T) {
          const uint32_t ql = L.ql[i];
          const uint32_t slot = L.qbase[ql] + atomicAdd(&L.qc[ql], 1u);
          if (slot < (uint32_t)capc) cand[(int64_t)(q0 + ql) * capc + slot] = L.key[i];
        }
      } else {
        score_chunk<false, SB>(rec, r0, r1, btag, bb, sk, qsk, tau, L, q0, cand, ccnt, capc);
      }
      __syncthreads();
    }
  }
}

// Smallest bin b of h[0..HBINS) whose inclusive prefix sum reaches `want`
// (HBINS - 1 if none), and the sum of all bins; by the whole workgroup, two
// bins a thread (BF_SEL_T * 2 >= HBINS).
__device__ __forceinline__ uint32_t hist_cut(const uint32_t* h, uint32_t want, uint32_t* scan_tmp, uint32_t* s_cut,
                                             uint32_t* total) {
  const int b0 = 2 * threadIdx.x, b1 = b0 + 1;
  const uint32_t c0 = b0 < HBINS ? h[b0] : 0u, c1 = b1 < HBINS ? h[b1] : 0u;
  if (threadIdx.x == 0) *s_cut = HBINS - 1;
  const uint32_t ex = block_excl_scan<BF_SEL_T>(c0 + c1, scan_tmp, total);  // has barriers
  if (ex < want && ex + c0 >= want) atomicMin(s_cut, (uint32_t)b0);
  else if (ex + c0 < want && ex + c0 + c1 >= want) atomicMin(s_cut, (uint32_t)b1);
  __syncthreads();
  return *s_cut;
}

// C2 of a query from its candidate list, or the query flagged for the
// entry-by-entry filter.  The list (at most capc keys) is read once into
// registers, PER keys a thread.  A key's position is inserted into an LDS hash
// set (2 capc slots, linear probing): the first insertion of a position marks
// the distinct key (one position always carries the same distance).  The
// distinct keys' distance histogram gives the cut at k2 distinct keys; only
// the distinct keys within the cut are sorted (in the same LDS).  The sorted
// distinct keys' first k2 are C2 when at least k2 distinct keys passed, or
// all of them when tau let every entry pass; otherwise the query is flagged.
template <int PER>
__global__ __launch_bounds__(BF_SEL_T) void k_bselect(const uint64_t* __restrict__ cand,
                                                      const uint32_t* __restrict__ ccnt,
                                                      const uint32_t* __restrict__ tau, int capc, int k2,
                                                      uint32_t* __restrict__ c2, int32_t* __restrict__ c2n,
                                                      uint32_t* __restrict__ flag) {
  extern __shared__ uint64_t keys[];  // capc keys; first the hash set's 2 capc slots
  uint32_t* hs = (uint32_t*)keys;
  __shared__ uint32_t hist[HBINS];
  __shared__ uint32_t scan_tmp[BF_SEL_T / 64 + 1];
  __shared__ uint32_t s_cut, s_cnt;
  const int64_t q = blockIdx.x;
  const uint32_t n = ccnt[q];
  if (n > (uint32_t)capc) {
    if (threadIdx.x == 0) flag[q] = 1;
    return;
  }
  const uint64_t* cq = cand + q * capc;
  uint64_t v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const uint32_t i = threadIdx.x + (uint32_t)j * BF_SEL_T;
    v[j] = i < n ? cq[i] : ~0ull;
  }
  const uint32_t hmask = 2u * (uint32_t)capc - 1u;
  for (uint32_t i = threadIdx.x; i <= hmask; i += BF_SEL_T) hs[i] = NONE32;
  for (int i = threadIdx.x; i < HBINS; i += BF_SEL_T) hist[i] = 0;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  uint32_t first = 0;  // bit j: v[j] is its position's first key
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if (threadIdx.x + (uint32_t)j * BF_SEL_T < n) {
      const uint32_t pos = (uint32_t)v[j];
      uint32_t slot = (pos * 0x9E3779B1u) & hmask;
      for (;;) {  // the set has 2 capc >= 2 n slots, so a free one exists
        const uint32_t old = atomicCAS(&hs[slot], NONE32, pos);
        if (old == NONE32) {
          first |= 1u << j;
          break;
        }
        if (old == pos) break;
        slot = (slot + 1u) & hmask;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < PER; ++j)
    if (first >> j & 1u) atomicAdd(&hist[(uint32_t)(v[j] >> 32)], 1u);
  __syncthreads();
  uint32_t distinct;
  const uint32_t cut = hist_cut(hist, (uint32_t)k2, scan_tmp, &s_cut, &distinct);
  if (distinct < (uint32_t)k2 && tau[q] < HBINS - 1) {
    if (threadIdx.x == 0) flag[q] = 1;
    return;
  }
  // the hash set is no longer read: its LDS takes the distinct keys within the cut
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const bool take = (first >> j & 1u) && (uint32_t)(v[j] >> 32) <= cut;
    const uint64_t m = __ballot(take);
    if (m) {
      const int lane = threadIdx.x & 63, leader = __ffsll((unsigned long long)m) - 1;
      uint32_t at = 0;
      if (lane == leader) at = atomicAdd(&s_cnt, (uint32_t)__popcll(m));
      at = (uint32_t)__shfl((int)at, leader);
      if (take) keys[at + (uint32_t)__popcll(m & lanemask_lt())] = v[j];
    }
  }
  __syncthreads();
  const int m = (int)s_cnt;
  int n2 = 1;
  while (n2 < m) n2 <<= 1;
  for (int i = m + threadIdx.x; i < n2; i += BF_SEL_T) keys[i] = ~0ull;
  __syncthreads();
  bitonic_u64(keys, n2);
  const int took = min(k2, m);
  for (int i = threadIdx.x; i < k2; i += BF_SEL_T) c2[q * k2 + i] = i < took ? (uint32_t)keys[i] : NONE32;
  if (threadIdx.x == 0) {
    c2n[q] = took;
    flag[q] = 0;
  }
}

}  // namespace

// Bucket bits: buckets of 2^bb positions (64 * 2^bb bytes of sketches), at
// most 2,048 of them (LDS counters of the count and scatter kernels).
int bfilter_bucket_bits(int64_t N) {
  int bb = 15;
  const char* env = getenv("HF_FILTER_BUCKET_BITS");
  if (env) bb = std::max(8, std::min(24, atoi(env)));
  while ((ceil_div(N, (int64_t)1 << bb)) > 2048) ++bb;
  return bb;
}

// Candidate-list capacity: the threshold passes about 7 k2 entries (3.5 k2
// aimed at, plus the sample's margin and the ties at the threshold).
int bfilter_capacity(int k2) {
  int c = 2048;
  while (c < 7 * k2) c <<= 1;
  return c;
}

bool bfilter_usable(int64_t N, int T, int k2) {
  const char* env = getenv("HF_FILTER");
  if (env && strcmp(env, "direct") == 0) return false;
  // candidate lists sorted in LDS; at most 2^(32 - bb) queries a batch
  return bfilter_capacity(k2) <= 16384 && T <= 4096 && N >= 1;
}

int64_t bfilter_max_batch(int64_t N) { return (int64_t)1 << (32 - bfilter_bucket_bits(N)); }

hf_status bfilter_run(const hf_forest* f, int T, int len, int64_t nb, const uint32_t* win, const uint64_t* qsk,
                      int k2, uint32_t* c2, int32_t* c2n, uint32_t* flag, Workspace& ws) {
  hipStream_t s = ws.stream;
  const int64_t N = f->N;
  const int bb = bfilter_bucket_bits(N);
  const int nbk = (int)ceil_div(N, (int64_t)1 << bb);
  const int nbx = (int)ceil_div(nbk, BF_XCD);
  const int capc = bfilter_capacity(k2);
  const int64_t entries = nb * (int64_t)T * len;
  uint32_t *tau, *cnt, *tot, *base, *cumx, *next, *rec, *ccnt;
  uint64_t* cand;
  HF_TRY(ws.alloc(&tau, (size_t)nb));
  HF_TRY(ws.alloc(&cnt, (size_t)nbk * nb));
  HF_TRY(ws.alloc(&tot, (size_t)nbk));
  HF_TRY(ws.alloc(&base, (size_t)nbk));
  HF_TRY(ws.alloc(&cumx, (size_t)BF_XCD * (nbx + 1)));
  HF_TRY(ws.alloc(&next, (size_t)BF_XCD));
  HF_TRY(ws.alloc(&rec, (size_t)entries));
  HF_TRY(ws.alloc(&ccnt, (size_t)nb));
  HF_TRY(ws.alloc(&cand, (size_t)nb * capc));
  // threshold from about 1/32 of the trees (all of them for small forests)
  const int tstride = std::max(1, T / 32);
  const int Ts = (int)ceil_div(T, tstride);
  // a near neighbour sits in the windows of many trees, so the lowest
  // distances hold many repeats: aim at 3.5 k2 entries for k2 distinct ones
  const float need_s = 3.5f * (float)k2 * (float)Ts / (float)T;
  k_tau<<<(unsigned)nb, BF_T, 0, s>>>(f->tree_perm, N, T, len, tstride, Ts, win, f->sk_pos, qsk, need_s, tau);
  HF_LAUNCH_CHECK();
  EntryMap em{f->tree_perm, N, len, ((1ull << 32) + (uint64_t)len - 1) / (uint64_t)len};
  const size_t lds = sizeof(uint32_t) * ((size_t)nbk + T);
  k_bcount<<<(unsigned)nb, BF_T, lds, s>>>(em, T, win, bb, nbk, nb, cnt, ccnt);
  HF_LAUNCH_CHECK();
  k_brow_scan<<<(unsigned)nbk, BS_T, 0, s>>>(cnt, nb, tot);
  HF_LAUNCH_CHECK();
  // records per chunk of the scoring kernel's work lists
  constexpr uint32_t chunk = 8192;
  k_bplan<<<1, BS_T, 0, s>>>(tot, nbk, nbx, chunk, base, cumx, next);
  HF_LAUNCH_CHECK();
  int dev = 0, ncu = 256, max_lds = 64 * 1024;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // entries counting-sorted per pass of the scatter kernel by 1024 threads:
  // 32,768 at a time when LDS holds them, else 16,384.  Longer passes give
  // each (bucket, query) run fewer, longer pieces: the stage took 10.7
  // against 11.2 ms per 10,000 queries at 1,280 x 70 (512 x 32, two
  // workgroups a CU: no faster than 1024 x 16)
  const size_t sc_fixed = 3 * (size_t)nbk + T;
  const bool sc_big = sizeof(uint32_t) * (sc_fixed + 32768) + 1024 <= (size_t)max_lds;
  const size_t sc_lds = sizeof(uint32_t) * (sc_fixed + (sc_big ? 32768 : 16384));
  if (sc_big) {
    HIP_TRY(hipFuncSetAttribute((const void*)k_bscatter<1024, 32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sc_lds));
    k_bscatter<1024, 32><<<(unsigned)nb, 1024, sc_lds, s>>>(em, T, win, bb, nbk, nb, cnt, base, rec);
  } else {
    if (sc_lds + 1024 > 64 * 1024)  // dynamic + static LDS above the default limit
      HIP_TRY(hipFuncSetAttribute((const void*)k_bscatter<1024, 16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)sc_lds));
    k_bscatter<1024, 16><<<(unsigned)nb, 1024, sc_lds, s>>>(em, T, win, bb, nbk, nb, cnt, base, rec);
  }
  HF_LAUNCH_CHECK();
  const unsigned grid = (unsigned)std::max(BF_XCD, (ncu * 8 + BF_XCD - 1) / BF_XCD * BF_XCD);
  // two record blocks of 64 in flight per wavefront (three or four: lower
  // occupancy, slower)
  k_bscore<2><<<grid, BF_T, 0, s>>>(rec, base, tot, cumx, nbx, bb, chunk, next, f->sk_pos, qsk, tau, cand, ccnt,
                                    capc);
  HF_LAUNCH_CHECK();
  const size_t sel_lds = sizeof(uint64_t) * (size_t)capc;
  switch (capc / BF_SEL_T) {
#define HF_BSEL(P)                                                                                            \
  case P:                                                                                                     \
    if (sel_lds + 1024 > 64 * 1024)                                                                           \
      HIP_TRY(hipFuncSetAttribute((const void*)k_bselect<P>, hipFuncAttributeMaxDynamicSharedMemorySize,      \
                                  (int)sel_lds));                                                             \
    k_bselect<P><<<(unsigned)nb, BF_SEL_T, sel_lds, s>>>(cand, ccnt, tau, capc, k2, c2, c2n, flag);           \
    break;
    HF_BSEL(4)
    HF_BSEL(8)
    HF_BSEL(16)
    HF_BSEL(32)
#undef HF_BSEL
    default:
      set_error("candidate capacity %d has no selection kernel", capc);
      return HF_ERR_UNSUPPORTED;
  }
  HF_LAUNCH_CHECK();
  return HF_OK;
}

}  // namespace hf
