// k-NN graph from windows along several Hilbert orders (Section 4.1,
// Algorithm 2).  Per order: Hilbert sort of all points, then a band kernel.
//
// Orders are pipelined: a second stream sorts and gathers order t+1 while the
// band kernel of order t runs on the caller's stream.
//
// Band kernel: a workgroup owns 64 consecutive positions of the order, a
// wavefront 16 of them.  Their rows (fp16, gathered through the order) stay in
// registers as the A operand of v_mfma_f32_16x16x32_f16; the rows of each
// 16-position block within +-w stream through a shared LDS tile as the B
// operand, so every MFMA tile is a 16x16 block of dot products along the
// band.  All 64 lanes screen the tile's pairs against each row's k-th entry;
// cosines (FP32 accumulate, FP32 norms) of the survivors with 0 < |i-j| <= w
// are queued per row in LDS and merged by the row's owner lane into that
// point's top-k list (cosine desc, id asc), held in registers while the wave
// runs and in HBM between orders.  A candidate already in the list is skipped; one that
// was evicted earlier is evicted again (its score is fixed), so the list
// stays the top-k of the union of all windows seen.
#include <math.h>
#include <stdlib.h>

#include "hf_internal.h"

namespace hf {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

// Row norms into nrm[p * stride].  With stride 4 the rest of each record
// (the band kernel's point record: norm, k-th cosine of the point's list,
// the counts of its two mailboxes) is set to -inf (the mark of a list not
// yet full) and two zero counts.
__global__ void k_norms(const __half* __restrict__ X, int64_t N, int d, float* __restrict__ nrm,
                        int stride = 1) {
  int64_t p = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (p >= N) return;
  float a = 0.f;
  for (int i = __lane_id(); i < d; i += 64) {
    float v = __half2float(X[p * d + i]);
    a = fmaf(v, v, a);
  }
  for (int m = 32; m >= 1; m >>= 1) a += __shfl_xor(a, m);
  if (__lane_id() == 0) {
    if (stride == 4)
      ((float4*)nrm)[p] = make_float4(sqrtf(a), -INFINITY, 0.f, 0.f);
    else
      nrm[p * stride] = sqrtf(a);
  }
}

// The band kernel's working lists: per point the KMAX (cosine, id) slots of
// its top-k list as a TopList holds them (KMAX - k sentinels, then the k
// entries, the k-th in the last slot), 8 bytes a slot: one 128-byte line a
// point at KMAX = 16.
__global__ void k_init_slots(uint2* __restrict__ slots, int64_t n, int kmax, int k) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n * kmax; i += (int64_t)gridDim.x * 256) {
    const bool sentinel = (int)(i % kmax) < kmax - k;
    slots[i] = sentinel ? make_uint2(__float_as_uint(INFINITY), (uint32_t)-2)
                        : make_uint2(__float_as_uint(-INFINITY), (uint32_t)-1);
  }
}

// The lists out of the working slots: ids (-1 where fewer than k) and cosines.
__global__ void k_slots_out(const uint2* __restrict__ slots, int64_t n, int kmax, int k,
                            int32_t* __restrict__ ids, float* __restrict__ sc) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n * k; i += (int64_t)gridDim.x * 256) {
    const int64_t p = i / k;
    const uint2 e = slots[p * kmax + kmax - k + (i - p * k)];
    sc[i] = __uint_as_float(e.x);
    ids[i] = (int32_t)e.y;
  }
}

__device__ __forceinline__ bool better(float s1, int32_t c1, float s2, int32_t c2) {
  return s1 > s2 || (s1 == s2 && (uint32_t)c1 < (uint32_t)c2);
}

// Top-k list of one row in registers, best first.  Rows with k < KMAX
// start with KMAX - k sentinels (+inf, id -2) that nothing displaces, so the
// k-th entry is always the last slot; empty slots are (-inf, -1).
template <int KMAX>
struct TopList {
  float ls[KMAX];
  int32_t li[KMAX];
  __device__ __forceinline__ float ws() const { return ls[KMAX - 1]; }
  __device__ __forceinline__ int32_t wi() const { return li[KMAX - 1]; }
  // slot i of the list holds entry i - (KMAX - k) of a k-list
  __device__ __forceinline__ void load(const float* sc, const int32_t* id, int k, bool valid) {
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      const int e = i - (KMAX - k);
      ls[i] = e < 0 ? INFINITY : -INFINITY;
      li[i] = e < 0 ? -2 : -1;
      if (valid && e >= 0) {
        ls[i] = sc[e];
        li[i] = id[e];
      }
    }
  }
  // whole slot arrays (sentinels included), 16-byte vectors of two slots
  __device__ __forceinline__ void load_slots(const uint4* src) {
#pragma unroll
    for (int j = 0; j < KMAX / 2; ++j) {
      const uint4 v = src[j];
      ls[2 * j] = __uint_as_float(v.x);
      li[2 * j] = (int32_t)v.y;
      ls[2 * j + 1] = __uint_as_float(v.z);
      li[2 * j + 1] = (int32_t)v.w;
    }
  }
  __device__ __forceinline__ void save_slots(uint4* dst) const {
#pragma unroll
    for (int j = 0; j < KMAX / 2; ++j)
      dst[j] = make_uint4(__float_as_uint(ls[2 * j]), (uint32_t)li[2 * j], __float_as_uint(ls[2 * j + 1]),
                          (uint32_t)li[2 * j + 1]);
  }
  __device__ __forceinline__ void save(float* sc, int32_t* id, int k) const {
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      const int e = i - (KMAX - k);
      if (e >= 0) {
        sc[e] = ls[i];
        id[e] = li[i];
      }
    }
  }
  // (s, c) enters unless it is listed already; the slots it beats (a suffix
  // of the list, empty slots included) shift down by one
  __device__ __forceinline__ void insert(float s, int32_t c) {
    bool dup = false;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) dup |= li[i] == c;
    if (dup) return;
    bool prev = false;
    float ps = 0.f;
    int32_t pi = 0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      const bool b = li[i] == -1 || better(s, c, ls[i], li[i]);
      const float os = ls[i];
      const int32_t oi = li[i];
      ls[i] = b ? (prev ? ps : s) : os;
      li[i] = b ? (prev ? pi : c) : oi;
      ps = os;
      pi = oi;
      prev = b;
    }
  }
};

// The top-k list of one row spread over four lanes of a wavefront: lane
// R + 16 j holds slots SPL j .. SPL j + SPL - 1 of row R, in the slot layout
// of TopList (KMAX - k sentinels first, the k-th entry in the last slot).
// The four lanes of a row insert together: each counts the slots of its own
// that stay ahead of the candidate, two xor-shuffles give the position, and
// every slot past it takes its predecessor (the first slot of a lane takes
// the last of the lane before).
template <int KMAX>
struct RowList {
  static constexpr int SPL = KMAX / 4;
  float ls[SPL];
  int32_t li[SPL];
  __device__ __forceinline__ void init(int k, int j) {
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
      const bool sentinel = SPL * j + q < KMAX - k;
      ls[q] = sentinel ? INFINITY : -INFINITY;
      li[q] = sentinel ? -2 : -1;
    }
  }
  // `row`: the point's KMAX / 2 16-byte vectors of slots
  __device__ __forceinline__ void load(const uint4* row, int j) {
#pragma unroll
    for (int v = 0; v < SPL / 2; ++v) {
      const uint4 x = row[j * (SPL / 2) + v];
      ls[2 * v] = __uint_as_float(x.x);
      li[2 * v] = (int32_t)x.y;
      ls[2 * v + 1] = __uint_as_float(x.z);
      li[2 * v + 1] = (int32_t)x.w;
    }
  }
  __device__ __forceinline__ void save(uint4* row, int j) const {
#pragma unroll
    for (int v = 0; v < SPL / 2; ++v)
      row[j * (SPL / 2) + v] = make_uint4(__float_as_uint(ls[2 * v]), (uint32_t)li[2 * v],
                                          __float_as_uint(ls[2 * v + 1]), (uint32_t)li[2 * v + 1]);
  }
  // called by the four lanes of the row together, with the same (s, c)
  __device__ __forceinline__ void insert(float s, int32_t c, int j) {
    int dup = 0, ahead = 0;
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
      dup |= li[q] == c;
      ahead += li[q] != -1 && !better(s, c, ls[q], li[q]);
    }
    dup |= __shfl_xor(dup, 16);
    dup |= __shfl_xor(dup, 32);
    ahead += __shfl_xor(ahead, 16);
    ahead += __shfl_xor(ahead, 32);
    const int src = (__lane_id() + 48) & 63;  // the row's lane before this one
    const float ps = __shfl(ls[SPL - 1], src);
    const int32_t pi = __shfl(li[SPL - 1], src);
    if (dup || ahead >= KMAX) return;
#pragma unroll
    for (int q = SPL - 1; q >= 0; --q) {
      const int g = SPL * j + q;
      const float os = q > 0 ? ls[q - 1] : ps;
      const int32_t oi = q > 0 ? li[q - 1] : pi;
      ls[q] = g > ahead ? os : (g == ahead ? s : ls[q]);
      li[q] = g > ahead ? oi : (g == ahead ? c : li[q]);
    }
  }
};

__device__ __forceinline__ half8 load_row8(const __half* __restrict__ X, int64_t r, int d, int k0) {
  if (r < 0 || k0 >= d) return (half8)(0);
  uint4 raw = *(const uint4*)(X + r * d + k0);
  return __builtin_bit_cast(half8, raw);
}

// Pairs sent to a point by the band kernel of one order, for its owner to
// merge in the next order: per point a count (point p's at n[4 p], a word of
// its record) and up to w (cosine, id) entries.
struct Mailbox {
  uint32_t* n;
  uint2* e;
};

// A workgroup (four wavefronts) owns 64 consecutive positions; wavefront v
// owns rows R0+16v .. +15.  Column blocks of 16 positions stream through a
// double-buffered LDS tile shared by the four wavefronts, BPS blocks per
// step, fetched two steps ahead (16-byte coalesced).  Rows are padded by 16
// bytes in LDS so the 16 lanes reading one column fragment hit distinct
// banks.  Rows are read from X through the order: the point ids of a tile
// reach LDS three steps ahead of its rows, so no global load waits on another.
//
// SYM: each pair of the band is computed once, by the owner of its lower
// position i: columns i+1 .. i+w only (blocks v .. v+wr of 4+wr).  The pair
// is screened against both points' thresholds (the column point's is read
// from its list in HBM: any value it held is a valid lower bound); the row
// side is queued as below, the column side goes to the column point's
// mailbox `mo`, which its owner merges in the next order (`mi`, whose counts
// it clears).  Otherwise every row meets columns i-w .. i+w (blocks
// v .. v+2wr of 4+2wr) and pairs are computed from both sides.
template <int KMAX, int KS, bool SYM>
__global__ __launch_bounds__(256, KMAX <= 16 && KS <= 12 ? 2 : 1) void k_band(const __half* __restrict__ X, int64_t N, int d,
                                              const uint32_t* __restrict__ order,
                                              float4* __restrict__ pt, int w, int k,
                                              uint4* __restrict__ slots, Mailbox mi, Mailbox mo) {
  constexpr int BPS = 2;           // column blocks per step
  constexpr int TR = 16 * BPS;     // tile rows
  // LDS row stride (halves): 32 bytes past a multiple of 256 bytes when
  // 4 | KS, so the B-fragment reads (16 rows x 4 chunks of 16 bytes) hit
  // distinct banks; 16 bytes past costs four conflict cycles a read
  constexpr int RS = KS * 32 + 16;
  constexpr int CPR = KS * 4;      // 16-byte chunks per tile row
  constexpr int CH = (TR * CPR + 255) / 256;  // chunks per thread per tile
  __shared__ __attribute__((aligned(16))) _Float16 tile[2][TR * RS];
  __shared__ int32_t tcid[3][TR];  // point ids of the tile rows of step q: slot q % 3
  __shared__ float tnrm[2][TR];
  __shared__ float tthr[2][TR];    // SYM: column thresholds in dot units / row norm
  constexpr int QCAP = 32;  // queued pairs per row (a block adds at most 16)
  __shared__ float qcs[4][16][QCAP];
  __shared__ int32_t qid[4][16][QCAP];
  __shared__ uint32_t qn[4][16];
  const int wv = threadIdx.x / 64, l = __lane_id();
  // workgroups are dealt to the eight XCDs in turn: give each XCD a
  // contiguous run of position blocks so neighbours share its L2
  const unsigned G = gridDim.x, per = G / 8, rem = G % 8, x8 = blockIdx.x % 8, j8 = blockIdx.x / 8;
  const unsigned tileb = x8 < rem ? x8 * (per + 1) + j8 : rem * (per + 1) + (x8 - rem) * per + j8;
  const int64_t R0 = (int64_t)tileb * 64;
  const int64_t r0 = R0 + 16 * wv;
  const int ri = l % 16, kg = l / 16;
  const int wr = (w + 15) / 16;
  const int cbmax = SYM ? wr : 2 * wr;  // a wavefront's blocks: v .. v + cbmax
  const int nsteps = (4 + cbmax + BPS - 1) / BPS;
  const int64_t C0 = SYM ? R0 : R0 - 16 * (int64_t)wr;  // first column of block 0
  auto margin = [](float x) { return x - fabsf(x) * 0x1p-20f; };

  // Tile pipeline.  Chunk x of a tile is row x / CPR, halves 8*(x % CPR).
  // The ids of the rows of step q reach LDS slot q % 3 two steps ahead; the
  // rows are fetched into registers at the start of the step before theirs
  // and stored to LDS at its end (the barriers between steps order LDS only,
  // so the loads stay in flight through the step's work).
  // Every global load of the pipeline is issued unconditionally, by every
  // thread and at every step (out-of-range steps, rows, ids and columns read
  // an in-range address), and masked when the stage is stored: a branch on a
  // loaded value, or a load some paths skip, makes the wait for it cover
  // every load issued before it, the prefetched rows included.
  struct Stage {
    uint4 v[CH];
    float n, ts;
  };
  Stage st;
  const int tr = threadIdx.x % TR;  // the tile row whose id, norm and threshold a thread loads
  auto tile_row = [&](int q) { return C0 + TR * (int64_t)q + tr; };
  auto load_ids = [&](int q) {
    const int64_t row = tile_row(q);
    return (int32_t)order[row < 0 ? 0 : (row >= N ? N - 1 : row)];
  };
  auto put_ids = [&](int q, int32_t id) {
    if (threadIdx.x < TR) {
      const int64_t row = tile_row(q);
      tcid[q % 3][tr] = row >= 0 && row < N ? id : -1;
    }
  };
  // Thread t moves tile row t / TPR, chunks t % TPR + TPR j: one id and
  // one row address per thread, contiguous 16-byte chunks per TPR lanes.
  // Rows past the array read point 0 and stay unmasked (every pair with
  // them fails the bounds test); chunks past d are zeroed.
  constexpr int TPR = 256 / TR;                 // threads per tile row
  static_assert(TR * TPR == 256 && (CPR + TPR - 1) / TPR == CH, "tile load layout");
  const int trow = threadIdx.x / TPR, tc = threadIdx.x % TPR;
  const bool dense = d == 32 * KS;
  auto fetch = [&](int q) {
    const int32_t id = tcid[q % 3][trow];
    const int64_t ic = id < 0 ? 0 : id;
    const __half* src = X + ic * d;
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int c = tc + TPR * j;
      if (c < CPR) st.v[j] = *(const uint4*)(src + (dense || 8 * c < d ? 8 * c : 0));
    }
    const float2 rec = *(const float2*)&pt[ic];
    st.n = rec.x;
    st.ts = rec.y;
  };
  auto store = [&](int q) {
    const int slot = q & 1;
    _Float16* dst = &tile[slot][trow * RS];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int c = tc + TPR * j;
      if (c < CPR) {
        uint4 v = st.v[j];
        if (!dense && 8 * c >= d) v = make_uint4(0, 0, 0, 0);
        *(uint4*)(dst + 8 * c) = v;
      }
    }
    if (tc == 0) {
      const bool ok = tcid[q % 3][trow] >= 0;
      tnrm[slot][trow] = ok ? st.n : 1.f;
      // column threshold: the k-th cosine of the column point's list (any
      // value it held is a valid lower bound) in dot units over the row norm
      if constexpr (SYM) tthr[slot][trow] = ok && st.ts != -INFINITY ? margin(st.ts * st.n) : -INFINITY;
    }
  };

  // Prologue: ids of the first two steps and the owners' ids, then (one
  // memory latency later) the owners' lists and mailbox counts and the rows
  // of the first step, all in flight together.  (Every order has nsteps >= 3.)
  const int32_t id0 = load_ids(0), id1 = load_ids(1);
  // the owner lane (l < 16) holds the list of row r0 + l
  const int64_t own = r0 + l;
  const bool owner = l < 16 && own < N;
  const int64_t own_id = owner ? (int64_t)order[own] : 0;
  put_ids(0, id0);
  put_ids(1, id1);
  // the wavefront's rows, as the MFMA A operand (with SYM taken from the
  // tile when its first column block, its own rows, arrives)
  half8 A[KS];
  if constexpr (!SYM) {
    const int64_t arow = r0 + ri < N ? (int64_t)order[r0 + ri] : -1;
#pragma unroll
    for (int s = 0; s < KS; ++s) A[s] = load_row8(X, arow, d, 32 * s + 8 * kg);
  }
  const float own_n = owner ? pt[own_id].x : 1.f;  // (the record's line also holds the mail count)
  // row ri's list, over lanes ri + 16 j (j = kg)
  const bool row_ok = r0 + ri < N;
  const int64_t row_id = __shfl((int32_t)own_id, ri);
  const float row_n = __shfl(own_n, ri);
  RowList<KMAX> L;
  if (row_ok)
    L.load(slots + row_id * (KMAX / 2), kg);
  else
    L.init(k, kg);
  // The pairs the point received in the previous order are merged after the
  // last step (the list is the top-k of everything merged into it, whatever
  // the order; a threshold without them only lets more pairs through): the
  // count is loaded now and used then.
  uint32_t nmail = 0;
  if constexpr (SYM) nmail = mi.n[own_id * 4];
  block_lds_sync();
  fetch(0);
  // row threshold in dot-product units, lowered by a relative 2^-20 (far
  // beyond the rounding of either side, so a pair below it cannot beat the
  // k-th entry), for the screening test of all lanes; lane (kg, ri) keeps
  // copies for rows 4kg..4kg+3.  The k-th entry of row R is the last slot
  // of lane R + 48.
  constexpr int SPL = RowList<KMAX>::SPL;
  float wsn = margin(L.ls[SPL - 1] * row_n);
  int open = L.li[SPL - 1] < 0;
  float rthr[4], rown[4];
  int ropen[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    rthr[r] = __shfl(wsn, 48 + 4 * kg + r);
    ropen[r] = __shfl(open, 48 + 4 * kg + r);
    rown[r] = __shfl(own_n, 4 * kg + r);
  }
  // Pairs that pass the screening wait in a per-row queue; the owners merge
  // the queues into their lists when one fills up and after the last step.
  // The lists end as the top-k of all candidates whatever the order of the
  // merges, and a late threshold only lets more pairs through the screening.
  if (l < 16) qn[wv][l] = 0;
  wave_lds_sync();
  auto drain = [&]() {
    // the four lanes of row ri take its queue entries together
    const uint32_t n = row_ok ? qn[wv][ri] : 0u;
    for (uint32_t i = 0; __ballot(i < n); ++i)
      if (i < n) L.insert(qcs[wv][ri][i], qid[wv][ri][i], kg);
    wave_lds_sync();
    if (l < 16) qn[wv][l] = 0;
    wsn = margin(L.ls[SPL - 1] * row_n);
    open = L.li[SPL - 1] < 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      rthr[r] = __shfl(wsn, 48 + 4 * kg + r);
      ropen[r] = __shfl(open, 48 + 4 * kg + r);
    }
    wave_lds_sync();
  };
  store(0);

  for (int q = 0; q < nsteps; ++q) {
    // tile q is in slot q & 1, the ids of steps q and q + 1 are in LDS
    block_lds_sync();
    // the ids before the rows, so that the wait for them does not cover the rows
    const int32_t id2 = load_ids(q + 2 < nsteps ? q + 2 : nsteps - 1);
    fetch(q + 1 < nsteps ? q + 1 : nsteps - 1);
#pragma unroll
    for (int hb = 0; hb < BPS; ++hb) {
      const int blk = BPS * q + hb;
      const int cb = blk - wv;
      if (cb < 0 || cb > cbmax || r0 >= N) continue;
      const int slot = q & 1;
      const int64_t c0 = C0 + 16 * (int64_t)blk;
      const _Float16* bt = &tile[slot][(16 * hb + ri) * RS + 8 * kg];
      if (SYM && cb == 0) {
        // (the empty asm keeps this a branch: selects on all of A would cost
        // every block 4 KS instructions)
        asm volatile("");
#pragma unroll
        for (int s = 0; s < KS; ++s) A[s] = *(const half8*)(bt + 32 * s);
      }
      float4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const half8 B = *(const half8*)(bt + 32 * s);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[s], B, acc, 0, 0, 0);
      }
      // D layout: lane (kg, ri) holds rows 4kg+r (r < 4) of column ri.
      // Screening in registers against the rows' (and with SYM the
      // columns') thresholds; the band and array bounds are tested per pair
      // only in blocks that cross them.
      const float cn = tnrm[slot][16 * hb + ri];
      const int64_t o = c0 - r0;  // pair offsets of the block: o - 15 .. o + 15
      const bool inner = c0 >= 0 && c0 + 16 <= N && r0 + 16 <= N &&
                         ((o >= 16 && o + 15 <= w) || (!SYM && o <= -16 && o - 15 >= -w));
      bool prow[4], pcol[4];
      const float ct = SYM ? tthr[slot][16 * hb + ri] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        prow[r] = (ropen[r] != 0) | (acc[r] >= rthr[r] * cn);
        pcol[r] = SYM && ((ct == -INFINITY) | (acc[r] >= ct * rown[r]));
      }
      if (!inner) {
        const int off = (int)o + ri;  // column offset from row 0 of the tile
        const bool col_ok = c0 + ri >= 0 && c0 + ri < N;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int R = 4 * kg + r;
          const int delta = off - R;
          const bool in = col_ok & (r0 + R < N) & (delta <= w) &
                          (SYM ? delta >= 1 : (delta != 0) & (-delta <= w));
          prow[r] &= in;
          pcol[r] &= in;
        }
      }
      if (__ballot(prow[0] | prow[1] | prow[2] | prow[3] | pcol[0] | pcol[1] | pcol[2] | pcol[3])) {
        const int32_t cid = tcid[q % 3][16 * hb + ri];
        bool full = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int32_t rid = __shfl((int32_t)own_id, 4 * kg + r);
          if (prow[r] | pcol[r]) {
            // the exact cosine, as the row's owner would compute it
            const float cs = acc[r] / (rown[r] * cn);
            if (prow[r]) {
              const int R = 4 * kg + r;
              const uint32_t j = atomicAdd(&qn[wv][R], 1u);
              qcs[wv][R][j] = cs;
              qid[wv][R][j] = cid;
              full |= j >= (uint32_t)(QCAP - 16);
            }
            if (SYM && pcol[r]) {
              // a point receives at most w pairs per order: one per position before it
              const uint32_t j = atomicAdd(&mo.n[(int64_t)cid * 4], 1u);
              mo.e[(int64_t)cid * w + j] = make_uint2(__float_as_uint(cs), (uint32_t)rid);
            }
          }
        }
        wave_lds_sync();
        // a block queues at most 16 per row: drain once a row holds more
        // than QCAP - 16
        if (__ballot(full)) drain();
      }
    }
    if (q + 1 < nsteps) store(q + 1);
    if (q + 2 < nsteps) put_ids(q + 2, id2);
  }
  if (r0 < N) drain();
  if constexpr (SYM) {
    const uint32_t n = row_ok ? (uint32_t)__shfl((int32_t)nmail, ri) : 0u;
    for (uint32_t i = 0; __ballot(i < n); ++i) {
      if (i < n) {
        const uint2 e = mi.e[row_id * w + i];
        L.insert(__uint_as_float(e.x), (int32_t)e.y, kg);
      }
    }
    if (owner) mi.n[own_id * 4] = 0;
  }
  if (row_ok) L.save(slots + row_id * (KMAX / 2), kg);
  const float kth = __shfl(L.ls[SPL - 1], 48 + (l & 15));
  if (owner) pt[own_id].y = kth;  // -inf while the list is not full
}

// The pairs sent in the last order, merged into every point's list.
template <int KMAX>
__global__ __launch_bounds__(256) void k_mailbox_final(Mailbox m, int64_t N, int w,
                                                       uint4* __restrict__ slots) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  const uint32_t n = m.n[p * 4];
  if (n == 0) return;
  TopList<KMAX> L;
  L.load_slots(slots + p * (KMAX / 2));
  for (uint32_t i = 0; i < n; ++i) {
    const uint2 e = m.e[p * w + i];
    const float cs = __uint_as_float(e.x);
    const int32_t c = (int32_t)e.y;
    if (L.wi() < 0 || better(cs, c, L.ws(), L.wi())) L.insert(cs, c);
  }
  L.save_slots(slots + p * (KMAX / 2));
  m.n[p * 4] = 0;
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, ceil_div(n, 256)));
}

template <int KMAX, bool SYM>
hf_status launch_band(int ks, const __half* X, int64_t N, int d, const uint32_t* order,
                      float4* pt, int w, int k, uint4* slots, Mailbox mi, Mailbox mo, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(N, 64));
  switch (ks) {
#define HF_KS(n) \
  case n: k_band<KMAX, n, SYM><<<grid, 256, 0, s>>>(X, N, d, order, pt, w, k, slots, mi, mo); break;
    HF_KS(1) HF_KS(2) HF_KS(3) HF_KS(4) HF_KS(5) HF_KS(6) HF_KS(7) HF_KS(8) HF_KS(9) HF_KS(10)
    HF_KS(11) HF_KS(12) HF_KS(13) HF_KS(14) HF_KS(15) HF_KS(16) HF_KS(20) HF_KS(24) HF_KS(32)
#undef HF_KS
    default:
      set_error("graph band kernel: unsupported d");
      return HF_ERR_UNSUPPORTED;
  }
  HF_LAUNCH_CHECK();
  return HF_OK;
}

}  // namespace

// Algorithm 2 with the sketch stage: per order a Hilbert sort, the Hamming
// band and the list merge; after the last order the cosine top-k of every
// point's k2 list.
static hf_status graph_prefilter(const void* X, int64_t N, int d, const hf_graph_params& p, int e,
                                 int32_t* ids, float* scores, int32_t* c2_ids, hipStream_t s) {
  Workspace ws(s);
  const int w = (int)p.window, k2 = (int)p.k2;
  uint64_t* sk;
  HF_TRY(ws.alloc(&sk, (size_t)N * 8));
  if (p.sketch == HF_SKETCH_LEARNED) {
    HF_TRY(lhash_encode_dev(p.lhash, X, HF_F16, N, sk, s));
  } else if (p.sketch == HF_SKETCH_SIGN) {
    HF_TRY(sign_sketch(X, HF_F16, N, d, sk, s));
  } else if (d % 16 == 0 && getenv("HF_SRP_VALU") == nullptr) {
    // the int8 matrix-core kernel (the same bits as the vector-ALU one)
    int8_t* Rb = nullptr;
    HF_TRY(srp_matrix_i8_upload(d, p.sketch_seed, &Rb, s));
    const hf_status st = srp_sketch_mfma(X, HF_F16, N, d, e, Rb, sk, s);
    const hipError_t sy = hipStreamSynchronize(s);
    (void)hipFree(Rb);
    HF_TRY(st);
    HIP_TRY(sy);
  } else {
    HF_TRY(srp_sketch(X, HF_F16, N, d, e, p.sketch_seed, sk, ws));
  }
  uint8_t* codes;
  float* nrm;
  uint32_t* order;
  uint64_t* lists;
  HF_TRY(ws.alloc(&codes, (size_t)(N * d)));
  HF_TRY(ws.alloc(&nrm, (size_t)N));
  HF_TRY(ws.alloc(&order, (size_t)N));
  HF_TRY(ws.alloc(&lists, (size_t)N * k2));
  // staging of one chunk of positions: 2w keys each, HF_GRAPH_STAGE_MIB
  // (default 1024) MiB at most
  int64_t stage_mib = 1024;
  if (const char* v = getenv("HF_GRAPH_STAGE_MIB")) stage_mib = std::max<int64_t>(1, atoll(v));
  int64_t chunk = (stage_mib << 17) / (2 * w);
  chunk = std::max<int64_t>(256, chunk / 256 * 256);
  chunk = std::min<int64_t>(chunk, N);
  uint64_t* stage;
  uint32_t* cnt;
  HF_TRY(ws.alloc(&stage, (size_t)(2 * w) * chunk));
  HF_TRY(ws.alloc(&cnt, (size_t)chunk));
  HF_TRY(quantize(X, HF_F16, N * d, e, codes, s));
  uint32_t* msb = nullptr;
  if (msb_words(d) > 0) {
    HF_TRY(ws.alloc(&msb, (size_t)(N * msb_words(d))));
    HF_TRY(msb_plane(codes, N, d, msb, s));
  }
  k_norms<<<(unsigned)ceil_div(N, 4), 256, 0, s>>>((const __half*)X, N, d, nrm);
  HF_LAUNCH_CHECK();
  HF_TRY(gpf_init_lists(lists, N * k2, s));
  const int T = (int)p.n_orders;
  std::vector<int32_t> perm((size_t)T * d);
  std::vector<uint8_t> refl((size_t)T * d);
  make_curves(p.seed, T, d, perm.data(), refl.data());
  int32_t* dperm;
  uint8_t* drefl;
  HF_TRY(ws.alloc(&dperm, (size_t)T * d));
  HF_TRY(ws.alloc(&drefl, (size_t)T * d));
  HIP_TRY(hipMemcpyAsync(dperm, perm.data(), 4 * (size_t)T * d, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(drefl, refl.data(), (size_t)T * d, hipMemcpyHostToDevice, s));
  for (int t = 0; t < T; ++t) {
    Workspace wt(s);
    {
      StageTimer tm(ST_GSORT, s);
      HF_TRY(hilbert_sort_dev(codes, msb, N, d, dperm + (size_t)t * d, drefl + (size_t)t * d, order, nullptr, wt));
    }
    HF_TRY(gpf_order(sk, order, N, w, k2, lists, chunk, stage, cnt, s));
  }
  HF_TRY(gpf_final(X, nrm, N, d, lists, k2, (int)p.k, ids, scores, c2_ids, s));
  HIP_TRY(hipStreamSynchronize(s));
  return HF_OK;
}

hf_status graph_launch(const void* Xv, hf_dtype dt, int64_t N, int d, const hf_graph_params& p, int e,
                       int32_t* ids, float* scores, int32_t* c2_ids, hipStream_t s) {
  (void)dt;
  if (p.k2 != 0) return graph_prefilter(Xv, N, d, p, e, ids, scores, c2_ids, s);
  const __half* X = (const __half*)Xv;
  int ks = (d + 31) / 32;
  if (ks > 16) ks = ks <= 20 ? 20 : (ks <= 24 ? 24 : (ks <= 32 ? 32 : 0));
  if (ks == 0) {
    set_error("graph band kernel: d > 1024 not built");
    return HF_ERR_UNSUPPORTED;
  }
  // A second stream sorts order t+1 while the band kernel of order t runs:
  // the orders are double-buffered.
  // (the workspace is declared first so that it is released last, after the
  // guard below has waited for the second stream)
  Workspace ws(s);
  struct Pipe {
    hipStream_t s2 = nullptr;
    hipEvent_t ready = nullptr, sorted[2] = {nullptr, nullptr}, banded[2] = {nullptr, nullptr};
    ~Pipe() {
      if (s2) (void)hipStreamSynchronize(s2);
      for (hipEvent_t e : {ready, sorted[0], sorted[1], banded[0], banded[1]})
        if (e) (void)hipEventDestroy(e);
      if (s2) (void)hipStreamDestroy(s2);
    }
  } pp;
  HIP_TRY(hipStreamCreateWithFlags(&pp.s2, hipStreamNonBlocking));
  for (hipEvent_t* e : {&pp.ready, &pp.sorted[0], &pp.sorted[1], &pp.banded[0], &pp.banded[1]})
    HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
  hipStream_t s2 = pp.s2;
  uint8_t* codes;
  float4* pt;  // per point: norm, k-th cosine of its list (-inf until full), two mail counts
  uint32_t* order[2];
  for (int b = 0; b < 2; ++b) HF_TRY(ws.alloc(&order[b], (size_t)N));
  HF_TRY(ws.alloc(&codes, (size_t)(N * d)));
  HF_TRY(ws.alloc(&pt, (size_t)N));
  HF_TRY(quantize(X, HF_F16, N * d, e, codes, s));
  uint32_t* msb = nullptr;
  if (msb_words(d) > 0) {
    HF_TRY(ws.alloc(&msb, (size_t)(N * msb_words(d))));
    HF_TRY(msb_plane(codes, N, d, msb, s));
  }
  k_norms<<<(unsigned)ceil_div(N, 4), 256, 0, s>>>(X, N, d, (float*)pt, 4);
  const int kmax = p.k <= 16 ? 16 : 32;
  uint4* slots;
  HF_TRY(ws.alloc(&slots, (size_t)N * kmax / 2));
  k_init_slots<<<grid_for(N * kmax), 256, 0, s>>>((uint2*)slots, N, kmax, (int)p.k);
  HF_LAUNCH_CHECK();
  // Each pair of the band is computed once when the two mailboxes (per point
  // w entries of 8 bytes; the counts are words of the point records) fit in
  // HF_GRAPH_MAILBOX_MIB (default 32768) MiB; otherwise from both sides.
  const int w = (int)p.window;
  int64_t mb_mib = 32768;
  if (const char* v = getenv("HF_GRAPH_MAILBOX_MIB")) mb_mib = std::max<int64_t>(0, atoll(v));
  const bool sym = 2 * N * 8 * (int64_t)w <= (mb_mib << 20);
  Mailbox mb[2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  if (sym) {
    for (int b = 0; b < 2; ++b) {
      mb[b].n = (uint32_t*)pt + 2 + b;  // zeroed with the records
      HF_TRY(ws.alloc(&mb[b].e, (size_t)N * w));
    }
  }
  const int T = (int)p.n_orders;
  std::vector<int32_t> perm((size_t)T * d);
  std::vector<uint8_t> refl((size_t)T * d);
  make_curves(p.seed, T, d, perm.data(), refl.data());
  int32_t* dperm;
  uint8_t* drefl;
  HF_TRY(ws.alloc(&dperm, (size_t)T * d));
  HF_TRY(ws.alloc(&drefl, (size_t)T * d));
  HIP_TRY(hipMemcpyAsync(dperm, perm.data(), 4 * (size_t)T * d, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(drefl, refl.data(), (size_t)T * d, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(pp.ready, s));
  HIP_TRY(hipStreamWaitEvent(s2, pp.ready, 0));
  // sort order t into buffer t & 1 on the second stream
  auto prepare = [&](int t) -> hf_status {
    const int b = t & 1;
    if (t >= 2) HIP_TRY(hipStreamWaitEvent(s2, pp.banded[b], 0));  // band t-2 is done with b
    {
      Workspace wt(s2);
      StageTimer tm(ST_GSORT, s2);
      HF_TRY(hilbert_sort_dev(codes, msb, N, d, dperm + (size_t)t * d, drefl + (size_t)t * d, order[b], nullptr,
                              wt));
    }
    HIP_TRY(hipEventRecord(pp.sorted[b], s2));
    return HF_OK;
  };
  HF_TRY(prepare(0));
  for (int t = 0; t < T; ++t) {
    const int b = t & 1;
    HIP_TRY(hipStreamWaitEvent(s, pp.sorted[b], 0));
    {
      // the band of order t fills mailbox t & 1 and empties the other
      StageTimer tm(ST_GBAND, s);
      const Mailbox mi = mb[b ^ 1], mo = mb[b];
      const int k = (int)p.k;
      // The first two orders score every pair from both sides: nearly every
      // pair passes against lists still empty or weak, and two-sided
      // pushes go to the LDS queues instead of returning global atomics on
      // the mailboxes.  (Order 2 finds order 1's mailbox empty.)
      const bool sym_t = sym && t >= 2;
      hf_status st;
      if (k <= 16)
        st = sym_t ? launch_band<16, true>(ks, X, N, d, order[b], pt, w, k, slots, mi, mo, s)
                   : launch_band<16, false>(ks, X, N, d, order[b], pt, w, k, slots, mi, mo, s);
      else
        st = sym_t ? launch_band<32, true>(ks, X, N, d, order[b], pt, w, k, slots, mi, mo, s)
                   : launch_band<32, false>(ks, X, N, d, order[b], pt, w, k, slots, mi, mo, s);
      HF_TRY(st);
    }
    HIP_TRY(hipEventRecord(pp.banded[b], s));
    if (t + 1 < T) HF_TRY(prepare(t + 1));
  }
  {
    // the last order's mailboxes, then the lists out of the working slots
    StageTimer tm(ST_GMAIL, s);
    if (sym) {
      const Mailbox m = mb[(T - 1) & 1];
      if (p.k <= 16)
        k_mailbox_final<16><<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(m, N, w, slots);
      else
        k_mailbox_final<32><<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(m, N, w, slots);
    }
    k_slots_out<<<grid_for(N * p.k), 256, 0, s>>>((const uint2*)slots, N, kmax, (int)p.k, ids, scores);
    HF_LAUNCH_CHECK();
  }
  HIP_TRY(hipStreamSynchronize(s2));
  HIP_TRY(hipStreamSynchronize(s));
  return HF_OK;
}

}  // namespace hf
