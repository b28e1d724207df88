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

__global__ void k_norms(const __half* __restrict__ X, int64_t N, int d, float* __restrict__ nrm) {
  int64_t p = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (p >= N) return;
  float a = 0.f;
  for (int i = __lane_id(); i < d; i += 64) {
    float v = __half2float(X[p * d + i]);
    a = fmaf(v, v, a);
  }
  for (int m = 32; m >= 1; m >>= 1) a += __shfl_xor(a, m);
  if (__lane_id() == 0) nrm[p] = sqrtf(a);
}

__global__ void k_init_lists(int32_t* __restrict__ ids, float* __restrict__ sc, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    ids[i] = -1;
    sc[i] = -INFINITY;
  }
}

// Rows (and their norms) re-laid in the order's sequence so the band tiles
// read contiguous memory.
__global__ void k_gather_sorted(const __half* __restrict__ X, const float* __restrict__ nrm,
                                const uint32_t* __restrict__ order, int64_t N, int d,
                                __half* __restrict__ Xs, float* __restrict__ ns) {
  const int64_t nv = d / 8;  // 16-byte vectors per row
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N * nv; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / nv, c = i - r * nv;
    const uint32_t id = order[r];
    ((uint4*)Xs)[r * nv + c] = ((const uint4*)(X + (int64_t)id * d))[c];
    if (c == 0) ns[r] = nrm[id];
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

__device__ __forceinline__ half8 load_row8(const __half* __restrict__ X, int64_t r, int d, int k0) {
  if (r < 0 || k0 >= d) return (half8)(0);
  uint4 raw = *(const uint4*)(X + r * d + k0);
  return __builtin_bit_cast(half8, raw);
}

// A workgroup (four wavefronts) owns 64 consecutive positions; wavefront v
// owns rows R0+16v .. +15.  Column blocks of 16 positions stream through a
// double-buffered LDS tile shared by the four wavefronts, BPS blocks per
// step (loaded once, one step ahead, 16-byte coalesced); wavefront v uses
// blocks v .. v+2*wr of the workgroup's 4+2*wr.  Rows are padded by 16 bytes
// in LDS so the 16 lanes reading one column fragment hit distinct banks.
template <int KMAX, int KS>
__global__ __launch_bounds__(256) void k_band(const __half* __restrict__ Xs, int64_t N, int d,
                                              const uint32_t* __restrict__ order,
                                              const float* __restrict__ ns, int w, int k,
                                              int32_t* __restrict__ gids, float* __restrict__ gsc) {
  constexpr int BPS = 2;           // column blocks per step
  constexpr int TR = 16 * BPS;     // tile rows
  constexpr int RS = KS * 32 + 8;  // LDS row stride (halves)
  constexpr int CPR = KS * 4;      // 16-byte chunks per tile row
  constexpr int CH = (TR * CPR + 255) / 256;  // chunks per thread per tile
  __shared__ __attribute__((aligned(16))) _Float16 tile[2][TR * RS];
  __shared__ int32_t tcid[2][TR];
  __shared__ float tnrm[2][TR];
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
  const int64_t arow = r0 + ri < N ? r0 + ri : -1;
  half8 A[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) A[s] = load_row8(Xs, arow, d, 32 * s + 8 * kg);
  // the owner lane (l < 16) holds the list of row r0 + l
  TopList<KMAX> L;
  const int64_t own = r0 + l;
  const bool owner = l < 16 && own < N;
  const int64_t own_id = owner ? (int64_t)order[own] : 0;
  const float own_n = owner ? ns[own] : 1.f;
  L.load(gsc + own_id * k, gids + own_id * k, k, owner);
  // row threshold in dot-product units, lowered by a relative 2^-20 (far
  // beyond the rounding of either side, so a pair below it cannot beat the
  // k-th entry), for the screening test of all lanes; lane (kg, ri) keeps
  // copies for rows 4kg..4kg+3
  auto margin = [](float x) { return x - fabsf(x) * 0x1p-20f; };
  float wsn = margin(L.ws() * own_n);
  int open = L.wi() < 0;
  float rthr[4], rown[4];
  int ropen[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    rthr[r] = __shfl(wsn, 4 * kg + r);
    ropen[r] = __shfl(open, 4 * kg + r);
    rown[r] = __shfl(own_n, 4 * kg + r);
  }
  // Pairs that pass the screening wait in a per-row queue; the owners merge
  // the queues into their lists when one fills up and after the last step.
  // The lists end as the top-k of all candidates whatever the order of the
  // merges, and a late threshold only lets more pairs through the screening.
  if (l < 16) qn[wv][l] = 0;
  wave_lds_sync();
  auto drain = [&]() {
    const uint32_t n = owner ? qn[wv][l] : 0u;
    for (uint32_t i = 0; __ballot(i < n); ++i) {
      if (i < n) {
        const float cs = qcs[wv][l][i];
        const int32_t c = qid[wv][l][i];
        if (L.wi() < 0 || better(cs, c, L.ws(), L.wi())) L.insert(cs, c);
      }
    }
    if (l < 16) qn[wv][l] = 0;
    wsn = margin(L.ws() * own_n);
    open = L.wi() < 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      rthr[r] = __shfl(wsn, 4 * kg + r);
      ropen[r] = __shfl(open, 4 * kg + r);
    }
    wave_lds_sync();
  };
  const int wr = (w + 15) / 16;
  const int nsteps = (4 + 2 * wr + BPS - 1) / BPS;
  const int64_t C0 = R0 - 16 * (int64_t)wr;  // first column of block 0
  // cooperative tile load: chunk x of the tile is row x / CPR, halves 8*(x % CPR).
  // A tile of whole rows inside the array (d = 32 KS) is one contiguous run
  // of memory: chunk x is 16-byte vector x from the tile's first row.
  uint4 stg[CH];
  int32_t scid = -1;
  float snrm = 1.f;
  const bool dense = d == KS * 32;
  auto fetch = [&](int q) {
    const int64_t cb0 = C0 + TR * (int64_t)q;
    if (dense && cb0 >= 0 && cb0 + TR <= N) {
      const uint4* src = (const uint4*)(Xs + cb0 * d);
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int x = threadIdx.x + 256 * i;
        stg[i] = make_uint4(0, 0, 0, 0);
        if ((i + 1) * 256 <= TR * CPR || x < TR * CPR) stg[i] = src[x];
      }
    } else {
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int x = threadIdx.x + 256 * i;
        const int rr = x / CPR, k0 = 8 * (x % CPR);
        const int64_t row = cb0 + rr;
        stg[i] = make_uint4(0, 0, 0, 0);
        if (x < TR * CPR && row >= 0 && row < N && k0 < d) stg[i] = *(const uint4*)(Xs + row * d + k0);
      }
    }
    scid = -1;
    snrm = 1.f;
    if (threadIdx.x < TR) {
      const int64_t row = cb0 + threadIdx.x;
      if (row >= 0 && row < N) {
        scid = (int32_t)order[row];
        snrm = ns[row];
      }
    }
  };
  auto store = [&](int slot) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int x = threadIdx.x + 256 * i;
      if (x < TR * CPR) *(uint4*)(&tile[slot][(x / CPR) * RS + 8 * (x % CPR)]) = stg[i];
    }
    if (threadIdx.x < TR) {
      tcid[slot][threadIdx.x] = scid;
      tnrm[slot][threadIdx.x] = snrm;
    }
  };
  fetch(0);
  store(0);
  for (int q = 0; q < nsteps; ++q) {
    __syncthreads();  // tile q is in slot q & 1; slot (q + 1) & 1 is free
    if (q + 1 < nsteps) fetch(q + 1);
#pragma unroll
    for (int hb = 0; hb < BPS; ++hb) {
    const int blk = BPS * q + hb;
    const int cb = blk - wv;
    if (cb >= 0 && cb <= 2 * wr && r0 < N) {
      const int slot = q & 1;
      const int64_t c0 = C0 + 16 * (int64_t)blk;
      float4v acc = {0.f, 0.f, 0.f, 0.f};
      const _Float16* bt = &tile[slot][(16 * hb + ri) * RS + 8 * kg];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const half8 B = *(const half8*)(bt + 32 * s);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[s], B, acc, 0, 0, 0);
      }
      // D layout: lane (kg, ri) holds rows 4kg+r (r < 4) of column ri.
      // Screening in registers against the rows' thresholds; the band and
      // array bounds are tested per pair only in blocks that cross them.
      const float cn = tnrm[slot][16 * hb + ri];
      const int64_t o = c0 - r0;  // pair offsets of the block: o - 15 .. o + 15
      const bool inner = c0 >= 0 && c0 + 16 <= N && r0 + 16 <= N &&
                         ((o >= 16 && o + 15 <= w) || (o <= -16 && o - 15 >= -w));
      bool pass[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) pass[r] = (ropen[r] != 0) | (acc[r] >= rthr[r] * cn);
      if (!inner) {
        const int off = (int)o + ri;  // column offset from row 0 of the tile
        const bool col_ok = c0 + ri >= 0 && c0 + ri < N;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int R = 4 * kg + r;
          const int delta = off - R;
          pass[r] &= col_ok & (r0 + R < N) & (delta != 0) & (delta <= w) & (-delta <= w);
        }
      }
      if (__ballot(pass[0] | pass[1] | pass[2] | pass[3])) {
        const int32_t cid = tcid[slot][16 * hb + ri];
        bool full = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (pass[r]) {
            // the exact cosine, as the row's owner would compute it, queued
            const int R = 4 * kg + r;
            const uint32_t j = atomicAdd(&qn[wv][R], 1u);
            qcs[wv][R][j] = acc[r] / (rown[r] * cn);
            qid[wv][R][j] = cid;
            full |= j >= (uint32_t)(QCAP - 16);
          }
        }
        wave_lds_sync();
        // a block queues at most 16 per row: drain once a row holds more
        // than QCAP - 16
        if (__ballot(full)) drain();
      }
    }
    }
    if (q + 1 < nsteps) store((q + 1) & 1);
  }
  if (r0 < N) drain();
  if (owner) L.save(gsc + own_id * k, gids + own_id * k, k);
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, ceil_div(n, 256)));
}

template <int KMAX>
hf_status launch_band(int ks, const __half* X, int64_t N, int d, const uint32_t* order,
                      const float* nrm, int w, int k, int32_t* ids, float* sc, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(N, 64));
  switch (ks) {
#define HF_KS(n) \
  case n: k_band<KMAX, n><<<grid, 256, 0, s>>>(X, N, d, order, nrm, w, k, ids, sc); break;
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
  // A second stream sorts and gathers order t+1 while the band kernel of
  // order t runs: orders, re-laid rows and norms are double-buffered.
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
  float* nrm;
  uint32_t* order[2];
  __half* Xs[2];
  float* ns[2];
  for (int b = 0; b < 2; ++b) {
    HF_TRY(ws.alloc(&Xs[b], (size_t)(N * d)));
    HF_TRY(ws.alloc(&ns[b], (size_t)N));
    HF_TRY(ws.alloc(&order[b], (size_t)N));
  }
  HF_TRY(ws.alloc(&codes, (size_t)(N * d)));
  HF_TRY(ws.alloc(&nrm, (size_t)N));
  HF_TRY(quantize(X, HF_F16, N * d, e, codes, s));
  uint32_t* msb = nullptr;
  if (msb_words(d) > 0) {
    HF_TRY(ws.alloc(&msb, (size_t)(N * msb_words(d))));
    HF_TRY(msb_plane(codes, N, d, msb, s));
  }
  k_norms<<<(unsigned)ceil_div(N, 4), 256, 0, s>>>(X, N, d, nrm);
  k_init_lists<<<grid_for(N * p.k), 256, 0, s>>>(ids, scores, N * p.k);
  HF_LAUNCH_CHECK();
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
  // sort and gather order t into buffer t & 1 on the second stream
  auto prepare = [&](int t) -> hf_status {
    const int b = t & 1;
    if (t >= 2) HIP_TRY(hipStreamWaitEvent(s2, pp.banded[b], 0));  // band t-2 is done with b
    {
      Workspace wt(s2);
      StageTimer tm(ST_GSORT, s2);
      HF_TRY(hilbert_sort_dev(codes, msb, N, d, dperm + (size_t)t * d, drefl + (size_t)t * d, order[b], nullptr,
                              wt));
    }
    {
      StageTimer tg(ST_GGATHER, s2);
      k_gather_sorted<<<grid_for(N * (d / 8)), 256, 0, s2>>>(X, nrm, order[b], N, d, Xs[b], ns[b]);
      HF_LAUNCH_CHECK();
    }
    HIP_TRY(hipEventRecord(pp.sorted[b], s2));
    return HF_OK;
  };
  HF_TRY(prepare(0));
  for (int t = 0; t < T; ++t) {
    const int b = t & 1;
    HIP_TRY(hipStreamWaitEvent(s, pp.sorted[b], 0));
    {
      StageTimer tm(ST_GBAND, s);
      if (p.k <= 16)
        HF_TRY(launch_band<16>(ks, Xs[b], N, d, order[b], ns[b], (int)p.window, (int)p.k, ids, scores, s));
      else
        HF_TRY(launch_band<32>(ks, Xs[b], N, d, order[b], ns[b], (int)p.window, (int)p.k, ids, scores, s));
    }
    HIP_TRY(hipEventRecord(pp.banded[b], s));
    if (t + 1 < T) HF_TRY(prepare(t + 1));
  }
  HIP_TRY(hipStreamSynchronize(s2));
  HIP_TRY(hipStreamSynchronize(s));
  return HF_OK;
}

}  // namespace hf
