// Stable LSD radix sort of (uint64 key, uint32 value) pairs, 8 bits per pass.
//
// Per pass: (1) each 4096-element tile counts its digits into a digit-major
// table counts[digit][tile]; (2) an exclusive scan of that table gives every
// (digit, tile) its global offset, which keeps equal digits in input order
// across tiles; (3) each tile ranks its elements stably (wavefront ballots
// find equal digits inside a 64-element row, per-wave running counters carry
// the rank across rows and waves), stages them in LDS grouped by digit and
// writes each digit run out contiguously.  Every global load of a tile is
// issued before the ranking starts: a load between the ballots would be
// waited for row by row.
#include "hf_internal.h"

namespace hf {
namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ROWS = 16;                       // 64-element rows per wave
constexpr int RS_TILE = RS_THREADS * RS_ROWS;     // 4096
constexpr int RS_WAVE_SPAN = 64 * RS_ROWS;        // elements per wave

__global__ __launch_bounds__(RS_THREADS) void rs_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                      int shift, uint32_t* __restrict__ counts,
                                                      int64_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  uint32_t dg[RS_ROWS];
#pragma unroll
  for (int i = 0; i < RS_ROWS; ++i) {
    const int64_t idx = base + (int64_t)i * RS_THREADS + threadIdx.x;
    dg[i] = (uint32_t)(keys[idx < n ? idx : n - 1] >> shift) & 255u;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RS_ROWS; ++i)
    if (base + (int64_t)i * RS_THREADS + threadIdx.x < n) atomicAdd(&h[dg[i]], 1u);
  __syncthreads();
  counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RS_THREADS) void rs_scatter(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t n, int shift,
    const uint32_t* __restrict__ offs, int64_t ntiles, uint64_t* __restrict__ okeys,
    uint32_t* __restrict__ ovals) {
  __shared__ uint64_t skey[RS_TILE];
  __shared__ uint32_t sval[RS_TILE];
  __shared__ uint32_t wcnt[RS_WAVES][256];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t scan_tmp[RS_THREADS / 64 + 1];

  const int w = threadIdx.x / 64, l = __lane_id();
  const int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
  uint64_t k[RS_ROWS];
  uint32_t v[RS_ROWS];
  uint32_t rank[RS_ROWS];
  // the tile's global offset of digit threadIdx.x
  const uint32_t off = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
#pragma unroll
  for (int r = 0; r < RS_ROWS; ++r) {
    const int64_t idx = tile0 + (int64_t)w * RS_WAVE_SPAN + r * 64 + l;
    const int64_t ic = idx < n ? idx : n - 1;
    k[r] = keys[ic];
    v[r] = vals[ic];
  }
  for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_THREADS) (&wcnt[0][0])[i] = 0;
  __syncthreads();

  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < RS_ROWS; ++r) {
    int64_t idx = tile0 + (int64_t)w * RS_WAVE_SPAN + r * 64 + l;
    bool ok = idx < n;
    uint32_t dg = (uint32_t)(k[r] >> shift) & 255u;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bal = __ballot((dg >> b) & 1u);
      peers &= ((dg >> b) & 1u) ? bal : ~bal;
    }
    uint32_t before = (uint32_t)__popcll(peers & lt);
    uint32_t cnt = (uint32_t)__popcll(peers);
    int leader = peers ? (int)__ffsll((long long)peers) - 1 : 0;
    uint32_t old = 0;
    if (ok && l == leader) {
      old = wcnt[w][dg];
      wcnt[w][dg] = old + cnt;
    }
    old = __shfl(old, leader);
    rank[r] = old + before;
  }
  __syncthreads();
  // per digit: exclusive prefix over waves, then over digits (tile-local start)
  {
    uint32_t dg = threadIdx.x, run = 0;
#pragma unroll
    for (int ww = 0; ww < RS_WAVES; ++ww) {
      uint32_t c = wcnt[ww][dg];
      wcnt[ww][dg] = run;
      run += c;
    }
    uint32_t tot;
    dstart[dg] = block_excl_scan<RS_THREADS>(run, scan_tmp, &tot);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_ROWS; ++r) {
    int64_t idx = tile0 + (int64_t)w * RS_WAVE_SPAN + r * 64 + l;
    if (idx < n) {
      uint32_t dg = (uint32_t)(k[r] >> shift) & 255u;
      uint32_t p = dstart[dg] + wcnt[w][dg] + rank[r];
      skey[p] = k[r];
      sval[p] = v[r];
    }
  }
  __syncthreads();
  // the counters are spent: digit d's output position of LDS slot i is
  // wcnt[0][d] + i
  wcnt[0][threadIdx.x] = off - dstart[threadIdx.x];
  __syncthreads();
  int64_t m = n - tile0;
  if (m > RS_TILE) m = RS_TILE;
  for (int i = threadIdx.x; i < m; i += RS_THREADS) {
    uint64_t kk = skey[i];
    uint32_t dg = (uint32_t)(kk >> shift) & 255u;
    uint32_t dst = wcnt[0][dg] + (uint32_t)i;
    okeys[dst] = kk;
    ovals[dst] = sval[i];
  }
}

}  // namespace

hf_status radix_sort_pairs(uint64_t** keys, uint32_t** vals, uint64_t** alt_keys,
                           uint32_t** alt_vals, int64_t n, int bit_lo, int bit_hi, Workspace& ws) {
  if (n <= 1 || bit_hi <= bit_lo) return HF_OK;
  int64_t ntiles = ceil_div(n, RS_TILE);
  uint32_t *counts, *offs;
  HF_TRY(ws.alloc(&counts, (size_t)(256 * ntiles)));
  HF_TRY(ws.alloc(&offs, (size_t)(256 * ntiles)));
  for (int shift = bit_lo; shift < bit_hi; shift += 8) {
    rs_hist<<<dim3((unsigned)ntiles), RS_THREADS, 0, ws.stream>>>(*keys, n, shift, counts, ntiles);
    HF_LAUNCH_CHECK();
    HF_TRY(excl_scan_u32(counts, offs, 256 * ntiles, nullptr, ws));
    rs_scatter<<<dim3((unsigned)ntiles), RS_THREADS, 0, ws.stream>>>(*keys, *vals, n, shift, offs,
                                                                     ntiles, *alt_keys, *alt_vals);
    HF_LAUNCH_CHECK();
    uint64_t* tk = *keys;
    *keys = *alt_keys;
    *alt_keys = tk;
    uint32_t* tv = *vals;
    *vals = *alt_vals;
    *alt_vals = tv;
  }
  return HF_OK;
}

}  // namespace hf
