// Device-wide exclusive prefix sum of uint32 (reduce, scan of partials,
// down-sweep), used by the radix sort, compactions and the trie levels.
#include "hf_internal.h"

namespace hf {
namespace {

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

__global__ __launch_bounds__(SC_THREADS) void scan_reduce(const uint32_t* __restrict__ in,
                                                          int64_t n, uint32_t* __restrict__ part) {
  __shared__ uint32_t lds[SC_THREADS / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * SC_TILE;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    int64_t idx = base + (int64_t)i * SC_THREADS + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  uint32_t tot;
  block_excl_scan<SC_THREADS>(s, lds, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: exclusive scan of the partials in place, any length.
__global__ __launch_bounds__(1024) void scan_partials(uint32_t* part, int64_t n,
                                                      uint32_t* total) {
  __shared__ uint32_t lds[1024 / 64 + 1];
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += 1024) {
    int64_t idx = base + threadIdx.x;
    uint32_t v = idx < n ? part[idx] : 0;
    uint32_t tot;
    uint32_t ex = block_excl_scan<1024>(v, lds, &tot);
    if (idx < n) part[idx] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(SC_THREADS) void scan_down(const uint32_t* __restrict__ in,
                                                        uint32_t* __restrict__ out, int64_t n,
                                                        const uint32_t* __restrict__ part) {
  __shared__ uint32_t lds[SC_THREADS / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
  uint32_t v[SC_ITEMS];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    int64_t idx = base + i;
    v[i] = idx < n ? in[idx] : 0;
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = part[blockIdx.x] + block_excl_scan<SC_THREADS>(s, lds, &tot);
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
}

}  // namespace

hf_status excl_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev,
                        Workspace& ws) {
  if (n <= 0) {
    if (total_dev) HIP_TRY(hipMemsetAsync(total_dev, 0, 4, ws.stream));
    return HF_OK;
  }
  int64_t nb = ceil_div(n, SC_TILE);
  uint32_t* part;
  HF_TRY(ws.alloc(&part, (size_t)nb));
  scan_reduce<<<dim3((unsigned)nb), SC_THREADS, 0, ws.stream>>>(in, n, part);
  HF_LAUNCH_CHECK();
  scan_partials<<<1, 1024, 0, ws.stream>>>(part, nb, total_dev);
  HF_LAUNCH_CHECK();
  scan_down<<<dim3((unsigned)nb), SC_THREADS, 0, ws.stream>>>(in, out, n, part);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

}  // namespace hf
