// Achievable ceilings of one MI355X for the access patterns of the search and
// graph kernels, measured with plain kernels (one JSON object per line):
//   copy    - streaming read + write of a 4 GiB buffer (16-byte lanes);
//   gather  - random records from an array the size of the 23M-point sketch
//             table: 64-byte records (a sketch), 128-byte records (a whole L2
//             line) and 768-byte records (an fp16 row of 384 dimensions);
//             record indexes come from a hash of the entry number; and
//             64-byte records from a 2 MiB table that every L2 holds;
//   mfma    - independent chains of 32x32x16 fp16 MFMAs with fp32
//             accumulation in every wave of a full grid.
// The published peaks are the denominators of the rooflines; these figures
// say how much of them a kernel with the same access pattern can reach.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define CK(x)                                                                                  \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) {                                                                    \
      fprintf(stderr, "%s:%d %s\n", __FILE__, __LINE__, hipGetErrorString(e_));                \
      exit(1);                                                                                 \
    }                                                                                          \
  } while (0)

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ a, uint4* __restrict__ b,
                                              int64_t n) {
  const int64_t s = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += s) b[i] = a[i];
}

// 64-bit mix (the finaliser of splitmix64) of the entry number -> record index
__device__ __forceinline__ uint32_t rec_of(uint64_t i, uint64_t nr) {
  uint64_t z = i + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (uint32_t)(z % nr);
}

__global__ void k_fill(uint32_t* __restrict__ pos, int64_t n, uint64_t nr) {
  const int64_t s = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += s) pos[i] = rec_of(i, nr);
}

// L lanes per record of 16*L*V bytes, V 16-byte loads per lane; four records
// in flight per lane group; a popcount per record keeps the loads alive.
template <int L, int V>
__global__ __launch_bounds__(256) void k_gather(const uint4* __restrict__ tab,
                                                const uint32_t* __restrict__ pos, int64_t n,
                                                uint32_t* __restrict__ out) {
  const int ln = threadIdx.x % L;
  const int64_t g0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) / L;
  const int64_t gs = (int64_t)gridDim.x * (256 / L);
  uint32_t acc = 0;
  for (int64_t g = g0; g < n; g += 4 * gs) {
    uint32_t p[4];
    uint4 v[4][V];
#pragma unroll
    for (int u = 0; u < 4; ++u) p[u] = pos[g + u * gs < n ? g + u * gs : n - 1];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < V; ++j) v[u][j] = tab[(uint64_t)p[u] * (L * V) + (uint64_t)j * L + ln];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const uint32_t c = __popc(v[u][j].x) + __popc(v[u][j].y) + __popc(v[u][j].z) + __popc(v[u][j].w);
        acc += g + u * gs < n ? c : 0u;
      }
  }
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

// Each wave: C independent 32x32 accumulators, `iters` rounds of C MFMAs.
template <int C>
__global__ __launch_bounds__(256) void k_mfma(const v8h* __restrict__ in, int iters,
                                              float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  v8h a = in[lane], b = in[64 + lane];
  v16f acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[c][e];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

struct Timer {
  hipEvent_t a, b;
  Timer() {
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&b));
  }
  void start() { CK(hipEventRecord(a)); }
  float stop() {
    CK(hipEventRecord(b));
    CK(hipEventSynchronize(b));
    float ms;
    CK(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
};

static int g_blocks = 8192;

template <int L, int V>
static void gather(const char* name, const uint4* tab, uint64_t tab_bytes, uint32_t* pos, int64_t n,
                   uint32_t* out, int reps) {
  const uint64_t rec = 16ull * L * V, nr = tab_bytes / rec;
  k_fill<<<4096, 256>>>(pos, n, nr);
  CK(hipGetLastError());
  k_gather<L, V><<<g_blocks, 256>>>(tab, pos, n, out);
  CK(hipGetLastError());
  Timer t;
  t.start();
  for (int r = 0; r < reps; ++r) k_gather<L, V><<<g_blocks, 256>>>(tab, pos, n, out);
  const float ms = t.stop() / reps;
  printf("{\"probe\": \"%s\", \"record_bytes\": %llu, \"records\": %llu, \"table_bytes\": %llu, "
         "\"ms\": %.4f, \"grecords_per_s\": %.3f, \"record_gb_per_s\": %.1f}\n",
         name, (unsigned long long)rec, (unsigned long long)n, (unsigned long long)(nr * rec), ms,
         n / ms / 1e6, n * (double)rec / ms / 1e6);
  fflush(stdout);
}

int main() {
  const int reps = 5;
  int dev;
  hipDeviceProp_t prop;
  CK(hipGetDevice(&dev));
  CK(hipGetDeviceProperties(&prop, dev));
  printf("{\"device\": \"%s\", \"arch\": \"%s\", \"compute_units\": %d}\n", prop.name, prop.gcnArchName,
         prop.multiProcessorCount);
  fflush(stdout);

  // copy: 4 GiB -> 4 GiB
  {
    const int64_t n = (4ll << 30) / 16;
    uint4 *a, *b;
    CK(hipMalloc(&a, n * 16));
    CK(hipMalloc(&b, n * 16));
    CK(hipMemset(a, 1, n * 16));
    k_copy<<<g_blocks * 4, 256>>>(a, b, n);
    CK(hipGetLastError());
    Timer t;
    t.start();
    for (int r = 0; r < reps; ++r) k_copy<<<g_blocks * 4, 256>>>(a, b, n);
    const float ms = t.stop() / reps;
    printf("{\"probe\": \"copy\", \"bytes_moved\": %lld, \"ms\": %.4f, \"gb_per_s\": %.1f}\n", 2 * n * 16, ms,
           2.0 * n * 16 / ms / 1e6);
    fflush(stdout);
    CK(hipFree(a));
    CK(hipFree(b));
  }

  // gathers from a table of 23,000,000 x 64 bytes
  {
    const uint64_t tab_bytes = 23000000ull * 64;
    const int64_t n = 200000000;
    uint4* tab;
    uint32_t *pos, *out;
    CK(hipMalloc(&tab, tab_bytes));
    CK(hipMalloc(&pos, n * 4));
    CK(hipMalloc(&out, (size_t)g_blocks * 256 * 4));
    CK(hipMemset(tab, 0x5a, tab_bytes));
    gather<4, 1>("gather_64B", tab, tab_bytes, pos, n, out, reps);
    gather<8, 1>("gather_128B", tab, tab_bytes, pos, n, out, reps);
    gather<16, 3>("gather_768B", tab, tab_bytes, pos, n / 8, out, reps);
    // the same 64-byte gathers from a 2 MiB table: every XCD's L2 holds it
    gather<4, 1>("gather_64B_l2", tab, 2ull << 20, pos, n, out, reps);
    CK(hipFree(tab));
    CK(hipFree(pos));
    CK(hipFree(out));
  }

  // fp16 MFMA
  {
    v8h* in;
    float* out;
    const int blocks = prop.multiProcessorCount * 8, iters = 5000, C = 4;
    CK(hipMalloc(&in, 128 * sizeof(v8h)));
    CK(hipMemset(in, 0x3c, 128 * sizeof(v8h)));  // every half 0x3c3c (about 1.06)
    CK(hipMalloc(&out, (size_t)blocks * 256 * 4));
    k_mfma<C><<<blocks, 256>>>(in, iters / 10, out);
    CK(hipGetLastError());
    Timer t;
    t.start();
    k_mfma<C><<<blocks, 256>>>(in, iters, out);
    const float ms = t.stop();
    const double flop = (double)blocks * 4 * iters * C * (2.0 * 32 * 32 * 16);
    printf("{\"probe\": \"mfma_f16_32x32x16\", \"flop\": %.4g, \"ms\": %.4f, \"tflop_per_s\": %.1f}\n", flop, ms,
           flop / ms / 1e9);
    fflush(stdout);
    CK(hipFree(in));
    CK(hipFree(out));
  }
  return 0;
}
