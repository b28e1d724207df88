// 512-bit sign-of-random-projection sketches (the binary sketches of Section
// 3.1, compared by Hamming distance).  Projections are exact integers:
// z_j = sum_i R[j][i] * xq_i with R in {-1,+1} and xq_i the coordinate in
// fixed point (scale 2^(e+5), round-to-nearest-even, clamped to +-8191), so
// the sign bits do not depend on summation order.
#include <math.h>

#include "hf_internal.h"

namespace hf {
namespace {

constexpr int SK_DCH = 128;  // dimensions staged per step

// BPT projection bits per thread: 512 / BPT threads per point, 256 threads
// per block.  BPT = 64 (a thread per output word) for large batches;
// BPT = 16 for small ones (query batches), which puts four times as many
// threads on the same sums; lanes 4w .. 4w+3 of a point then OR their
// 16-bit parts into word w.
template <class T, int BPT>
__global__ __launch_bounds__(256) void srp_kernel(const T* __restrict__ X, int64_t N, int d,
                                                  float scale, const uint64_t* __restrict__ Rt,
                                                  uint64_t* __restrict__ out) {
  constexpr int TPP = 512 / BPT, PTS = 256 / TPP, SUB = 64 / BPT;
  __shared__ int16_t sx[PTS][SK_DCH];
  __shared__ uint64_t sr[SK_DCH][8];
  const int pt = threadIdx.x / TPP, tp = threadIdx.x % TPP, w = tp / SUB, sub = tp % SUB;
  const int64_t p0 = (int64_t)blockIdx.x * PTS;
  int32_t z[BPT];
#pragma unroll
  for (int j = 0; j < BPT; ++j) z[j] = 0;
  for (int i0 = 0; i0 < d; i0 += SK_DCH) {
    const int ni = min(SK_DCH, d - i0);
    for (int e = threadIdx.x; e < PTS * SK_DCH; e += 256) {
      int r = e / SK_DCH, c = e % SK_DCH;
      int16_t v = 0;
      if (c < ni && p0 + r < N) {
        float x;
        if constexpr (sizeof(T) == 2)
          x = __half2float(X[(p0 + r) * d + i0 + c]);
        else
          x = X[(p0 + r) * d + i0 + c];
        float q = rintf(x * scale);
        q = fminf(fmaxf(q, -8191.0f), 8191.0f);
        v = (int16_t)q;
      }
      sx[r][c] = v;
    }
    for (int e = threadIdx.x; e < SK_DCH * 8; e += 256) {
      int r = e / 8, c = e % 8;
      sr[r][c] = r < ni ? Rt[(int64_t)(i0 + r) * 8 + c] : 0ull;
    }
    __syncthreads();
    for (int i = 0; i < ni; ++i) {
      int32_t x = sx[pt][i];
      const uint64_t r = sr[i][w] >> (BPT * sub);
#pragma unroll
      for (int j = 0; j < BPT; ++j) z[j] += ((r >> j) & 1ull) ? x : -x;
    }
    __syncthreads();
  }
  uint64_t word = 0;
#pragma unroll
  for (int j = 0; j < BPT; ++j)
    if (z[j] >= 0) word |= 1ull << j;
  if constexpr (SUB > 1) {
    word <<= BPT * sub;
#pragma unroll
    for (int m = 1; m < SUB; m <<= 1) word |= shfl_xor_u64(word, m);
  }
  if (sub == 0 && p0 + pt < N) out[(p0 + pt) * 8 + w] = word;
}

}  // namespace

// Projection signs, transposed for the kernel: Rt[i*8 + w] bit jj is the sign
// of R[64w + jj][i], i.e. bit (64w+jj)*d + i of the SplitMix64 stream.
static std::vector<uint64_t> srp_matrix(int d, uint64_t sketch_seed) {
  int64_t nbits = 512LL * d;
  std::vector<uint64_t> stream((size_t)ceil_div(nbits, 64));
  uint64_t st = sketch_seed;
  for (auto& w : stream) w = splitmix64_next(&st);
  std::vector<uint64_t> Rt((size_t)d * 8, 0ull);
  for (int j = 0; j < 512; ++j)
    for (int i = 0; i < d; ++i) {
      int64_t b = (int64_t)j * d + i;
      if ((stream[(size_t)(b >> 6)] >> (b & 63)) & 1ull) Rt[(size_t)i * 8 + j / 64] |= 1ull << (j % 64);
    }
  return Rt;
}

hf_status srp_matrix_upload(int d, uint64_t sketch_seed, uint64_t** out, size_t* bytes, hipStream_t s) {
  std::vector<uint64_t> Rt = srp_matrix(d, sketch_seed);
  HIP_TRY(hipMalloc(out, Rt.size() * 8));
  HIP_TRY(hipMemcpyAsync(*out, Rt.data(), Rt.size() * 8, hipMemcpyHostToDevice, s));
  // the host copy must outlive the async upload
  HIP_TRY(hipStreamSynchronize(s));
  *bytes = Rt.size() * 8;
  return HF_OK;
}

hf_status srp_sketch(const void* X, hf_dtype dt, int64_t N, int d, int e, uint64_t sketch_seed,
                     uint64_t* out, Workspace& ws, const uint64_t* R_dev) {
  if (N <= 0) return HF_OK;
  float scale = ldexpf(1.0f, e + 5);
  auto launch = [&](const uint64_t* R) -> hf_status {
    // batches below 256K points: 16 bits per thread (a large batch fills the
    // chip at 64 bits per thread, with less staging per point)
    if (N < (1 << 18)) {
      const unsigned grid = (unsigned)ceil_div(N, 8);
      if (dt == HF_F16)
        srp_kernel<__half, 16><<<grid, 256, 0, ws.stream>>>((const __half*)X, N, d, scale, R, out);
      else
        srp_kernel<float, 16><<<grid, 256, 0, ws.stream>>>((const float*)X, N, d, scale, R, out);
    } else {
      const unsigned grid = (unsigned)ceil_div(N, 32);
      if (dt == HF_F16)
        srp_kernel<__half, 64><<<grid, 256, 0, ws.stream>>>((const __half*)X, N, d, scale, R, out);
      else
        srp_kernel<float, 64><<<grid, 256, 0, ws.stream>>>((const float*)X, N, d, scale, R, out);
    }
    HF_LAUNCH_CHECK();
    return HF_OK;
  };
  if (R_dev) return launch(R_dev);  // resident (a forest's): nothing to generate, upload or wait for
  std::vector<uint64_t> Rt = srp_matrix(d, sketch_seed);
  uint64_t* dRt;
  HF_TRY(ws.alloc(&dRt, Rt.size()));
  HIP_TRY(hipMemcpyAsync(dRt, Rt.data(), Rt.size() * 8, hipMemcpyHostToDevice, ws.stream));
  HF_TRY(launch(dRt));
  // the host copy of Rt must outlive the async upload
  HIP_TRY(hipStreamSynchronize(ws.stream));
  return HF_OK;
}

}  // namespace hf
