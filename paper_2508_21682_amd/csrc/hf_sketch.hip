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

// The same projections on the int8 matrix cores.  xq = 64 hi + lo with
// hi = floor(xq / 64) in [-128, 127] and lo in [0, 63], both int8, so
//   z = sum_i (64 R_i) hi_i + R_i lo_i,
// one exact int32-accumulating chain of v_mfma_i32_16x16x64_i8 whose 64-long
// K axis holds 32 coordinates twice: the hi bytes against 64 R (+-64 fits in
// int8) and the lo bytes against R.  A workgroup of four wavefronts scores 64
// points against all 512 projections; wavefront w owns projections
// [128 w, 128 w + 128) for all 64 points (4 row tiles x 8 column tiles), so
// each LDS fragment it reads feeds several products.  Per 32-coordinate step
// the points' hi | lo bytes (64 x 64) and the step's 64 R | R bytes
// (512 x 64) are staged in LDS; the next step's global loads are issued
// before the current step's products.  Sign bits are gathered with ballots.
typedef int int4v __attribute__((ext_vector_type(4)));
// LDS row: 32 hi | 32 lo bytes + 32 pad, so rows sit 32 bytes past a multiple
// of 256 and the 16-row x 4-chunk fragment reads hit distinct banks; sign-bit
// rows of 36 halfwords (the four lanes storing one ballot write rows 4 apart)
constexpr int SM_ROWS = 64, SM_K = 32, SM_PAD = 96, SM_BS = 36;

template <class T>
__device__ __forceinline__ void srp_load_x(const T* __restrict__ X, int64_t row, int d, int c, uint4 (&v)[2]) {
  v[0] = v[1] = make_uint4(0, 0, 0, 0);
  if (row < 0) return;
  if constexpr (sizeof(T) == 2) {
    v[0] = *(const uint4*)(X + row * d + c);
  } else {
    v[0] = *(const uint4*)(X + row * d + c);
    v[1] = *(const uint4*)(X + row * d + c + 4);
  }
}

__device__ __forceinline__ uint32_t srp_q(float x, float scale) {
  float q = rintf(x * scale);
  q = fminf(fmaxf(q, -8191.0f), 8191.0f);
  return (uint32_t)(int)q;
}

template <class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void srp_mfma_kernel(const T* __restrict__ X, int64_t N, int d, float scale,
                                                       const int8_t* __restrict__ Rb,
                                                       uint64_t* __restrict__ out) {
  __shared__ __align__(16) int8_t s_x[SM_ROWS * SM_PAD];
  __shared__ __align__(16) int8_t s_r[512 * SM_PAD];
  __shared__ __align__(16) uint16_t s_bits[SM_ROWS * SM_BS];
  const int wv = threadIdx.x / 64, l = __lane_id(), ri = l % 16, g = l / 16;
  const int64_t p0 = (int64_t)blockIdx.x * SM_ROWS;
  // staging roles: row xr, coordinates 8 xc .. 8 xc + 7 of the step; and
  // projection rows rj + 128 m (m = 0..3), 16 coordinates at 16 rc
  const int xr = threadIdx.x / 4, xc = threadIdx.x % 4;
  const int64_t xrow = p0 + xr < N ? p0 + xr : -1;
  const int rj = threadIdx.x / 2, rc = threadIdx.x % 2;
  int4v acc[4][8];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) acc[rt][cb] = (int4v){0, 0, 0, 0};
  uint4 xv[2], rv[4];
  auto issue = [&](int k0) {
    const int cx = k0 + 8 * xc;
    srp_load_x<T>(X, cx < d ? xrow : -1, d, cx, xv);
    const int cr = k0 + 16 * rc;
#pragma unroll
    for (int m = 0; m < 4; ++m)
      rv[m] = cr < d ? *(const uint4*)(Rb + (int64_t)(rj + 128 * m) * d + cr) : make_uint4(0, 0, 0, 0);
  };
  issue(0);
  for (int k0 = 0; k0 < d; k0 += SM_K) {
    __syncthreads();  // the previous step's fragments have been read
    {
      float f[8];
      if constexpr (sizeof(T) == 2) {
        const __half2* h = (const __half2*)&xv[0];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float2 t = __half22float2(h[j]);
          f[2 * j] = t.x;
          f[2 * j + 1] = t.y;
        }
      } else {
        const float* a = (const float*)&xv[0];
#pragma unroll
        for (int j = 0; j < 8; ++j) f[j] = a[j];
      }
      uint32_t hi[2] = {0, 0}, lo[2] = {0, 0};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t q = srp_q(f[j], scale);
        const uint32_t h = (uint32_t)((int)q >> 6);  // floor(xq / 64)
        hi[j / 4] |= (h & 0xFFu) << (8 * (j % 4));
        lo[j / 4] |= (q & 0x3Fu) << (8 * (j % 4));
      }
      *(uint2*)(s_x + xr * SM_PAD + 8 * xc) = make_uint2(hi[0], hi[1]);
      *(uint2*)(s_x + xr * SM_PAD + 32 + 8 * xc) = make_uint2(lo[0], lo[1]);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const uint4 r = rv[m];
        // bytes +1 / -1 times 64: 0x40 / 0xC0 (zero bytes stay zero)
        const uint4 r64 = make_uint4((r.x << 6) & 0xC0C0C0C0u, (r.y << 6) & 0xC0C0C0C0u, (r.z << 6) & 0xC0C0C0C0u,
                                     (r.w << 6) & 0xC0C0C0C0u);
        int8_t* row = s_r + (rj + 128 * m) * SM_PAD;
        *(uint4*)(row + 16 * rc) = r64;
        *(uint4*)(row + 32 + 16 * rc) = r;
      }
    }
    __syncthreads();
    if (k0 + SM_K < d) issue(k0 + SM_K);
    int4v a[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) a[rt] = *(const int4v*)(s_x + (16 * rt + ri) * SM_PAD + 16 * g);
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) {
      const int4v b = *(const int4v*)(s_r + (128 * wv + 16 * cb + ri) * SM_PAD + 16 * g);
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) acc[rt][cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[rt], b, acc[rt][cb], 0, 0, 0);
    }
  }
  // lane l holds points 16 rt + 4 g + r, projection 128 wv + 16 cb + ri; the
  // ballot's bits 16 g' + i are point 16 rt + 4 g' + r, projection
  // 128 wv + 16 cb + i: one 16-bit part of one point's sketch
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int cb = 0; cb < 8; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint64_t m = __ballot(acc[rt][cb][r] >= 0);
        if (l < 4) s_bits[(16 * rt + 4 * l + r) * SM_BS + 8 * wv + cb] = (uint16_t)(m >> (16 * l));
      }
  __syncthreads();
  for (int e = threadIdx.x; e < SM_ROWS * 8; e += 256) {
    const int r = e / 8, w = e % 8;
    if (p0 + r < N) out[(p0 + r) * 8 + w] = *(const uint64_t*)(s_bits + r * SM_BS + 4 * w);
  }
}

}  // namespace

// Projection signs as int8 (+1 / -1) rows: Rb[j * d + i] = sign of R[j][i].
static std::vector<int8_t> srp_matrix_i8(int d, uint64_t sketch_seed) {
  int64_t nbits = 512LL * d;
  std::vector<uint64_t> stream((size_t)ceil_div(nbits, 64));
  uint64_t st = sketch_seed;
  for (auto& w : stream) w = splitmix64_next(&st);
  std::vector<int8_t> Rb((size_t)512 * d);
  for (int64_t b = 0; b < nbits; ++b) Rb[(size_t)b] = ((stream[(size_t)(b >> 6)] >> (b & 63)) & 1ull) ? 1 : -1;
  return Rb;
}

hf_status srp_matrix_i8_upload(int d, uint64_t sketch_seed, int8_t** out, hipStream_t s) {
  std::vector<int8_t> Rb = srp_matrix_i8(d, sketch_seed);
  HIP_TRY(hipMalloc(out, Rb.size()));
  HIP_TRY(hipMemcpyAsync(*out, Rb.data(), Rb.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return HF_OK;
}

hf_status srp_sketch_mfma(const void* X, hf_dtype dt, int64_t N, int d, int e, const int8_t* Rb, uint64_t* out,
                          hipStream_t s) {
  if (N <= 0) return HF_OK;
  const float scale = ldexpf(1.0f, e + 5);
  const unsigned grid = (unsigned)ceil_div(N, SM_ROWS);
  if (dt == HF_F16)
    srp_mfma_kernel<__half><<<grid, 256, 0, s>>>((const __half*)X, N, d, scale, Rb, out);
  else
    srp_mfma_kernel<float><<<grid, 256, 0, s>>>((const float*)X, N, d, scale, Rb, out);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

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
  if (d % 16 == 0 && getenv("HF_SRP_VALU") == nullptr) {
    // the int8 matrix-core kernel, its projection in the call's workspace
    std::vector<int8_t> Rb = srp_matrix_i8(d, sketch_seed);
    int8_t* dRb;
    HF_TRY(ws.alloc(&dRb, Rb.size()));
    HIP_TRY(hipMemcpyAsync(dRb, Rb.data(), Rb.size(), hipMemcpyHostToDevice, ws.stream));
    HF_TRY(srp_sketch_mfma(X, dt, N, d, e, dRb, out, ws.stream));
    // the host copy of Rb must outlive the async upload
    HIP_TRY(hipStreamSynchronize(ws.stream));
    return HF_OK;
  }
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
