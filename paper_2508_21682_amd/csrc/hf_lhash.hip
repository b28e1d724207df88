// Learned hash (not in the paper): an MLP d -> hidden -> 512 whose output
// signs replace the SRP sketch bits.
//
// Forward (encode and training): two MFMA layers (v_mfma_f32_16x16x32_bf16)
// with BF16 inputs and weights and FP32 accumulation; a wavefront computes 16
// rows x 256 outputs, weights streamed from L2.  The hidden activations are
// relu(z1) rounded to BF16.
// Training: codes c = tanh(slope*z2); an InfoNCE loss over the in-batch pairs
// plus a bit-balance term; the backward pass is a chain of FP32 GEMMs (FP32
// MFMA from LDS tiles) and element-wise kernels; AdamW keeps FP32 master
// weights and refreshes the BF16 copies after every step.
#include <math.h>

#include <type_traits>

#include <string.h>

#include "hf_internal.h"

struct hf_lhash {
  uint32_t magic;
  int device;
  int d, hid;
  float *W1, *b1, *W2, *b2;  // FP32 master weights: W1 hid x d, W2 512 x hid
  uint16_t *W1b, *W2b;       // BF16 copies used by the forward
  uint16_t *W1p, *W2p;       // the same BF16 values in MFMA fragment order
  float* mom[4];             // Adam first moments (W1, b1, W2, b2)
  float* vel[4];             // Adam second moments
  int64_t step;
};
constexpr uint32_t HF_LHASH_MAGIC = 0x48464c48u;  // "HFLH"

namespace hf {
namespace {

typedef float float4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_to_f(uint32_t b) { return __uint_as_float(b << 16); }

inline unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, ceil_div(n, 256)));
}

__global__ void k_f32_to_bf16(const float* __restrict__ w, int64_t n, uint16_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = (uint16_t)bf16_rne(w[i]);
}

// BF16 weights W (ncol x K, row-major; ncol % 16 == 0, K % 32 == 0) in the
// order the B operand of v_mfma_f32_16x16x32_bf16 takes them: for column tile
// ct and K step ks, 64 lanes x 8 values, lane l holding W[16 ct + l % 16]
// [32 ks + 8 (l / 16) + j], so a wavefront's fragment is 1 KB in one run.
__global__ void k_pack_frag(const uint16_t* __restrict__ W, int ncol, int K, uint16_t* __restrict__ out) {
  const int64_t n = (int64_t)ncol * K;
  const int ksn = K / 32;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int j = (int)(i % 8), l = (int)(i / 8 % 64);
    const int64_t blk = i / 512;
    const int ks = (int)(blk % ksn), ct = (int)(blk / ksn);
    out[i] = W[(int64_t)(16 * ct + l % 16) * K + 32 * ks + 8 * (l / 16) + j];
  }
}

// 8 consecutive input values of row r starting at column k (zero past K) as BF16.
template <class T>
__device__ __forceinline__ uint4 load8_bf16(const T* __restrict__ X, int64_t r, int K, int k) {
  if (r < 0 || k >= K) return make_uint4(0, 0, 0, 0);
  const T* p = X + r * K + k;
  float f[8];
  if constexpr (sizeof(T) == 2 && !std::is_same<T, uint16_t>::value) {
    uint4 raw = *(const uint4*)p;
    const __half2* h = (const __half2*)&raw;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float2 v = __half22float2(h[j]);
      f[2 * j] = v.x;
      f[2 * j + 1] = v.y;
    }
  } else if constexpr (std::is_same<T, uint16_t>::value) {
    return *(const uint4*)p;  // already BF16
  } else {
    float4 a = *(const float4*)p, b = *(const float4*)(p + 4);
    f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w; f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
  }
  uint4 o;
  o.x = bf16_rne(f[0]) | (bf16_rne(f[1]) << 16);
  o.y = bf16_rne(f[2]) | (bf16_rne(f[3]) << 16);
  o.z = bf16_rne(f[4]) | (bf16_rne(f[5]) << 16);
  o.w = bf16_rne(f[6]) | (bf16_rne(f[7]) << 16);
  return o;
}

// One layer: Y[r][c] = sum_k A[r][k] * W[c][k] + bias[c] for a 16-row block
// and up to 256 columns per pass.  MODE 1: relu, BF16 store to H (M x ncol);
// MODE 2: FP32 store to Z (optional) and sign bits to SK (optional, 8 words/row).
template <class T, int MODE>
__global__ __launch_bounds__(256) void k_mlp(const T* __restrict__ A, int64_t M, int K,
                                             const uint16_t* __restrict__ W, const float* __restrict__ bias,
                                             int ncol, uint16_t* __restrict__ H, float* __restrict__ Z,
                                             uint64_t* __restrict__ SK) {
  __shared__ uint32_t bits[4][16][16];  // per wave: 16 rows x 512 bits
  const int wv = threadIdx.x / 64, l = __lane_id(), ri = l % 16, g = l / 16;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
  if (r0 >= M) return;  // waves are independent
  const int64_t arow = r0 + ri < M ? r0 + ri : -1;
  if (MODE == 2 && SK) {
    for (int i = l; i < 16 * 16; i += 64) (&bits[wv][0][0])[i] = 0u;
  }
  const int ksteps = (K + 31) / 32;
  for (int c0 = 0; c0 < ncol; c0 += 256) {
    const int nb = min(16, (ncol - c0) / 16);
    float4v acc[16];
#pragma unroll
    for (int cb = 0; cb < 16; ++cb) acc[cb] = (float4v){0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < ksteps; ++s) {
      const int k = 32 * s + 8 * g;
      const uint4 a = load8_bf16<T>(A, arow, K, k);
#pragma unroll
      for (int cb = 0; cb < 16; ++cb) {
        if (cb < nb) {
          const int c = c0 + cb * 16 + ri;
          const uint4 b = k < K ? *(const uint4*)(W + (int64_t)c * K + k) : make_uint4(0, 0, 0, 0);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                            __builtin_bit_cast(bf16x8, b), acc[cb], 0, 0, 0);
        }
      }
    }
    // D layout: lane l holds rows 4*(l/16)+r, column l%16 of each block
#pragma unroll
    for (int cb = 0; cb < 16; ++cb) {
      if (cb < nb) {
        const int c = c0 + cb * 16 + ri;
        const float bc = bias[c];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = r0 + 4 * g + r;
          const float v = acc[cb][r] + bc;
          if (row < M) {
            if (MODE == 1) {
              H[row * ncol + c] = (uint16_t)bf16_rne(v > 0.f ? v : 0.f);
            } else {
              if (Z) Z[row * ncol + c] = v;
              if (SK && v >= 0.f) atomicOr(&bits[wv][4 * g + r][c >> 5], 1u << (c & 31));
            }
          }
        }
      }
    }
  }
  if (MODE == 2 && SK) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int i = l; i < 16 * 16; i += 64) {
      const int row = i / 16, w = i % 16;
      if (r0 + row < M) ((uint32_t*)SK)[(r0 + row) * 16 + w] = bits[wv][row][w];
    }
  }
}

// 8 values of T as BF16, from the raw bytes of one (half) or two (float) uint4
template <class T>
__device__ __forceinline__ uint4 raw_to_bf16(uint4 r0, uint4 r1) {
  float f[8];
  if constexpr (sizeof(T) == 2) {
    const __half2* h = (const __half2*)&r0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float2 v = __half22float2(h[j]);
      f[2 * j] = v.x;
      f[2 * j + 1] = v.y;
    }
  } else {
    const float* a = (const float*)&r0;
    const float* b = (const float*)&r1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      f[j] = a[j];
      f[4 + j] = b[j];
    }
  }
  uint4 o;
  o.x = bf16_rne(f[0]) | (bf16_rne(f[1]) << 16);
  o.y = bf16_rne(f[2]) | (bf16_rne(f[3]) << 16);
  o.z = bf16_rne(f[4]) | (bf16_rne(f[5]) << 16);
  o.w = bf16_rne(f[6]) | (bf16_rne(f[7]) << 16);
  return o;
}

// Columns [col0, col0 + 16 NC) (col0 % 16 == 0) of a dense layer for the
// 128 rows held in LDS (row stride AS, K inputs) into acc, from weights in
// fragment order (k_pack_frag); the weight fragments of step k + 32 are
// loaded while step k's products run.
template <int K, int NC>
__device__ __forceinline__ void ws_layer(const uint16_t* __restrict__ sa, int AS, const uint16_t* __restrict__ Wp,
                                         int col0, int ri, int g, float4v (&acc)[8][NC]) {
#pragma unroll
  for (int rt = 0; rt < 8; ++rt)
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) acc[rt][cb] = (float4v){0.f, 0.f, 0.f, 0.f};
  // fragment (ct, ks) starts at 512 (ct K / 32 + ks); a step of k is k * 16
  const uint16_t* wp = Wp + (int64_t)(col0 / 16) * K * 16 + 8 * (ri + 16 * g);
  uint4 bw[NC], bn[NC];
#pragma unroll
  for (int cb = 0; cb < NC; ++cb) bw[cb] = *(const uint4*)(wp + (int64_t)cb * 16 * K);
  // not unrolled: the LDS fragment loads of later steps are not hoisted
#pragma unroll 1
  for (int k = 0; k < K; k += 32) {
    if (k + 32 < K) {
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) bn[cb] = *(const uint4*)(wp + (int64_t)cb * 16 * K + 16 * (k + 32));
    }
#pragma unroll
    for (int rt = 0; rt < 8; ++rt) {
      const uint4 a = *(const uint4*)(sa + (16 * rt + ri) * AS + k + 8 * g);
#pragma unroll
      for (int cb = 0; cb < NC; ++cb)
        acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                              __builtin_bit_cast(bf16x8, bw[cb]), acc[rt][cb], 0, 0, 0);
    }
    if (k + 32 < K) {
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) bw[cb] = bn[cb];
    }
  }
}

// Encoder, persistent form: one workgroup of eight wavefronts per CU walks
// blocks of 128 rows.  Per block the rows (BF16) sit in LDS and each
// wavefront computes a column slice of a layer for all 128 rows (layer 1: 32
// hidden units; layer 2: 64 outputs in two passes of 32), so a weight element
// is read from L2 once per 128 rows, each wavefront's weight fragment as one
// contiguous kilobyte (k_pack_frag); the hidden activations then overwrite
// the rows in LDS.  The next block's rows (fp16 input) are loaded into
// registers while the current block's products run.  Same summation order as
// the two-kernel path, so the sketches are equal.
constexpr int WS_ROWS = 128, WS_T = 512, WS_PASSES = 2;
template <class T, int D, int HID>
__global__ __launch_bounds__(WS_T) void k_mlp_ws(const T* __restrict__ X, int64_t M,
                                                 const uint16_t* __restrict__ W1, const float* __restrict__ b1,
                                                 const uint16_t* __restrict__ W2, const float* __restrict__ b2,
                                                 uint64_t* __restrict__ SK) {
  // row strides of 32 bytes past a multiple of 256: the A-fragment reads
  // (16 rows x 4 chunks of 16 bytes) then hit distinct banks; 16 bytes past
  // costs four conflict cycles a read
  constexpr int XS = D + 16, HS = HID + 16;
  static_assert((2 * XS) % 256 == 32 && (2 * HS) % 256 == 32, "row padding");
  constexpr int XH = WS_ROWS * (XS > HS ? XS : HS);
  constexpr int NC1 = HID / 8 / 16;              // layer-1 column tiles per wavefront
  constexpr int PER = WS_ROWS * (D / 8) / WS_T;  // 8-value chunks a thread stages
  constexpr bool PREF = sizeof(T) == 2;          // fp16 rows prefetched a block ahead
  static_assert(PER * WS_T == WS_ROWS * (D / 8) && HID % 128 == 0 && D % 32 == 0, "shape");
  __shared__ __align__(16) uint16_t s_xh[XH];
  // sign bits, 36 halfwords a row: the four lanes that store one ballot write
  // rows 4 apart, which a 32-halfword stride would put in one bank
  constexpr int BS = 36;
  __shared__ __align__(16) uint16_t s_bits[WS_ROWS * BS];
  const int wv = threadIdx.x / 64, l = __lane_id(), ri = l % 16, g = l / 16;
  const int64_t nblk = (M + WS_ROWS - 1) / WS_ROWS;
  uint4 xr[PREF ? PER : 1];
  auto load_rows = [&](int64_t blk) {
    const int64_t r0 = blk * WS_ROWS;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + WS_T * i, r = e / (D / 8), c8 = e % (D / 8);
      const int64_t row = r0 + r < M ? r0 + r : M - 1;
      xr[PREF ? i : 0] = *(const uint4*)(X + row * D + 8 * c8);
      if constexpr (!PREF) {
        // float rows: converted and stored at once (no prefetch)
        const uint4 hi = *(const uint4*)(X + row * D + 8 * c8 + 4);
        uint4 v = raw_to_bf16<T>(xr[0], hi);
        if (r0 + r >= M) v = make_uint4(0, 0, 0, 0);
        *(uint4*)(s_xh + r * XS + 8 * c8) = v;
      }
    }
  };
  if (PREF && blockIdx.x < nblk) load_rows(blockIdx.x);
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t r0 = blk * WS_ROWS;
    __syncthreads();  // the previous block's hidden units and sign bits are consumed
    if constexpr (PREF) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + WS_T * i, r = e / (D / 8), c8 = e % (D / 8);
        uint4 v = raw_to_bf16<T>(xr[i], make_uint4(0, 0, 0, 0));
        if (r0 + r >= M) v = make_uint4(0, 0, 0, 0);
        *(uint4*)(s_xh + r * XS + 8 * c8) = v;
      }
    } else {
      load_rows(blk);
    }
    __syncthreads();
    if (PREF && blk + gridDim.x < nblk) load_rows(blk + gridDim.x);
    {
      float4v acc[8][NC1];
      ws_layer<D, NC1>(s_xh, XS, W1, wv * NC1 * 16, ri, g, acc);
      __syncthreads();  // every wavefront is done with the rows
#pragma unroll
      for (int cb = 0; cb < NC1; ++cb) {
        const int c = wv * NC1 * 16 + cb * 16 + ri;
        const float bc = b1[c];
#pragma unroll
        for (int rt = 0; rt < 8; ++rt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float v = acc[rt][cb][r] + bc;
            s_xh[(16 * rt + 4 * g + r) * HS + c] = (uint16_t)bf16_rne(v > 0.f ? v : 0.f);
          }
      }
    }
    __syncthreads();
    constexpr int PS = WS_PASSES, NCP = 4 / PS;  // layer-2 passes and their column tiles
#pragma unroll
    for (int ps = 0; ps < PS; ++ps) {
      // outputs [64 wv + 16 NCP ps, + 16 NCP): the ballot's bits 16 g' + i
      // are row 16 rt + 4 g' + r, output c0 + i
      float4v acc[8][NCP];
      ws_layer<HID, NCP>(s_xh, HS, W2, 64 * wv + 16 * NCP * ps, ri, g, acc);
#pragma unroll
      for (int cb = 0; cb < NCP; ++cb) {
        const int c0 = 64 * wv + 16 * NCP * ps + 16 * cb;
        const float bc = b2[c0 + ri];
#pragma unroll
        for (int rt = 0; rt < 8; ++rt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint64_t m = __ballot(acc[rt][cb][r] + bc >= 0.f);
            if (l < 4) s_bits[(16 * rt + 4 * l + r) * BS + c0 / 16] = (uint16_t)(m >> (16 * l));
          }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < WS_ROWS * 8; e += WS_T) {
      const int r = e / 8, w = e % 8;
      if (r0 + r < M) SK[(r0 + r) * 8 + w] = *(const uint64_t*)(s_bits + r * BS + 4 * w);
    }
  }
}

// C = alpha * op(A) * op(B) + beta * C, FP32, row-major storage; op(A)[m][k] =
// A[m*sam + k*sak], op(B)[k][n] = B[k*sbk + n*sbn]; on v_mfma_f32_16x16x4_f32
// (FP32 operands and sums).  64x64 tiles, four wavefronts of 32x32 (2 x 2 MFMA
// tiles); K in LDS steps of 16.
// Lane l of a 16x16x4 product holds A[l % 16][l / 16] and B[l / 16][l % 16]
// and returns C[4 (l / 16) + r][l % 16] in register r.  Tile loads run along
// whichever index of the operand has unit stride, so they are coalesced.
__global__ __launch_bounds__(256) void k_sgemm(int M, int N, int K, float alpha, const float* __restrict__ A,
                                               int64_t sam, int64_t sak, const float* __restrict__ B,
                                               int64_t sbk, int64_t sbn, float beta, float* __restrict__ C,
                                               int64_t ldc) {
  constexpr int LS = 64 + 16;  // row stride of the LDS tiles
  __shared__ float As[16][LS];
  __shared__ float Bs[16][LS];
  const int l = __lane_id(), wv = threadIdx.x / 64, wm = wv / 2, wn = wv % 2;
  const int i16 = l % 16, kq = l / 16;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const bool a_k = sak == 1, b_k = sbk == 1;  // unit stride along k
  float4v acc[2][2];
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn) acc[tm][tn] = (float4v){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = threadIdx.x + 256 * u;
      {
        const int kk = a_k ? i % 16 : i / 64, mm = a_k ? i / 16 : i % 64;
        const int m = m0 + mm, k = k0 + kk;
        As[kk][mm] = (m < M && k < K) ? A[(int64_t)m * sam + (int64_t)k * sak] : 0.f;
      }
      {
        const int kk = b_k ? i % 16 : i / 64, nn = b_k ? i / 16 : i % 64;
        const int n = n0 + nn, k = k0 + kk;
        Bs[kk][nn] = (n < N && k < K) ? B[(int64_t)k * sbk + (int64_t)n * sbn] : 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      float a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[kk + kq][32 * wm + 16 * t + i16];
        b[t] = Bs[kk + kq][32 * wn + 16 * t + i16];
      }
#pragma unroll
      for (int tm = 0; tm < 2; ++tm)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn)
          acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[tm], b[tn], acc[tm][tn], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + 32 * wm + 16 * tm + 4 * kq + r, n = n0 + 32 * wn + 16 * tn + i16;
        if (m < M && n < N) {
          float* c = C + (int64_t)m * ldc + n;
          *c = alpha * acc[tm][tn][r] + (beta != 0.f ? beta * *c : 0.f);
        }
      }
}

__global__ void k_tanh(const float* __restrict__ z, int64_t n, float slope, float* __restrict__ c) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    c[i] = tanhf(slope * z[i]);
}

// Row-wise softmax gradient of the InfoNCE loss: G = (softmax(S/tau) - I) / (tau*B);
// per-row loss terms to rl.  With hard negatives (Hn non-null) row i has one
// more logit Hn[i], whose gradient goes to Gn[i].  One wavefront per row.
__global__ void k_infonce(const float* __restrict__ S, const float* __restrict__ Hn, int B, float tau,
                          float* __restrict__ G, float* __restrict__ Gn, float* __restrict__ rl) {
  const int i = blockIdx.x * 4 + threadIdx.x / 64;
  if (i >= B) return;
  const float* s = S + (int64_t)i * B;
  float mx = Hn ? Hn[i] / tau : -INFINITY;
  for (int j = __lane_id(); j < B; j += 64) mx = fmaxf(mx, s[j] / tau);
  for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  float sum = 0.f;
  for (int j = __lane_id(); j < B; j += 64) sum += expf(s[j] / tau - mx);
  for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o);
  if (Hn) sum += expf(Hn[i] / tau - mx);
  for (int j = __lane_id(); j < B; j += 64)
    G[(int64_t)i * B + j] = (expf(s[j] / tau - mx) / sum - (i == j ? 1.f : 0.f)) / (tau * (float)B);
  if (__lane_id() == 0) {
    if (Hn) Gn[i] = expf(Hn[i] / tau - mx) / sum / (tau * (float)B);
    rl[i] = (mx + logf(sum) - s[i] / tau) / (float)B;
  }
}

// Hn[i] = <Cq_i, Cn_i> / 512 (a wavefront per row).
__global__ void k_rowdot(const float* __restrict__ Cq, const float* __restrict__ Cn, int B,
                         float* __restrict__ Hn) {
  const int i = blockIdx.x * 4 + threadIdx.x / 64;
  if (i >= B) return;
  float a = 0.f;
  for (int b = __lane_id(); b < 512; b += 64) a += Cq[(int64_t)i * 512 + b] * Cn[(int64_t)i * 512 + b];
  for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
  if (__lane_id() == 0) Hn[i] = a / 512.f;
}

// The negative logit's part of the code gradients: dCq_i += Gn_i Cn_i / 512,
// dCn_i = Gn_i Cq_i / 512.
__global__ void k_neg_grad(const float* __restrict__ Cq, const float* __restrict__ Cn, const float* __restrict__ Gn,
                           int B, float* __restrict__ dCq, float* __restrict__ dCn) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < (int64_t)B * 512; t += (int64_t)gridDim.x * 256) {
    const float g = Gn[t / 512] / 512.f;
    dCq[t] += g * Cn[t];
    dCn[t] = g * Cq[t];
  }
}

__global__ void k_zero_f32(float* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.f;
}

// Column means of C (R x 512) and the balance part of the loss.
__global__ void k_colmean(const float* __restrict__ C, int R, float* __restrict__ m) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= 512) return;
  float a = 0.f;
  for (int r = 0; r < R; ++r) a += C[(int64_t)r * 512 + b];
  m[b] = a / (float)R;
}

// dZ2 = (dC + lambda*2*m/R) * slope * (1 - c^2)
__global__ void k_dz2(const float* __restrict__ dC, const float* __restrict__ C, const float* __restrict__ m,
                      int R, float lambda, float slope, float* __restrict__ dZ) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < (int64_t)R * 512; i += (int64_t)gridDim.x * 256) {
    const float c = C[i];
    dZ[i] = (dC[i] + lambda * 2.f * m[i % 512] / (float)R) * slope * (1.f - c * c);
  }
}

__global__ void k_bf16_rows_to_f32(const uint16_t* __restrict__ h, int64_t n, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = bf16_to_f(h[i]);
}

template <class T>
__global__ void k_rows_to_bf16f(const T* __restrict__ X, int64_t n, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    float v;
    if constexpr (sizeof(T) == 2)
      v = __half2float(X[i]);
    else
      v = X[i];
    out[i] = bf16_to_f(bf16_rne(v));
  }
}

// dZ1 = dH * [h > 0]  (h = bf16(relu(z1)) > 0 exactly when z1 > 0)
__global__ void k_relu_grad(const float* __restrict__ dH, const uint16_t* __restrict__ h, int64_t n,
                            float* __restrict__ dZ) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dZ[i] = h[i] ? dH[i] : 0.f;
}

__global__ void k_colsum(const float* __restrict__ X, int R, int n, float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  float a = 0.f;
  for (int r = 0; r < R; ++r) a += X[(int64_t)r * n + c];
  out[c] = a;
}

// loss = sum of row terms + lambda * sum_b m_b^2
__global__ void k_loss(const float* __restrict__ rl, int B, const float* __restrict__ m, float lambda,
                       float* __restrict__ out) {
  __shared__ float s[256];
  float a = 0.f;
  for (int i = threadIdx.x; i < B; i += 256) a += rl[i];
  for (int b = threadIdx.x; b < 512; b += 256) a += lambda * m[b] * m[b];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out += s[0];
}

__global__ void k_adamw(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float wd,
                        float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * w[i]);
  }
}

template <class T>
__global__ void k_gather(const T* __restrict__ X, int d, const uint32_t* __restrict__ idx, int64_t n,
                         T* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n * d; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / d;
    out[i] = X[(int64_t)idx[r] * d + (i - r * d)];
  }
}

hf_status sgemm(hipStream_t s, int M, int N, int K, float alpha, const float* A, int64_t sam, int64_t sak,
                const float* B, int64_t sbk, int64_t sbn, float beta, float* C, int64_t ldc) {
  dim3 grid((unsigned)ceil_div(N, 64), (unsigned)ceil_div(M, 64));
  k_sgemm<<<grid, 256, 0, s>>>(M, N, K, alpha, A, sam, sak, B, sbk, sbn, beta, C, ldc);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

template <class T, int MODE>
hf_status mlp_layer(hipStream_t s, const T* A, int64_t M, int K, const uint16_t* W, const float* bias, int ncol,
                    uint16_t* H, float* Z, uint64_t* SK) {
  if (M <= 0) return HF_OK;
  k_mlp<T, MODE><<<(unsigned)ceil_div(M, 64), 256, 0, s>>>(A, M, K, W, bias, ncol, H, Z, SK);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

// Forward of n rows of X: hidden activations to H (n x hid BF16); z2 (n x 512)
// to Z and/or sign bits to SK.
hf_status lhash_forward(const hf_lhash* L, const void* X, hf_dtype dt, int64_t n, uint16_t* H, float* Z,
                        uint64_t* SK, hipStream_t s) {
  if (dt == HF_F16)
    HF_TRY((mlp_layer<__half, 1>(s, (const __half*)X, n, L->d, L->W1b, L->b1, L->hid, H, nullptr, nullptr)));
  else
    HF_TRY((mlp_layer<float, 1>(s, (const float*)X, n, L->d, L->W1b, L->b1, L->hid, H, nullptr, nullptr)));
  HF_TRY((mlp_layer<uint16_t, 2>(s, H, n, L->hid, L->W2b, L->b2, 512, nullptr, Z, SK)));
  return HF_OK;
}

hf_status refresh_bf16(hf_lhash* L, hipStream_t s) {
  const int64_t n1 = (int64_t)L->hid * L->d, n2 = 512LL * L->hid;
  k_f32_to_bf16<<<grid_for(n1), 256, 0, s>>>(L->W1, n1, L->W1b);
  k_f32_to_bf16<<<grid_for(n2), 256, 0, s>>>(L->W2, n2, L->W2b);
  HF_LAUNCH_CHECK();
  if (L->W1p) {
    k_pack_frag<<<grid_for(n1), 256, 0, s>>>(L->W1b, L->hid, L->d, L->W1p);
    k_pack_frag<<<grid_for(n2), 256, 0, s>>>(L->W2b, 512, L->hid, L->W2p);
    HF_LAUNCH_CHECK();
  }
  return HF_OK;
}

// Loss (added to *loss_dev) and gradients (device) of one batch of B pairs:
// rows A[0..B) and P[0..B), and hard negatives Ng[0..B) when Ng is non-null.
hf_status lhash_grad(const hf_lhash* L, const void* A, const void* P, const void* Ng, hf_dtype dt, int B,
                     const hf_lhash_train_params& tp, float* loss_dev, float* gW1, float* gb1, float* gW2,
                     float* gb2, Workspace& ws) {
  hipStream_t s = ws.stream;
  const int R = (Ng ? 3 : 2) * B, hid = L->hid, d = L->d;
  const size_t esz = dt == HF_F16 ? 2 : 4;
  uint16_t* H;
  float *Z, *Cc, *S, *G, *dC, *m, *rl, *dZ, *Hf, *dH, *Xf;
  HF_TRY(ws.alloc(&H, (size_t)R * hid));
  HF_TRY(ws.alloc(&Z, (size_t)R * 512));
  HF_TRY(ws.alloc(&Cc, (size_t)R * 512));
  HF_TRY(ws.alloc(&S, (size_t)B * B));
  HF_TRY(ws.alloc(&G, (size_t)B * B));
  HF_TRY(ws.alloc(&dC, (size_t)R * 512));
  HF_TRY(ws.alloc(&m, 512));
  HF_TRY(ws.alloc(&rl, (size_t)B));
  HF_TRY(ws.alloc(&dZ, (size_t)R * 512));
  HF_TRY(ws.alloc(&Hf, (size_t)R * hid));
  HF_TRY(ws.alloc(&dH, (size_t)R * hid));
  HF_TRY(ws.alloc(&Xf, (size_t)R * d));
  HF_TRY(lhash_forward(L, A, dt, B, H, Z, nullptr, s));
  HF_TRY(lhash_forward(L, P, dt, B, H + (size_t)B * hid, Z + (size_t)B * 512, nullptr, s));
  if (Ng) HF_TRY(lhash_forward(L, Ng, dt, B, H + (size_t)2 * B * hid, Z + (size_t)2 * B * 512, nullptr, s));
  k_tanh<<<grid_for((int64_t)R * 512), 256, 0, s>>>(Z, (int64_t)R * 512, tp.slope, Cc);
  HF_LAUNCH_CHECK();
  const float* Cq = Cc;
  const float* Cp = Cc + (size_t)B * 512;
  // S = Cq Cp^T / 512
  HF_TRY(sgemm(s, B, B, 512, 1.f / 512.f, Cq, 512, 1, Cp, 1, 512, 0.f, S, B));
  float *Hn = nullptr, *Gn = nullptr;
  if (Ng) {
    HF_TRY(ws.alloc(&Hn, (size_t)B));
    HF_TRY(ws.alloc(&Gn, (size_t)B));
    k_rowdot<<<(unsigned)ceil_div(B, 4), 256, 0, s>>>(Cq, Cc + (size_t)2 * B * 512, B, Hn);
  }
  k_infonce<<<(unsigned)ceil_div(B, 4), 256, 0, s>>>(S, Hn, B, tp.tau, G, Gn, rl);
  HF_LAUNCH_CHECK();
  // dCq = G Cp / 512 ; dCp = G^T Cq / 512
  HF_TRY(sgemm(s, B, 512, B, 1.f / 512.f, G, B, 1, Cp, 512, 1, 0.f, dC, 512));
  HF_TRY(sgemm(s, B, 512, B, 1.f / 512.f, G, 1, B, Cq, 512, 1, 0.f, dC + (size_t)B * 512, 512));
  if (Ng) {
    k_neg_grad<<<grid_for((int64_t)B * 512), 256, 0, s>>>(Cq, Cc + (size_t)2 * B * 512, Gn, B, dC,
                                                           dC + (size_t)2 * B * 512);
    HF_LAUNCH_CHECK();
  }
  k_colmean<<<2, 256, 0, s>>>(Cc, R, m);
  k_loss<<<1, 256, 0, s>>>(rl, B, m, tp.balance, loss_dev);
  k_dz2<<<grid_for((int64_t)R * 512), 256, 0, s>>>(dC, Cc, m, R, tp.balance, tp.slope, dZ);
  k_bf16_rows_to_f32<<<grid_for((int64_t)R * hid), 256, 0, s>>>(H, (int64_t)R * hid, Hf);
  HF_LAUNCH_CHECK();
  // dW2 = dZ^T H ; db2 = colsum(dZ)
  HF_TRY(sgemm(s, 512, hid, R, 1.f, dZ, 1, 512, Hf, hid, 1, 0.f, gW2, hid));
  k_colsum<<<2, 256, 0, s>>>(dZ, R, 512, gb2);
  // dH = dZ W2b (the forward used the BF16 weights) ; dZ1 = dH * [h > 0]
  float* W2f;
  HF_TRY(ws.alloc(&W2f, (size_t)512 * hid));
  k_bf16_rows_to_f32<<<grid_for(512LL * hid), 256, 0, s>>>(L->W2b, 512LL * hid, W2f);
  HF_LAUNCH_CHECK();
  HF_TRY(sgemm(s, R, hid, 512, 1.f, dZ, 512, 1, W2f, hid, 1, 0.f, dH, hid));
  k_relu_grad<<<grid_for((int64_t)R * hid), 256, 0, s>>>(dH, H, (int64_t)R * hid, dH);
  // dW1 = dZ1^T bf16(X) ; db1 = colsum(dZ1)
  const void* srcs[3] = {A, P, Ng};
  for (int part = 0; part < R / B; ++part) {
    if (dt == HF_F16)
      k_rows_to_bf16f<__half><<<grid_for((int64_t)B * d), 256, 0, s>>>((const __half*)srcs[part], (int64_t)B * d,
                                                                        Xf + (size_t)part * B * d);
    else
      k_rows_to_bf16f<float><<<grid_for((int64_t)B * d), 256, 0, s>>>((const float*)srcs[part], (int64_t)B * d,
                                                                       Xf + (size_t)part * B * d);
  }
  HF_LAUNCH_CHECK();
  HF_TRY(sgemm(s, hid, d, R, 1.f, dH, 1, hid, Xf, d, 1, 0.f, gW1, d));
  k_colsum<<<(unsigned)ceil_div(hid, 256), 256, 0, s>>>(dH, R, hid, gb1);
  HF_LAUNCH_CHECK();
  (void)esz;
  return HF_OK;
}

void lhash_release(hf_lhash* L) {
  if (!L) return;
  void* ptrs[] = {L->W1, L->b1, L->W2, L->b2, L->W1b, L->W2b, L->W1p, L->W2p, L->mom[0], L->mom[1], L->mom[2], L->mom[3],
                  L->vel[0], L->vel[1], L->vel[2], L->vel[3]};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  L->magic = 0;
  delete L;
}

hf_status check_lhash(const hf_lhash* L) {
  if (!L || L->magic != HF_LHASH_MAGIC) {
    set_error("invalid learned-hash handle");
    return HF_ERR_INVALID_HANDLE;
  }
  return HF_OK;
}

}  // namespace

hf_status lhash_encode_dev(const hf_lhash* L, const void* X, hf_dtype dt, int64_t N, uint64_t* sk, hipStream_t s,
                           Workspace* ext) {
  HF_TRY(check_lhash(L));
  if (N <= 0) return HF_OK;
  const char* form = getenv("HF_MLP");  // "two": the two-kernel path
  if (L->d == 384 && L->hid == 256 && L->W1p && !(form && strcmp(form, "two") == 0)) {
    int dev = 0, ncu = 256;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(N, WS_ROWS), ncu);
    if (dt == HF_F16)
      k_mlp_ws<__half, 384, 256><<<grid, WS_T, 0, s>>>((const __half*)X, N, L->W1p, L->b1, L->W2p, L->b2, sk);
    else
      k_mlp_ws<float, 384, 256><<<grid, WS_T, 0, s>>>((const float*)X, N, L->W1p, L->b1, L->W2p, L->b2, sk);
    HF_LAUNCH_CHECK();
    return HF_OK;
  }
  Workspace own(s);
  Workspace& ws = ext ? *ext : own;
  const int64_t chunk = std::min<int64_t>(N, 1 << 20);
  uint16_t* H;
  HF_TRY(ws.alloc(&H, (size_t)chunk * L->hid));
  const size_t esz = dt == HF_F16 ? 2 : 4;
  for (int64_t r0 = 0; r0 < N; r0 += chunk) {
    const int64_t n = std::min(chunk, N - r0);
    HF_TRY(lhash_forward(L, (const char*)X + r0 * L->d * esz, dt, n, H, nullptr, sk + r0 * 8, s));
  }
  return HF_OK;
}

int lhash_dim(const hf_lhash* L) { return (L && L->magic == HF_LHASH_MAGIC) ? L->d : 0; }
int lhash_hidden(const hf_lhash* L) { return (L && L->magic == HF_LHASH_MAGIC) ? L->hid : 0; }

}  // namespace hf

using namespace hf;

extern "C" {

hf_status hf_lhash_create(int32_t d, int32_t hidden, const float* W1, const float* b1, const float* W2,
                          const float* b2, hf_lhash** out) {
  clear_error();
  HF_ARG(W1 && b1 && W2 && b2 && out, "null pointer");
  HF_ARG(d >= 8 && d <= 4096 && d % 8 == 0, "d must be a multiple of 8 in [8, 4096]");
  HF_ARG(hidden >= 16 && hidden <= 2048 && hidden % 16 == 0, "hidden must be a multiple of 16 in [16, 2048]");
  *out = nullptr;
  hf_lhash* L = new hf_lhash();
  L->magic = HF_LHASH_MAGIC;
  HIP_TRY(hipGetDevice(&L->device));
  L->d = d;
  L->hid = hidden;
  const size_t n[4] = {(size_t)hidden * d, (size_t)hidden, (size_t)512 * hidden, 512};
  float** w[4] = {&L->W1, &L->b1, &L->W2, &L->b2};
  const float* src[4] = {W1, b1, W2, b2};
  struct Guard {
    hf_lhash* L;
    ~Guard() {
      if (L) lhash_release(L);
    }
  } guard{L};
  for (int i = 0; i < 4; ++i) {
    HIP_TRY(hipMalloc(w[i], 4 * n[i]));
    HIP_TRY(hipMemcpy(*w[i], src[i], 4 * n[i], hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&L->mom[i], 4 * n[i]));
    HIP_TRY(hipMalloc(&L->vel[i], 4 * n[i]));
    HIP_TRY(hipMemset(L->mom[i], 0, 4 * n[i]));
    HIP_TRY(hipMemset(L->vel[i], 0, 4 * n[i]));
  }
  HIP_TRY(hipMalloc(&L->W1b, 2 * n[0]));
  HIP_TRY(hipMalloc(&L->W2b, 2 * n[2]));
  if (d % 32 == 0 && hidden % 32 == 0) {
    HIP_TRY(hipMalloc(&L->W1p, 2 * n[0]));
    HIP_TRY(hipMalloc(&L->W2p, 2 * n[2]));
  }
  HF_TRY(refresh_bf16(L, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  guard.L = nullptr;
  *out = L;
  return HF_OK;
}

void hf_lhash_free(hf_lhash* L) {
  if (L && L->magic == HF_LHASH_MAGIC) lhash_release(L);
}

hf_status hf_lhash_get(const hf_lhash* L, float* W1, float* b1, float* W2, float* b2) {
  clear_error();
  HF_TRY(check_lhash(L));
  HF_ARG(W1 && b1 && W2 && b2, "null pointer");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(W1, L->W1, 4 * (size_t)L->hid * L->d, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(b1, L->b1, 4 * (size_t)L->hid, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(W2, L->W2, 4 * (size_t)512 * L->hid, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(b2, L->b2, 4 * 512, hipMemcpyDeviceToHost));
  return HF_OK;
}

hf_status hf_lhash_encode(const hf_lhash* L, const void* X_dev, hf_dtype dtype, int64_t N, int32_t d,
                          uint64_t* sk_dev, void* stream) {
  clear_error();
  HF_TRY(check_lhash(L));
  HF_ARG(X_dev && sk_dev, "null pointer");
  HF_ARG(dtype == HF_F16 || dtype == HF_F32, "bad dtype");
  HF_ARG(d == L->d, "d (%d) differs from the network's input size (%d)", d, L->d);
  HF_ARG(N >= 0 && N < (1ll << 31), "N out of range");
  return lhash_encode_dev(L, X_dev, dtype, N, sk_dev, (hipStream_t)stream);
}

static hf_status check_tp(const hf_lhash_train_params* tp) {
  HF_ARG(tp && tp->struct_size == sizeof(hf_lhash_train_params), "bad train params");
  HF_ARG(tp->batch >= 2 && tp->batch <= 8192, "batch must be in [2, 8192]");
  HF_ARG(tp->tau > 0.f && tp->slope > 0.f, "tau and slope must be > 0");
  return HF_OK;
}

hf_status hf_lhash_grad(const hf_lhash* L, const void* A_dev, const void* B_dev, const void* N_dev, hf_dtype dtype,
                        int64_t npairs, int32_t d, const hf_lhash_train_params* tp, float* loss_host, float* gW1_dev,
                        float* gb1_dev, float* gW2_dev, float* gb2_dev, void* stream) {
  clear_error();
  HF_TRY(check_lhash(L));
  HF_TRY(check_tp(tp));
  HF_ARG(A_dev && B_dev && loss_host && gW1_dev && gb1_dev && gW2_dev && gb2_dev, "null pointer");
  HF_ARG(d == L->d && npairs >= 2 && npairs <= 8192, "bad sizes");
  HF_ARG(dtype == HF_F16 || dtype == HF_F32, "bad dtype");
  hipStream_t s = (hipStream_t)stream;
  Workspace ws(s);
  float* loss;
  HF_TRY(ws.alloc(&loss, 1));
  k_zero_f32<<<1, 64, 0, s>>>(loss, 1);
  HF_TRY(lhash_grad(L, A_dev, B_dev, N_dev, dtype, (int)npairs, *tp, loss, gW1_dev, gb1_dev, gW2_dev, gb2_dev, ws));
  HIP_TRY(hipMemcpyAsync(loss_host, loss, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return HF_OK;
}

hf_status hf_lhash_train(hf_lhash* L, const void* A_dev, const void* B_dev, const void* N_dev, hf_dtype dtype,
                         int64_t npairs, int32_t d, const hf_lhash_train_params* tp, float* loss_curve_host,
                         void* stream) {
  clear_error();
  HF_TRY(check_lhash(L));
  HF_TRY(check_tp(tp));
  HF_ARG(A_dev && B_dev, "null pointer");
  HF_ARG(d == L->d && npairs >= (int64_t)tp->batch && npairs < (1ll << 31), "bad sizes");
  HF_ARG(dtype == HF_F16 || dtype == HF_F32, "bad dtype");
  hipStream_t s = (hipStream_t)stream;
  Workspace ws(s);
  const int B = (int)tp->batch;
  const size_t esz = dtype == HF_F16 ? 2 : 4;
  const int64_t n[4] = {(int64_t)L->hid * d, L->hid, 512LL * L->hid, 512};
  float *g[4], *loss;
  for (int i = 0; i < 4; ++i) HF_TRY(ws.alloc(&g[i], (size_t)n[i]));
  HF_TRY(ws.alloc(&loss, 1));
  void *Ab, *Bb, *Nb = nullptr;
  uint32_t* idx;
  HF_TRY(ws.alloc((char**)&Ab, (size_t)B * d * esz));
  HF_TRY(ws.alloc((char**)&Bb, (size_t)B * d * esz));
  if (N_dev) HF_TRY(ws.alloc((char**)&Nb, (size_t)B * d * esz));
  HF_TRY(ws.alloc(&idx, (size_t)npairs));
  std::vector<uint32_t> perm((size_t)npairs);
  uint64_t st = tp->seed;
  const int64_t steps_per_epoch = npairs / B;
  for (uint32_t ep = 0; ep < tp->epochs; ++ep) {
    for (int64_t i = 0; i < npairs; ++i) perm[(size_t)i] = (uint32_t)i;
    if (tp->keep_blocks) {
      std::vector<int64_t> blocks((size_t)steps_per_epoch);
      for (int64_t b = 0; b < steps_per_epoch; ++b) blocks[(size_t)b] = b;
      for (int64_t b = steps_per_epoch - 1; b >= 1; --b)
        std::swap(blocks[(size_t)b], blocks[(size_t)(splitmix64_next(&st) % (uint64_t)(b + 1))]);
      for (int64_t b = 0; b < steps_per_epoch; ++b)
        for (int i = 0; i < B; ++i) perm[(size_t)(b * B + i)] = (uint32_t)(blocks[(size_t)b] * B + i);
    } else {
      for (int64_t i = npairs - 1; i >= 1; --i)
        std::swap(perm[(size_t)i], perm[(size_t)(splitmix64_next(&st) % (uint64_t)(i + 1))]);
    }
    HIP_TRY(hipMemcpyAsync(idx, perm.data(), 4 * (size_t)npairs, hipMemcpyHostToDevice, s));
    k_zero_f32<<<1, 64, 0, s>>>(loss, 1);  // the epoch's loss, summed on the device
    for (int64_t it = 0; it < steps_per_epoch; ++it) {
      const uint32_t* bi = idx + it * B;
      if (dtype == HF_F16) {
        k_gather<__half><<<grid_for((int64_t)B * d), 256, 0, s>>>((const __half*)A_dev, d, bi, B, (__half*)Ab);
        k_gather<__half><<<grid_for((int64_t)B * d), 256, 0, s>>>((const __half*)B_dev, d, bi, B, (__half*)Bb);
        if (N_dev)
          k_gather<__half><<<grid_for((int64_t)B * d), 256, 0, s>>>((const __half*)N_dev, d, bi, B, (__half*)Nb);
      } else {
        k_gather<float><<<grid_for((int64_t)B * d), 256, 0, s>>>((const float*)A_dev, d, bi, B, (float*)Ab);
        k_gather<float><<<grid_for((int64_t)B * d), 256, 0, s>>>((const float*)B_dev, d, bi, B, (float*)Bb);
        if (N_dev)
          k_gather<float><<<grid_for((int64_t)B * d), 256, 0, s>>>((const float*)N_dev, d, bi, B, (float*)Nb);
      }
      HF_LAUNCH_CHECK();
      Workspace wstep(s);
      HF_TRY(lhash_grad(L, Ab, Bb, Nb, dtype, B, *tp, loss, g[0], g[1], g[2], g[3], wstep));
      L->step += 1;
      const float c1 = 1.f - powf(tp->beta1, (float)L->step), c2 = 1.f - powf(tp->beta2, (float)L->step);
      float* w[4] = {L->W1, L->b1, L->W2, L->b2};
      for (int i = 0; i < 4; ++i) {
        const float wd = (i == 0 || i == 2) ? tp->weight_decay : 0.f;
        k_adamw<<<grid_for(n[i]), 256, 0, s>>>(w[i], g[i], L->mom[i], L->vel[i], n[i], tp->lr, tp->beta1, tp->beta2,
                                               tp->eps, wd, c1, c2);
      }
      HF_LAUNCH_CHECK();
      HF_TRY(refresh_bf16(L, s));
    }
    if (loss_curve_host) {
      float h = 0.f;
      HIP_TRY(hipMemcpyAsync(&h, loss, 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      loss_curve_host[ep] = h / (float)steps_per_epoch;
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  return HF_OK;
}

}  // extern "C"
