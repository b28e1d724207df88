// Precision form of the final selection: the expansion set E of a query is
// scored in BF16 or FP8 (OCP e4m3 with one scale per vector) on MFMA with FP32
// accumulation, the best S "survivors" are rescored in FP32 from the stored
// rows, and the top-k of those is the result.  FP64 appears only in the audit
// kernel, which recomputes given (query, id) scores exactly.
//
// MFMA use: a wavefront scores 16 rows of E at a time; the rows are the A
// operand (one row per lane mod 16) and the query, replicated over the 16
// columns, is the B operand, so every column of the 16x16 result holds the 16
// scores.  The path is bound by HBM (one read of each row), not by the matrix
// cores.
#include <math.h>

#include "hf_internal.h"
#include "hf_select.h"

namespace hf {
namespace {

typedef float float4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int int8v __attribute__((ext_vector_type(8)));

// Round-to-nearest-even float -> bfloat16 bits (finite input).
__device__ __forceinline__ uint32_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// Float -> OCP FP8 e4m3 bits: bias 7, subnormal step 2^-9, largest finite
// 448 (0x7E), round to nearest even, saturating (no NaN produced).
__device__ __forceinline__ uint32_t e4m3_bits(float y) {
  const uint32_t sign = (__float_as_uint(y) >> 31) << 7;
  const float a = fabsf(y);
  if (!(a < 448.0f)) return sign | 0x7Eu;
  if (a < 0.015625f) return sign | (uint32_t)rintf(a * 512.0f);  // 8 -> 0x08, the smallest normal
  int ex;
  frexpf(a, &ex);
  int E = ex - 1;  // a in [2^E, 2^(E+1))
  int m = (int)rintf((ldexpf(a, -E) - 1.0f) * 8.0f);
  if (m == 8) {
    m = 0;
    E += 1;
  }
  if (E > 8 || (E == 8 && m > 6)) return sign | 0x7Eu;
  return sign | (uint32_t)(((E + 7) << 3) | m);
}

template <class T>
__device__ __forceinline__ float ldf(const T* p, int64_t i) {
  if constexpr (sizeof(T) == 2)
    return __half2float(p[i]);
  else
    return p[i];
}

template <class T>
__global__ void k_make_bf16(const T* __restrict__ X, int64_t n, uint16_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = (uint16_t)bf16_bits(ldf(X, i));
}

// One wavefront per row: scale s = max|x| / 448 (FP32, 1 if the row is 0),
// codes of x / s.
template <class T>
__global__ void k_make_fp8(const T* __restrict__ X, int64_t N, int d, uint8_t* __restrict__ out,
                           float* __restrict__ scale) {
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (r >= N) return;
  float m = 0.f;
  for (int i = __lane_id(); i < d; i += 64) m = fmaxf(m, fabsf(ldf(X, r * d + i)));
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  const float s = m > 0.f ? __fdiv_rn(m, 448.0f) : 1.0f;
  for (int i = __lane_id(); i < d; i += 64) out[r * d + i] = (uint8_t)e4m3_bits(__fdiv_rn(ldf(X, r * d + i), s));
  if (__lane_id() == 0) scale[r] = s;
}

constexpr int LP_T = 512;

// PREC 1 = BF16 (KS = d/32 MFMA steps of K = 32), 2 = FP8 (KS = d/128 steps of K = 128).
template <class T, int PREC, int KS>
__global__ __launch_bounds__(LP_T) void k_rerank_lp(
    const T* __restrict__ Xp, const void* __restrict__ Xlp, const float* __restrict__ s8,
    int64_t N, int d, const T* __restrict__ Q, const uint32_t* __restrict__ c2,
    const int32_t* __restrict__ c2n, int k2, int h, int k, int S, int k2p, int emax, int sp,
    const uint32_t* __restrict__ pos2id, int32_t* __restrict__ ids, float* __restrict__ scores,
    uint32_t* __restrict__ surv_pos, float* __restrict__ surv_score, int32_t* __restrict__ en_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* sq = (float*)smem;                                   // d
  uint32_t* sc = (uint32_t*)(sq + ((d + 3) & ~3));            // k2p
  uint32_t* st = sc + k2p;                                    // k2p
  uint32_t* off = st + k2p;                                   // k2p + 4
  uint32_t* ekey = off + k2p + 4;                             // emax
  uint64_t* sel = (uint64_t*)(((uintptr_t)(ekey + emax) + 7) & ~(uintptr_t)7);  // sp
  uint64_t* fin = sel + sp;                                   // sp
  __shared__ uint32_t hist[256];
  __shared__ uint32_t scan_tmp[LP_T / 64 + 1];
  __shared__ uint32_t s_E, s_prefix, s_lt, s_want, s_nsel;
  __shared__ float s_qmax[LP_T / 64];

  const int64_t q = blockIdx.x;
  const int n2 = c2n[q];
  const int l = __lane_id(), wv = threadIdx.x / 64, g = l / 16;
  for (int i = threadIdx.x; i < d; i += LP_T) sq[i] = ldf(Q, q * d + i);
  for (int i = threadIdx.x; i < k2p; i += LP_T) sc[i] = i < n2 ? c2[q * k2 + i] : NONE32;
  __syncthreads();
  bitonic_u32(sc, k2p);
  expansion_intervals<LP_T>(sc, n2, h, N, st, off, scan_tmp, &s_E);
  const uint32_t E = s_E;

  // the query in the MFMA B layout, per lane
  float qscale = 1.f;
  if constexpr (PREC == 2) {
    float m = 0.f;
    for (int i = threadIdx.x; i < d; i += LP_T) m = fmaxf(m, fabsf(sq[i]));
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if (l == 0) s_qmax[wv] = m;
    __syncthreads();
    m = 0.f;
#pragma unroll
    for (int i = 0; i < LP_T / 64; ++i) m = fmaxf(m, s_qmax[i]);
    qscale = m > 0.f ? __fdiv_rn(m, 448.0f) : 1.0f;
  }
  uint32_t qb[KS][PREC == 1 ? 4 : 8];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    if constexpr (PREC == 1) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k0 = 32 * s + 8 * g + 2 * v;
        const uint32_t lo = k0 < d ? bf16_bits(sq[k0]) : 0u;
        const uint32_t hi = k0 + 1 < d ? bf16_bits(sq[k0 + 1]) : 0u;
        qb[s][v] = lo | (hi << 16);
      }
    } else {
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int kk = 128 * s + 32 * g + 4 * v + b;
          const uint32_t c = kk < d ? e4m3_bits(__fdiv_rn(sq[kk], qscale)) : 0u;
          w |= c << (8 * b);
        }
        qb[s][v] = w;
      }
    }
  }
  // low-precision scores of E: 16 rows per wavefront step
  for (uint32_t e0 = (uint32_t)wv * 16; e0 < E; e0 += (LP_T / 64) * 16) {
    const uint32_t e = e0 + (l % 16);
    const bool ok = e < E;
    const uint32_t p = ok ? epos(st, off, n2, e) : 0u;
    // FP8: the row's scale, fetched with its codes (lane l holds row l % 16)
    float rs = 1.f;
    if constexpr (PREC == 2) rs = s8[p];  // (position 0 when past E: never used)
    float4v acc = {0.f, 0.f, 0.f, 0.f};
    // Row loads are unconditional (rows past E read position 0 and their
    // scores are not stored; chunks past d are zeroed after the load): a
    // load some lanes skip would be waited for chunk by chunk.
    if constexpr (PREC == 1) {
      const uint16_t* row = (const uint16_t*)Xlp + (int64_t)p * d;
      uint4 a[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k0 = 32 * s + 8 * g;
        a[s] = *(const uint4*)(row + (k0 < d ? k0 : 0));
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        if (32 * s + 8 * g >= d) a[s] = make_uint4(0, 0, 0, 0);
        uint4 b = make_uint4(qb[s][0], qb[s][1], qb[s][2], qb[s][3]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[s]),
                                                      __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
      }
    } else {
      const uint8_t* row = (const uint8_t*)Xlp + (int64_t)p * d;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k0 = 128 * s + 32 * g;
        uint4 a0 = *(const uint4*)(row + (k0 < d ? k0 : 0));
        uint4 a1 = *(const uint4*)(row + (k0 + 16 < d ? k0 + 16 : 0));
        if (k0 >= d) a0 = make_uint4(0, 0, 0, 0);
        if (k0 + 16 >= d) a1 = make_uint4(0, 0, 0, 0);
        int8v A = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
        int8v B = {(int)qb[s][0], (int)qb[s][1], (int)qb[s][2], (int)qb[s][3],
                   (int)qb[s][4], (int)qb[s][5], (int)qb[s][6], (int)qb[s][7]};
        // format 0 = FP8 e4m3 for both operands; block scales 2^0 (E8M0 127)
        acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(A, B, acc, 0, 0, 0, 127, 0, 127);
      }
    }
    // lane l holds rows 4*(l/16)+r of the block (every column is the same)
    float rsc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) rsc[r] = __shfl(rs, 4 * g + r);
    if (l % 16 == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t er = e0 + 4 * g + r;
        if (er < E) {
          float v = acc[r];
          if constexpr (PREC == 2) v = v * (rsc[r] * qscale);
          ekey[er] = ~float_to_ordered(v);
        }
      }
    }
  }
  __syncthreads();
  // survivors: the S best low-precision scores (ties by position)
  const uint32_t ns = (uint32_t)min<int64_t>(S, E);
  select_smallest<LP_T>(ekey, E, ns, sel, hist, scan_tmp, &s_prefix, &s_lt, &s_want, &s_nsel);
  for (int i = (int)ns + threadIdx.x; i < sp; i += LP_T) sel[i] = ~0ull;
  __syncthreads();
  bitonic_u64(sel, sp);
  if (surv_pos) {
    for (int i = threadIdx.x; i < S; i += LP_T) {
      const bool v = i < (int)ns;
      surv_pos[q * S + i] = v ? epos(st, off, n2, (uint32_t)sel[i]) : NONE32;
      surv_score[q * S + i] = v ? ordered_to_float(~(uint32_t)(sel[i] >> 32)) : -INFINITY;
    }
  }
  // FP32 rescoring of the survivors from the stored rows
  {
    const int grp = threadIdx.x / 16, gl = threadIdx.x % 16;
    for (int i = grp; i < (int)ns; i += LP_T / 16) {
      const uint32_t p = epos(st, off, n2, (uint32_t)sel[i]);
      const T* row = Xp + (int64_t)p * d;
      float a = 0.f;
      for (int c = gl; c < d; c += 16) a = fmaf(ldf(row, c), sq[c], a);
      a += __shfl_xor(a, 8);
      a += __shfl_xor(a, 4);
      a += __shfl_xor(a, 2);
      a += __shfl_xor(a, 1);
      if (gl == 0) fin[i] = ((uint64_t)(~float_to_ordered(a)) << 32) | p;
    }
  }
  for (int i = (int)ns + threadIdx.x; i < sp; i += LP_T) fin[i] = ~0ull;
  __syncthreads();
  bitonic_u64(fin, sp);
  for (int i = threadIdx.x; i < k; i += LP_T) {
    if (i < (int)ns) {
      const uint64_t v = fin[i];
      ids[q * k + i] = (int32_t)pos2id[(uint32_t)v];
      scores[q * k + i] = ordered_to_float(~(uint32_t)(v >> 32));
    } else {
      ids[q * k + i] = -1;
      scores[q * k + i] = -INFINITY;
    }
  }
  if (threadIdx.x == 0 && en_out) en_out[q] = (int32_t)E;
}

// FP64 audit: exact inner products of (query, id) pairs.
template <class T>
__global__ void k_audit(const T* __restrict__ X, int d, const T* __restrict__ Q, int64_t nq,
                        const int32_t* __restrict__ ids, int k, double* __restrict__ out) {
  const int64_t it = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (it >= nq * k) return;
  const int64_t q = it / k;
  const int32_t id = ids[it];
  double a = 0.0;
  if (id >= 0)
    for (int i = __lane_id(); i < d; i += 64) a += (double)ldf(Q, q * d + i) * (double)ldf(X, (int64_t)id * d + i);
  for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
  if (__lane_id() == 0) out[it] = id >= 0 ? a : 0.0;
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, ceil_div(n, 256)));
}

}  // namespace

hf_status make_lowprec(hf_forest* f, hf_precision prec, hipStream_t s) {
  const int64_t n = f->N * f->d;
  if (prec == HF_PREC_BF16) {
    if (f->X_bf16) return HF_OK;
    HIP_TRY(hipMalloc(&f->X_bf16, 2 * (size_t)n));
    if (f->dtype == HF_F16)
      k_make_bf16<__half><<<grid_for(n), 256, 0, s>>>((const __half*)f->X_pos, n, (uint16_t*)f->X_bf16);
    else
      k_make_bf16<float><<<grid_for(n), 256, 0, s>>>((const float*)f->X_pos, n, (uint16_t*)f->X_bf16);
    HF_LAUNCH_CHECK();
    f->device_bytes += 2 * n;
  } else {
    if (f->X_fp8) return HF_OK;
    HIP_TRY(hipMalloc(&f->X_fp8, (size_t)n));
    HIP_TRY(hipMalloc(&f->s_fp8, 4 * (size_t)f->N));
    const unsigned grid = (unsigned)ceil_div(f->N, 4);
    if (f->dtype == HF_F16)
      k_make_fp8<__half><<<grid, 256, 0, s>>>((const __half*)f->X_pos, f->N, f->d, (uint8_t*)f->X_fp8, f->s_fp8);
    else
      k_make_fp8<float><<<grid, 256, 0, s>>>((const float*)f->X_pos, f->N, f->d, (uint8_t*)f->X_fp8, f->s_fp8);
    HF_LAUNCH_CHECK();
    f->device_bytes += n + 4 * f->N;
  }
  HIP_TRY(hipStreamSynchronize(s));
  return HF_OK;
}

hf_status rerank_lp_launch(const hf_forest* f, hf_precision prec, const void* Qb, int64_t nb,
                           const uint32_t* c2b, const int32_t* c2nb, int k2, int h, int k, int S,
                           int32_t* idsb, float* scb, uint32_t* surv_pos, float* surv_score,
                           int32_t* enb, hipStream_t s) {
  const int d = f->d;
  const int ks = prec == HF_PREC_BF16 ? d / 32 : (d + 127) / 128;
  const int k2p = [&] { int v = 1; while (v < k2) v <<= 1; return v; }();
  const int sp = [&] { int v = 1; while (v < S) v <<= 1; return v; }();
  const int64_t emax = std::min<int64_t>((int64_t)k2 * (2 * h + 1), f->N);
  const size_t smem = sizeof(float) * (((size_t)d + 3) & ~(size_t)3) + 4 * (3 * (size_t)k2p + 4) +
                      4 * (size_t)emax + 8 + 16 * (size_t)sp;
  if (smem > 160 * 1024) {
    set_error("low-precision rerank needs %zu bytes of LDS (k2*(2h+1) or survivors too large)", smem);
    return HF_ERR_UNSUPPORTED;
  }
  const void* kern = nullptr;
#define HF_LP(TY, P, K) \
  if (ks == K) kern = (const void*)k_rerank_lp<TY, P, K>;
  if (f->dtype == HF_F16) {
    if (prec == HF_PREC_BF16) {
      HF_LP(__half, 1, 4) HF_LP(__half, 1, 8) HF_LP(__half, 1, 12) HF_LP(__half, 1, 16) HF_LP(__half, 1, 24) HF_LP(__half, 1, 32)
    } else {
      HF_LP(__half, 2, 1) HF_LP(__half, 2, 2) HF_LP(__half, 2, 3) HF_LP(__half, 2, 4) HF_LP(__half, 2, 6) HF_LP(__half, 2, 8)
    }
  } else {
    if (prec == HF_PREC_BF16) {
      HF_LP(float, 1, 4) HF_LP(float, 1, 8) HF_LP(float, 1, 12) HF_LP(float, 1, 16) HF_LP(float, 1, 24) HF_LP(float, 1, 32)
    } else {
      HF_LP(float, 2, 1) HF_LP(float, 2, 2) HF_LP(float, 2, 3) HF_LP(float, 2, 4) HF_LP(float, 2, 6) HF_LP(float, 2, 8)
    }
  }
#undef HF_LP
  if (!kern || d % 32 != 0) {
    set_error("precision form needs d in {128, 256, 384, 512, 768, 1024} (got %d)", d);
    return HF_ERR_UNSUPPORTED;
  }
  if (smem > 64 * 1024) HIP_TRY(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  const void* Xp = f->X_pos;
  const void* Xlp = prec == HF_PREC_BF16 ? f->X_bf16 : f->X_fp8;
  const float* s8 = f->s_fp8;
  int64_t N = f->N;
  int d_ = d, emax_ = (int)emax;
  void* args[] = {(void*)&Xp, (void*)&Xlp, (void*)&s8, &N, &d_, (void*)&Qb, (void*)&c2b, (void*)&c2nb,
                  &k2, &h, &k, &S, (void*)&k2p, &emax_, (void*)&sp, (void*)&f->pos2id, (void*)&idsb,
                  (void*)&scb, (void*)&surv_pos, (void*)&surv_score, (void*)&enb};
  HIP_TRY(hipLaunchKernel(kern, dim3((unsigned)nb), dim3(LP_T), args, smem, s));
  return HF_OK;
}

hf_status audit_launch(const void* X, hf_dtype dt, int d, const void* Q, int64_t nq, const int32_t* ids,
                       int k, double* out, hipStream_t s) {
  const unsigned grid = (unsigned)ceil_div(nq * k, 4);
  if (dt == HF_F16)
    k_audit<__half><<<grid, 256, 0, s>>>((const __half*)X, d, (const __half*)Q, nq, ids, k, out);
  else
    k_audit<float><<<grid, 256, 0, s>>>((const float*)X, d, (const float*)Q, nq, ids, k, out);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

}  // namespace hf
