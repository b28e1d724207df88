// Precision form of the final selection: the expansion set E of a query is
// scored in BF16 or FP8 (OCP e4m3 with one scale per vector) with FP32
// accumulation, the best S "survivors" are rescored in FP32 from the stored
// rows, and the top-k of those is the result.  FP64 appears only in the audit
// kernel, which recomputes given (query, id) scores exactly.
//
// Scoring E is one query against |E| distinct rows: a matrix-vector product,
// bound by reading the rows (BF16: 2d bytes, FP8: d + 4 bytes a row), so it
// runs on the vector ALUs: a 16-lane group per row, 16-byte loads, several
// rows in flight per group, exact products of the rounded values summed in
// FP32.
#include <math.h>

#include "hf_internal.h"
#include "hf_select.h"

namespace hf {
namespace {


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

constexpr int LP_T = 256;

constexpr int LP_ROWS = 4;
typedef float float2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf16_val(uint32_t b) { return __uint_as_float(b << 16); }

// Value of an OCP e4m3 code (bias 7, subnormals 2^-9 m; 0x7F never occurs).
__device__ __forceinline__ float e4m3_val(uint32_t c) {
  const uint32_t E = (c >> 3) & 15u, m = c & 7u;
  const float v = E ? __uint_as_float(((E + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;
  return (c & 0x80u) ? -v : v;
}

// PREC 1 = BF16, 2 = FP8; MCH 16-byte chunks of a low-precision row per lane
// of a GL-lane group (16 for BF16 rows, 8 for the half-as-long FP8 rows, so
// every lane loads whole chunks and twice as many FP8 rows are in flight),
// RCH of a stored row per lane of a 16-lane group (rescoring).
template <class T, int PREC, int MCH, int RCH, int GL>
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
  float* sqr = (float*)(((uintptr_t)(fin + sp) + 15) & ~(uintptr_t)15);  // d: the rounded query
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

  // the query rounded to the format (FP8: codes of q / qscale), as floats
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
  for (int i = threadIdx.x; i < d; i += LP_T)
    sqr[i] = PREC == 1 ? bf16_val(bf16_bits(sq[i])) : e4m3_val(e4m3_bits(__fdiv_rn(sq[i], qscale)));
  __syncthreads();
  // low-precision scores of E: a 16-lane group per row, 16-byte chunks of
  // the row (8 BF16 or 16 FP8 values), LP_ROWS rows in flight per group;
  // products of rounded values are exact in FP32, sums accumulate in FP32
  {
    const int grp = threadIdx.x / GL, gl = threadIdx.x % GL;
    constexpr int NG = LP_T / GL;
    constexpr int EPC = PREC == 1 ? 8 : 16;  // values per 16-byte chunk
    const int nch = d / EPC;
    for (uint32_t e0 = (uint32_t)grp * LP_ROWS; e0 < E; e0 += NG * LP_ROWS) {
      uint4 raw[LP_ROWS][MCH];
      float rs[LP_ROWS];
#pragma unroll
      for (int u = 0; u < LP_ROWS; ++u) {
        const uint32_t e = e0 + u;
        const uint32_t p = e < E ? epos(st, off, n2, e) : 0u;
        const unsigned char* row = (const unsigned char*)Xlp + (int64_t)p * d * (PREC == 1 ? 2 : 1);
#pragma unroll
        for (int m = 0; m < MCH; ++m) {
          const int c = gl + GL * m;
          raw[u][m] = *(const uint4*)(row + 16 * (c < nch ? c : 0));
        }
        rs[u] = PREC == 2 ? s8[p] : 1.f;
      }
#pragma unroll
      for (int u = 0; u < LP_ROWS; ++u) {
        float a = 0.f;
#pragma unroll
        for (int m = 0; m < MCH; ++m) {
          const int c = gl + GL * m;
          if (c < nch) {
            const float4* q4 = (const float4*)(sqr + c * EPC);  // 16-byte LDS reads
            const uint32_t w[4] = {raw[u][m].x, raw[u][m].y, raw[u][m].z, raw[u][m].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              if constexpr (PREC == 1) {
                const float4 qa = q4[j >> 1];
                const float q0 = (j & 1) ? qa.z : qa.x, q1 = (j & 1) ? qa.w : qa.y;
                a = fmaf(bf16_val(w[j] & 0xFFFFu), q0, a);
                a = fmaf(bf16_val(w[j] >> 16), q1, a);
              } else {
                // gfx950 converts OCP e4m3 pairs to FP32 in one instruction
                const float4 qa = q4[j];
                const float2v lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[j], false);
                const float2v hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[j], true);
                a = fmaf(lo.x, qa.x, a);
                a = fmaf(lo.y, qa.y, a);
                a = fmaf(hi.x, qa.z, a);
                a = fmaf(hi.y, qa.w, a);
              }
            }
          }
        }
#pragma unroll
        for (int o = GL / 2; o >= 1; o >>= 1) a += __shfl_xor(a, o);
        if (PREC == 2) a = a * (rs[u] * qscale);
        if (gl == 0 && e0 + u < E) ekey[e0 + u] = ~float_to_ordered(a);
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
  // FP32 rescoring of the survivors from the stored rows (16-byte chunks)
  {
    const int grp = threadIdx.x / 16, gl = threadIdx.x % 16;
    constexpr int EPC = 16 / sizeof(T);
    const int nch = d / EPC;
    for (int i = grp; i < (int)ns; i += LP_T / 16) {
      const uint32_t p = epos(st, off, n2, (uint32_t)sel[i]);
      const unsigned char* row = (const unsigned char*)(Xp + (int64_t)p * d);
      uint4 raw[RCH];
#pragma unroll
      for (int m = 0; m < RCH; ++m) {
        const int c = gl + 16 * m;
        raw[m] = *(const uint4*)(row + 16 * (c < nch ? c : 0));
      }
      float a = 0.f;
#pragma unroll
      for (int m = 0; m < RCH; ++m) {
        const int c = gl + 16 * m;
        if (c < nch) {
          const float* qq = sq + c * EPC;
          if constexpr (sizeof(T) == 2) {
            const __half2* hv = (const __half2*)&raw[m];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float2 f2 = __half22float2(hv[j]);
              a = fmaf(f2.x, qq[2 * j], a);
              a = fmaf(f2.y, qq[2 * j + 1], a);
            }
          } else {
            const float* fv = (const float*)&raw[m];
#pragma unroll
            for (int j = 0; j < 4; ++j) a = fmaf(fv[j], qq[j], a);
          }
        }
      }
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
  const int k2p = [&] { int v = 1; while (v < k2) v <<= 1; return v; }();
  const int sp = [&] { int v = 1; while (v < S) v <<= 1; return v; }();
  const int64_t emax = std::min<int64_t>((int64_t)k2 * (2 * h + 1), f->N);
  const size_t smem = sizeof(float) * (((size_t)d + 3) & ~(size_t)3) + 4 * (3 * (size_t)k2p + 4) +
                      4 * (size_t)emax + 8 + 16 * (size_t)sp + 4 * (size_t)d + 16;
  if (smem > 160 * 1024) {
    set_error("low-precision rerank needs %zu bytes of LDS (k2*(2h+1) or survivors too large)", smem);
    return HF_ERR_UNSUPPORTED;
  }
  const void* kern = nullptr;
  // chunks per lane: low-precision rows (BF16: d/8 chunks over 16 lanes,
  // FP8: d/16 over 8) and stored rows (fp16: d/8, fp32: d/4, over 16 lanes)
#define HF_LP(DV, TY, P, M, R)                                               \
  if (d == DV && prec == (P == 1 ? HF_PREC_BF16 : HF_PREC_FP8))               \
    kern = (const void*)k_rerank_lp<TY, P, M, R, P == 1 ? 16 : 8>;
  if (f->dtype == HF_F16) {
    HF_LP(128, __half, 1, 1, 1) HF_LP(256, __half, 1, 2, 2) HF_LP(384, __half, 1, 3, 3) HF_LP(512, __half, 1, 4, 4)
    HF_LP(768, __half, 1, 6, 6) HF_LP(1024, __half, 1, 8, 8)
    HF_LP(128, __half, 2, 1, 1) HF_LP(256, __half, 2, 2, 2) HF_LP(384, __half, 2, 3, 3) HF_LP(512, __half, 2, 4, 4)
    HF_LP(768, __half, 2, 6, 6) HF_LP(1024, __half, 2, 8, 8)
  } else {
    HF_LP(128, float, 1, 1, 2) HF_LP(256, float, 1, 2, 4) HF_LP(384, float, 1, 3, 6) HF_LP(512, float, 1, 4, 8)
    HF_LP(768, float, 1, 6, 12) HF_LP(1024, float, 1, 8, 16)
    HF_LP(128, float, 2, 1, 2) HF_LP(256, float, 2, 2, 4) HF_LP(384, float, 2, 3, 6) HF_LP(512, float, 2, 4, 8)
    HF_LP(768, float, 2, 6, 12) HF_LP(1024, float, 2, 8, 16)
  }
#undef HF_LP
  if (!kern) {
    set_error("precision form needs d in {128, 256, 384, 512, 768, 1024} (got %d)", d);
    return HF_ERR_UNSUPPORTED;
  }
  if (smem + 1024 > 64 * 1024) HIP_TRY(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
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
