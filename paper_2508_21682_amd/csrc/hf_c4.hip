// The paper's compressed layout (Section 3.1): sketches of one bit per
// coordinate and 4-bit vector codes that share that bit, with the final
// distances computed from the codes and the unquantized query.
//
//   sketch bit i = [x_i >= 0]: the coordinate's sign, which is also the top
//     bit of its 8-bit ordering code, so the forest's sign plane (kept for
//     the exact query positions) is the sketch and the codes' sign bit at
//     once; the Hamming filter reads a copy padded with zeros to 512 bits;
//   magnitude m_i = #{k in 1..7 : 8 |x_i| >= k max_j |x_j|}, three bit
//     planes per row, compared in FP64 (exact for fp16 and fp32 values);
//   scale s = max_j |x_j| / 8 (exact in FP32);
//   value of coordinate i = (+-1) (m_i + 1/2) s.
// Rows hold sign words (d/32, in the sign plane) plus 3 magnitude words per
// sign word and one FP32 scale: 4 d/8 + 4 bytes instead of 2 d.
#include <math.h>

#include "hf_internal.h"
#include "hf_select.h"

namespace hf {
namespace {

template <class T>
__device__ __forceinline__ float ldf(const T* X, int64_t i) {
  if constexpr (sizeof(T) == 2)
    return __half2float(X[i]);
  else
    return X[i];
}

// Sign sketches: a wavefront per row, bit i from a ballot over 64 coordinates.
template <class T>
__global__ __launch_bounds__(256) void k_sign_sketch(const T* __restrict__ X, int64_t N, int d,
                                                     uint64_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (r >= N) return;
  const int l = __lane_id();
  for (int w = 0; w < HF_SKETCH_WORDS; ++w) {
    const int i = w * 64 + l;
    const bool b = i < d && ldf(X, r * d + i) >= 0.0f;
    const uint64_t m = __ballot(b);
    if (l == 0) out[r * HF_SKETCH_WORDS + w] = m;
  }
}

// Magnitude planes (mag[(r * nw + w) * 3 + plane], 32 coordinates a word) and
// scales: a wavefront per row.
template <class T>
__global__ __launch_bounds__(256) void k_make_c4(const T* __restrict__ X, int64_t N, int d, int nw,
                                                 uint32_t* __restrict__ mag, float* __restrict__ scale) {
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (r >= N) return;
  const int l = __lane_id();
  float mx = 0.0f;
  for (int i = l; i < d; i += 64) mx = fmaxf(mx, fabsf(ldf(X, r * d + i)));
  for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  const double mxd = (double)mx;
  for (int g = 0; g < nw; g += 2) {  // 64 coordinates per step: words g and g + 1
    const int i = g * 32 + l;
    int m = 0;
    if (i < d) {
      const double a = 8.0 * fabs((double)ldf(X, r * d + i));
#pragma unroll
      for (int k = 1; k <= 7; ++k) m += a >= (double)k * mxd ? 1 : 0;
    }
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
      const uint64_t bits = __ballot((m >> pl) & 1);
      if (l == 0) {
        mag[(r * nw + g) * 3 + pl] = (uint32_t)bits;
        if (g + 1 < nw) mag[(r * nw + g + 1) * 3 + pl] = (uint32_t)(bits >> 32);
      }
    }
  }
  if (l == 0) scale[r] = mx * 0.125f;
}

// Final stage from the codes: C2 sorted by position, expanded by +-h into
// merged intervals, each row scored by a 16-lane group (lane j: coordinates
// 32j .. 32j+31 from sign word j and its three magnitude words, 4 rows in
// flight per group), the k best (score desc, position asc) selected.
constexpr int C4_T = 256, C4_ROWS = 4;
template <class T>
__global__ __launch_bounds__(C4_T) void k_rerank_c4(const uint32_t* __restrict__ sgn,
                                                    const uint32_t* __restrict__ mag,
                                                    const float* __restrict__ scale, int nw, int64_t N, int d,
                                                    const T* __restrict__ Q, const uint32_t* __restrict__ c2,
                                                    const int32_t* __restrict__ c2n, int k2, int h, int k, int k2p,
                                                    int emax, int kp, const uint32_t* __restrict__ pos2id,
                                                    int32_t* __restrict__ ids, float* __restrict__ scores,
                                                    int32_t* __restrict__ en_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  // the query transposed: sq[b * 17 + w] = q[32 w + b] (zero past d), so the
  // 16 lanes of a group, reading word w = lane at one bit b, hit 16 banks
  float* sq = (float*)smem;                         // 32 x 17
  uint32_t* sc = (uint32_t*)(sq + 32 * 17);         // k2p
  uint32_t* st = sc + k2p;                          // k2p
  uint32_t* off = st + k2p;                         // k2p + 1
  uint32_t* ekey = off + k2p + 4;                   // emax
  uint64_t* sel = (uint64_t*)(((uintptr_t)(ekey + emax) + 7) & ~(uintptr_t)7);  // kp
  __shared__ uint32_t hist[256];
  __shared__ uint32_t scan_tmp[C4_T / 64 + 1];
  __shared__ uint32_t s_E, s_lt, s_eq_need, s_nsel, s_prefix;

  const int64_t q = blockIdx.x;
  const int n2 = c2n[q];
  for (int i = threadIdx.x; i < 32 * 17; i += C4_T) {
    const int b = i / 17, w = i % 17, c = 32 * w + b;
    sq[i] = (w < nw && c < d) ? ldf(Q, q * d + c) : 0.0f;
  }
  for (int i = threadIdx.x; i < k2p; i += C4_T) sc[i] = i < n2 ? c2[q * k2 + i] : NONE32;
  __syncthreads();
  bitonic_u32(sc, k2p);
  expansion_intervals<C4_T>(sc, n2, h, N, st, off, scan_tmp, &s_E);
  const uint32_t E = s_E;
  {
    const int g = threadIdx.x / 16, gl = threadIdx.x % 16;
    constexpr int NG = C4_T / 16;
    for (uint32_t e0 = (uint32_t)g * C4_ROWS; e0 < E; e0 += NG * C4_ROWS) {
      uint32_t sw[C4_ROWS];
      uint3 mw[C4_ROWS];
      uint32_t prow[C4_ROWS];
#pragma unroll
      for (int u = 0; u < C4_ROWS; ++u) {
        const uint32_t e = e0 + u;
        const uint32_t p = e < E ? epos(st, off, n2, e) : 0u;
        prow[u] = p;
        // unconditional loads (rows past E read position 0, lanes past the
        // row's words read word 0), masked afterwards
        const int64_t w = (int64_t)p * nw + (gl < nw ? gl : 0);
        sw[u] = sgn[w];
        mw[u] = *(const uint3*)(mag + w * 3);
      }
#pragma unroll
      for (int u = 0; u < C4_ROWS; ++u)
        if (!(e0 + u < E && gl < nw)) {
          sw[u] = 0u;
          mw[u] = make_uint3(0, 0, 0);
        }
      float sfac[C4_ROWS];
#pragma unroll
      for (int u = 0; u < C4_ROWS; ++u) sfac[u] = scale[prow[u]];
#pragma unroll
      for (int u = 0; u < C4_ROWS; ++u) {
        float a = 0.0f;
        if (gl < nw) {
          const float* qq = sq + gl;
#pragma unroll
          for (int b = 0; b < 32; ++b) {
            const uint32_t m = ((mw[u].x >> b) & 1u) | (((mw[u].y >> b) & 1u) << 1) | (((mw[u].z >> b) & 1u) << 2);
            const float v = (float)m + 0.5f;
            a = fmaf(qq[17 * b], ((sw[u] >> b) & 1u) ? v : -v, a);
          }
        }
        a += __shfl_xor(a, 8);
        a += __shfl_xor(a, 4);
        a += __shfl_xor(a, 2);
        a += __shfl_xor(a, 1);
        if (gl == 0 && e0 + u < E) ekey[e0 + u] = ~float_to_ordered(a * sfac[u]);
      }
    }
  }
  __syncthreads();
  const uint32_t kk = (uint32_t)min<int64_t>(k, E);
  select_smallest<C4_T>(ekey, E, kk, sel, hist, scan_tmp, &s_prefix, &s_lt, &s_eq_need, &s_nsel);
  __syncthreads();
  for (int i = (int)kk + threadIdx.x; i < kp; i += C4_T) sel[i] = ~0ull;
  __syncthreads();
  bitonic_u64(sel, kp);
  for (int i = threadIdx.x; i < k; i += C4_T) {
    if (i < (int)kk) {
      const uint64_t v = sel[i];
      const uint32_t p = epos(st, off, n2, (uint32_t)v);
      ids[q * k + i] = (int32_t)pos2id[p];
      scores[q * k + i] = ordered_to_float(~(uint32_t)(v >> 32));
    } else {
      ids[q * k + i] = -1;
      scores[q * k + i] = -INFINITY;
    }
  }
  if (threadIdx.x == 0 && en_out) en_out[q] = (int32_t)E;
}

unsigned rows_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, 4)); }

}  // namespace

hf_status sign_sketch(const void* X, hf_dtype dt, int64_t N, int d, uint64_t* out, hipStream_t s) {
  if (N <= 0) return HF_OK;
  if (d > HF_SKETCH_BITS) {
    set_error("sign sketches hold one bit per coordinate: d must be <= %d", HF_SKETCH_BITS);
    return HF_ERR_UNSUPPORTED;
  }
  if (dt == HF_F16)
    k_sign_sketch<__half><<<rows_grid(N), 256, 0, s>>>((const __half*)X, N, d, out);
  else
    k_sign_sketch<float><<<rows_grid(N), 256, 0, s>>>((const float*)X, N, d, out);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

hf_status make_c4(hf_forest* f, hipStream_t s) {
  if (f->c4_mag) return HF_OK;
  if (f->sgn_words == 0) {
    set_error("the compressed layout needs d <= 512");
    return HF_ERR_UNSUPPORTED;
  }
  const int nw = f->sgn_words;
  HIP_TRY(hipMalloc(&f->c4_mag, sizeof(uint32_t) * 3 * (size_t)nw * f->N));
  HIP_TRY(hipMalloc(&f->c4_scale, sizeof(float) * (size_t)f->N));
  if (f->dtype == HF_F16)
    k_make_c4<__half><<<rows_grid(f->N), 256, 0, s>>>((const __half*)f->X_pos, f->N, f->d, nw, f->c4_mag,
                                                      f->c4_scale);
  else
    k_make_c4<float><<<rows_grid(f->N), 256, 0, s>>>((const float*)f->X_pos, f->N, f->d, nw, f->c4_mag,
                                                     f->c4_scale);
  HF_LAUNCH_CHECK();
  HIP_TRY(hipStreamSynchronize(s));
  f->device_bytes += 12 * (int64_t)nw * f->N + 4 * f->N;
  return HF_OK;
}

hf_status rerank_c4_launch(const hf_forest* f, const void* Qb, int64_t nb, const uint32_t* c2b, const int32_t* c2nb,
                           int k2, int h, int k, int32_t* idsb, float* scb, int32_t* enb, hipStream_t s) {
  const int nw = f->sgn_words, d = f->d;
  const int k2p = [&] { int v = 1; while (v < k2) v <<= 1; return v; }();
  const int kp = [&] { int v = 1; while (v < k) v <<= 1; return v; }();
  const int64_t emax = std::min<int64_t>((int64_t)k2 * (2 * h + 1), f->N);
  const size_t smem = sizeof(float) * 32 * 17 + sizeof(uint32_t) * (3 * (size_t)k2p + 4) +
                      sizeof(uint32_t) * (size_t)emax + 8 + sizeof(uint64_t) * (size_t)kp;
  if (smem > 160 * 1024) {
    set_error("rerank needs %zu bytes of LDS (k2*(2h+1) too large)", smem);
    return HF_ERR_UNSUPPORTED;
  }
  const void* kern = f->dtype == HF_F16 ? (const void*)k_rerank_c4<__half> : (const void*)k_rerank_c4<float>;
  if (smem + 2048 > 64 * 1024)
    HIP_TRY(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  const uint32_t* sg = f->sgn_pos;
  const uint32_t* mg = f->c4_mag;
  const float* scl = f->c4_scale;
  const uint32_t* p2i = f->pos2id;
  int64_t N = f->N;
  int nw_ = nw, d_ = d, k2_ = k2, h_ = h, k_ = k, k2p_ = k2p, emax_ = (int)emax, kp_ = kp;
  void* args[] = {(void*)&sg, (void*)&mg, (void*)&scl, &nw_, &N, &d_, (void*)&Qb, (void*)&c2b, (void*)&c2nb,
                  &k2_, &h_, &k_, &k2p_, &emax_, &kp_, (void*)&p2i, (void*)&idsb, (void*)&scb, (void*)&enb};
  HIP_TRY(hipLaunchKernel(kern, dim3((unsigned)nb), dim3(C4_T), args, smem, s));
  return HF_OK;
}

}  // namespace hf
