// 8-bit ordering codes: min/max reduction for the power-of-two scale, and the
// element-wise quantiser u = clamp(floor(x * 2^e) + 128, 0, 255).
#include <math.h>

#include "hf_internal.h"

namespace hf {
namespace {

__device__ __forceinline__ float load_f(const void* X, hf_dtype dt, int64_t i) {
  return dt == HF_F16 ? __half2float(((const __half*)X)[i]) : ((const float*)X)[i];
}

// Partial min/max per block, plus a non-finite flag.
__global__ __launch_bounds__(256) void minmax_kernel(const void* __restrict__ X, hf_dtype dt,
                                                    int64_t n, float* __restrict__ pmin,
                                                    float* __restrict__ pmax,
                                                    int* __restrict__ bad) {
  float mn = INFINITY, mx = -INFINITY;
  int nf = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    float v = load_f(X, dt, i);
    if (!isfinite(v)) nf = 1;
    mn = fminf(mn, v);
    mx = fmaxf(mx, v);
  }
  for (int m = 32; m >= 1; m >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, m));
    mx = fmaxf(mx, __shfl_xor(mx, m));
  }
  __shared__ float smn[4], smx[4];
  int w = threadIdx.x / 64;
  if (__lane_id() == 0) {
    smn[w] = mn;
    smx[w] = mx;
  }
  if (__any(nf) && __lane_id() == 0) atomicOr(bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i) {
      mn = fminf(mn, smn[i]);
      mx = fmaxf(mx, smx[i]);
    }
    pmin[blockIdx.x] = fminf(smn[0], mn);
    pmax[blockIdx.x] = fmaxf(smx[0], mx);
  }
}

// Exact: x * 2^e is a power-of-two scaling of a finite float (ldexpf), and the
// floor and clamp are exact.
template <class T>
__global__ __launch_bounds__(256) void quantize_kernel(const T* __restrict__ X, int64_t n, int e,
                                                       uint8_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    float v;
    if constexpr (sizeof(T) == 2)
      v = __half2float(X[i]);
    else
      v = X[i];
    float f = floorf(ldexpf(v, e)) + 128.0f;
    f = fminf(fmaxf(f, 0.0f), 255.0f);
    out[i] = (uint8_t)f;
  }
}

}  // namespace

hf_status minmax(const void* X, hf_dtype dt, int64_t n, float* mn_host, float* mx_host,
                 int* nonfinite_host, Workspace& ws) {
  int blocks = (int)std::min<int64_t>(2048, std::max<int64_t>(1, ceil_div(n, 256)));
  float *pmin, *pmax;
  int* bad;
  HF_TRY(ws.alloc(&pmin, blocks));
  HF_TRY(ws.alloc(&pmax, blocks));
  HF_TRY(ws.alloc(&bad, 1));
  HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), ws.stream));
  minmax_kernel<<<blocks, 256, 0, ws.stream>>>(X, dt, n, pmin, pmax, bad);
  HF_LAUNCH_CHECK();
  std::vector<float> a(blocks), b(blocks);
  int h_bad = 0;
  HIP_TRY(hipMemcpyAsync(a.data(), pmin, blocks * 4, hipMemcpyDeviceToHost, ws.stream));
  HIP_TRY(hipMemcpyAsync(b.data(), pmax, blocks * 4, hipMemcpyDeviceToHost, ws.stream));
  HIP_TRY(hipMemcpyAsync(&h_bad, bad, 4, hipMemcpyDeviceToHost, ws.stream));
  HIP_TRY(hipStreamSynchronize(ws.stream));
  float mn = INFINITY, mx = -INFINITY;
  for (int i = 0; i < blocks; ++i) {
    mn = std::min(mn, a[i]);
    mx = std::max(mx, b[i]);
  }
  *mn_host = mn;
  *mx_host = mx;
  *nonfinite_host = h_bad;
  return HF_OK;
}

// Largest e in [-8, 24] with 2^e*max < 128 and 2^e*min >= -128; -8 if none.
// Products of a float with a power of two are exact in double.
int choose_exp(float mn, float mx) {
  for (int e = 24; e >= -8; --e)
    if (ldexp((double)mx, e) < 128.0 && ldexp((double)mn, e) >= -128.0) return e;
  return -8;
}

hf_status quantize(const void* X, hf_dtype dt, int64_t n, int e, uint8_t* out, hipStream_t s) {
  if (n <= 0) return HF_OK;
  int blocks = (int)std::min<int64_t>(65536, ceil_div(n, 256));
  if (dt == HF_F16)
    quantize_kernel<__half><<<blocks, 256, 0, s>>>((const __half*)X, n, e, out);
  else
    quantize_kernel<float><<<blocks, 256, 0, s>>>((const float*)X, n, e, out);
  HF_LAUNCH_CHECK();
  return HF_OK;
}

}  // namespace hf
