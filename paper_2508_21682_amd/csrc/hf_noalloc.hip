// hf_search_noalloc: Algorithm 1 with every scratch buffer carved from one
// fixed device array, for callers that cannot allocate device memory.
//
// The array below is a file-scope __device__ variable: the loader gives every
// GPU the library runs on its own copy, held until the process ends.  Host
// code never passes the variable's name to a kernel or copy (on the host it
// only stands for the symbol); each device's address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
#include <mutex>

#include "hf_internal.h"

namespace hf {
namespace {

constexpr size_t kScratchBytes = (size_t)HF_NOALLOC_SCRATCH_MIB << 20;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch`.
hf_status scratch_region(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d outside the %d devices the scratch table covers", dev, kMaxDevices);
    return HF_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned no address for the scratch array");
      return HF_ERR_DEVICE;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return HF_OK;
}

}  // namespace
}  // namespace hf

using namespace hf;

extern "C" {

hf_status hf_search_noalloc(const hf_forest* f, const void* Q_dev, hf_dtype dtype, int64_t nq,
                            const hf_search_params* params, int32_t* ids_dev, float* scores_dev, void* stream) {
  clear_error();
  HF_TRY(search_args_ok(f, Q_dev, dtype, nq, params, ids_dev, scores_dev));
  const hf_search_params& p = *params;
  const size_t one = search_scratch_bytes(f, 1, p);
  if (one > kScratchBytes) {
    set_error("one query needs %zu bytes of scratch (n_trees * k1, k2 too large); the fixed region holds %zu",
              one, kScratchBytes);
    return HF_ERR_UNSUPPORTED;
  }
  // the largest query count whose scratch fits (scratch grows with the count)
  int64_t lo = 1, hi = nq;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (search_scratch_bytes(f, mid, p) <= kScratchBytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t chunk = lo;
  void* region = nullptr;
  HF_TRY(scratch_region(&region));
  hipStream_t s = (hipStream_t)stream;
  const size_t esz = f->dtype == HF_F16 ? 2 : 4;
  // chunks run in stream order, so each may reuse the whole region
  for (int64_t q0 = 0; q0 < nq; q0 += chunk) {
    const int64_t nb = std::min(chunk, nq - q0);
    Workspace arena(s, region, kScratchBytes);
    HF_TRY(search_launch(f, (const char*)Q_dev + q0 * f->d * esz, nb, p, ids_dev + q0 * p.k,
                         scores_dev + q0 * p.k, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, s,
                         &arena));
  }
  return HF_OK;
}

}  // extern "C"
