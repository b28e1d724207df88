// C ABI entry points of libhf: argument checks, forest construction order
// (Algorithm 1 preprocessing), introspection and error reporting.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>

#include "hf_internal.h"

namespace hf {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }

// ------------------------------------------------------------------ timing
namespace {
struct TimedSpan {
  int stage;
  hipEvent_t a, b;
};
thread_local bool t_on = false;
thread_local std::vector<TimedSpan> t_spans;
thread_local std::vector<hipEvent_t> t_open(ST_COUNT, nullptr);
const char* kStageNames[ST_COUNT] = {"query_codes", "query_sketch", "descend", "hamming", "select",
                                     "rerank", "graph_sort", "graph_band", "build_sort", "build_trie",
                                     "build_sketch", "lowprec_score", "graph_hamming", "graph_merge",
                                     "graph_final", "graph_mailbox"};
}  // namespace

bool timing_on() { return t_on; }

void timing_mark(int stage, bool begin, hipStream_t s) {
  if (!t_on) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  if (begin) {
    t_open[stage] = e;
  } else if (t_open[stage]) {
    t_spans.push_back({stage, t_open[stage], e});
    t_open[stage] = nullptr;
  } else {
    (void)hipEventDestroy(e);
  }
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).
uint64_t splitmix64_next(uint64_t* state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One stream for all trees, consumed in tree order: a Fisher-Yates shuffle of
// the axes (i = d-1 .. 1, j = next mod (i+1)), then ceil(d/64) reflection words.
void make_curves(uint64_t seed, int T, int d, int32_t* perm, uint8_t* refl) {
  uint64_t st = seed;
  for (int t = 0; t < T; ++t) {
    int32_t* p = perm + (int64_t)t * d;
    for (int i = 0; i < d; ++i) p[i] = i;
    for (int i = d - 1; i >= 1; --i) {
      uint64_t j = splitmix64_next(&st) % (uint64_t)(i + 1);
      std::swap(p[i], p[j]);
    }
    for (int w = 0; w < (d + 63) / 64; ++w) {
      uint64_t bits = splitmix64_next(&st);
      for (int b = 0; b < 64 && w * 64 + b < d; ++b)
        refl[(int64_t)t * d + w * 64 + b] = (uint8_t)((bits >> b) & 1u);
    }
  }
}

hf_status graph_launch(const void* X, hf_dtype dt, int64_t N, int d, const hf_graph_params& p,
                       int e, int32_t* ids, float* scores, int32_t* c2_ids, hipStream_t s);

namespace {

__global__ void k_inverse(const uint32_t* __restrict__ order, int64_t n, uint32_t* __restrict__ pos) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    pos[order[i]] = (uint32_t)i;
}

__global__ void k_map(const uint32_t* __restrict__ order, const uint32_t* __restrict__ pos, int64_t n,
                      uint32_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = pos[order[i]];
}

// Gather rows (16-byte vectors when the row size allows it).
__global__ void k_gather_rows(const unsigned char* __restrict__ X, int64_t row_bytes,
                              const uint32_t* __restrict__ ids, int64_t n,
                              unsigned char* __restrict__ out) {
  if (row_bytes % 16 == 0) {
    const int64_t nv = row_bytes / 16;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n * nv; i += (int64_t)gridDim.x * 256) {
      int64_t r = i / nv, c = i % nv;
      ((uint4*)out)[r * nv + c] = ((const uint4*)(X + (int64_t)ids[r] * row_bytes))[c];
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n * row_bytes; i += (int64_t)gridDim.x * 256) {
      int64_t r = i / row_bytes, c = i % row_bytes;
      out[i] = X[(int64_t)ids[r] * row_bytes + c];
    }
  }
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, ceil_div(n, 256)));
}

bool valid_dtype(hf_dtype dt) { return dt == HF_F16 || dt == HF_F32; }
size_t dsize(hf_dtype dt) { return dt == HF_F16 ? 2 : 4; }

hf_status data_exp(const void* X, hf_dtype dt, int64_t n, int32_t want, int* e, Workspace& ws) {
  float mn, mx;
  int bad;
  HF_TRY(minmax(X, dt, n, &mn, &mx, &bad, ws));
  if (bad) {
    set_error("input holds a non-finite value");
    return HF_ERR_INVALID_INPUT;
  }
  *e = want == HF_QUANT_AUTO ? choose_exp(mn, mx) : want;
  return HF_OK;
}

void forest_release(hf_forest* f) {
  if (!f) return;
  void* ptrs[] = {f->X_pos, f->sk_pos, f->pos2id, f->tree_perm, f->nodes, f->curve_perm, f->curve_refl,
                  f->X_bf16, f->X_fp8, f->s_fp8, f->node_off_dev, f->srp_R, f->srp_Rb, f->node_aux, f->sgn_pos,
                  f->c4_mag, f->c4_scale};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  f->magic = 0;
  delete f;
}

hf_status check_forest(const hf_forest* f) {
  if (!f || f->magic != HF_FOREST_MAGIC) {
    set_error("invalid forest handle");
    return HF_ERR_INVALID_HANDLE;
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != f->device) {
    set_error("forest lives on device %d, current device is %d", f->device, dev);
    return HF_ERR_INVALID_HANDLE;
  }
  return HF_OK;
}

}  // namespace

ScratchAlloc g_scratch = {{nullptr, nullptr, nullptr}, false};
ScratchAlloc scratch_allocator() { return g_scratch; }
}  // namespace hf

using namespace hf;

extern "C" {

const char* hf_status_str(hf_status s) {
  switch (s) {
    case HF_OK: return "ok";
    case HF_ERR_INVALID_ARG: return "invalid argument";
    case HF_ERR_INVALID_INPUT: return "invalid input data";
    case HF_ERR_OOM: return "out of device memory";
    case HF_ERR_DEVICE: return "device error";
    case HF_ERR_INVALID_HANDLE: return "invalid handle";
    case HF_ERR_UNSUPPORTED: return "unsupported parameters";
  }
  return "unknown status";
}

const char* hf_last_error(void) { return g_err.c_str(); }

hf_status hf_set_allocator(const hf_allocator* a) {
  hf::clear_error();
  if (!a) {
    hf::g_scratch.on = false;
    return HF_OK;
  }
  HF_ARG(a->alloc && a->free, "an allocator needs both alloc and free");
  hf::g_scratch.a = *a;
  hf::g_scratch.on = true;
  return HF_OK;
}

hf_status hf_timing_enable(int32_t on) {
  t_on = on != 0;
  return HF_OK;
}

hf_status hf_timing_read(float* ms_host, int32_t* launches_host) {
  clear_error();
  HF_ARG(ms_host && launches_host, "null pointer");
  for (int i = 0; i < ST_COUNT; ++i) {
    ms_host[i] = 0.f;
    launches_host[i] = 0;
  }
  for (auto& sp : t_spans) {
    float ms = 0.f;
    HIP_TRY(hipEventSynchronize(sp.b));
    HIP_TRY(hipEventElapsedTime(&ms, sp.a, sp.b));
    ms_host[sp.stage] += ms;
    launches_host[sp.stage] += 1;
    (void)hipEventDestroy(sp.a);
    (void)hipEventDestroy(sp.b);
  }
  t_spans.clear();
  return HF_OK;
}

const char* hf_timing_stage_name(int32_t stage) {
  return (stage >= 0 && stage < ST_COUNT) ? kStageNames[stage] : "";
}

hf_status hf_curves(uint64_t seed, int32_t T, int32_t d, int32_t* perm_host, uint8_t* refl_host) {
  clear_error();
  HF_ARG(T >= 1 && T <= 1 << 20, "T must be in [1, 2^20] (got %d)", T);
  HF_ARG(d >= 1 && d <= 4096, "d must be in [1, 4096] (got %d)", d);
  HF_ARG(perm_host && refl_host, "null output");
  make_curves(seed, T, d, perm_host, refl_host);
  return HF_OK;
}

hf_status hf_quant_exp(const void* X_dev, hf_dtype dtype, int64_t n_elems, int32_t* e_out_host,
                       void* stream) {
  clear_error();
  HF_ARG(X_dev && e_out_host, "null pointer");
  HF_ARG(valid_dtype(dtype), "bad dtype %d", (int)dtype);
  HF_ARG(n_elems >= 1, "n_elems must be >= 1");
  Workspace ws((hipStream_t)stream);
  int e;
  HF_TRY(data_exp(X_dev, dtype, n_elems, HF_QUANT_AUTO, &e, ws));
  *e_out_host = e;
  return HF_OK;
}

hf_status hf_quantize(const void* X_dev, hf_dtype dtype, int64_t n_elems, int32_t e, uint8_t* codes_dev,
                      void* stream) {
  clear_error();
  HF_ARG(X_dev && codes_dev, "null pointer");
  HF_ARG(valid_dtype(dtype), "bad dtype %d", (int)dtype);
  HF_ARG(n_elems >= 0, "n_elems must be >= 0");
  HF_ARG(e >= -8 && e <= 24, "e must be in [-8, 24]");
  return quantize(X_dev, dtype, n_elems, e, codes_dev, (hipStream_t)stream);
}

hf_status hf_hilbert_sort(const uint8_t* codes_dev, int64_t N, int32_t d, uint64_t seed, uint32_t tree,
                          uint32_t* order_dev, uint32_t* split_dev, void* stream) {
  clear_error();
  HF_ARG(codes_dev && order_dev, "null pointer");
  HF_ARG(N >= 1 && N < (1ll << 31), "N must be in [1, 2^31)");
  HF_ARG(d >= 1 && d <= 4096, "d must be in [1, 4096]");
  HF_ARG(tree < (1u << 20), "tree index too large");
  hipStream_t s = (hipStream_t)stream;
  Workspace ws(s);
  std::vector<int32_t> perm((size_t)(tree + 1) * d);
  std::vector<uint8_t> refl((size_t)(tree + 1) * d);
  make_curves(seed, (int)tree + 1, d, perm.data(), refl.data());
  int32_t* dperm;
  uint8_t* drefl;
  HF_TRY(ws.alloc(&dperm, d));
  HF_TRY(ws.alloc(&drefl, d));
  HIP_TRY(hipMemcpyAsync(dperm, perm.data() + (size_t)tree * d, 4 * d, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(drefl, refl.data() + (size_t)tree * d, d, hipMemcpyHostToDevice, s));
  uint32_t* msb = nullptr;
  if (msb_words(d) > 0) {
    HF_TRY(ws.alloc(&msb, (size_t)(N * msb_words(d))));
    HF_TRY(msb_plane(codes_dev, N, d, msb, s));
  }
  HF_TRY(hilbert_sort_dev(codes_dev, msb, N, d, dperm, drefl, order_dev, split_dev, ws));
  HIP_TRY(hipStreamSynchronize(s));
  return HF_OK;
}

hf_status hf_srp_sketch(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d, int32_t e,
                        uint64_t sketch_seed, uint64_t* out_dev, void* stream) {
  clear_error();
  HF_ARG(X_dev && out_dev, "null pointer");
  HF_ARG(valid_dtype(dtype), "bad dtype");
  HF_ARG(N >= 0 && N < (1ll << 31), "N out of range");
  HF_ARG(d >= 1 && d <= 4096, "d must be in [1, 4096]");
  HF_ARG(e >= -8 && e <= 24, "e must be in [-8, 24]");
  Workspace ws((hipStream_t)stream);
  return srp_sketch(X_dev, dtype, N, d, e, sketch_seed, out_dev, ws);
}

hf_status hf_build_forest(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d,
                          const hf_forest_params* params, void* stream, hf_forest** out) {
  clear_error();
  HF_ARG(X_dev && params && out, "null pointer");
  HF_ARG(params->struct_size == sizeof(hf_forest_params), "struct_size mismatch");
  HF_ARG(valid_dtype(dtype), "bad dtype");
  HF_ARG(N >= 1 && N < (1ll << 31), "N must be in [1, 2^31)");
  HF_ARG(d >= 1 && d <= 4096, "d must be in [1, 4096]");
  HF_ARG(params->n_trees >= 1 && params->n_trees <= 4096, "n_trees must be in [1, 4096]");
  HF_ARG(params->leaf_max >= 1, "leaf_max must be >= 1");
  HF_ARG(params->quant_exp == HF_QUANT_AUTO || (params->quant_exp >= -8 && params->quant_exp <= 24),
         "quant_exp must be HF_QUANT_AUTO or in [-8, 24]");
  HF_ARG(params->sketch == HF_SKETCH_SRP || params->sketch == HF_SKETCH_LEARNED || params->sketch == HF_SKETCH_SIGN,
         "bad sketch kind");
  if (params->sketch == HF_SKETCH_LEARNED) {
    HF_ARG(params->lhash != nullptr, "learned sketches need a hash");
    HF_ARG(lhash_dim(params->lhash) == d, "the hash's input size differs from d");
  }
  if (params->sketch == HF_SKETCH_SIGN && d > HF_SKETCH_BITS) {
    set_error("sign sketches need d <= %d", HF_SKETCH_BITS);
    return HF_ERR_UNSUPPORTED;
  }
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  const int T = (int)params->n_trees;
  hf_forest* f = new hf_forest();
  f->magic = HF_FOREST_MAGIC;
  HIP_TRY(hipGetDevice(&f->device));
  f->N = N;
  f->d = d;
  f->T = T;
  f->M = (int)params->leaf_max;
  f->dtype = dtype;
  f->seed = params->seed;
  f->sketch_seed = params->sketch_seed;
  struct Guard {
    hf_forest* f;
    ~Guard() {
      if (f) forest_release(f);
    }
  } guard{f};
  Workspace ws(s);
  int e;
  HF_TRY(data_exp(X_dev, dtype, N * d, params->quant_exp, &e, ws));
  f->e = e;
  uint8_t* codes;
  HF_TRY(ws.alloc(&codes, (size_t)(N * d)));
  HF_TRY(quantize(X_dev, dtype, N * d, e, codes, s));
  std::vector<int32_t> perm((size_t)T * d);
  std::vector<uint8_t> refl((size_t)T * d);
  make_curves(params->seed, T, d, perm.data(), refl.data());
  const size_t esz = dsize(dtype);
  HIP_TRY(hipMalloc(&f->curve_perm, sizeof(int32_t) * T * d));
  HIP_TRY(hipMalloc(&f->curve_refl, (size_t)T * d));
  HIP_TRY(hipMalloc(&f->X_pos, esz * N * d));
  HIP_TRY(hipMalloc(&f->sk_pos, sizeof(uint64_t) * 8 * N));
  HIP_TRY(hipMalloc(&f->pos2id, sizeof(uint32_t) * N));
  HIP_TRY(hipMalloc(&f->tree_perm, sizeof(uint32_t) * (size_t)T * N));
  HIP_TRY(hipMemcpyAsync(f->curve_perm, perm.data(), sizeof(int32_t) * T * d, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(f->curve_refl, refl.data(), (size_t)T * d, hipMemcpyHostToDevice, s));
  uint32_t* pos;
  HF_TRY(ws.alloc(&pos, N));
  uint32_t* msb = nullptr;
  if (msb_words(d) > 0) {
    HF_TRY(ws.alloc(&msb, (size_t)(N * msb_words(d))));
    HF_TRY(msb_plane(codes, N, d, msb, s));
  }
  std::vector<uint32_t*> tnodes(T, nullptr), taux(T, nullptr);
  std::vector<int64_t> tcount(T, 0);
  struct NodeGuard {
    std::vector<uint32_t*>& v;
    ~NodeGuard() {
      for (auto p : v)
        if (p) (void)hipFree(p);
    }
  } ng{tnodes}, ga{taux};
  const bool progress = getenv("HF_PROGRESS") != nullptr;
  for (int t = 0; t < T; ++t) {
    if (progress && (t % 16 == 0 || t == T - 1)) {
      fprintf(stderr, "[libhf] building tree %d/%d\n", t + 1, T);
      fflush(stderr);
    }
    Workspace wt(s);
    uint32_t *order, *split;
    HF_TRY(wt.alloc(&order, N));
    HF_TRY(wt.alloc(&split, N));
    const int32_t* pt = f->curve_perm + (size_t)t * d;
    const uint8_t* rt = f->curve_refl + (size_t)t * d;
    {
      StageTimer tm(ST_BSORT, s);
      HF_TRY(hilbert_sort_dev(codes, msb, N, d, pt, rt, order, split, wt));
    }
    {
      StageTimer tm(ST_BTRIE, s);
      HF_TRY(build_trie(codes, N, d, f->M, pt, rt, order, split, &tnodes[t], &taux[t], &tcount[t], wt));
    }
    uint32_t* tp = f->tree_perm + (size_t)t * N;
    if (t == 0) {
      HIP_TRY(hipMemcpyAsync(f->pos2id, order, 4 * N, hipMemcpyDeviceToDevice, s));
      k_inverse<<<grid_for(N), 256, 0, s>>>(order, N, pos);
      HF_LAUNCH_CHECK();
    }
    k_map<<<grid_for(N), 256, 0, s>>>(order, pos, N, tp);
    HF_LAUNCH_CHECK();
  }
  f->node_off.assign(T + 1, 0);
  for (int t = 0; t < T; ++t) f->node_off[t + 1] = f->node_off[t] + tcount[t];
  HIP_TRY(hipMalloc(&f->nodes, sizeof(uint32_t) * 2 * (size_t)f->node_off[T]));
  HIP_TRY(hipMalloc(&f->node_off_dev, sizeof(int64_t) * (size_t)(T + 1)));
  HIP_TRY(hipMemcpyAsync(f->node_off_dev, f->node_off.data(), sizeof(int64_t) * (size_t)(T + 1),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMalloc(&f->node_aux, sizeof(uint32_t) * 2 * (size_t)f->node_off[T]));
  for (int t = 0; t < T; ++t) {
    HIP_TRY(hipMemcpyAsync(f->nodes + 2 * f->node_off[t], tnodes[t], 8 * (size_t)tcount[t],
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(f->node_aux + 2 * f->node_off[t], taux[t], 8 * (size_t)tcount[t],
                           hipMemcpyDeviceToDevice, s));
  }
  // coordinate signs (top bits of the codes) in master order, for the exact
  // position of queries along each tree's curve
  f->sgn_words = msb ? msb_words(d) : 0;
  if (msb) {
    HIP_TRY(hipMalloc(&f->sgn_pos, sizeof(uint32_t) * (size_t)f->sgn_words * N));
    k_gather_rows<<<grid_for(N * f->sgn_words / 4 + 1), 256, 0, s>>>((const unsigned char*)msb,
                                                                     (int64_t)(4 * f->sgn_words), f->pos2id, N,
                                                                     (unsigned char*)f->sgn_pos);
    HF_LAUNCH_CHECK();
  }
  k_gather_rows<<<grid_for(N * d * esz / 16 + 1), 256, 0, s>>>((const unsigned char*)X_dev,
                                                               (int64_t)(esz * d), f->pos2id, N,
                                                               (unsigned char*)f->X_pos);
  HF_LAUNCH_CHECK();
  size_t r_bytes = 0;
  HF_TRY(srp_matrix_upload(d, params->sketch_seed, &f->srp_R, &r_bytes, s));
  if (d % 16 == 0) {
    HF_TRY(srp_matrix_i8_upload(d, params->sketch_seed, &f->srp_Rb, s));
    r_bytes += 512 * (size_t)d;
  }
  {
    StageTimer tm(ST_BSKETCH, s);
    if (params->sketch == HF_SKETCH_LEARNED)
      HF_TRY(lhash_encode_dev(params->lhash, f->X_pos, dtype, N, f->sk_pos, s));
    else if (params->sketch == HF_SKETCH_SIGN)
      HF_TRY(sign_sketch(f->X_pos, dtype, N, d, f->sk_pos, s));
    else if (f->srp_Rb && getenv("HF_SRP_VALU") == nullptr)
      HF_TRY(srp_sketch_mfma(f->X_pos, dtype, N, d, e, f->srp_Rb, f->sk_pos, s));
    else
      HF_TRY(srp_sketch(f->X_pos, dtype, N, d, e, params->sketch_seed, f->sk_pos, ws, f->srp_R));
  }
  f->sketch_kind = (int)params->sketch;
  f->lhash = params->sketch == HF_SKETCH_LEARNED ? params->lhash : nullptr;
  HIP_TRY(hipStreamSynchronize(s));
  f->device_bytes = (int64_t)(esz * N * d + 64 * N + 4 * N + 4 * (size_t)T * N +
                              16 * (size_t)f->node_off[T] + 5 * (size_t)T * d + 8 * (size_t)(T + 1) + r_bytes +
                              4 * (size_t)f->sgn_words * N);
  guard.f = nullptr;
  *out = f;
  return HF_OK;
}

void hf_forest_free(hf_forest* f) {
  if (f && f->magic == HF_FOREST_MAGIC) forest_release(f);
}

hf_status hf_forest_get_info(const hf_forest* f, hf_forest_info* info) {
  clear_error();
  HF_TRY(check_forest(f));
  HF_ARG(info, "null pointer");
  info->N = f->N;
  info->d = f->d;
  info->n_trees = f->T;
  info->leaf_max = f->M;
  info->quant_exp = f->e;
  info->dtype = (int32_t)f->dtype;
  info->device = f->device;
  info->total_nodes = f->node_off[f->T];
  info->device_bytes = f->device_bytes;
  return HF_OK;
}

hf_status hf_forest_perm(const hf_forest* f, uint32_t t, uint32_t* perm_dev, void* stream) {
  clear_error();
  HF_TRY(check_forest(f));
  HF_ARG(perm_dev && t < (uint32_t)f->T, "bad tree index or null pointer");
  HIP_TRY(hipMemcpyAsync(perm_dev, f->tree_perm + (size_t)t * f->N, 4 * f->N, hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return HF_OK;
}

hf_status hf_forest_nodes(const hf_forest* f, uint32_t t, uint32_t* nodes_dev, int64_t* count_host,
                          void* stream) {
  clear_error();
  HF_TRY(check_forest(f));
  HF_ARG(t < (uint32_t)f->T, "bad tree index");
  int64_t n = f->node_off[t + 1] - f->node_off[t];
  if (count_host) *count_host = n;
  if (nodes_dev)
    HIP_TRY(hipMemcpyAsync(nodes_dev, f->nodes + 2 * f->node_off[t], 8 * (size_t)n,
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return HF_OK;
}

hf_status hf_forest_node_splits(const hf_forest* f, uint32_t t, uint32_t* splits_dev, int64_t* count_host,
                                void* stream) {
  clear_error();
  HF_TRY(check_forest(f));
  HF_ARG(t < (uint32_t)f->T, "bad tree index");
  const int64_t n = f->node_off[t + 1] - f->node_off[t];
  if (count_host) *count_host = n;
  if (splits_dev)
    HIP_TRY(hipMemcpyAsync(splits_dev, f->node_aux + 2 * f->node_off[t], 8 * (size_t)n, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
  return HF_OK;
}

hf_status hf_forest_pos2id(const hf_forest* f, uint32_t* pos2id_dev, void* stream) {
  clear_error();
  HF_TRY(check_forest(f));
  HF_ARG(pos2id_dev, "null pointer");
  HIP_TRY(hipMemcpyAsync(pos2id_dev, f->pos2id, 4 * f->N, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return HF_OK;
}

hf_status hf_forest_sketches(const hf_forest* f, uint64_t* sk_dev, void* stream) {
  clear_error();
  HF_TRY(check_forest(f));
  HF_ARG(sk_dev, "null pointer");
  HIP_TRY(hipMemcpyAsync(sk_dev, f->sk_pos, 64 * f->N, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return HF_OK;
}

static hf_status check_search(const hf_forest* f, const void* Q, hf_dtype dtype, int64_t nq,
                              const hf_search_params* p, const void* ids, const void* scores) {
  HF_TRY(check_forest(f));
  HF_ARG(p && Q && ids && scores, "null pointer");
  HF_ARG(p->struct_size == sizeof(hf_search_params), "struct_size mismatch");
  HF_ARG(dtype == f->dtype, "query dtype differs from the forest's");
  HF_ARG(nq >= 1 && nq < (1ll << 31), "nq out of range");
  HF_ARG(p->k >= 1 && p->k <= 1024, "k must be in [1, 1024]");
  HF_ARG(p->k1 >= 1, "k1 must be >= 1");
  HF_ARG(p->k2 >= p->k && p->k2 <= 4096, "k2 must be in [k, 4096]");
  HF_ARG(p->h <= 1024, "h must be <= 1024");
  HF_ARG(p->precision <= HF_PREC_C4, "bad precision %u", p->precision);
  if (p->precision == HF_PREC_C4 && !f->c4_mag) {
    set_error("the forest has no 4-bit codes: call hf_forest_add_precision(HF_PREC_C4) first");
    return HF_ERR_INVALID_ARG;
  }
  if (p->precision == HF_PREC_BF16 && !f->X_bf16) {
    set_error("the forest has no BF16 copy: call hf_forest_add_precision first");
    return HF_ERR_INVALID_ARG;
  }
  if (p->precision == HF_PREC_FP8 && !f->X_fp8) {
    set_error("the forest has no FP8 copy: call hf_forest_add_precision first");
    return HF_ERR_INVALID_ARG;
  }
  if (p->precision == HF_PREC_BF16 || p->precision == HF_PREC_FP8) {
    const uint32_t S = p->survivors ? p->survivors : 4 * p->k;
    HF_ARG(S >= p->k && S <= 4096, "survivors must be in [k, 4096]");
  }
  HF_ARG(p->trees <= (uint32_t)f->T, "trees (%u) exceeds the forest's %d trees", p->trees, f->T);
  HF_ARG(p->position <= HF_POS_EXACT, "bad position %u", p->position);
  if (p->position == HF_POS_EXACT && f->sgn_words == 0) {
    set_error("exact query positions need d <= 512");
    return HF_ERR_UNSUPPORTED;
  }
  if ((int64_t)(p->trees ? (int)p->trees : f->T) * (int64_t)std::min<int64_t>(p->k1, f->N) > (1ll << 30)) {
    set_error("n_trees * k1 too large");
    return HF_ERR_UNSUPPORTED;
  }
  return HF_OK;
}

hf_status hf_search(const hf_forest* f, const void* Q_dev, hf_dtype dtype, int64_t nq,
                    const hf_search_params* params, int32_t* ids_dev, float* scores_dev, void* stream) {
  clear_error();
  HF_TRY(check_search(f, Q_dev, dtype, nq, params, ids_dev, scores_dev));
  return search_launch(f, Q_dev, nq, *params, ids_dev, scores_dev, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr, (hipStream_t)stream);
}

hf_status hf_search_debug(const hf_forest* f, const void* Q_dev, hf_dtype dtype, int64_t nq,
                          const hf_search_params* params, int32_t* ids_dev, float* scores_dev,
                          uint32_t* win_dev, uint32_t* c2_dev, int32_t* c2n_dev, int32_t* en_dev,
                          void* stream) {
  clear_error();
  HF_TRY(check_search(f, Q_dev, dtype, nq, params, ids_dev, scores_dev));
  return search_launch(f, Q_dev, nq, *params, ids_dev, scores_dev, win_dev, c2_dev, c2n_dev, en_dev,
                       nullptr, nullptr, (hipStream_t)stream);
}

hf_status hf_forest_set_sketch(hf_forest* f, hf_sketch_kind kind, const hf_lhash* lhash, void* stream) {
  clear_error();
  HF_TRY(check_forest(f));
  HF_ARG(kind == HF_SKETCH_SRP || kind == HF_SKETCH_LEARNED || kind == HF_SKETCH_SIGN, "bad sketch kind");
  hipStream_t s = (hipStream_t)stream;
  if (kind == HF_SKETCH_LEARNED) {
    HF_ARG(lhash != nullptr, "learned sketches need a hash");
    HF_ARG(lhash_dim(lhash) == f->d, "the hash's input size differs from the forest's d");
    HF_TRY(lhash_encode_dev(lhash, f->X_pos, f->dtype, f->N, f->sk_pos, s));
  } else if (kind == HF_SKETCH_SIGN) {
    HF_TRY(sign_sketch(f->X_pos, f->dtype, f->N, f->d, f->sk_pos, s));
  } else if (f->srp_Rb && getenv("HF_SRP_VALU") == nullptr) {
    HF_TRY(srp_sketch_mfma(f->X_pos, f->dtype, f->N, f->d, f->e, f->srp_Rb, f->sk_pos, s));
  } else {
    Workspace ws(s);
    HF_TRY(srp_sketch(f->X_pos, f->dtype, f->N, f->d, f->e, f->sketch_seed, f->sk_pos, ws, f->srp_R));
  }
  HIP_TRY(hipStreamSynchronize(s));
  f->sketch_kind = (int)kind;
  f->lhash = kind == HF_SKETCH_LEARNED ? lhash : nullptr;
  return HF_OK;
}

hf_status hf_forest_add_precision(hf_forest* f, hf_precision prec, void* stream) {
  clear_error();
  HF_TRY(check_forest(f));
  HF_ARG(prec == HF_PREC_BF16 || prec == HF_PREC_FP8 || prec == HF_PREC_C4, "precision must be BF16, FP8 or C4");
  if (prec == HF_PREC_C4) return make_c4(f, (hipStream_t)stream);
  return make_lowprec(f, prec, (hipStream_t)stream);
}

hf_status hf_search_lowprec_debug(const hf_forest* f, const void* Q_dev, hf_dtype dtype, int64_t nq,
                                  const hf_search_params* params, int32_t* ids_dev, float* scores_dev,
                                  uint32_t* surv_pos_dev, float* surv_score_dev, void* stream) {
  clear_error();
  HF_TRY(check_search(f, Q_dev, dtype, nq, params, ids_dev, scores_dev));
  HF_ARG(params->precision != HF_PREC_FP32, "precision must be BF16 or FP8");
  HF_ARG(surv_pos_dev && surv_score_dev, "null pointer");
  return search_launch(f, Q_dev, nq, *params, ids_dev, scores_dev, nullptr, nullptr, nullptr, nullptr,
                       surv_pos_dev, surv_score_dev, (hipStream_t)stream);
}

hf_status hf_audit_scores(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d, const void* Q_dev,
                          int64_t nq, const int32_t* ids_dev, int32_t k, double* out_dev, void* stream) {
  clear_error();
  HF_ARG(X_dev && Q_dev && ids_dev && out_dev, "null pointer");
  HF_ARG(valid_dtype(dtype), "bad dtype");
  HF_ARG(N >= 1 && d >= 1 && d <= 4096 && nq >= 1 && k >= 1, "bad sizes");
  return audit_launch(X_dev, dtype, d, Q_dev, nq, ids_dev, k, out_dev, (hipStream_t)stream);
}

static hf_status knn_graph(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d, const hf_graph_params* p,
                           int32_t* ids_dev, float* scores_dev, int32_t* c2_dev, void* stream) {
  clear_error();
  HF_ARG(X_dev && p && ids_dev && scores_dev, "null pointer");
  HF_ARG(p->struct_size == sizeof(hf_graph_params), "struct_size mismatch");
  HF_ARG(valid_dtype(dtype), "bad dtype");
  HF_ARG(N >= 2 && N < (1ll << 31), "N must be in [2, 2^31)");
  HF_ARG(d >= 1 && d <= 4096, "d must be in [1, 4096]");
  HF_ARG(p->n_orders >= 1 && p->n_orders <= 4096, "n_orders must be in [1, 4096]");
  HF_ARG(p->window >= 1 && p->window <= 512 && 2 * (int64_t)p->window < N, "window must be in [1, 512] and 2w < N");
  HF_ARG(p->k >= 1 && p->k <= 32, "k must be in [1, 32]");
  HF_ARG(p->k2 == 0 || (p->k2 >= p->k && p->k2 <= 256), "k2 must be 0 or in [k, 256]");
  HF_ARG(p->quant_exp == HF_QUANT_AUTO || (p->quant_exp >= -8 && p->quant_exp <= 24), "bad quant_exp");
  HF_ARG(p->k2 == 0 || p->sketch == HF_SKETCH_SRP || p->sketch == HF_SKETCH_LEARNED || p->sketch == HF_SKETCH_SIGN,
         "bad sketch kind");
  if (p->k2 > 0 && p->sketch == HF_SKETCH_SIGN && d > HF_SKETCH_BITS) {
    set_error("sign sketches need d <= %d", HF_SKETCH_BITS);
    return HF_ERR_UNSUPPORTED;
  }
  HF_ARG(((uintptr_t)X_dev & 15) == 0, "X_dev must be 16-byte aligned");
  if (dtype != HF_F16 || d % 8 != 0) {
    set_error("the graph kernels take fp16 rows with d a multiple of 8");
    return HF_ERR_UNSUPPORTED;
  }
  if (p->k2 > 0 && p->sketch == HF_SKETCH_LEARNED) {
    HF_ARG(p->lhash != nullptr, "learned sketches need a hash");
    HF_ARG(lhash_dim(p->lhash) == d, "the hash's input size differs from d");
  }
  hipStream_t s = (hipStream_t)stream;
  int e;
  {
    Workspace ws(s);
    HF_TRY(data_exp(X_dev, dtype, N * d, p->quant_exp, &e, ws));
  }
  return graph_launch(X_dev, dtype, N, d, *p, e, ids_dev, scores_dev, c2_dev, s);
}

hf_status hf_knn_graph(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d, const hf_graph_params* p,
                       int32_t* ids_dev, float* scores_dev, void* stream) {
  return knn_graph(X_dev, dtype, N, d, p, ids_dev, scores_dev, nullptr, stream);
}

hf_status hf_knn_graph_debug(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d, const hf_graph_params* p,
                             int32_t* ids_dev, float* scores_dev, int32_t* c2_dev, void* stream) {
  clear_error();
  HF_ARG(p && p->k2 > 0 && c2_dev, "the debug graph needs k2 > 0 and a C2 buffer");
  return knn_graph(X_dev, dtype, N, d, p, ids_dev, scores_dev, c2_dev, stream);
}

}  // extern "C"

namespace hf {
hf_status search_args_ok(const hf_forest* f, const void* Q, hf_dtype dtype, int64_t nq, const hf_search_params* p,
                         const void* ids, const void* scores) {
  return check_search(f, Q, dtype, nq, p, ids, scores);
}
}  // namespace hf
