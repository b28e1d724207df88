// Internal declarations of libhf: status handling, device helpers and the
// host launchers each .hip file provides.  Not part of the public ABI.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/hf.h"

namespace hf {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
void clear_error();

struct Err {
  hf_status s;
};

#define HF_TRY(expr)                                   \
  do {                                                 \
    hf_status _s = (expr);                             \
    if (_s != HF_OK) return _s;                        \
  } while (0)

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      ::hf::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),       \
                      __FILE__, __LINE__);                                         \
      return _e == hipErrorOutOfMemory ? HF_ERR_OOM : HF_ERR_DEVICE;               \
    }                                                                              \
  } while (0)

#define HF_LAUNCH_CHECK() HIP_TRY(hipGetLastError())

#define HF_ARG(cond, ...)               \
  do {                                  \
    if (!(cond)) {                      \
      ::hf::set_error(__VA_ARGS__);     \
      return HF_ERR_INVALID_ARG;        \
    }                                   \
  } while (0)

// ---------------------------------------------------------------- workspace
// The caller's scratch allocator (hf_set_allocator); `on` false: hipMallocAsync.
struct ScratchAlloc {
  hf_allocator a;
  bool on;
};
ScratchAlloc scratch_allocator();

// Device buffers owned by one call; freed (stream-ordered) on scope exit,
// through the allocator that was registered when the call started.  In arena
// mode (the second constructor) buffers are carved, 256-byte aligned, from a
// caller-provided device region and nothing is allocated or freed.
struct Workspace {
  hipStream_t stream;
  ScratchAlloc al;
  std::vector<void*> ptrs;
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  explicit Workspace(hipStream_t s) : stream(s), al(scratch_allocator()) {}
  Workspace(hipStream_t s, void* region, size_t bytes)
      : stream(s), al{{nullptr, nullptr, nullptr}, false}, arena((char*)region), arena_cap(bytes) {}
  ~Workspace() {
    for (void* p : ptrs) {
      if (al.on)
        al.a.free(p, al.a.ctx, (void*)stream);
      else
        (void)hipFreeAsync(p, stream);
    }
  }
  // bytes an arena needs for buffers of these sizes (each rounded up to 256)
  static size_t arena_bytes(size_t bytes) { return (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255; }
  template <class T>
  hf_status alloc(T** out, size_t count) {
    void* p = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 16;
    if (arena) {
      const size_t need = arena_bytes(bytes);
      if (arena_used + need > arena_cap) {
        set_error("scratch region of %zu bytes exhausted (%zu more needed)", arena_cap,
                  arena_used + need - arena_cap);
        return HF_ERR_UNSUPPORTED;
      }
      *out = reinterpret_cast<T*>(arena + arena_used);
      arena_used += need;
      return HF_OK;
    }
    if (al.on) {
      p = al.a.alloc(bytes, al.a.ctx, (void*)stream);
      if (!p) {
        set_error("the caller's allocator returned no memory for %zu bytes", bytes);
        return HF_ERR_OOM;
      }
      ptrs.push_back(p);
      *out = static_cast<T*>(p);
      return HF_OK;
    }
    hipError_t e = hipMallocAsync(&p, bytes, stream);
    if (e != hipSuccess) {
      set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
      return HF_ERR_OOM;
    }
    ptrs.push_back(p);
    *out = static_cast<T*>(p);
    return HF_OK;
  }
};

// ------------------------------------------------------------ device helpers
constexpr int WAVE = 64;
constexpr uint32_t NONE32 = 0xFFFFFFFFu;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// quad_perm DPP moves: lane i of each quad reads lane sel[i] of the quad
template <int CTRL>
__device__ __forceinline__ uint32_t quad_perm(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t quad_bcast(uint32_t v, int u) {
  return u == 0 ? quad_perm<0x00>(v) : u == 1 ? quad_perm<0x55>(v) : u == 2 ? quad_perm<0xAA>(v) : quad_perm<0xFF>(v);
}
constexpr int QP_XOR1 = 0xB1;  // [1, 0, 3, 2]
constexpr int QP_XOR2 = 0x4E;  // [2, 3, 0, 1]
__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl(lo, src);
  hi = __shfl(hi, src);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl_xor(lo, m);
  hi = __shfl_xor(hi, m);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int m = 32; m >= 1; m >>= 1) {
    uint64_t o = shfl_xor_u64(v, m);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v) {
  for (int m = 32; m >= 1; m >>= 1) v |= shfl_xor_u64(v, m);
  return v;
}

// Inclusive scan of uint32 over one wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  int l = __lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_up(v, off);
    if (l >= off) v += o;
  }
  return v;
}

// Exclusive scan over a block of THREADS threads (one value each); `lds` holds
// THREADS/64 + 1 words.  Returns the exclusive prefix, *total the sum.
template <int THREADS>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
  constexpr int NW = THREADS / 64;
  int w = threadIdx.x / 64, l = __lane_id();
  uint32_t inc = wave_incl_scan(v);
  if (l == 63) lds[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int i = 0; i < NW; ++i) {
      uint32_t t = lds[i];
      lds[i] = run;
      run += t;
    }
    lds[NW] = run;
  }
  __syncthreads();
  uint32_t r = lds[w] + inc - v;
  *total = lds[NW];
  __syncthreads();
  return r;
}

// float -> uint32 whose unsigned order is the float order (NaN-free input).
__device__ __forceinline__ uint32_t float_to_ordered(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// LDS written and read by the same wavefront only: order the accesses
// without a block barrier.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup barrier that orders LDS accesses only: global loads in flight
// stay in flight across it (__syncthreads waits for every outstanding one).
__device__ __forceinline__ void block_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

inline int bits_for(uint64_t max_value) {
  int b = 0;
  while (b < 64 && (max_value >> b) != 0) ++b;
  return b;
}

// ---------------------------------------------------------------- launchers
// hf_scan.hip
hf_status excl_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev,
                        Workspace& ws);
// hf_radix.hip: stable LSD sort of (key, val) pairs on key bits [bit_lo, bit_hi).
// Sorted pairs end in (*keys, *vals), which may be swapped with (alt_keys, alt_vals).
hf_status radix_sort_pairs(uint64_t** keys, uint32_t** vals, uint64_t** alt_keys,
                           uint32_t** alt_vals, int64_t n, int bit_lo, int bit_hi, Workspace& ws);
// hf_quant.hip
hf_status minmax(const void* X, hf_dtype dt, int64_t n, float* mn_host, float* mx_host,
                 int* nonfinite_host, Workspace& ws);
int choose_exp(float mn, float mx);
hf_status quantize(const void* X, hf_dtype dt, int64_t n, int e, uint8_t* out, hipStream_t s);
// hf_keys.hip
// msb: optional top-bit plane (msb_words(d) words per point) for top-level chunks.
int msb_words(int d);
hf_status msb_plane(const uint8_t* codes, int64_t N, int d, uint32_t* msb, hipStream_t s);
hf_status key_chunks(const uint8_t* codes, const uint32_t* msb, int d, const int32_t* perm,
                     const uint8_t* refl, const uint32_t* items, int64_t n_items, int chunk,
                     uint64_t* out, hipStream_t s);
// Window starts of the (query, tree) pairs listed in deep (q << 32 | t; *ndeep
// of them, on the device) whose exact position needs keys below the top level.
hf_status rank_deep(const hf_forest* f, const uint8_t* qcodes, int64_t nq, int T, int k1, const uint64_t* deep,
                    const uint32_t* ndeep, uint32_t* win, hipStream_t s);
hf_status node_tests(const uint8_t* codes, int d, const int32_t* perm, const uint8_t* refl,
                     const uint32_t* points, const uint32_t* bits, int64_t n, uint32_t* out_w1,
                     hipStream_t s);
// hf_sort.hip: Hilbert sort with a curve already on the device.
// msb (nullable): top-bit plane of the codes, computed once per code set.
hf_status hilbert_sort_dev(const uint8_t* codes, const uint32_t* msb, int64_t N, int d,
                           const int32_t* perm, const uint8_t* refl, uint32_t* order, uint32_t* split,
                           Workspace& ws);
// hf_trie.hip: pre-order trie records (2 words each) from a sorted order and its split bits.
// aux_out: 2 words per node (hipMalloc, caller frees): internal {split
// position m, split bit b}, leaf {lo, 0xFFFFFFFF}.
hf_status build_trie(const uint8_t* codes, int64_t N, int d, int M, const int32_t* perm,
                     const uint8_t* refl, const uint32_t* order, const uint32_t* split,
                     uint32_t** nodes_out, uint32_t** aux_out, int64_t* n_nodes, Workspace& ws);
// hf_sketch.hip
// SRP sketches of N rows; R_dev: a resident projection matrix (a forest's),
// else it is generated from sketch_seed, uploaded and waited for
hf_status srp_sketch(const void* X, hf_dtype dt, int64_t N, int d, int e, uint64_t sketch_seed,
                     uint64_t* out, Workspace& ws, const uint64_t* R_dev = nullptr);
// the same sketches on the int8 matrix cores (d a multiple of 16), with the
// projection signs as 512 x d int8 rows (srp_matrix_i8_upload, hipMalloc)
hf_status srp_sketch_mfma(const void* X, hf_dtype dt, int64_t N, int d, int e, const int8_t* Rb, uint64_t* out,
                          hipStream_t s);
hf_status srp_matrix_i8_upload(int d, uint64_t sketch_seed, int8_t** out, hipStream_t s);
// the projection matrix of (d, sketch_seed) in a new device buffer (hipMalloc)
hf_status srp_matrix_upload(int d, uint64_t sketch_seed, uint64_t** out, size_t* bytes, hipStream_t s);
// stage timing (hf_api.hip): events around a launch when timing is on
enum Stage { ST_QCODES = 0, ST_QSKETCH, ST_DESCEND, ST_HAM, ST_SELECT, ST_RERANK, ST_GSORT, ST_GBAND,
             ST_BSORT, ST_BTRIE, ST_BSKETCH, ST_LOWPREC, ST_GHAM, ST_GMERGE, ST_GFINAL, ST_GMAIL, ST_COUNT };
bool timing_on();
void timing_mark(int stage, bool begin, hipStream_t s);
struct StageTimer {
  int st;
  hipStream_t s;
  StageTimer(int stage, hipStream_t stream) : st(stage), s(stream) { timing_mark(st, true, s); }
  ~StageTimer() { timing_mark(st, false, s); }
};
// hf_lowprec.hip
hf_status make_lowprec(hf_forest* f, hf_precision prec, hipStream_t s);
hf_status rerank_lp_launch(const hf_forest* f, hf_precision prec, const void* Qb, int64_t nb,
                           const uint32_t* c2b, const int32_t* c2nb, int k2, int h, int k, int S,
                           int32_t* idsb, float* scb, uint32_t* surv_pos, float* surv_score,
                           int32_t* enb, hipStream_t s);
hf_status audit_launch(const void* X, hf_dtype dt, int d, const void* Q, int64_t nq, const int32_t* ids,
                       int k, double* out, hipStream_t s);
// hf_gprefilter.hip: sketch prefilter of the graph.  lists: N x k2 keys
// (Hamming << 32 | id), ascending, empty slots all-ones.
constexpr int GRAPH_K2_MAX = 256;
hf_status gpf_init_lists(uint64_t* lists, int64_t n, hipStream_t s);
// One order: stage holds 2w x chunk keys, cnt chunk counters.
hf_status gpf_order(const uint64_t* sk, const uint32_t* order, int64_t N, int w, int k2, uint64_t* lists,
                    int64_t chunk, uint64_t* stage, uint32_t* cnt, hipStream_t s);
// Final cosine top-k of every list; c2_ids (nullable) receives the listed ids (-1 if empty).
hf_status gpf_final(const void* X, const float* nrm, int64_t N, int d, const uint64_t* lists, int k2, int k,
                    int32_t* ids, float* sc, int32_t* c2_ids, hipStream_t s);
// hf_lhash.hip
// ws (nullable): where the hidden-layer staging comes from (a call's own
// workspace otherwise)
hf_status lhash_encode_dev(const hf_lhash* L, const void* X, hf_dtype dt, int64_t N, uint64_t* sk, hipStream_t s,
                           Workspace* ws = nullptr);
// hf_search.hip: Algorithm 1 for nq queries; scratch from ws when given
hf_status search_launch(const hf_forest* f, const void* Q, int64_t nq, const hf_search_params& p,
                        int32_t* ids, float* scores, uint32_t* win_out, uint32_t* c2_out,
                        int32_t* c2n_out, int32_t* en_out, uint32_t* surv_pos, float* surv_score,
                        hipStream_t s, Workspace* ws = nullptr);
// hf_c4.hip: the paper's compressed layout (sign sketches, 4-bit codes)
hf_status sign_sketch(const void* X, hf_dtype dt, int64_t N, int d, uint64_t* out, hipStream_t s);
hf_status make_c4(hf_forest* f, hipStream_t s);
hf_status rerank_c4_launch(const hf_forest* f, const void* Qb, int64_t nb, const uint32_t* c2b, const int32_t* c2nb,
                           int k2, int h, int k, int32_t* idsb, float* scb, int32_t* enb, hipStream_t s);
// hf_bfilter.hip: the Hamming filter by master-position bucket.  Writes C2
// and its count for the queries it completes and flag[q] = 0 for them,
// flag[q] = 1 for the queries the entry-by-entry filter must redo.
bool bfilter_usable(int64_t N, int T, int k2);
int64_t bfilter_max_batch(int64_t N);
hf_status bfilter_run(const hf_forest* f, int T, int len, int64_t nb, const uint32_t* win, const uint64_t* qsk,
                      int k2, uint32_t* c2, int32_t* c2n, uint32_t* flag, Workspace& ws);
// hf_api.hip: the argument checks of hf_search
hf_status search_args_ok(const hf_forest* f, const void* Q, hf_dtype dtype, int64_t nq, const hf_search_params* p,
                         const void* ids, const void* scores);
// scratch bytes search_launch takes from an arena for nq queries
size_t search_scratch_bytes(const hf_forest* f, int64_t nq, const hf_search_params& p);
int lhash_dim(const hf_lhash* L);
int lhash_hidden(const hf_lhash* L);
// host helpers (hf_api.hip)
void make_curves(uint64_t seed, int T, int d, int32_t* perm, uint8_t* refl);
uint64_t splitmix64_next(uint64_t* state);

}  // namespace hf

// Forest handle.
struct hf_forest {
  uint32_t magic;
  int device;
  int64_t N;
  int32_t d, T, M, e;
  hf_dtype dtype;
  uint64_t seed, sketch_seed;
  void* X_pos;           // N x d rows in master order (dtype)
  uint64_t* sk_pos;      // N x 8 sketch words in master order
  uint32_t* pos2id;      // N
  uint32_t* tree_perm;   // T x N master positions
  uint32_t* nodes;       // all trees' records, 2 words per node
  uint32_t* node_aux;    // per node {m, b} (internal) or {lo, NONE} (leaf), same offsets
  uint32_t* sgn_pos;     // N x sgn_words top bits of the codes (coordinate signs), master order
  int sgn_words;         // 32-bit words per row of sgn_pos (0: d too large, no exact rank)
  uint32_t* c4_mag;      // N x sgn_words x 3 magnitude bit planes of the 4-bit codes, or null
  float* c4_scale;       // N scales of the 4-bit codes (max |x| / 8)
  std::vector<int64_t> node_off;  // T+1 offsets (in nodes)
  int64_t* node_off_dev; // the same offsets on the device
  uint64_t* srp_R;       // SRP projection matrix of (d, sketch_seed) on the device
  int8_t* srp_Rb;        // the same signs as 512 x d int8 rows (matrix-core sketches), or null
  int32_t* curve_perm;   // T x d
  uint8_t* curve_refl;   // T x d
  void* X_bf16;          // N x d bfloat16 copy of X_pos (precision form), or null
  void* X_fp8;           // N x d e4m3 codes of X_pos, or null
  float* s_fp8;          // N per-row scales of X_fp8
  int sketch_kind;       // hf_sketch_kind of sk_pos
  const hf_lhash* lhash; // encoder of queries when sketch_kind is learned (not owned)
  int64_t device_bytes;
};
constexpr uint32_t HF_FOREST_MAGIC = 0x48464f52u;  // "HFOR"
