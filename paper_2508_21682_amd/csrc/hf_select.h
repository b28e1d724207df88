// Block-level selection helpers shared by the rerank kernels: bitonic sorts
// in LDS, the merged expansion intervals of a sorted candidate list, and an
// exact k-smallest selection of 32-bit keys (radix select + ordered ties).
#pragma once

#include "hf_internal.h"

namespace hf {

// Bitonic sort of a[0..n2) in LDS by the whole workgroup (n2 a power of two,
// blockDim.x a multiple of 64).  A stage compares n2/2 pairs, pair p on
// thread p mod blockDim.x: elements i = ((p & ~(j-1)) << 1) | (p & (j-1))
// and i + j.  While j <= 32 the pairs of one wavefront's p-range stay in a
// 128-element run that this wavefront alone touches in every such stage, so
// those stages are separated by wavefront syncs; a workgroup barrier follows
// every stage with j >= 64, every stage before one, and the last stage.
template <class T>
__device__ __forceinline__ void bitonic_lds(T* a, int n2) {
  const int half = n2 >> 1;
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int p = threadIdx.x; p < half; p += blockDim.x) {
        const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
        const T x = a[i], y = a[i + j];
        if ((x > y) == ((i & k) == 0)) {
          a[i] = y;
          a[i + j] = x;
        }
      }
      const int jn = j > 1 ? j >> 1 : k;  // j of the next stage (k doubles after j = 1)
      if (j > 32 || jn > 32 || (j == 1 && k == n2))
        __syncthreads();
      else
        wave_lds_sync();
    }
}

__device__ __forceinline__ void bitonic_u32(uint32_t* a, int n2) { bitonic_lds(a, n2); }

__device__ __forceinline__ void bitonic_u64(uint64_t* a, int n2) { bitonic_lds(a, n2); }

__device__ __forceinline__ float ordered_to_float(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __uint_as_float(u);
}

// Position of expansion entry e: interval i with off[i] <= e < off[i+1].
__device__ __forceinline__ uint32_t epos(const uint32_t* st, const uint32_t* off, int n2, uint32_t e) {
  int lo = 0, hi = n2 - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return st[lo] + (e - off[lo]);
}

// Merged intervals [max(0,r-h), min(N-1,r+h)] of the sorted distinct positions
// sc[0..n2): interval i starts at st[i] and holds off[i+1]-off[i] positions
// that no earlier interval holds; off[n2] = |E| (also stored in *s_E).
template <int THREADS>
__device__ __forceinline__ void expansion_intervals(const uint32_t* sc, int n2, int h, int64_t N,
                                                    uint32_t* st, uint32_t* off, uint32_t* scan_tmp,
                                                    uint32_t* s_E) {
  const int per = (n2 + THREADS - 1) / THREADS;
  const int a0 = threadIdx.x * per, a1 = min(n2, a0 + per);
  uint32_t mine = 0;
  for (int i = a0; i < a1; ++i) {
    int64_t r = sc[i];
    int64_t a = r - h < 0 ? 0 : r - h, z = r + h > N - 1 ? N - 1 : r + h;
    if (i > 0) {
      int64_t pz = (int64_t)sc[i - 1] + h;
      pz = pz > N - 1 ? N - 1 : pz;
      if (a < pz + 1) a = pz + 1;
    }
    st[i] = (uint32_t)a;
    off[i] = z >= a ? (uint32_t)(z - a + 1) : 0u;
    mine += off[i];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan<THREADS>(mine, scan_tmp, &tot);
  for (int i = a0; i < a1; ++i) {
    uint32_t c = off[i];
    off[i] = run;
    run += c;
  }
  if (threadIdx.x == 0) {
    off[n2] = tot;
    *s_E = tot;
  }
  __syncthreads();
}

// The kk smallest of keys[0..E) as (key << 32 | index) in sel[0..kk), ties
// taken in index order: an 8-bit radix select finds the kk-th key, keys below
// it are collected, then the first equal ones by index.  sel is not sorted.
template <int THREADS>
__device__ __forceinline__ void select_smallest(const uint32_t* keys, uint32_t E, uint32_t kk,
                                                uint64_t* sel, uint32_t* hist, uint32_t* scan_tmp,
                                                uint32_t* s_prefix, uint32_t* s_lt, uint32_t* s_want,
                                                uint32_t* s_nsel) {
  if (threadIdx.x == 0) {
    *s_prefix = 0;
    *s_lt = 0;
    *s_want = kk;
    *s_nsel = 0;
  }
  __syncthreads();
  for (int pass = 0; pass < 4 && kk > 0; ++pass) {
    const int shift = 24 - 8 * pass;
    const uint32_t hi_mask = pass == 0 ? 0u : (0xFFFFFFFFu << (32 - 8 * pass));
    const uint32_t prefix = *s_prefix;
    for (int i = threadIdx.x; i < 256; i += THREADS) hist[i] = 0;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < E; e += THREADS) {
      const uint32_t key = keys[e];
      if ((key & hi_mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t want = *s_want, cum = 0;
      int b = 0;
      for (; b < 256; ++b) {
        if (cum + hist[b] >= want) break;
        cum += hist[b];
      }
      *s_prefix = prefix | ((uint32_t)b << shift);
      *s_lt += cum;
      *s_want = want - cum;
    }
    __syncthreads();
  }
  const uint32_t thr = *s_prefix, n_lt = *s_lt;
  const int per = (int)((E + THREADS - 1) / THREADS);
  const int a0 = threadIdx.x * per, a1 = min((int)E, a0 + per);
  uint32_t myeq = 0;
  for (int e = a0; e < a1; ++e) {
    const uint32_t key = keys[e];
    if (kk > 0 && key < thr) {
      const uint32_t slot = atomicAdd(s_nsel, 1u);
      sel[slot] = ((uint64_t)key << 32) | (uint32_t)e;
    } else if (kk > 0 && key == thr) {
      ++myeq;
    }
  }
  uint32_t tot;
  uint32_t r = block_excl_scan<THREADS>(myeq, scan_tmp, &tot);
  const uint32_t need_eq = kk - n_lt;
  for (int e = a0; e < a1; ++e) {
    if (kk > 0 && keys[e] == thr) {
      if (r < need_eq) sel[n_lt + r] = ((uint64_t)thr << 32) | (uint32_t)e;
      ++r;
    }
  }
  __syncthreads();
}

}  // namespace hf
