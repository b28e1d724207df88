/*
 * Hilbert-forest ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously correct CPU implementation of what the Hilbert
 * forest computes (Imamura et al., "Hilbert Forest in the SISAP 2025 Indexing
 * Challenge", arXiv 2508.21682).  Only the tests, the package smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code with the
 * HIP library: keys are computed in full (all d*B bits) by Skilling's
 * transform, sorts use qsort on full keys, node tests are found by toggling
 * bits, sets are formed with marker arrays, scores are FP64.
 *
 * Parity status of each function is given in its header comment.  All
 * readings of places where the paper is silent are the ones the library
 * documents (power-of-two 8-bit quantiser, SplitMix64 curve seeds, axis
 * permutation + reflection, leaf midpoint window, set semantics for C1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HFO_SKETCH_WORDS 8 /* 512-bit sketches */

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number     */
/* generators", OOPSLA 2014): add the golden-gamma constant, then mix.       */
/* Pinned by the published first outputs for seed 0 (tests).                 */
/* ------------------------------------------------------------------------ */
static uint64_t sm64_next(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t hfo_splitmix64(uint64_t seed, int64_t index) {
  uint64_t s = seed, z = 0;
  for (int64_t i = 0; i <= index; ++i) z = sm64_next(&s);
  return z;
}

/* ------------------------------------------------------------------------ */
/* Curves, one per tree (Alg. 1 and Alg. 2: a random axis order per tree or */
/* order).  One SplitMix64 stream seeded with `seed` is                      */
/* consumed tree after tree: first a Fisher-Yates shuffle of the identity    */
/* (for i = d-1 down to 1: j = next mod (i+1), swap), then ceil(d/64) words  */
/* whose bits (LSB first) say which tree axes are reflected (x -> 255 - x).  */
/* Pinned: permutation property + published SplitMix64 outputs.             */
/* ------------------------------------------------------------------------ */
void hfo_curves(uint64_t seed, int32_t T, int32_t d, int32_t *perm, uint8_t *refl) {
  uint64_t s = seed;
  for (int32_t t = 0; t < T; ++t) {
    int32_t *p = perm + (int64_t)t * d;
    for (int32_t i = 0; i < d; ++i) p[i] = i;
    for (int32_t i = d - 1; i >= 1; --i) {
      uint64_t j = sm64_next(&s) % (uint64_t)(i + 1);
      int32_t tmp = p[i];
      p[i] = p[j];
      p[j] = tmp;
    }
    for (int32_t w = 0; w < (d + 63) / 64; ++w) {
      uint64_t bits = sm64_next(&s);
      for (int32_t b = 0; b < 64 && w * 64 + b < d; ++b)
        refl[(int64_t)t * d + w * 64 + b] = (uint8_t)((bits >> b) & 1u);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Stored values.  dtype 0 = IEEE binary16, 1 = binary32; both are exact in  */
/* binary64.  Pinned against numpy's float16 conversion for all 65536 codes. */
/* ------------------------------------------------------------------------ */
double hfo_f16_to_f64(uint16_t h) {
  int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
  double v;
  if (e == 0)
    v = ldexp((double)m, -24);
  else if (e == 31)
    v = m ? NAN : INFINITY;
  else
    v = ldexp((double)(m + 1024), e - 25);
  return s ? -v : v;
}

static double val(const void *x, int32_t dtype, int64_t i) {
  if (dtype == 0) return hfo_f16_to_f64(((const uint16_t *)x)[i]);
  return (double)((const float *)x)[i];
}

/* ------------------------------------------------------------------------ */
/* 8-bit ordering codes (the quantization step of Alg. 1 / Alg. 2; the paper */
/* gives no codec for the ordering, so one power-of-two scale is used):      */
/*   e = largest integer in [-8, 24] with 2^e*max < 128 and 2^e*min >= -128  */
/*       over the data (-8 if none);  u = clamp(floor(x*2^e) + 128, 0, 255). */
/* Returns INT32_MIN if any value is not finite.                             */
/* Pinned: exact by construction (power-of-two scale, floor); tests check    */
/* the defining inequalities and hand-computed codes.                        */
/* ------------------------------------------------------------------------ */
int32_t hfo_quant_exp(const void *x, int32_t dtype, int64_t n) {
  double mx = -INFINITY, mn = INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    double v = val(x, dtype, i);
    if (!isfinite(v)) return INT32_MIN;
    if (v > mx) mx = v;
    if (v < mn) mn = v;
  }
  if (n == 0) return 24;
  for (int32_t e = 24; e >= -8; --e)
    if (ldexp(mx, e) < 128.0 && ldexp(mn, e) >= -128.0) return e;
  return -8;
}

void hfo_quantize(const void *x, int32_t dtype, int64_t n, int32_t e, uint8_t *out) {
  for (int64_t i = 0; i < n; ++i) {
    double f = floor(ldexp(val(x, dtype, i), e)) + 128.0;
    out[i] = (uint8_t)(f < 0.0 ? 0.0 : (f > 255.0 ? 255.0 : f));
  }
}

/* ------------------------------------------------------------------------ */
/* Hilbert index by Skilling's transform (J. Skilling, "Programming the      */
/* Hilbert curve", AIP Conf. Proc. 707, 2004), restated:                     */
/*  1. for levels L = B-1 down to 1 (mask P = 2^L - 1), for axes i = 0..d-1: */
/*     if bit L of X[i] is set, invert the low bits of X[0] (X[0] ^= P),     */
/*     otherwise exchange the low bits of X[0] and X[i];                     */
/*  2. Gray-encode: X[i] ^= X[i-1] for i = 1..d-1, then XOR every axis with  */
/*     t = XOR of (2^L - 1) over the levels L >= 1 where X[d-1] has bit L;   */
/*  3. read the bits level-major, MSB first: key bit (B-1-L)*d + j is bit L  */
/*     of X[j].  Words hold 64 key bits each, key bit 0 in the word's MSB.   */
/* The Hilbert sort (Section 2) orders points by this index.                 */
/* Pinned: bijection, unit steps, sub-cube contiguity and origin start for   */
/* small (d, B); B = 1 is the Gray code; d = 1 is the identity; the 2-D      */
/* order-2 curve against a hand-drawn table.                                 */
/* ------------------------------------------------------------------------ */
void hfo_key(const uint8_t *v, int32_t d, int32_t B, uint64_t *key) {
  uint8_t *X = (uint8_t *)malloc((size_t)d);
  memcpy(X, v, (size_t)d);
  for (int32_t L = B - 1; L >= 1; --L) {
    uint8_t Q = (uint8_t)(1u << L), P = (uint8_t)(Q - 1u);
    for (int32_t i = 0; i < d; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        uint8_t t = (uint8_t)((X[0] ^ X[i]) & P);
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  for (int32_t i = 1; i < d; ++i) X[i] ^= X[i - 1];
  uint8_t t = 0;
  for (int32_t L = B - 1; L >= 1; --L)
    if (X[d - 1] & (1u << L)) t ^= (uint8_t)((1u << L) - 1u);
  for (int32_t i = 0; i < d; ++i) X[i] ^= t;
  int64_t words = ((int64_t)d * B + 63) / 64;
  memset(key, 0, (size_t)words * 8);
  for (int32_t L = B - 1; L >= 0; --L)
    for (int32_t j = 0; j < d; ++j) {
      int64_t b = (int64_t)(B - 1 - L) * d + j;
      if ((X[j] >> L) & 1u) key[b >> 6] |= 1ull << (63 - (b & 63));
    }
  free(X);
}

/* Tree coordinates: v[i] = u[perm[i]] XOR (255 * refl[i]). */
static void tree_coords(const uint8_t *u, int32_t d, const int32_t *perm, const uint8_t *refl,
                        uint8_t *v) {
  for (int32_t i = 0; i < d; ++i) v[i] = (uint8_t)(u[perm[i]] ^ (refl[i] ? 0xFFu : 0u));
}

void hfo_tree_keys(const uint8_t *codes, int64_t N, int32_t d, const int32_t *perm,
                   const uint8_t *refl, uint64_t *keys) {
  int64_t W = ((int64_t)d * 8 + 63) / 64;
#pragma omp parallel
  {
    uint8_t *v = (uint8_t *)malloc((size_t)d);
#pragma omp for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
      tree_coords(codes + p * d, d, perm, refl, v);
      hfo_key(v, d, 8, keys + p * W);
    }
    free(v);
  }
}

/* ------------------------------------------------------------------------ */
/* Hilbert sort (Section 2): order = argsort by (key, id), keys compared as  */
/* bit strings.  Pinned: output is a permutation with non-decreasing keys    */
/* and ids increasing among equal keys (checked independently in tests).     */
/* ------------------------------------------------------------------------ */
static const uint64_t *g_sort_keys;
static int64_t g_sort_words;

static int cmp_key_id(const void *a, const void *b) {
  uint32_t ia = *(const uint32_t *)a, ib = *(const uint32_t *)b;
  const uint64_t *ka = g_sort_keys + (int64_t)ia * g_sort_words;
  const uint64_t *kb = g_sort_keys + (int64_t)ib * g_sort_words;
  for (int64_t w = 0; w < g_sort_words; ++w)
    if (ka[w] != kb[w]) return ka[w] < kb[w] ? -1 : 1;
  return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

void hfo_sort(const uint64_t *keys, int64_t N, int32_t W, uint32_t *order) {
  for (int64_t i = 0; i < N; ++i) order[i] = (uint32_t)i;
  g_sort_keys = keys;
  g_sort_words = W;
  qsort(order, (size_t)N, sizeof(uint32_t), cmp_key_id);
}

/* ------------------------------------------------------------------------ */
/* Leaf-compressed Hilbert tree (Section 2 "Hilbert tree"; Section 3.1 leaf  */
/* compression of subtrees of about M points).  Read as a binary trie over   */
/* the sorted keys:                                                          */
/*   [lo,hi) is a leaf if hi-lo <= M or all its keys are equal; otherwise    */
/*   b = first bit where the keys of order[lo] and order[hi-1] differ,       */
/*   m = first index in [lo,hi) whose key has bit b set, children [lo,m),    */
/*   [m,hi).  The node test (a, L, flip) says: key bit b of any point in the */
/*   range equals bit L of its code on data axis a, XOR flip.  It is found   */
/*   by brute force: the unique tree axis j such that toggling bit L of      */
/*   v[order[lo]][j] keeps key bits < b and flips bit b; a = perm[j].        */
/* Layout: pre-order, left subtree first; two u32 words per node:            */
/*   internal: w0 = index of the right child, w1 = a | L<<16 | flip<<19;     */
/*   leaf:     w0 = lo,                       w1 = 1<<31 | (hi-lo).          */
/* aux (nullable), two words per node: internal {m, b}, leaf {lo, ~0}.      */
/* Returns the node count, or -1 if `cap` is too small, -2 if a node test is */
/* not unique (cannot happen for Skilling keys; kept as an assertion).       */
/* Pinned by invariants in tests (ranges partition [0,N), split bits, every  */
/* data point descends to the leaf holding it, test valid at both ends).     */
/* ------------------------------------------------------------------------ */
typedef struct {
  const uint64_t *keys;
  const uint32_t *order;
  int64_t W;
  int32_t d, M;
  uint32_t *nodes, *aux;
  int64_t cap, count;
  int64_t *pending; /* node index -> (lo, b) for internal nodes, to fill tests later */
  int64_t *pend_lo, *pend_b;
  int64_t npend;
} trie_ctx;

static int keybit(const uint64_t *k, int64_t b) { return (int)((k[b >> 6] >> (63 - (b & 63))) & 1u); }

static int64_t first_diff(const uint64_t *a, const uint64_t *b, int64_t W) {
  for (int64_t w = 0; w < W; ++w)
    if (a[w] != b[w]) {
      uint64_t x = a[w] ^ b[w];
      int64_t z = 0;
      while (!((x >> (63 - z)) & 1u)) ++z;
      return w * 64 + z;
    }
  return -1;
}

static int64_t trie_rec(trie_ctx *c, int64_t lo, int64_t hi) {
  int64_t me = c->count++;
  if (me >= c->cap) return -1;
  const uint64_t *klo = c->keys + (int64_t)c->order[lo] * c->W;
  const uint64_t *khi = c->keys + (int64_t)c->order[hi - 1] * c->W;
  int64_t b = (hi - lo <= c->M) ? -1 : first_diff(klo, khi, c->W);
  if (b < 0) {
    c->nodes[2 * me] = (uint32_t)lo;
    c->nodes[2 * me + 1] = 0x80000000u | (uint32_t)(hi - lo);
    if (c->aux) {
      c->aux[2 * me] = (uint32_t)lo;
      c->aux[2 * me + 1] = 0xFFFFFFFFu;
    }
    return 0;
  }
  int64_t m = lo;
  while (!keybit(c->keys + (int64_t)c->order[m] * c->W, b)) ++m;
  if (c->aux) {
    c->aux[2 * me] = (uint32_t)m;
    c->aux[2 * me + 1] = (uint32_t)b;
  }
  c->pending[c->npend] = me;
  c->pend_lo[c->npend] = lo;
  c->pend_b[c->npend] = b;
  c->npend++;
  if (trie_rec(c, lo, m) < 0) return -1;
  c->nodes[2 * me] = (uint32_t)c->count; /* right child comes next in pre-order */
  return trie_rec(c, m, hi);
}

int64_t hfo_trie(const uint64_t *keys, const uint32_t *order, int64_t N, int32_t d, int32_t M,
                 const uint8_t *codes, const int32_t *perm, const uint8_t *refl, uint32_t *nodes,
                 int64_t cap, uint32_t *aux) {
  trie_ctx c;
  c.keys = keys;
  c.order = order;
  c.W = ((int64_t)d * 8 + 63) / 64;
  c.d = d;
  c.M = M;
  c.nodes = nodes;
  c.aux = aux;
  c.cap = cap;
  c.count = 0;
  c.npend = 0;
  c.pending = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap + 1));
  c.pend_lo = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap + 1));
  c.pend_b = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap + 1));
  int64_t rc = trie_rec(&c, 0, N);
  int bad = 0;
  if (rc >= 0) {
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (int64_t q = 0; q < c.npend; ++q) {
      int64_t me = c.pending[q], b = c.pend_b[q];
      uint32_t p = order[c.pend_lo[q]];
      int32_t L = 7 - (int32_t)(b / d);
      uint8_t *v = (uint8_t *)malloc((size_t)d);
      uint64_t *k0 = (uint64_t *)malloc((size_t)c.W * 8);
      uint64_t *k1 = (uint64_t *)malloc((size_t)c.W * 8);
      tree_coords(codes + (int64_t)p * d, d, perm, refl, v);
      hfo_key(v, d, 8, k0);
      int found = -1, nfound = 0;
      for (int32_t j = 0; j < d; ++j) {
        v[j] ^= (uint8_t)(1u << L);
        hfo_key(v, d, 8, k1);
        v[j] ^= (uint8_t)(1u << L);
        int64_t f = first_diff(k0, k1, c.W);
        if (f == b) {
          found = j;
          ++nfound;
        }
      }
      if (nfound != 1) {
        bad = 1;
      } else {
        int32_t a = perm[found];
        int flip = keybit(k0, b) ^ ((codes[(int64_t)p * d + a] >> L) & 1);
        nodes[2 * me + 1] = (uint32_t)a | ((uint32_t)L << 16) | ((uint32_t)flip << 19);
      }
      free(v);
      free(k0);
      free(k1);
    }
  }
  free(c.pending);
  free(c.pend_lo);
  free(c.pend_b);
  if (rc < 0) return -1;
  if (bad) return -2;
  return c.count;
}

/* ------------------------------------------------------------------------ */
/* Collective descent (Section 3.1: all queries located along each tree's    */
/* curve at once; Alg. 1 first stage).  From the root, bit = ((u_q[a] >> L) & 1)  */
/* ^ flip; 0 goes left (next node), 1 goes right.  At the leaf [lo,hi) the   */
/* query's position is read as the leaf midpoint and the k1 candidates as    */
/* the centred window: s = clamp(floor((lo+hi)/2) - floor(k1/2), 0,          */
/* max(0, N-k1)).  Pinned: every data point descends to its own leaf (test). */
/* ------------------------------------------------------------------------ */
void hfo_window_starts(const uint32_t *nodes, const uint8_t *qcodes, int64_t nq, int32_t d,
                       int64_t N, int32_t k1, uint32_t *out, int64_t out_stride) {
  for (int64_t q = 0; q < nq; ++q) {
    const uint8_t *u = qcodes + q * d;
    int64_t idx = 0;
    for (;;) {
      uint32_t w0 = nodes[2 * idx], w1 = nodes[2 * idx + 1];
      if (w1 >> 31) {
        int64_t mid = (int64_t)w0 + (int64_t)((w1 & 0x7FFFFFFFu) >> 1);
        int64_t s = mid - k1 / 2, smax = N - k1 > 0 ? N - k1 : 0;
        if (s < 0) s = 0;
        if (s > smax) s = smax;
        out[q * out_stride] = (uint32_t)s;
        break;
      }
      uint32_t a = w1 & 0xFFFFu, L = (w1 >> 16) & 7u, flip = (w1 >> 19) & 1u;
      uint32_t bit = ((u[a] >> L) & 1u) ^ flip;
      idx = bit ? (int64_t)w0 : idx + 1;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Exact position of a query along a tree's curve (Section 2: a point's      */
/* place in Hilbert order can be found in O(log n); Alg. 1 first stage takes */
/* the k1 candidates around it).  Read as the insertion rank of the query's  */
/* key among the tree's sorted keys, before any equal key: rank = number of  */
/* data points whose key is strictly smaller.  Found by binary search over   */
/* the sorted order with full keys of both sides.  Window start              */
/* s = clamp(rank - floor(k1/2), 0, max(0, N-k1)).                            */
/* keys: N x W keys of the tree's curve indexed by point id; order: the      */
/* tree's sorted ids.  Pinned: rank equals the count of smaller keys by      */
/* brute force, and a data point with a unique key ranks at its own place.   */
/* ------------------------------------------------------------------------ */
static int key_cmp(const uint64_t *a, const uint64_t *b, int64_t W) {
  for (int64_t w = 0; w < W; ++w)
    if (a[w] != b[w]) return a[w] < b[w] ? -1 : 1;
  return 0;
}

void hfo_exact_ranks(const uint64_t *keys, const uint32_t *order, int64_t N, int32_t d, const uint8_t *qcodes,
                     int64_t nq, const int32_t *perm, const uint8_t *refl, int32_t k1, uint32_t *rank_out,
                     uint32_t *start_out) {
  const int64_t W = ((int64_t)d * 8 + 63) / 64;
#pragma omp parallel
  {
    uint8_t *v = (uint8_t *)malloc((size_t)d);
    uint64_t *kq = (uint64_t *)malloc((size_t)W * 8);
#pragma omp for schedule(static)
    for (int64_t q = 0; q < nq; ++q) {
      tree_coords(qcodes + q * d, d, perm, refl, v);
      hfo_key(v, d, 8, kq);
      int64_t lo = 0, hi = N; /* first index whose key is >= the query's */
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (key_cmp(keys + (int64_t)order[mid] * W, kq, W) < 0)
          lo = mid + 1;
        else
          hi = mid;
      }
      int64_t s = lo - k1 / 2, smax = N - k1 > 0 ? N - k1 : 0;
      if (s < 0) s = 0;
      if (s > smax) s = smax;
      if (rank_out) rank_out[q] = (uint32_t)lo;
      if (start_out) start_out[q] = (uint32_t)s;
    }
    free(v);
    free(kq);
  }
}

/* ------------------------------------------------------------------------ */
/* 512-bit sign-of-random-projection sketches (Section 3.1 uses binary       */
/* sketches compared by Hamming distance; their construction is not given). */
/* R[j][i] in {-1,+1} is bit (j*d + i) of the concatenated SplitMix64        */
/* outputs seeded with `sketch_seed` (LSB first, 1 -> +1);                   */
/* xq_i = clamp(rne(x_i * 2^(e+5)), -8191, 8191) with e the data's code      */
/* exponent; z_j = sum_i R[j][i]*xq_i (exact integer); sketch bit j =        */
/* [z_j >= 0], stored in word j/64 at bit j%64.                              */
/* Pinned: sign symmetry sketch(-x) = ~sketch(x) where no z_j is 0, the     */
/* integer sum against an independent numpy matmul (tests).                  */
/* ------------------------------------------------------------------------ */
void hfo_srp(const void *x, int32_t dtype, int64_t N, int32_t d, int32_t e, uint64_t sketch_seed,
             uint64_t *out) {
  int64_t nbits = 512LL * d, nw = (nbits + 63) / 64;
  uint64_t *R = (uint64_t *)malloc((size_t)nw * 8);
  uint64_t s = sketch_seed;
  for (int64_t w = 0; w < nw; ++w) R[w] = sm64_next(&s);
#pragma omp parallel
  {
    int64_t *xq = (int64_t *)malloc(sizeof(int64_t) * (size_t)d);
#pragma omp for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
      for (int32_t i = 0; i < d; ++i) {
        double r = nearbyint(ldexp(val(x, dtype, p * d + i), e + 5));
        if (r > 8191.0) r = 8191.0;
        if (r < -8191.0) r = -8191.0;
        xq[i] = (int64_t)r;
      }
      uint64_t *o = out + p * HFO_SKETCH_WORDS;
      memset(o, 0, HFO_SKETCH_WORDS * 8);
      for (int32_t j = 0; j < 512; ++j) {
        int64_t z = 0;
        for (int32_t i = 0; i < d; ++i) {
          int64_t b = (int64_t)j * d + i;
          z += ((R[b >> 6] >> (b & 63)) & 1u) ? xq[i] : -xq[i];
        }
        if (z >= 0) o[j >> 6] |= 1ull << (j & 63);
      }
    }
    free(xq);
  }
  free(R);
}

static int hamming(const uint64_t *a, const uint64_t *b) {
  int h = 0;
  for (int w = 0; w < HFO_SKETCH_WORDS; ++w) h += __builtin_popcountll(a[w] ^ b[w]);
  return h;
}

/* ------------------------------------------------------------------------ */
/* Second stage and final selection of Alg. 1, one query at a time:          */
/*   C1 = union over trees of tree_perm[t][s .. s+k1) (a set of master       */
/*        positions; the paper's count n*k1 includes duplicates);            */
/*   C2 = first min(k2, |C1|) of C1 ordered by (Hamming(sk_q, sk_r), r);     */
/*   E  = union over r in C2 of [max(0, r-h), min(N-1, r+h)] (master order); */
/*   S  = top-k of E by (inner product desc, r asc) in FP64, mapped to ids.  */
/* x_pos(r) = X[pos2id[r]].  Pinned: T=1, k1>=N, k2>=N, h=0 reduces to the   */
/* exact brute-force k-NN (tests); C1/C2/E by set algebra on tiny inputs.    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t key;
  int64_t r;
  double s;
} cand;

static int cmp_ham_pos(const void *a, const void *b) {
  const cand *x = (const cand *)a, *y = (const cand *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->r < y->r ? -1 : (x->r > y->r ? 1 : 0);
}

static int cmp_score_desc_pos(const void *a, const void *b) {
  const cand *x = (const cand *)a, *y = (const cand *)b;
  if (x->s != y->s) return x->s > y->s ? -1 : 1;
  return x->r < y->r ? -1 : (x->r > y->r ? 1 : 0);
}

void hfo_search_stage2(const void *X, int32_t dtype, int64_t N, int32_t d, const uint32_t *pos2id,
                       const uint32_t *tree_perm, int32_t T, const uint32_t *winstart,
                       const uint64_t *sk_pos, const void *Q, const uint64_t *qsk, int64_t nq,
                       int32_t k1, int32_t k2, int32_t h, int32_t k, int32_t *ids, double *scores,
                       uint32_t *c2, int32_t *c2n, int32_t *c1n, int32_t *en) {
  int64_t len = k1 < N ? k1 : N;
#pragma omp parallel
  {
    uint8_t *mark = (uint8_t *)calloc((size_t)N, 1);
    cand *buf = (cand *)malloc(sizeof(cand) * (size_t)(T * len + (int64_t)k2 * (2 * h + 1) + 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
      const uint64_t *sq = qsk + q * HFO_SKETCH_WORDS;
      int64_t n1 = 0;
      for (int32_t t = 0; t < T; ++t) {
        const uint32_t *P = tree_perm + (int64_t)t * N;
        int64_t s = winstart[q * T + t];
        for (int64_t i = s; i < s + len; ++i) {
          uint32_t r = P[i];
          if (!mark[r]) {
            mark[r] = 1;
            buf[n1].r = r;
            buf[n1].key = hamming(sq, sk_pos + (int64_t)r * HFO_SKETCH_WORDS);
            ++n1;
          }
        }
      }
      for (int64_t i = 0; i < n1; ++i) mark[buf[i].r] = 0;
      qsort(buf, (size_t)n1, sizeof(cand), cmp_ham_pos);
      int64_t n2 = n1 < k2 ? n1 : k2;
      if (c2)
        for (int64_t i = 0; i < k2; ++i) c2[q * k2 + i] = i < n2 ? (uint32_t)buf[i].r : 0xFFFFFFFFu;
      if (c2n) c2n[q] = (int32_t)n2;
      if (c1n) c1n[q] = (int32_t)n1;
      /* expansion in master order */
      cand *E = buf + n2;
      int64_t ne = 0;
      for (int64_t i = 0; i < n2; ++i) {
        int64_t r = buf[i].r, a = r - h < 0 ? 0 : r - h, z = r + h > N - 1 ? N - 1 : r + h;
        for (int64_t x = a; x <= z; ++x)
          if (!mark[x]) {
            mark[x] = 1;
            E[ne].r = x;
            ++ne;
          }
      }
      for (int64_t i = 0; i < ne; ++i) mark[E[i].r] = 0;
      if (en) en[q] = (int32_t)ne;
      for (int64_t i = 0; i < ne; ++i) {
        int64_t row = (int64_t)pos2id[E[i].r];
        double acc = 0.0;
        for (int32_t j = 0; j < d; ++j) acc += val(Q, dtype, q * d + j) * val(X, dtype, row * d + j);
        E[i].s = acc;
      }
      qsort(E, (size_t)ne, sizeof(cand), cmp_score_desc_pos);
      for (int32_t i = 0; i < k; ++i) {
        ids[q * k + i] = i < ne ? (int32_t)pos2id[E[i].r] : -1;
        scores[q * k + i] = i < ne ? E[i].s : -INFINITY;
      }
    }
    free(mark);
    free(buf);
  }
}

/* ------------------------------------------------------------------------ */
/* The paper's compressed layout (Section 3.1): 384-bit sketches for 384-d   */
/* data and 4-bit vector codes that share one bit with the sketch, the rerank */
/* computed from the codes with the query left unquantized.  Read as:        */
/*  sketch bit i = [x_i >= 0] (one bit per coordinate, stored in word i/64   */
/*    at bit i%64, d bits; the Hamming filter compares these);               */
/*  code i = that sign bit plus a 3-bit magnitude m_i = the number of        */
/*    k in 1..7 with 8|x_i| >= k * max_j |x_j| (uniform levels of width      */
/*    s = max|x| / 8 per vector; m = 7 for the largest element);             */
/*  value of code i = (+-1) * (m_i + 1/2) * s, the sign from the sketch bit. */
/* A zero vector has s = 0 and every value 0.                                */
/* Pinned: m against exact rational arithmetic, reconstruction within s/2,  */
/* sign sketches against Python bit packing (tests).                         */
/* ------------------------------------------------------------------------ */
void hfo_c4_encode(const void *x, int32_t dtype, int64_t N, int32_t d, uint64_t *sign_out, uint8_t *mag_out,
                   double *scale_out) {
  const int64_t W = (d + 63) / 64;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < N; ++p) {
    double mx = 0.0;
    for (int32_t i = 0; i < d; ++i) {
      double a = fabs(val(x, dtype, p * d + i));
      if (a > mx) mx = a;
    }
    scale_out[p] = mx / 8.0;
    uint64_t *sg = sign_out + p * W;
    for (int64_t w = 0; w < W; ++w) sg[w] = 0;
    for (int32_t i = 0; i < d; ++i) {
      double v = val(x, dtype, p * d + i);
      if (v >= 0.0) sg[i >> 6] |= 1ull << (i & 63);
      int m = 0;
      for (int k = 1; k <= 7; ++k)
        if (8.0 * fabs(v) >= (double)k * mx) m = k;
      mag_out[p * d + i] = (uint8_t)m;
    }
  }
}

/* Value of code i of row p (see above). */
static double c4_value(const uint64_t *sign, const uint8_t *mag, const double *scale, int64_t p, int32_t d,
                       int32_t i) {
  const int64_t W = (d + 63) / 64;
  double v = ((double)mag[p * d + i] + 0.5) * scale[p];
  return ((sign[p * W + (i >> 6)] >> (i & 63)) & 1u) ? v : -v;
}

/* Alg. 1 stages two and three in the compressed layout, one query at a     */
/* time: C1 as in hfo_search_stage2; C2 = the first k2 of C1 by (Hamming     */
/* distance of the d-bit sign sketches, position); E = C2 expanded by h;     */
/* S = top-k of E by (sum_i q_i * code value_i desc, position asc), with the  */
/* stored query values.  Rows indexed by master position.                    */
void hfo_search_c4(int64_t N, int32_t d, const uint32_t *pos2id, const uint32_t *tree_perm, int32_t T,
                   const uint32_t *winstart, const uint64_t *sign_pos, const uint8_t *mag_pos,
                   const double *scale_pos, const void *Q, int32_t qdtype, int64_t nq, int32_t k1, int32_t k2,
                   int32_t h, int32_t k, int32_t *ids, double *scores, uint32_t *c2, int32_t *c2n, int32_t *en) {
  const int64_t W = (d + 63) / 64;
  int64_t len = k1 < N ? k1 : N;
#pragma omp parallel
  {
    uint8_t *mark = (uint8_t *)calloc((size_t)N, 1);
    cand *buf = (cand *)malloc(sizeof(cand) * (size_t)(T * len + (int64_t)k2 * (2 * h + 1) + 1));
    uint64_t *qs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)W);
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
      for (int64_t w = 0; w < W; ++w) qs[w] = 0;
      for (int32_t i = 0; i < d; ++i)
        if (val(Q, qdtype, q * d + i) >= 0.0) qs[i >> 6] |= 1ull << (i & 63);
      int64_t n1 = 0;
      for (int32_t t = 0; t < T; ++t) {
        const uint32_t *P = tree_perm + (int64_t)t * N;
        int64_t s = winstart[q * T + t];
        for (int64_t i = s; i < s + len; ++i) {
          uint32_t r = P[i];
          if (!mark[r]) {
            mark[r] = 1;
            int hd = 0;
            for (int64_t w = 0; w < W; ++w) hd += __builtin_popcountll(qs[w] ^ sign_pos[(int64_t)r * W + w]);
            buf[n1].r = r;
            buf[n1].key = hd;
            ++n1;
          }
        }
      }
      for (int64_t i = 0; i < n1; ++i) mark[buf[i].r] = 0;
      qsort(buf, (size_t)n1, sizeof(cand), cmp_ham_pos);
      int64_t n2 = n1 < k2 ? n1 : k2;
      if (c2)
        for (int64_t i = 0; i < k2; ++i) c2[q * k2 + i] = i < n2 ? (uint32_t)buf[i].r : 0xFFFFFFFFu;
      if (c2n) c2n[q] = (int32_t)n2;
      cand *E = buf + n2;
      int64_t ne = 0;
      for (int64_t i = 0; i < n2; ++i) {
        int64_t r = buf[i].r, a = r - h < 0 ? 0 : r - h, z = r + h > N - 1 ? N - 1 : r + h;
        for (int64_t x = a; x <= z; ++x)
          if (!mark[x]) {
            mark[x] = 1;
            E[ne].r = x;
            ++ne;
          }
      }
      for (int64_t i = 0; i < ne; ++i) mark[E[i].r] = 0;
      if (en) en[q] = (int32_t)ne;
      for (int64_t i = 0; i < ne; ++i) {
        double acc = 0.0;
        for (int32_t j = 0; j < d; ++j)
          acc += val(Q, qdtype, q * d + j) * c4_value(sign_pos, mag_pos, scale_pos, E[i].r, d, j);
        E[i].s = acc;
      }
      qsort(E, (size_t)ne, sizeof(cand), cmp_score_desc_pos);
      for (int32_t i = 0; i < k; ++i) {
        ids[q * k + i] = i < ne ? (int32_t)pos2id[E[i].r] : -1;
        scores[q * k + i] = i < ne ? E[i].s : -INFINITY;
      }
    }
    free(mark);
    free(buf);
    free(qs);
  }
}

/* ------------------------------------------------------------------------ */
/* Precision form emulation (not in the paper).                              */
/*  bf16: x rounded to 8 significant bits, nearest, ties to even.            */
/*  fp8 (OCP e4m3): value of code c = sign * (m/8) * 2^-6 for exponent field */
/*  0, (1 + m/8) * 2^(E-7) otherwise; 0x7F is NaN and never produced.  A      */
/*  value is encoded as the finite code nearest to it (ties: even code),     */
/*  saturating at 448.  Per-vector scale s = max|x| / 448 in binary32 (1 for */
/*  a zero vector), codes of x / s computed in binary32.                     */
/* Pinned: every code round-trips, encoding of midpoints goes to even codes, */
/* the largest value is 448 and the smallest subnormal 2^-9 (tests).        */
/* ------------------------------------------------------------------------ */
double hfo_bf16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  double f = frexp(x, &e); /* |f| in [0.5, 1) */
  return ldexp(nearbyint(f * 256.0), e - 8);
}

double hfo_e4m3_decode(uint8_t c) {
  int sign = c >> 7, E = (c >> 3) & 15, m = c & 7;
  double v;
  if ((c & 0x7F) == 0x7F) return NAN;
  if (E == 0)
    v = ldexp((double)m, -9);
  else
    v = ldexp(1.0 + m / 8.0, E - 7);
  return sign ? -v : v;
}

uint8_t hfo_e4m3_encode(float y) {
  uint8_t sign = signbit(y) ? 0x80 : 0;
  double a = fabs((double)y);
  int best = 0;
  double berr = INFINITY;
  for (int c = 0; c <= 0x7E; ++c) {
    double err = fabs(hfo_e4m3_decode((uint8_t)c) - a);
    if (err < berr || (err == berr && (c & 1) == 0)) {
      berr = err;
      best = c;
    }
  }
  if (a >= 448.0) best = 0x7E;
  return (uint8_t)(sign | best);
}

float hfo_fp8_scale(const void *x, int32_t dtype, int64_t row, int32_t d) {
  float m = 0.0f;
  for (int32_t i = 0; i < d; ++i) {
    float v = (float)fabs(val(x, dtype, row * d + i));
    if (v > m) m = v;
  }
  return m > 0.0f ? m / 448.0f : 1.0f;
}

/* Emulated low-precision inner product of query row q and data row r. */
static double lowprec_dot(const void *Q, const void *X, int32_t dtype, int64_t q, int64_t r,
                          int32_t d, int32_t prec) {
  double acc = 0.0;
  if (prec == 1) {
    for (int32_t i = 0; i < d; ++i)
      acc += hfo_bf16(val(Q, dtype, q * d + i)) * hfo_bf16(val(X, dtype, r * d + i));
    return acc;
  }
  float sq = hfo_fp8_scale(Q, dtype, q, d), sx = hfo_fp8_scale(X, dtype, r, d);
  for (int32_t i = 0; i < d; ++i) {
    double a = hfo_e4m3_decode(hfo_e4m3_encode((float)val(Q, dtype, q * d + i) / sq));
    double b = hfo_e4m3_decode(hfo_e4m3_encode((float)val(X, dtype, r * d + i) / sx));
    acc += a * b;
  }
  return (double)sq * (double)sx * acc;
}

/* Final selection of the precision form for one query: E scored in the     */
/* emulated precision, the first S by (score desc, position asc) survive,   */
/* then FP64 scores of the survivors give the top-k (score desc, pos asc).   */
void hfo_search_lowprec(const void *X, int32_t dtype, int64_t N, int32_t d, const uint32_t *pos2id,
                        const uint32_t *c2, const int32_t *c2n, int32_t k2, const void *Q, int64_t nq,
                        int32_t h, int32_t k, int32_t prec, int32_t S, int32_t *ids, double *scores,
                        uint32_t *surv_pos, double *surv_score) {
#pragma omp parallel
  {
    uint8_t *mark = (uint8_t *)calloc((size_t)N, 1);
    cand *E = (cand *)malloc(sizeof(cand) * (size_t)((int64_t)k2 * (2 * h + 1) + 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
      int64_t ne = 0;
      for (int32_t i = 0; i < c2n[q]; ++i) {
        int64_t r = c2[q * k2 + i], a = r - h < 0 ? 0 : r - h, z = r + h > N - 1 ? N - 1 : r + h;
        for (int64_t x = a; x <= z; ++x)
          if (!mark[x]) {
            mark[x] = 1;
            E[ne++].r = x;
          }
      }
      for (int64_t i = 0; i < ne; ++i) mark[E[i].r] = 0;
      for (int64_t i = 0; i < ne; ++i) E[i].s = lowprec_dot(Q, X, dtype, q, (int64_t)pos2id[E[i].r], d, prec);
      qsort(E, (size_t)ne, sizeof(cand), cmp_score_desc_pos);
      int64_t ns = ne < S ? ne : S;
      for (int32_t i = 0; i < S; ++i) {
        surv_pos[q * S + i] = i < ns ? (uint32_t)E[i].r : 0xFFFFFFFFu;
        surv_score[q * S + i] = i < ns ? E[i].s : -INFINITY;
      }
      for (int64_t i = 0; i < ns; ++i) {
        int64_t row = (int64_t)pos2id[E[i].r];
        double acc = 0.0;
        for (int32_t j = 0; j < d; ++j) acc += val(Q, dtype, q * d + j) * val(X, dtype, row * d + j);
        E[i].s = acc;
      }
      qsort(E, (size_t)ns, sizeof(cand), cmp_score_desc_pos);
      for (int32_t i = 0; i < k; ++i) {
        ids[q * k + i] = i < ns ? (int32_t)pos2id[E[i].r] : -1;
        scores[q * k + i] = i < ns ? E[i].s : -INFINITY;
      }
    }
    free(mark);
    free(E);
  }
}

/* ------------------------------------------------------------------------ */
/* Learned hash (not in the paper), FP64.                                    */
/*   z1 = W1 r(x) + b1, a = r(relu(z1)), z2 = W2 a + b2, bit j = [z2_j >= 0] */
/* with r() = bf16 rounding of inputs, weights and hidden activations when   */
/* `rounded` is set (the deployed network), identity otherwise.  W1 is      */
/* hidden x d, W2 is 512 x hidden, row-major.                                */
/* Training loss over B pairs (q_i, p_i), codes c = tanh(slope * z2):        */
/*   S_ij = <c(q_i), c(p_j)> / 512,                                          */
/*   L = (1/B) sum_i [ log sum_j exp(S_ij / tau) - S_ii / tau ]              */
/*       + lambda * sum_b m_b^2,  m_b = mean of c_b over all 2B codes.       */
/* Gradients by hand (chain rule, rounding treated as identity).             */
/* Pinned: central finite differences with rounded = 0 (tests).             */
/* ------------------------------------------------------------------------ */
static double rb(double x, int rounded) { return rounded ? hfo_bf16(x) : x; }

/* band_out (nullable): margin below which the sign of z2 may differ from an
 * FP32-accumulating implementation.  Sums of K products in FP32 differ from
 * the FP64 value by at most about (K/32 + 5) * 2^-24 * sum|terms|; 2^-16 *
 * sum|terms| bounds that for K <= 4096.  A hidden activation can then round to
 * a different bf16 value only if z1 lies within that bound of a rounding
 * boundary (or of 0, the relu kink); such activations may move by one bf16
 * step (or all of a), which moves z2_j by |W2[j][i]| times that. */
void hfo_mlp_forward(const void *x, int32_t dtype, int64_t n, int32_t d, int32_t hid,
                     const float *W1, const float *b1, const float *W2, const float *b2,
                     int32_t rounded, double *z1_out, double *a_out, double *z2_out,
                     double *band_out) {
#pragma omp parallel
  {
    double *move = (double *)malloc(sizeof(double) * hid);
#pragma omp for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
      double *z1 = z1_out + r * hid, *a = a_out + r * hid;
      for (int32_t j = 0; j < hid; ++j) {
        double acc = 0.0, mag = fabs((double)b1[j]);
        for (int32_t i = 0; i < d; ++i) {
          double t = rb(W1[(int64_t)j * d + i], rounded) * rb(val(x, dtype, r * d + i), rounded);
          acc += t;
          mag += fabs(t);
        }
        z1[j] = acc + b1[j];
        a[j] = rb(z1[j] > 0.0 ? z1[j] : 0.0, rounded);
        double delta = ldexp(mag, -16);
        move[j] = 0.0;
        if (fabs(z1[j]) <= delta) {
          move[j] = fabs(a[j]) + delta; /* relu kink: a may be 0 or a small value */
        } else if (z1[j] > 0.0 && rounded) {
          /* a in [2^(e-1), 2^e): bf16 values there are 2^(e-8) apart.  The
           * value below a is 2^(e-8) away too, except when a = 2^(e-1) is a
           * power of two, where the binade below has half that spacing. */
          int e;
          frexp(a[j], &e);
          double up = ldexp(1.0, e - 8);
          double down = a[j] == ldexp(1.0, e - 1) ? ldexp(1.0, e - 9) : up;
          double lo_mid = a[j] - down / 2, hi_mid = a[j] + up / 2;
          if (fabs(z1[j] - lo_mid) <= delta || fabs(z1[j] - hi_mid) <= delta) move[j] = up;
        }
      }
      for (int32_t j = 0; j < 512; ++j) {
        double acc = 0.0, mag = fabs((double)b2[j]), mv = 0.0;
        for (int32_t i = 0; i < hid; ++i) {
          double w = rb(W2[(int64_t)j * hid + i], rounded);
          acc += w * a[i];
          mag += fabs(w * a[i]);
          mv += fabs(w) * move[i];
        }
        z2_out[r * 512 + j] = acc + b2[j];
        if (band_out) band_out[r * 512 + j] = mv + ldexp(mag, -16);
      }
    }
    free(move);
  }
}

/* Loss and gradients with optional hard negatives Ng (nullable, B rows, one */
/* per query): the softmax of query i then runs over the B in-batch          */
/* positives and its own negative, H_i = <c(q_i), c(n_i)> / 512:             */
/*   L = (1/B) sum_i [ log( sum_j exp(S_ij/tau) + exp(H_i/tau) ) - S_ii/tau ] */
/*       + lambda * sum_b m_b^2, m = mean code over all rows (2B or 3B).     */
double hfo_lhash_grad(const void *A, const void *Bm, const void *Ng, int32_t dtype, int64_t B, int32_t d,
                      int32_t hid, const float *W1, const float *b1, const float *W2, const float *b2, double slope,
                      double tau, double lambda, int32_t rounded, double *gW1, double *gb1, double *gW2,
                      double *gb2) {
  const int64_t R = (Ng ? 3 : 2) * B; /* rows: the B queries, the B positives, the B negatives */
  double *z1 = (double *)malloc(sizeof(double) * R * hid);
  double *a = (double *)malloc(sizeof(double) * R * hid);
  double *z2 = (double *)malloc(sizeof(double) * R * 512);
  double *c = (double *)malloc(sizeof(double) * R * 512);
  double *dc = (double *)calloc((size_t)(R * 512), sizeof(double));
  double *S = (double *)malloc(sizeof(double) * B * (B + 1));
  double *m = (double *)calloc(512, sizeof(double));
  hfo_mlp_forward(A, dtype, B, d, hid, W1, b1, W2, b2, rounded, z1, a, z2, NULL);
  hfo_mlp_forward(Bm, dtype, B, d, hid, W1, b1, W2, b2, rounded, z1 + B * hid, a + B * hid, z2 + B * 512, NULL);
  if (Ng)
    hfo_mlp_forward(Ng, dtype, B, d, hid, W1, b1, W2, b2, rounded, z1 + 2 * B * hid, a + 2 * B * hid,
                    z2 + 2 * B * 512, NULL);
  for (int64_t i = 0; i < R * 512; ++i) c[i] = tanh(slope * z2[i]);
  /* logits of row i: columns j < B the positives, column B its negative */
  const int64_t nc = Ng ? B + 1 : B;
  for (int64_t i = 0; i < B; ++i)
    for (int64_t j = 0; j < nc; ++j) {
      const double *o = j < B ? c + (B + j) * 512 : c + (2 * B + i) * 512;
      double acc = 0.0;
      for (int32_t b = 0; b < 512; ++b) acc += c[i * 512 + b] * o[b];
      S[i * nc + j] = acc / 512.0;
    }
  double loss = 0.0;
  for (int64_t i = 0; i < B; ++i) {
    double mx = -INFINITY, sum = 0.0;
    for (int64_t j = 0; j < nc; ++j) mx = fmax(mx, S[i * nc + j] / tau);
    for (int64_t j = 0; j < nc; ++j) sum += exp(S[i * nc + j] / tau - mx);
    loss += (mx + log(sum) - S[i * nc + i] / tau) / (double)B;
    for (int64_t j = 0; j < nc; ++j) {
      double g = (exp(S[i * nc + j] / tau - mx) / sum - (i == j ? 1.0 : 0.0)) / (tau * (double)B);
      const int64_t orow = j < B ? B + j : 2 * B + i;
      for (int32_t b = 0; b < 512; ++b) {
        dc[i * 512 + b] += g * c[orow * 512 + b] / 512.0;
        dc[orow * 512 + b] += g * c[i * 512 + b] / 512.0;
      }
    }
  }
  for (int64_t r = 0; r < R; ++r)
    for (int32_t b = 0; b < 512; ++b) m[b] += c[r * 512 + b] / (double)R;
  for (int32_t b = 0; b < 512; ++b) loss += lambda * m[b] * m[b];
  for (int64_t r = 0; r < R; ++r)
    for (int32_t b = 0; b < 512; ++b) dc[r * 512 + b] += lambda * 2.0 * m[b] / (double)R;
  memset(gW1, 0, sizeof(double) * hid * d);
  memset(gb1, 0, sizeof(double) * hid);
  memset(gW2, 0, sizeof(double) * 512 * hid);
  memset(gb2, 0, sizeof(double) * 512);
  double *dz1 = (double *)malloc(sizeof(double) * hid);
  for (int64_t r = 0; r < R; ++r) {
    const void *src = r < B ? A : (r < 2 * B ? Bm : Ng);
    int64_t rr = r % B;
    for (int32_t i = 0; i < hid; ++i) dz1[i] = 0.0;
    for (int32_t j = 0; j < 512; ++j) {
      double cj = c[r * 512 + j];
      double dz2 = dc[r * 512 + j] * slope * (1.0 - cj * cj);
      gb2[j] += dz2;
      for (int32_t i = 0; i < hid; ++i) {
        gW2[(int64_t)j * hid + i] += dz2 * a[r * hid + i];
        dz1[i] += dz2 * rb(W2[(int64_t)j * hid + i], rounded);
      }
    }
    for (int32_t i = 0; i < hid; ++i) {
      double g = z1[r * hid + i] > 0.0 ? dz1[i] : 0.0;
      gb1[i] += g;
      for (int32_t k = 0; k < d; ++k) gW1[(int64_t)i * d + k] += g * rb(val(src, dtype, rr * d + k), rounded);
    }
  }
  free(dz1);
  free(z1);
  free(a);
  free(z2);
  free(c);
  free(dc);
  free(S);
  free(m);
  return loss;
}

/* ------------------------------------------------------------------------ */
/* k-NN graph rows (Alg. 2), for selected rows p only:                       */
/*   C1(p) = union over orders t of order_t[i-w .. i+w] without p, i being   */
/*           p's rank in order t (window clipped to the array);              */
/*   k2 > 0: C2(p) = first k2 of C1(p) by (Hamming, id); else C2 = C1;       */
/*   S(p)  = top-k of C2(p) by (cosine desc, id asc) in FP64.                */
/* c2_out (nullable, k2 > 0): C2(p) in (Hamming, id) order, -1 padded to k2. */
/* Pinned: w >= N reduces to the exact brute-force graph (tests).            */
/* ------------------------------------------------------------------------ */
static int cmp_key_r(const void *a, const void *b) { return cmp_ham_pos(a, b); }

void hfo_graph_rows(const void *X, int32_t dtype, int64_t N, int32_t d, const uint32_t *orders,
                    int32_t n, int32_t w, const int64_t *rows, int64_t nrows, int32_t k, int32_t k2,
                    const uint64_t *sk, int32_t *out_ids, double *out_scores, int32_t *c1n,
                    int32_t *c2_out) {
  uint32_t *rank = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N * n));
  for (int32_t t = 0; t < n; ++t)
    for (int64_t i = 0; i < N; ++i) rank[(int64_t)t * N + orders[(int64_t)t * N + i]] = (uint32_t)i;
  double *norm = (double *)malloc(sizeof(double) * (size_t)N);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < N; ++p) {
    double a = 0.0;
    for (int32_t j = 0; j < d; ++j) {
      double v = val(X, dtype, p * d + j);
      a += v * v;
    }
    norm[p] = sqrt(a);
  }
#pragma omp parallel
  {
    uint8_t *mark = (uint8_t *)calloc((size_t)N, 1);
    cand *buf = (cand *)malloc(sizeof(cand) * (size_t)((int64_t)n * (2 * w + 1) + 1));
#pragma omp for schedule(dynamic, 4)
    for (int64_t ri = 0; ri < nrows; ++ri) {
      int64_t p = rows[ri], n1 = 0;
      for (int32_t t = 0; t < n; ++t) {
        int64_t i = rank[(int64_t)t * N + p];
        int64_t a = i - w < 0 ? 0 : i - w, z = i + w > N - 1 ? N - 1 : i + w;
        for (int64_t j = a; j <= z; ++j) {
          uint32_t c = orders[(int64_t)t * N + j];
          if ((int64_t)c == p || mark[c]) continue;
          mark[c] = 1;
          buf[n1].r = c;
          buf[n1].key = sk ? hamming(sk + p * HFO_SKETCH_WORDS, sk + (int64_t)c * HFO_SKETCH_WORDS) : 0;
          ++n1;
        }
      }
      for (int64_t i = 0; i < n1; ++i) mark[buf[i].r] = 0;
      if (c1n) c1n[ri] = (int32_t)n1;
      int64_t n2 = n1;
      if (k2 > 0) {
        qsort(buf, (size_t)n1, sizeof(cand), cmp_key_r);
        if (n2 > k2) n2 = k2;
        if (c2_out)
          for (int32_t i = 0; i < k2; ++i) c2_out[ri * k2 + i] = i < n2 ? (int32_t)buf[i].r : -1;
      }
      for (int64_t i = 0; i < n2; ++i) {
        int64_t c = buf[i].r;
        double acc = 0.0;
        for (int32_t j = 0; j < d; ++j) acc += val(X, dtype, p * d + j) * val(X, dtype, c * d + j);
        buf[i].s = acc / (norm[p] * norm[c]);
      }
      qsort(buf, (size_t)n2, sizeof(cand), cmp_score_desc_pos);
      for (int32_t i = 0; i < k; ++i) {
        out_ids[ri * k + i] = i < n2 ? (int32_t)buf[i].r : -1;
        out_scores[ri * k + i] = i < n2 ? buf[i].s : -INFINITY;
      }
    }
    free(mark);
    free(buf);
  }
  free(rank);
  free(norm);
}
