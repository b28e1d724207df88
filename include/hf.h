/*
 * hf.h -- C ABI of the Hilbert-forest library (libhf.so) for AMD Instinct
 * MI355X (gfx950).
 *
 * The method is the Hilbert forest of Imamura et al., "Hilbert Forest in the
 * SISAP 2025 Indexing Challenge" (arXiv 2508.21682): points are ordered along
 * Hilbert curves (Section 2), a forest of leaf-compressed Hilbert trees gives
 * first-stage candidates for a whole query batch at once, binary sketches
 * filter them by Hamming distance and vector distance picks the result
 * (Section 3.1, Algorithm 1); a k-NN graph is built from windows along
 * several Hilbert orders (Section 4.1, Algorithm 2).
 *
 * Conventions for every call:
 *  - Pointers named *_dev are device pointers (HIP global memory) on the
 *    current device; pointers named *_host are host pointers.  The caller
 *    owns every input and output buffer.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued on it; device outputs are valid once the stream has completed.
 *    Calls that must read a device value back (marked "synchronises") wait
 *    for the stream before returning.
 *  - Matrices are row-major and dense: X[i*d + j].
 *  - Every call returns an hf_status and never throws.  On HF_ERR_INVALID_ARG
 *    nothing is launched and outputs are untouched; the reason is available
 *    from hf_last_error() (thread-local).
 *  - Sizes: 1 <= N < 2^31, 1 <= d <= 4096.
 */
#ifndef HF_H
#define HF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hf_status {
  HF_OK = 0,
  HF_ERR_INVALID_ARG = 1,     /* bad size, pointer or parameter */
  HF_ERR_INVALID_INPUT = 2,   /* input data not finite */
  HF_ERR_OOM = 3,             /* device allocation failed */
  HF_ERR_DEVICE = 4,          /* a HIP call failed (text in hf_last_error) */
  HF_ERR_INVALID_HANDLE = 5,  /* NULL or freed forest / hash handle */
  HF_ERR_UNSUPPORTED = 6      /* parameters outside what the kernels implement */
} hf_status;

typedef enum hf_dtype { HF_F16 = 0, HF_F32 = 1 } hf_dtype;

typedef enum hf_precision {
  HF_PREC_FP32 = 0, /* score every expanded candidate in FP32 */
  HF_PREC_BF16 = 1, /* score in BF16 on MFMA, FP32 rerank of survivors */
  HF_PREC_FP8 = 2,  /* score in FP8 e4m3 (per-row scale) on MFMA, FP32 rerank */
  HF_PREC_C4 = 3    /* Section 3.1's layout: score from 4-bit codes (sign + 3-bit magnitude)
                       with the query unquantized, FP32 accumulate */
} hf_precision;

/* Sketches compared by the Hamming filter:
 *  HF_SKETCH_SRP:     512 signs of seeded random projections (default);
 *  HF_SKETCH_LEARNED: 512 sign bits of a trained MLP (hf_lhash_*);
 *  HF_SKETCH_SIGN:    one bit per coordinate, [x_i >= 0] (Section 3.1's d-bit
 *                     sketches, the bit the 4-bit codes share), d <= 512,
 *                     zero padded to 512 bits. */
typedef enum hf_sketch_kind { HF_SKETCH_SRP = 0, HF_SKETCH_LEARNED = 1, HF_SKETCH_SIGN = 2 } hf_sketch_kind;

#define HF_QUANT_AUTO INT32_MIN
#define HF_SKETCH_BITS 512
#define HF_SKETCH_WORDS 8

typedef struct hf_forest hf_forest;
typedef struct hf_lhash hf_lhash;

/* Build parameters (Section 3.1, key hyperparameters: n trees; leaves of
 * about M points).  struct_size must be sizeof(hf_forest_params). */
typedef struct hf_forest_params {
  uint32_t struct_size;
  uint32_t n_trees;      /* n, 1..4096 (4N bytes of HBM each); tree 0's order is the master order */
  uint32_t leaf_max;     /* M >= 1: ranges of at most M points become leaves */
  int32_t quant_exp;     /* code exponent e, or HF_QUANT_AUTO (from the data) */
  uint64_t seed;         /* seeds the curves (axis permutation + reflection) */
  uint64_t sketch_seed;  /* seeds the SRP sketch projections */
  uint32_t sketch;       /* hf_sketch_kind */
  uint32_t reserved;
  const hf_lhash* lhash; /* learned hash when sketch == HF_SKETCH_LEARNED */
} hf_forest_params;

/* Search parameters (Section 3.1: k1 per tree, k2 by sketches, h neighbours
 * on each side in the master order).  struct_size = sizeof(hf_search_params). */
typedef struct hf_search_params {
  uint32_t struct_size;
  uint32_t k;         /* results per query, 1..1024 */
  uint32_t k1;        /* window per tree, >= 1 */
  uint32_t k2;        /* kept after the Hamming filter, k <= k2 <= 4096 */
  uint32_t h;         /* expansion half-width in master order */
  uint32_t precision; /* hf_precision */
  uint32_t survivors; /* low-precision survivors per query (0 = 4k) */
  uint32_t trees;     /* search trees 0..trees-1 only (0 = all n trees of the forest); tree t
                         is the same tree in any forest built with the same seed and data */
  uint32_t position;  /* hf_position: where a query sits along each tree's curve */
  uint32_t reserved;
} hf_search_params;

/* Where a query's window of k1 candidates is centred in each tree's order
 * (Algorithm 1, first stage; Section 2 locates a point along the curve):
 *  HF_POS_LEAF:  the midpoint of the leaf its descent reaches;
 *  HF_POS_EXACT: its exact insertion rank among the tree's sorted Hilbert
 *                keys, before any equal key (the number of data points with
 *                a smaller key); needs d <= 512. */
typedef enum hf_position { HF_POS_LEAF = 0, HF_POS_EXACT = 1 } hf_position;

/* Graph parameters (Section 4.1: n sorts, k1 candidates per point per sort
 * read as the window +-w, k2 kept by sketches; k = 15 in the paper). */
typedef struct hf_graph_params {
  uint32_t struct_size;
  uint32_t n_orders;   /* n, 1..4096 */
  uint32_t window;     /* w: positions i-w..i+w of each order, 1..512, 2w < N */
  uint32_t k;          /* neighbours per point, 1..32 */
  uint32_t k2;         /* 0 = no sketch stage; else Hamming top-k2 first, k <= k2 <= 256 */
  int32_t quant_exp;   /* code exponent e, or HF_QUANT_AUTO */
  uint32_t sketch;     /* hf_sketch_kind (used when k2 > 0) */
  uint64_t seed;       /* curves of the n orders */
  uint64_t sketch_seed;
  const hf_lhash* lhash;
} hf_graph_params;

/* ------------------------------------------------------------------ errors */
const char* hf_status_str(hf_status s);
/* Detail of the last failing call on this thread ("" if none). */
const char* hf_last_error(void);

/* ---------------------------------------------------------- building blocks */

/* Curves of trees 0..T-1 (Algorithms 1 and 2: a random axis order per tree or
 * order), computed on the host from one
 * SplitMix64 stream seeded with `seed`: per tree a Fisher-Yates shuffle of the
 * axes, then ceil(d/64) words whose bits (LSB first) mark reflected axes.
 * perm_host[t*d + i] = data axis read by tree axis i; refl_host[t*d + i] = 1
 * if that axis is reflected (x -> 255 - x).  Caller-owned, T*d entries each. */
hf_status hf_curves(uint64_t seed, int32_t T, int32_t d, int32_t* perm_host, uint8_t* refl_host);

/* Code exponent of a data set (the 8-bit fixed-point ordering codes): the
 * largest e in [-8, 24] with 2^e*max(X) < 128 and 2^e*min(X) >= -128 (e = -8
 * if none).  HF_ERR_INVALID_INPUT if X holds a non-finite value.
 * Synchronises. */
hf_status hf_quant_exp(const void* X_dev, hf_dtype dtype, int64_t n_elems, int32_t* e_out_host,
                       void* stream);

/* 8-bit ordering codes u = clamp(floor(x * 2^e) + 128, 0, 255), element-wise
 * (the quantization step of Algorithms 1 and 2, here only
 * used to order points). codes_dev: n_elems bytes. */
hf_status hf_quantize(const void* X_dev, hf_dtype dtype, int64_t n_elems, int32_t e,
                      uint8_t* codes_dev, void* stream);

/* Hilbert sort (Section 2) of N points with codes codes_dev (N x d bytes)
 * along curve `tree` of the stream seeded by `seed`: order_dev[i] = id of the
 * i-th point by (Skilling Hilbert index of the permuted/reflected codes, id).
 * split_dev (nullable, N-1 entries): split_dev[i] = index of the first key bit
 * where points order[i] and order[i+1] differ (key bit b = level 7 - b/d,
 * axis b%d, MSB first), or 0xFFFFFFFF if their keys are equal.
 * Synchronises (the tie refinement reads counts back). */
hf_status hf_hilbert_sort(const uint8_t* codes_dev, int64_t N, int32_t d, uint64_t seed,
                          uint32_t tree, uint32_t* order_dev, uint32_t* split_dev, void* stream);

/* 512-bit sign-of-random-projection sketches (the binary sketches compared by
 * Hamming distance in Section 3.1; their construction is not given in the
 * paper).  R[j][i] = +1 if bit j*d+i of the concatenated SplitMix64 outputs
 * seeded by sketch_seed is 1, else -1; xq_i = clamp(rne(x_i*2^(e+5)), -8191,
 * 8191); bit j = [sum_i R[j][i]*xq_i >= 0] stored in word j/64 at bit j%64.
 * out_dev: N x 8 uint64 words. */
hf_status hf_srp_sketch(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d, int32_t e,
                        uint64_t sketch_seed, uint64_t* out_dev, void* stream);

/* ------------------------------------------------------------------ forest */

/* Preprocessing of Algorithm 1: codes, master order (tree 0), sketches and
 * vectors re-laid in master order, then n leaf-compressed Hilbert trees whose
 * permutations hold master positions.  The forest keeps its own copies; X_dev
 * is not retained.  *out receives a handle to free with hf_forest_free.
 * Synchronises.  With HF_PROGRESS set in the environment, one line per tree
 * goes to stderr. */
hf_status hf_build_forest(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d,
                          const hf_forest_params* params, void* stream, hf_forest** out);
void hf_forest_free(hf_forest* f);

typedef struct hf_forest_info {
  int64_t N;
  int32_t d, n_trees, leaf_max, quant_exp;
  int32_t dtype;
  int32_t device;
  int64_t total_nodes;
  int64_t device_bytes; /* bytes the forest holds on its device */
} hf_forest_info;
hf_status hf_forest_get_info(const hf_forest* f, hf_forest_info* info_host);

/* Introspection (device outputs, caller-owned):
 *  perm: N uint32 master positions of tree t in Hilbert order (tree 0 = 0..N-1);
 *  nodes: the pre-order node records of tree t, 2 uint32 per node:
 *    internal: {index of right child, a | L<<16 | flip<<19}: key bit of a point
 *              = bit L of its code on data axis a, XOR flip; 0 = left child
 *              (the next record), 1 = right child;
 *    leaf:     {lo, 1<<31 | (hi - lo)}: positions [lo, hi) of the tree order.
 *    Pass nodes_dev = NULL to get the count only.
 *  pos2id: N uint32, original id of each master position;
 *  sketches: N x 8 uint64 in master order. */
hf_status hf_forest_perm(const hf_forest* f, uint32_t t, uint32_t* perm_dev, void* stream);
hf_status hf_forest_nodes(const hf_forest* f, uint32_t t, uint32_t* nodes_dev, int64_t* count_host,
                          void* stream);
hf_status hf_forest_pos2id(const hf_forest* f, uint32_t* pos2id_dev, void* stream);
/* Split records of tree t, 2 uint32 per node in the order of hf_forest_nodes:
 * internal {m, b}: the node's range [lo, hi) splits into [lo, m) and [m, hi)
 * at key bit b (the first bit where the range's end keys differ); leaf
 * {lo, 0xFFFFFFFF}.  count_host as for hf_forest_nodes. */
hf_status hf_forest_node_splits(const hf_forest* f, uint32_t t, uint32_t* splits_dev, int64_t* count_host,
                                void* stream);
hf_status hf_forest_sketches(const hf_forest* f, uint64_t* sk_dev, void* stream);

/* Algorithm 1 for a batch of nq queries (same dtype as the data):
 *  first stage: every query descends every tree (the whole batch located
 *    along every curve at once, Section 3.1); its window is the k1 tree positions centred on the
 *    midpoint of the leaf reached, shifted inside [0, N);
 *  second stage: C2 = the k2 candidates of the union of the windows with the
 *    smallest (Hamming distance of sketches, master position);
 *  final: E = C2 expanded by h master positions on each side; S = top-k of E
 *    by (inner product in FP32, descending; master position ascending).
 * ids_dev: nq x k original ids (-1 past the end when |E| < k); scores_dev:
 * nq x k FP32 inner products (-inf past the end). */
hf_status hf_search(const hf_forest* f, const void* Q_dev, hf_dtype dtype, int64_t nq,
                    const hf_search_params* params, int32_t* ids_dev, float* scores_dev,
                    void* stream);

/* hf_search plus the intermediate sets (all nullable, device, caller-owned):
 * win_dev nq x n window starts (n = params->trees, or all the forest's trees); c2_dev nq x k2 master positions in
 * (Hamming, position) order, 0xFFFFFFFF past c2n; c2n_dev nq counts; en_dev
 * nq sizes |E|. */
hf_status hf_search_debug(const hf_forest* f, const void* Q_dev, hf_dtype dtype, int64_t nq,
                          const hf_search_params* params, int32_t* ids_dev, float* scores_dev,
                          uint32_t* win_dev, uint32_t* c2_dev, int32_t* c2n_dev, int32_t* en_dev,
                          void* stream);

/* hf_search without any device allocation, for callers that cannot allocate
 * device memory (work under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, checks and results as hf_search.
 * Every scratch buffer is carved from one fixed array of
 * HF_NOALLOC_SCRATCH_MIB MiB that the library holds on each GPU it runs on
 * until the process ends; queries are processed in consecutive chunks sized
 * to fit it, in stream order.  A configuration whose single query needs more
 * than the array (about 2 * n_trees * k1 + 4 * (n_trees + k2) + d bytes)
 * returns HF_ERR_UNSUPPORTED without launching anything.  All calls on one
 * GPU share that GPU's array: calls that overlap in time on one GPU (on
 * different streams, or from different threads) race on it and must be
 * serialised by the caller.  The array keeps the last call's contents; no
 * result depends on them. */
#define HF_NOALLOC_SCRATCH_MIB 64
hf_status hf_search_noalloc(const hf_forest* f, const void* Q_dev, hf_dtype dtype, int64_t nq,
                            const hf_search_params* params, int32_t* ids_dev, float* scores_dev, void* stream);

/* Precision form (not in the paper): adds a BF16 copy (RNE of the stored
 * rows) or an FP8 copy (OCP e4m3, per-row scale s = max|x|/448 in FP32, codes
 * of x/s rounded to nearest even and saturated) of the master-ordered rows to
 * the forest, so hf_search can score the expansion set E with
 * params->precision = HF_PREC_BF16 / HF_PREC_FP8 on MFMA (FP32 accumulate),
 * keep the best `survivors` (default 4k; ties by position) and rerank those in
 * FP32 from the stored rows.  Adds 2 (BF16) or 1 + 4/d (FP8) bytes per
 * element to the forest.  Synchronises. */
hf_status hf_forest_add_precision(hf_forest* f, hf_precision prec, void* stream);

/* hf_search in a low precision, also returning the survivors: surv_pos_dev
 * nq x S master positions in (low-precision score desc, position) order,
 * 0xFFFFFFFF past |E|; surv_score_dev nq x S their low-precision scores. */
hf_status hf_search_lowprec_debug(const hf_forest* f, const void* Q_dev, hf_dtype dtype, int64_t nq,
                                  const hf_search_params* params, int32_t* ids_dev, float* scores_dev,
                                  uint32_t* surv_pos_dev, float* surv_score_dev, void* stream);

/* Error audit: FP64 inner products of query q with data row ids_dev[q*k + i]
 * (original order X_dev, N x d), written to out_dev (nq x k doubles; 0 for
 * id -1).  The only FP64 arithmetic on the GPU. */
hf_status hf_audit_scores(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d, const void* Q_dev,
                          int64_t nq, const int32_t* ids_dev, int32_t k, double* out_dev, void* stream);

/* ------------------------------------------------------------ learned hash */

/* Learned hash (not in the paper): sketch bit j of x = [z2_j >= 0] with
 * z1 = W1 bf16(x) + b1, a = bf16(relu(z1)), z2 = W2 a + b2 (BF16 weights and
 * inputs on MFMA, FP32 accumulate).  W1 is hidden x d, W2 is 512 x hidden,
 * row-major, given as FP32 host arrays (the master copy trained by
 * hf_lhash_train).  Handle from hf_lhash_create, freed by hf_lhash_free; it
 * must outlive any forest using it (hf_forest_set_sketch). */
typedef struct hf_lhash_train_params {
  uint32_t struct_size;
  uint32_t epochs;        /* passes over the pairs */
  uint32_t batch;         /* pairs per step, 2..8192 (in-batch negatives) */
  float lr, weight_decay; /* AdamW (decoupled decay on W1, W2) */
  float beta1, beta2, eps;
  float slope;            /* codes c = tanh(slope * z2) */
  float tau;              /* InfoNCE temperature on <c_q, c_p> / 512 */
  float balance;          /* weight of sum_b (mean_b c)^2 */
  uint32_t keep_blocks;   /* 0: shuffle all pairs each epoch; 1: batches are the
                             contiguous blocks of the given pair order (only the
                             order of the blocks is shuffled), so a caller that
                             orders pairs along a Hilbert order gets spatial
                             neighbours as in-batch negatives */
  uint64_t seed;          /* shuffles the pairs (or blocks) each epoch */
} hf_lhash_train_params;

hf_status hf_lhash_create(int32_t d, int32_t hidden, const float* W1_host, const float* b1_host,
                          const float* W2_host, const float* b2_host, hf_lhash** out);
void hf_lhash_free(hf_lhash* h);
/* Current FP32 master weights (synchronises). */
hf_status hf_lhash_get(const hf_lhash* h, float* W1_host, float* b1_host, float* W2_host, float* b2_host);
/* 512-bit learned sketches of N rows (N x 8 uint64, bit j in word j/64 at j%64). */
hf_status hf_lhash_encode(const hf_lhash* h, const void* X_dev, hf_dtype dtype, int64_t N, int32_t d,
                          uint64_t* sk_dev, void* stream);
/* Loss (host) and FP32 gradients (device, shapes of W1, b1, W2, b2) of the
 * training objective on one batch of npairs positive pairs (A_dev[i], B_dev[i])
 * and, if N_dev is non-null, one hard negative N_dev[i] per query:
 * (1/B) sum_i [log (sum_j exp(S_ij/tau) + exp(H_i/tau)) - S_ii/tau]
 * + balance * sum_b m_b^2, S_ij = <c(A_i), c(B_j)> / 512, H_i = <c(A_i), c(N_i)>
 * / 512 (the term absent without negatives), m = mean code over all rows.
 * Synchronises. */
hf_status hf_lhash_grad(const hf_lhash* h, const void* A_dev, const void* B_dev, const void* N_dev, hf_dtype dtype,
                        int64_t npairs, int32_t d, const hf_lhash_train_params* params, float* loss_host,
                        float* gW1_dev, float* gb1_dev, float* gW2_dev, float* gb2_dev, void* stream);
/* AdamW training on npairs pairs (rows of A_dev and B_dev, with the hard
 * negatives N_dev when non-null), `epochs` passes of shuffled batches;
 * loss_curve_host (nullable) receives the mean loss of each epoch.
 * Synchronises. */
hf_status hf_lhash_train(hf_lhash* h, const void* A_dev, const void* B_dev, const void* N_dev, hf_dtype dtype,
                         int64_t npairs, int32_t d, const hf_lhash_train_params* params, float* loss_curve_host,
                         void* stream);
/* Replaces the forest's sketches: HF_SKETCH_SRP (from its sketch_seed) or
 * HF_SKETCH_LEARNED (lhash encodes the master-ordered rows, and queries at
 * search time).  Synchronises. */
hf_status hf_forest_set_sketch(hf_forest* f, hf_sketch_kind kind, const hf_lhash* lhash, void* stream);

/* ------------------------------------------------------------------ timing */

/* Scratch allocator.  Every call takes its per-call scratch (device memory
 * beyond its inputs and outputs: query codes and sketches, window starts,
 * distances, candidate lists, sort and graph workspaces) on its stream and
 * gives it back, stream-ordered, once its work is enqueued.  By default that
 * is hipMallocAsync / hipFreeAsync on the device's default memory pool.  A
 * caller with its own device allocator (a framework's caching allocator, a
 * preallocated arena) registers it here:
 *   alloc(bytes, ctx, stream) returns device memory that work enqueued on
 *     `stream` after the call may use, or NULL (the call then fails with
 *     HF_ERR_OOM);
 *   free(ptr, ctx, stream) takes it back after the call has enqueued all of
 *     its work on `stream` (the memory may be reused by later work on that
 *     stream, in stream order).
 * a == NULL restores the default.  The setting is process-wide; change it
 * only while no call is in flight (a call keeps the allocator it started
 * with).  Long-lived storage (forests, learned hashes, precision copies)
 * stays on hipMalloc.  This is the interface of the caller-owned
 * allocator in the boundary of the search and graph calls. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx, void* stream);
  void (*free)(void* ptr, void* ctx, void* stream);
  void* ctx;
} hf_allocator;
hf_status hf_set_allocator(const hf_allocator* a);

/* Per-kernel timing with hipEvents recorded on the caller's stream around
 * each launch of the hot kernels (thread-local; off by default).  Stages:
 * 0 query codes, 1 query sketches, 2 descend, 3 hamming, 4 select, 5 rerank,
 * 6 graph sort, 7 graph band, 8 build sort, 9 build trie, 10 build sketch,
 * 11 lowprec score, 12 graph hamming band, 13 graph list merge, 14 graph
 * final cosine top-k, 15 graph mailbox merge after the last order. */
#define HF_N_STAGES 16
hf_status hf_timing_enable(int32_t on);
/* Waits for the recorded events, writes the summed milliseconds and launch
 * counts of every stage since the last read (arrays of HF_N_STAGES), clears. */
hf_status hf_timing_read(float* ms_host, int32_t* launches_host);
const char* hf_timing_stage_name(int32_t stage);

/* ------------------------------------------------------------------- graph */

/* Algorithm 2: for each of n orders (Hilbert sort along seeded curve t),
 * every point gets the points within +-w positions as candidates; the result
 * is, per point, the top-k of the union of its candidates (self excluded) by
 * (cosine similarity, descending; id ascending).  With k2 > 0 (the
 * second-stage filtering of Algorithm 2) the union is first cut to the k2
 * candidates with the smallest (Hamming distance of 512-bit sketches, id):
 * SRP sketches seeded by sketch_seed, or the learned hash `lhash`
 * (sketch = HF_SKETCH_LEARNED; the handle must outlive the call).
 * X_dev: N x d fp16, 16-byte aligned, d a multiple of 8 (HF_ERR_UNSUPPORTED
 * otherwise).  ids_dev: N x k int32 original ids (-1 if fewer candidates);
 * scores_dev: N x k FP32 cosines; both caller-owned.  Synchronises.
 * The sketch stage stages up to 2w keys per position for chunks of positions
 * whose staging fits HF_GRAPH_STAGE_MIB MiB (environment; default 1024).
 * Without it, each pair of a window is scored once when two per-point
 * mailboxes (8 N w bytes each) fit HF_GRAPH_MAILBOX_MIB MiB
 * (environment; default 32768), from both of its points otherwise; the
 * results are the same. */
hf_status hf_knn_graph(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d,
                       const hf_graph_params* params, int32_t* ids_dev, float* scores_dev,
                       void* stream);

/* hf_knn_graph with k2 > 0 that also writes every point's C2 (the k2
 * candidates by ascending (Hamming distance, id)): c2_dev N x k2 int32, -1
 * where fewer than k2 candidates exist.  Same limits and errors. */
hf_status hf_knn_graph_debug(const void* X_dev, hf_dtype dtype, int64_t N, int32_t d,
                             const hf_graph_params* params, int32_t* ids_dev, float* scores_dev,
                             int32_t* c2_dev, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HF_H */
