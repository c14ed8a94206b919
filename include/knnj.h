/*
 * knnj -- exact K-nearest-neighbour join of high-dimensional sparse vectors on
 * one AMD Instinct MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * The operation (Problem definition, Sec. 3): for every vector r of R, return
 * the k vectors s of S with the largest score dot(r, s) = sum_d r[d] * s[d]
 * (Eq. 1), where a sparse vector is a list of features (d, w), ascending d,
 * w > 0.  Reading used throughout: a neighbour must have score > 0
 * (Algorithms 1 and 2 start the pruning score at 0 and admit only scores above
 * it); neighbours are ordered by (score descending, S row id
 * ascending), which also decides ties at the k-th place; a query with fewer
 * than k positive-score vectors gets padding slots (id -1, score 0).
 *
 * Algorithms (Sec. 4): BF (Algorithm 2), IIB (inverted-index accumulation,
 * Algorithm 3) and IIIB (threshold-refined inverted index, Algorithm 4), run
 * as a block nested loop (Algorithm 1) over tiles of S.  All three return the
 * same result (Theorem 1).
 *
 * Memory: every array argument named "device" is HIP device memory that the
 * caller owns; the library never frees it.  The library owns the opaque
 * index and MLP objects (released with their _free calls).  Calls are
 * asynchronous on the given stream (a hipStream_t passed as void*, NULL for
 * the default stream) unless stated otherwise; output buffers are valid after
 * the stream is synchronised.
 *
 * Devices and overlap: an index or an MLP is used on the device that was
 * current when it was made (a call with another device current fails with
 * EINVAL).  An index holds the scratch memory of its joins (query order,
 * statistics, IIIB's per-block index), so joins on one index must not overlap:
 * issue them on one stream, or order them.  A join called with out_count NULL
 * uses a count buffer of the calling thread on the current device; two such
 * joins from one thread must not overlap either.  Different indexes may be
 * joined concurrently.
 *
 * Errors: every call returns a knnj_status; on failure nothing is written to
 * the outputs (unless stated) and knnj_last_error() returns a message for the
 * calling thread.
 */
#ifndef KNNJ_H
#define KNNJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KNNJ_OK = 0,
  KNNJ_EINVAL = -1,      /* bad argument or malformed CSR input */
  KNNJ_ENOMEM = -2,      /* device allocation failed */
  KNNJ_EDEVICE = -3,     /* a HIP runtime call failed */
  KNNJ_EOVERFLOW = -4,   /* an integer score could exceed 2^31 - 1 */
  KNNJ_EUNSUPPORTED = -5 /* valid input outside what the library supports */
} knnj_status;

/* Value type of a sparse matrix. */
typedef enum {
  KNNJ_U8 = 0,  /* uint8 weights in [1, 255]; scores are exact int32 */
  KNNJ_F32 = 1  /* finite float32 weights > 0; scores are float32 (fp64 sums, rounded) */
} knnj_dtype;

/* In-memory join algorithm run on each (query group, S tile) pair. */
typedef enum {
  KNNJ_IIB = 0, /* Algorithm 3: walk the whole posting list of every query feature */
  KNNJ_IIIB = 1 /* Algorithm 4: walk only the indexed part, then complete candidates */
} knnj_algo;

/*
 * Sparse matrix in CSR form, all arrays in device memory.
 *   indptr  int64[n_rows + 1], indptr[0] = 0, non-decreasing, indptr[n_rows] = nnz
 *   indices int32[nnz], strictly ascending within each row, each in [0, n_dims)
 *   values  uint8[nnz] (KNNJ_U8, every value >= 1) or float32[nnz] (KNNJ_F32,
 *           finite and > 0)
 * Rows may be empty.  A row may hold at most 4096 features.
 */
typedef struct {
  int64_t n_rows;
  int32_t n_dims;
  int32_t dtype; /* knnj_dtype */
  int64_t nnz;
  const int64_t* indptr;
  const int32_t* indices;
  const void* values;
} knnj_csr;

typedef struct knnj_index knnj_index;

/* Options of knnj_build_index (pass NULL for defaults). */
typedef struct {
  /* S tile width T: rows of S whose scores are accumulated together in one
   * workgroup's local memory (the block B_s of Algorithm 1).  0 selects the
   * default; otherwise a power of two in [256, 65536]. */
  int32_t tile_width;
  /* Also keep the dense_head dimensions with the longest lists as a dense
   * block per tile; the IIB join then computes their part of every score with
   * dot products (uint8: byte dot products, the same exact sums; float32: fp64
   * products of the float weights, each exact, summed in fp64 like the walk)
   * and walks only the other lists.  Pays off when a few dimensions hold most
   * postings.  0 = off; otherwise 64, 128, 192 or 256. */
  int32_t dense_head;
  int32_t reserved[6];
} knnj_index_opts;

/* Flags of knnj_join_opts.flags */
#define KNNJ_FLAG_NO_VALIDATE 1u /* skip the device check of R's CSR structure (no host sync) */
/* IIIB only, beyond the paper (its Sec. 6 asks for stronger refinement): skip the
 * completion of an s whose indexed partial score A[s] plus the bound of its
 * unindexed part cannot reach the threshold.  Results stay exact. */
#define KNNJ_FLAG_IIIB_BOUND 2u
/* Schedule of the IIB join.  Default: one launch per S tile with one workgroup
 * per query, queries in longest-first order (cost = the query's postings).
 * With this flag: one persistent launch per tile whose resident workgroups take
 * queries, in the same order, from a device counter.  Same results.  This
 * schedule walks every list: an index's dense head is not used by it. */
#define KNNJ_FLAG_PERSISTENT 4u
/* Ignore the index's dense head: walk every list (the plain Algorithm 3 walk). */
#define KNNJ_FLAG_NO_DENSE_HEAD 8u

/* Counters accumulated into knnj_join_opts.stats (device uint64[KNNJ_STAT_COUNT]). */
enum {
  KNNJ_STAT_POSTINGS = 0,   /* posting entries walked (IIB: the 2nd term of Eq. 4) */
  KNNJ_STAT_COMPLETION = 1, /* IIIB: unindexed features read to complete candidates */
  KNNJ_STAT_CANDIDATES = 2, /* IIIB: (query, s) pairs completed */
  KNNJ_STAT_FALLBACKS = 3,  /* queries recomputed without the seeded threshold */
  KNNJ_STAT_COUNT = 8
};

/* Options of knnj_join (pass NULL for defaults: IIB, validation on). */
typedef struct {
  int32_t algo;          /* knnj_algo */
  uint32_t flags;        /* KNNJ_FLAG_* */
  /* IIIB: rows of R per block whose statistics (dimension order and per-dimension
   * maximum weight, Algorithm 4's block statistics) define the refinement bound; 0 means
   * all of R is one block. */
  int64_t r_block_rows;
  /* Optional device float[n_rows of R]: a per-query guess of the k-th score used
   * to seed IIIB's threshold before any posting is read.  Results stay exact: a
   * query whose seed turns out too high is recomputed without it. */
  const float* theta_seed;
  /* Optional device uint64[KNNJ_STAT_COUNT]; counters are added to it. */
  uint64_t* stats;
  /* Optional device uint8[n_rows of R]: set to 1 for queries that fell back. */
  uint8_t* fallback_out;
  /* IIIB: index features whose bound reaches a ladder step this many steps
   * (factors of 2^(1/4)) below the threshold; 0 = the step at the threshold.
   * Any value keeps the result exact; it trades indexed postings for
   * completion work.  In [0, 63]. */
  int32_t level_drop;
  /* Optional upper bound on the longest row of R (0 = unknown).  Validation
   * measures it; without validation 4096 is assumed.  Sizes IIIB's local copy of
   * r when the dimensions are too many for a dense one. */
  int32_t r_max_row_nnz;
  /* Dense-head IIB join: S tiles taken by one launch (each workgroup keeps its
   * queries across them).  0 = default (4). */
  int32_t tiles_per_launch;
  int32_t reserved[3];
} knnj_join_opts;

/*
 * Build the inverted index of S (Algorithm 3, Create_Inverted_List_IIB): the
 * posting list I_d of every dimension, split by S tile so that one tile's
 * score accumulators fit in a workgroup's local memory; inside each
 * (tile, d) list the entries are in ascending S row id.  The index keeps its
 * own copy of everything it needs; S may be freed after the stream is
 * synchronised.  Validates S on the device and synchronises the stream.
 * Errors: EINVAL (malformed S, bad options), ENOMEM, EDEVICE, EUNSUPPORTED.
 */
knnj_status knnj_build_index(const knnj_csr* S, const knnj_index_opts* opt, void* stream, knnj_index** out);

/* Host-side facts about a built index (sizes; no device data copied). */
typedef struct {
  int64_t n_rows;
  int32_t n_dims;
  int32_t dtype;
  int64_t nnz;
  int32_t tile_width;
  int32_t n_tiles;
  int32_t max_row_nnz;
  int32_t dense_head;
} knnj_index_info;

knnj_status knnj_index_info_get(const knnj_index* ix, knnj_index_info* out);

/* Copy |I_d|, the length of every posting list over all of S (Sec. 4.3), into
 * out (device uint32[n_dims], caller-owned).  Asynchronous on stream. */
knnj_status knnj_index_list_lengths(const knnj_index* ix, uint32_t* out, void* stream);

void knnj_index_free(knnj_index* ix);

/*
 * Exact KNN join of R against the indexed S (Algorithm 1 with Algorithm 3 or 4
 * as the in-memory join).  k in [1, 1024].  Outputs (device, row-major, k per
 * query): out_ids int32[n_rows*k], out_scores int32 (U8) or float (F32)
 * [n_rows*k], out_count int32[n_rows] (may be NULL).  Row i holds
 * min(k, #{s : score > 0}) neighbours in (score desc, id asc) order, then
 * padding (-1, 0).
 * Validation: host checks of shapes and options; unless KNNJ_FLAG_NO_VALIDATE,
 * a device check of R's structure followed by a stream synchronisation.
 * Graph capture: with KNNJ_FLAG_NO_VALIDATE, out_count given and no more
 * queries than an earlier call of the same algorithm on the same index, a join
 * only enqueues kernels (no allocation, memset or synchronisation), so it can
 * be captured into a hipGraph.
 * Errors: EINVAL, EOVERFLOW (u8 scores could exceed 2^31-1), ENOMEM, EDEVICE.
 */
knnj_status knnj_join(const knnj_index* ix, const knnj_csr* R, int32_t k, const knnj_join_opts* opt,
                      int32_t* out_ids, void* out_scores, int32_t* out_count, void* stream);

/*
 * Brute-force join (Algorithm 2): every pair's score by a merge of the two
 * sorted feature lists.  Same outputs, validation and errors as knnj_join.
 */
knnj_status knnj_join_bf(const knnj_csr* S, const knnj_csr* R, int32_t k, int32_t* out_ids, void* out_scores,
                         int32_t* out_count, void* stream);

/* Phase times of knnj_join_blocked in milliseconds (host struct, filled when
 * the call returns).  Copies run on a stream of their own and overlap the
 * previous block's join, so the phases may add up to more than total_ms. */
typedef struct {
  int64_t n_blocks;
  double copy_ms;  /* host-to-device transfer of the S blocks (I/O) */
  double build_ms; /* per-block index builds, including their validation */
  double join_ms;  /* joins of R with each block */
  double merge_ms; /* merges of each block's k best into the running result */
  double total_ms;
} knnj_block_stats;

/*
 * Block nested loop with S in host memory (Algorithm 1, whose outer loop reads
 * S block by block into a buffer; Sec. 5 measures its I/O): S is taken in
 * blocks of block_rows rows in ascending row order.  Each block is copied to
 * the device (while the previous block is joined), indexed as by
 * knnj_build_index with index_opts, and joined with R as by knnj_join with
 * join_opts, each query starting from its running k-th score (pruneScore
 * carried across blocks, as Algorithm 1 carries it across S blocks); the rows
 * a block adds (ids offset by its first row) are then merged into the running
 * result under the same order (score desc, id asc).  The result equals
 * knnj_join on an index of all of S.
 * S: CSR in host memory (indptr, indices, values host pointers; page-locked
 * memory lets the copies run asynchronously); R and the outputs: device, as
 * for knnj_join, except that out_count must not be NULL.  join_opts->theta_seed must be NULL (a seed bounds the k-th
 * score over all of S, not over a block).  Device memory in use: about two
 * blocks of S, one block's index and one block's results.  Synchronises the
 * stream before it returns; block_stats (nullable, host) receives the phase
 * times.
 * Errors: as knnj_build_index and knnj_join; EINVAL for block_rows < 1 or a
 * seed.  A failure after the first block leaves the outputs holding a partial
 * result.
 */
knnj_status knnj_join_blocked(const knnj_csr* S_host, int64_t block_rows, const knnj_index_opts* index_opts,
                              const knnj_csr* R, int32_t k, const knnj_join_opts* join_opts, int32_t* out_ids,
                              void* out_scores, int32_t* out_count, knnj_block_stats* block_stats, void* stream);

/* ------------------------------------------------------------------------
 * Learned threshold seed (not in the paper; its Sec. 6 asks for stronger
 * refinement).  A 64-128-128-1 MLP (ReLU, bfloat16 weights, float32
 * accumulation) predicts a query's k-th score from 64 features; the prediction
 * is passed to knnj_join as theta_seed.  Correctness never depends on it: the
 * join's survivor check recomputes any query whose seed was too high.
 * ------------------------------------------------------------------------ */
typedef struct knnj_mlp knnj_mlp;

#define KNNJ_MLP_FEATURES 64
#define KNNJ_MLP_PARAMS 24961 /* W1[128][64] b1[128] W2[128][128] b2[128] w3[128] b3 */
#define KNNJ_MLP_NORM 129     /* feature mean[64], feature std[64], label scale */

typedef struct {
  int32_t epochs;  /* passes over the training set, >= 1 */
  int32_t batch;   /* minibatch size in [1, 65536] */
  float lr;        /* Adam step size */
  float tau;       /* pinball-loss quantile in (0, 1); small values bias the seed low */
  uint64_t seed;   /* shuffling seed */
  int32_t reserved[8];
} knnj_train_opts;

/* New network with He-uniform weights drawn from `seed` (host RNG), zero
 * biases, identity normalisation.  Errors: EINVAL, ENOMEM, EDEVICE. */
knnj_status knnj_mlp_create(uint64_t seed, knnj_mlp** out);
void knnj_mlp_free(knnj_mlp* m);

/* Features of every row of R (device float[n_rows][64]): log(1 + nnz), the
 * share of features in each of 16 weight bins, and the share in each of 47
 * bins of floor(2 log2(1 + |I_d|)) (list lengths from the index). */
knnj_status knnj_mlp_features(const knnj_index* ix, const knnj_csr* R, float* out, void* stream);

/* Train on n samples: X device float[n][64], y device float[n] (exact k-th
 * scores).  Sets the normalisation from X and y, then runs minibatch Adam on
 * the pinball loss.  epoch_loss (host float[epochs], nullable) receives each
 * epoch's mean batch loss.  Synchronises the stream. */
knnj_status knnj_mlp_train(knnj_mlp* m, const float* X, const float* y, int64_t n, const knnj_train_opts* opt,
                           float* epoch_loss, void* stream);

/* theta_out (device float[n]) = predicted k-th score of each row of X. */
knnj_status knnj_mlp_predict(const knnj_mlp* m, const float* X, int64_t n, float* theta_out, void* stream);

/* Gradient of the mean pinball loss over the n samples at the current working
 * weights, without updating them: grad_out device float[24961], loss_out device
 * float[1].  Synchronises the stream. */
knnj_status knnj_mlp_grad(knnj_mlp* m, const float* X, const float* y, int64_t n, float tau, float* grad_out,
                          float* loss_out, void* stream);

/* Host copies of the working (bfloat16-rounded) weights and the normalisation;
 * set_state rounds the given weights to bfloat16 for the working copy. */
knnj_status knnj_mlp_get_state(const knnj_mlp* m, float* params, float* norm);
knnj_status knnj_mlp_set_state(knnj_mlp* m, const float* params, const float* norm);

/* Thread-local description of the last failure ("" if none). */
const char* knnj_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KNNJ_H */
