// Block nested loop with S in host memory (Algorithm 1's outer loop over S
// blocks, pruneScore carried from block to block): each block is copied to the
// device on a stream of its own while the previous block is joined, indexed,
// joined with R starting from every query's running k-th score, and the rows
// it adds are merged into the running result.
#include <string.h>

#include <chrono>
#include <string>

#include "common.hpp"

namespace knnj {

knnj_status launch_init_out(int64_t n_rows, int32_t k, int32_t* ids, void* sc, int32_t* cnt, hipStream_t st);
knnj_status validate_csr(const knnj_csr* m, int32_t* dev_err, hipStream_t st, int32_t* max_row);
knnj_status join_impl(const knnj_index* h, const knnj_csr* R, int32_t k, const knnj_join_opts* opt, int32_t* ids,
                      void* sc, int32_t* cnt, void* stream, bool init_out);

// Rows of a block's indptr slice made relative to the block's first entry.
__global__ void k_rebase(int64_t n, int64_t base, int64_t* __restrict__ p) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] -= base;
}

// Start query q's block list from its running k-th score: a query that holds k
// neighbours gets k placeholders (id -1) at that score, so the block's join
// admits only rows scoring above it (a row of a later block that ties it ranks
// after it, as its id is larger) and prunes from the first tile on; any other
// query starts empty.
template <typename S>
__global__ void k_seed_block(int64_t n_q, int32_t k, const S* __restrict__ sc, const int32_t* __restrict__ cnt,
                             int32_t* __restrict__ b_ids, S* __restrict__ b_sc, int32_t* __restrict__ b_cnt) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n_q) return;
  const bool full = cnt[q] == k;
  const S th = full ? sc[q * k + k - 1] : S(0);
  for (int i = 0; i < k; ++i) {
    b_ids[q * k + i] = -1;
    b_sc[q * k + i] = th;
  }
  b_cnt[q] = full ? k : 0;
}

// Merge query q's block result (b_*, ids relative to the block, all above every
// id already held) into its running list (ids, sc, cnt), keeping the first k
// under (score desc, id asc).  One thread per query.  A forward pass counts
// how many of each list survive; the merge then runs backwards, so every write
// lands on a slot of the running list that has already been read.
template <typename S>
__global__ void k_merge_topk(int64_t n_q, int32_t k, int64_t id_off, const int32_t* __restrict__ b_ids,
                             const S* __restrict__ b_sc, const int32_t* __restrict__ b_cnt, int32_t* __restrict__ ids,
                             S* __restrict__ sc, int32_t* __restrict__ cnt) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n_q) return;
  const int32_t* bi = b_ids + q * k;
  // the block's own rows come first; placeholders (id -1) follow
  const int nbl = b_cnt[q];
  int nb = 0;
  while (nb < nbl && bi[nb] >= 0) ++nb;
  const int na = cnt[q];
  if (nb == 0) return;
  const S* bs = b_sc + q * k;
  int32_t* ai = ids + q * k;
  S* as = sc + q * k;
  // equal scores: the running list's ids are smaller, so it goes first
  int ia = 0, ib = 0;
  const int keep = na + nb < k ? na + nb : k;
  for (int i = 0; i < keep; ++i) {
    if (ib >= nb || (ia < na && as[ia] >= bs[ib])) ++ia;
    else ++ib;
  }
  for (int i = keep - 1; i >= 0; --i) {
    if (ib > 0 && (ia == 0 || bs[ib - 1] <= as[ia - 1])) {
      --ib;
      ai[i] = int32_t(int64_t(bi[ib]) + id_off);
      as[i] = bs[ib];
    } else {
      --ia;
      ai[i] = ai[ia];
      as[i] = as[ia];
    }
  }
  cnt[q] = keep;
}

namespace {

struct Staging {
  int64_t* indptr = nullptr;
  int32_t* indices = nullptr;
  void* values = nullptr;
};

// Resources of one blocked join, released on every exit path.
struct BlockedRun {
  Staging buf[2];
  int32_t* b_ids = nullptr;
  void* b_sc = nullptr;
  int32_t* b_cnt = nullptr;
  int32_t* dev_err = nullptr;
  hipStream_t copy = nullptr;
  hipEvent_t c0[2] = {nullptr, nullptr}, c1[2] = {nullptr, nullptr};
  hipEvent_t j0 = nullptr, j1 = nullptr, m1 = nullptr;
  knnj_index* ix = nullptr;
  ~BlockedRun() {
    (void)hipDeviceSynchronize();
    if (ix) knnj_index_free(ix);
    for (auto& b : buf) {
      (void)hipFree(b.indptr);
      (void)hipFree(b.indices);
      (void)hipFree(b.values);
    }
    (void)hipFree(b_ids);
    (void)hipFree(b_sc);
    (void)hipFree(b_cnt);
    (void)hipFree(dev_err);
    for (int i = 0; i < 2; ++i) {
      if (c0[i]) (void)hipEventDestroy(c0[i]);
      if (c1[i]) (void)hipEventDestroy(c1[i]);
    }
    if (j0) (void)hipEventDestroy(j0);
    if (j1) (void)hipEventDestroy(j1);
    if (m1) (void)hipEventDestroy(m1);
    if (copy) (void)hipStreamDestroy(copy);
  }
};

double since_ms(std::chrono::steady_clock::time_point t) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

float event_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.0f;
  return ms;
}

}  // namespace

}  // namespace knnj

using namespace knnj;

extern "C" knnj_status knnj_join_blocked(const knnj_csr* S, int64_t block_rows, const knnj_index_opts* index_opts,
                                         const knnj_csr* R, int32_t k, const knnj_join_opts* join_opts,
                                         int32_t* out_ids, void* out_scores, int32_t* out_count,
                                         knnj_block_stats* block_stats, void* stream) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!S || !R) return fail(KNNJ_EINVAL, "S or R is NULL");
  if (block_rows < 1) return fail(KNNJ_EINVAL, "block_rows must be >= 1");
  if (S->dtype != KNNJ_U8 && S->dtype != KNNJ_F32) return fail(KNNJ_EINVAL, "S: unknown dtype");
  if (S->n_rows < 0 || S->nnz < 0 || S->n_dims < 1) return fail(KNNJ_EINVAL, "S: negative size or n_dims < 1");
  if (!S->indptr || (S->nnz > 0 && (!S->indices || !S->values))) return fail(KNNJ_EINVAL, "S arrays are NULL");
  if (R->dtype != S->dtype || R->n_dims != S->n_dims) return fail(KNNJ_EINVAL, "R and S differ in dtype or n_dims");
  if (k < 1 || k > kMaxK) return fail(KNNJ_EINVAL, "k must be in [1, 1024]");
  if (R->n_rows < 0 || R->nnz < 0 || !R->indptr || (R->nnz > 0 && (!R->indices || !R->values)))
    return fail(KNNJ_EINVAL, "R: negative size or NULL arrays");
  if (R->n_rows > 0x7fffffffll) return fail(KNNJ_EUNSUPPORTED, "R: more than 2^31-1 rows");
  if (R->n_rows > 0 && (!out_ids || !out_scores || !out_count)) return fail(KNNJ_EINVAL, "outputs are NULL");
  knnj_join_opts jo;
  memset(&jo, 0, sizeof(jo));
  if (join_opts) jo = *join_opts;
  if (jo.theta_seed) return fail(KNNJ_EINVAL, "the blocked join takes no theta_seed");
  const int64_t* hp = S->indptr;
  if (hp[0] != 0 || hp[S->n_rows] != S->nnz) return fail(KNNJ_EINVAL, "S: indptr does not span [0, nnz]");
  hipStream_t st = (hipStream_t)stream;
  const int64_t n_r = R->n_rows;
  const size_t vbytes = S->dtype == KNNJ_U8 ? 1 : 4;
  BlockedRun run;
  knnj_block_stats bs;
  memset(&bs, 0, sizeof(bs));
  // R: validated once; later calls reuse its longest row
  KNNJ_HIP(hipMalloc(&run.dev_err, 4 * sizeof(int32_t)));
  if (!(jo.flags & KNNJ_FLAG_NO_VALIDATE)) {
    int32_t max_r = 0;
    knnj_status rc = validate_csr(R, run.dev_err, st, &max_r);
    if (rc != KNNJ_OK) return rc;
    jo.flags |= KNNJ_FLAG_NO_VALIDATE;
    jo.r_max_row_nnz = max_r > 0 ? max_r : 1;
  }
  if (n_r > 0) {
    knnj_status rc = launch_init_out(n_r, k, out_ids, out_scores, out_count, st);
    if (rc != KNNJ_OK) return rc;
  }
  const int64_t n_blocks = (S->n_rows + block_rows - 1) / block_rows;
  if (n_r == 0 || n_blocks == 0) {
    KNNJ_HIP(hipStreamSynchronize(st));
    bs.total_ms = since_ms(t_start);
    if (block_stats) *block_stats = bs;
    return KNNJ_OK;
  }
  // staging for the largest block, and one block's results
  int64_t max_nnz = 0;
  for (int64_t b = 0; b < n_blocks; ++b) {
    const int64_t r0 = b * block_rows, r1 = r0 + block_rows < S->n_rows ? r0 + block_rows : S->n_rows;
    if (hp[r1] < hp[r0]) return fail(KNNJ_EINVAL, "S: indptr is not ascending");
    if (hp[r1] - hp[r0] > max_nnz) max_nnz = hp[r1] - hp[r0];
  }
  const int64_t rows_cap = block_rows < S->n_rows ? block_rows : S->n_rows;
  for (auto& b : run.buf) {
    if (hipMalloc(&b.indptr, sizeof(int64_t) * (rows_cap + 1)) != hipSuccess ||
        hipMalloc(&b.indices, sizeof(int32_t) * (max_nnz > 0 ? max_nnz : 1)) != hipSuccess ||
        hipMalloc(&b.values, vbytes * (max_nnz > 0 ? max_nnz : 1)) != hipSuccess)
      return fail(KNNJ_ENOMEM, "device allocation of the S block buffers failed");
  }
  if (hipMalloc(&run.b_ids, sizeof(int32_t) * n_r * k) != hipSuccess ||
      hipMalloc(&run.b_sc, 4 * n_r * k) != hipSuccess || hipMalloc(&run.b_cnt, sizeof(int32_t) * n_r) != hipSuccess)
    return fail(KNNJ_ENOMEM, "device allocation of the block results failed");
  KNNJ_HIP(hipStreamCreateWithFlags(&run.copy, hipStreamNonBlocking));
  for (int i = 0; i < 2; ++i) {
    KNNJ_HIP(hipEventCreate(&run.c0[i]));
    KNNJ_HIP(hipEventCreate(&run.c1[i]));
  }
  KNNJ_HIP(hipEventCreate(&run.j0));
  KNNJ_HIP(hipEventCreate(&run.j1));
  KNNJ_HIP(hipEventCreate(&run.m1));
  // block b's rows and entries
  auto rows_of = [&](int64_t b, int64_t* r0, int64_t* r1) {
    *r0 = b * block_rows;
    *r1 = *r0 + block_rows < S->n_rows ? *r0 + block_rows : S->n_rows;
  };
  auto issue_copy = [&](int64_t b) -> knnj_status {
    int64_t r0, r1;
    rows_of(b, &r0, &r1);
    Staging& g = run.buf[b & 1];
    const int64_t e0 = hp[r0], ne = hp[r1] - hp[r0];
    KNNJ_HIP(hipEventRecord(run.c0[b & 1], run.copy));
    KNNJ_HIP(hipMemcpyAsync(g.indptr, hp + r0, sizeof(int64_t) * (r1 - r0 + 1), hipMemcpyHostToDevice, run.copy));
    if (ne > 0) {
      KNNJ_HIP(hipMemcpyAsync(g.indices, S->indices + e0, sizeof(int32_t) * ne, hipMemcpyHostToDevice, run.copy));
      KNNJ_HIP(hipMemcpyAsync(g.values, static_cast<const char*>(S->values) + vbytes * e0, vbytes * ne,
                              hipMemcpyHostToDevice, run.copy));
    }
    const int64_t n = r1 - r0 + 1;
    const int64_t nb = (n + kBlock - 1) / kBlock;
    k_rebase<<<unsigned(nb < 4096 ? nb : 4096), kBlock, 0, run.copy>>>(n, e0, g.indptr);
    KNNJ_HIP(hipGetLastError());
    KNNJ_HIP(hipEventRecord(run.c1[b & 1], run.copy));
    return KNNJ_OK;
  };
  // the previous block's join and merge times (read once the stream has passed them)
  auto take_join_times = [&]() {
    bs.join_ms += event_ms(run.j0, run.j1);
    bs.merge_ms += event_ms(run.j1, run.m1);
  };
  knnj_status rc = issue_copy(0);
  if (rc != KNNJ_OK) return rc;
  const unsigned merge_grid = unsigned((n_r + kBlock - 1) / kBlock);
  for (int64_t b = 0; b < n_blocks; ++b) {
    int64_t r0, r1;
    rows_of(b, &r0, &r1);
    Staging& g = run.buf[b & 1];
    KNNJ_HIP(hipStreamWaitEvent(st, run.c1[b & 1], 0));
    knnj_csr blk;
    blk.n_rows = r1 - r0;
    blk.n_dims = S->n_dims;
    blk.dtype = S->dtype;
    blk.nnz = hp[r1] - hp[r0];
    blk.indptr = g.indptr;
    blk.indices = g.indices;
    blk.values = g.values;
    // freeing the previous block's index waits for the device: its join and
    // merge are done (one index at a time in device memory)
    if (run.ix) {
      knnj_index_free(run.ix);
      run.ix = nullptr;
      take_join_times();
    }
    // the build validates the block and synchronises the stream, after this
    // block's copy has landed
    const auto tb = std::chrono::steady_clock::now();
    rc = knnj_build_index(&blk, index_opts, st, &run.ix);
    bs.build_ms += since_ms(tb);
    if (rc != KNNJ_OK) return rc;
    bs.copy_ms += event_ms(run.c0[b & 1], run.c1[b & 1]);
    knnj_index* ix = run.ix;
    // the next block's copy overlaps this block's join (its buffer was last read
    // by the build two blocks back, which has returned)
    if (b + 1 < n_blocks && (rc = issue_copy(b + 1)) != KNNJ_OK) return rc;
    KNNJ_HIP(hipEventRecord(run.j0, st));
    if (S->dtype == KNNJ_U8)
      k_seed_block<uint32_t><<<merge_grid, kBlock, 0, st>>>(n_r, k, (const uint32_t*)out_scores, out_count,
                                                             run.b_ids, (uint32_t*)run.b_sc, run.b_cnt);
    else
      k_seed_block<float><<<merge_grid, kBlock, 0, st>>>(n_r, k, (const float*)out_scores, out_count, run.b_ids,
                                                          (float*)run.b_sc, run.b_cnt);
    KNNJ_HIP(hipGetLastError());
    rc = join_impl(ix, R, k, &jo, run.b_ids, run.b_sc, run.b_cnt, st, false);
    if (rc != KNNJ_OK) return rc;
    KNNJ_HIP(hipEventRecord(run.j1, st));
    if (S->dtype == KNNJ_U8)
      k_merge_topk<uint32_t><<<merge_grid, kBlock, 0, st>>>(n_r, k, r0, run.b_ids, (const uint32_t*)run.b_sc,
                                                             run.b_cnt, out_ids, (uint32_t*)out_scores, out_count);
    else
      k_merge_topk<float><<<merge_grid, kBlock, 0, st>>>(n_r, k, r0, run.b_ids, (const float*)run.b_sc, run.b_cnt,
                                                          out_ids, (float*)out_scores, out_count);
    KNNJ_HIP(hipGetLastError());
    KNNJ_HIP(hipEventRecord(run.m1, st));
  }
  KNNJ_HIP(hipStreamSynchronize(st));
  take_join_times();
  bs.n_blocks = n_blocks;
  bs.total_ms = since_ms(t_start);
  if (block_stats) *block_stats = bs;
  return KNNJ_OK;
}
