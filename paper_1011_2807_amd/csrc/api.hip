// C-ABI entry points: argument checks, object lifetime, kernel sequencing.
#include <string.h>

#include <string>

#include "common.hpp"
#include "sched.hpp"

namespace knnj {

static thread_local std::string g_last_error;

knnj_status fail(knnj_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

knnj_status validate_csr(const knnj_csr* m, int32_t* dev_err, hipStream_t st, int32_t* max_row);
knnj_status build_postings(Index* ix, const int64_t* indptr, const int32_t* indices, const void* values,
                           hipStream_t st);
knnj_status launch_init_out(int64_t n_rows, int32_t k, int32_t* ids, void* sc, int32_t* cnt, hipStream_t st);
knnj_status launch_reduce_stats(const uint64_t* slots, uint64_t* out, hipStream_t st);
knnj_status launch_iib(const Index* ix, const knnj_csr* R, int32_t k, const int32_t* order, int32_t* ids, void* sc,
                       int32_t* cnt, uint64_t* slots, hipStream_t st);
knnj_status launch_iiib(Index* ix, const knnj_csr* R, int32_t k, const knnj_join_opts* opt, const int32_t* order,
                        int32_t max_r, int32_t* ids, void* sc, int32_t* cnt, uint64_t* slots, hipStream_t st);
knnj_status launch_iib_persistent(const Index* ix, const knnj_csr* R, int32_t k, const Sched& sch, int32_t* ids,
                                  void* sc, int32_t* cnt, uint64_t* slots, hipStream_t st);
knnj_status launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
knnj_status launch_lpt_order(int64_t n, const int64_t* r_ptr, const int32_t* r_idx, const uint32_t* list_len,
                             uint32_t* bucket, uint32_t* hist, int32_t* order, hipStream_t st);
knnj_status build_head(Index* ix, hipStream_t st);
knnj_status launch_iib_head(Index* ix, const knnj_csr* R, int32_t k, const int32_t* order, int32_t tiles_per_launch,
                            int32_t* ids, void* sc, int32_t* cnt, uint64_t* slots, hipStream_t st);
size_t head_smem_bytes(int tile, int k, int H, int dtype);
knnj_status launch_bf(const knnj_csr* S, const knnj_csr* R, int32_t k, int32_t* ids, void* sc, int32_t* cnt,
                      hipStream_t st);
size_t tile_smem_bytes(int tile, int k, size_t acc_b);

static knnj_status check_csr_host(const knnj_csr* m, const char* name) {
  if (!m) return fail(KNNJ_EINVAL, std::string(name) + " is NULL");
  if (m->dtype != KNNJ_U8 && m->dtype != KNNJ_F32) return fail(KNNJ_EINVAL, std::string(name) + ": unknown dtype");
  if (m->n_rows < 0 || m->nnz < 0 || m->n_dims < 1)
    return fail(KNNJ_EINVAL, std::string(name) + ": negative size or n_dims < 1");
  if (m->n_rows > 0x7fffffffll) return fail(KNNJ_EUNSUPPORTED, std::string(name) + ": more than 2^31-1 rows");
  if (!m->indptr) return fail(KNNJ_EINVAL, std::string(name) + ": indptr is NULL");
  if (m->nnz > 0 && (!m->indices || !m->values))
    return fail(KNNJ_EINVAL, std::string(name) + ": indices/values are NULL");
  return KNNJ_OK;
}

// Objects (index, MLP) are used on the device that was current when they were made.
knnj_status check_device(int owner, const char* what) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(KNNJ_EDEVICE, "hipGetDevice failed");
  if (dev != owner)
    return fail(KNNJ_EINVAL, std::string(what) + " was made on device " + std::to_string(owner) + ", but device " +
                                 std::to_string(dev) + " is current");
  return KNNJ_OK;
}

static int device_max_smem(int dev) {
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
  return v;
}

static void free_index(Index* ix) {
  if (!ix) return;
  (void)hipFree(ix->offsets);
  (void)hipFree(ix->post_u8);
  (void)hipFree(ix->post_s);
  (void)hipFree(ix->post_w);
  (void)hipFree(ix->list_len);
  (void)hipFree(ix->head_pos);
  (void)hipFree(ix->head_blk);
  (void)hipFree(ix->hj_cnt);
  (void)hipFree(ix->hj_d);
  (void)hipFree(ix->hj_w);
  (void)hipFree(ix->hj_rh);

  (void)hipFree(ix->s_indptr);
  (void)hipFree(ix->s_indices);
  (void)hipFree(ix->s_values);
  (void)hipFree(ix->iiib_post);
  (void)hipFree(ix->iiib_post_w);
  (void)hipFree(ix->iiib_post_s);
  (void)hipFree(ix->iiib_fwd);
  (void)hipFree(ix->iiib_fwd_w);
  (void)hipFree(ix->iiib_cut);
  (void)hipFree(ix->iiib_freq);
  (void)hipFree(ix->iiib_maxw);
  (void)hipFree(ix->iiib_big);
  (void)hipFree(ix->iiib_small);
  (void)hipFree(ix->iiib_out_tmp);
  (void)hipFree(ix->iiib_qlist);
  (void)hipFree(ix->iiib_seed2);
  (void)hipFree(ix->rec_tmp);
  (void)hipFree(ix->dev_err);
  (void)hipFree(ix->stat_slots);
  (void)hipFree(ix->js_order);
  (void)hipFree(ix->js_bucket);
  (void)hipFree(ix->js_heads);
  (void)hipFree(ix->js_small);
  delete ix;
}

}  // namespace knnj

using namespace knnj;

namespace knnj {
const uint32_t* index_list_len(const knnj_index* h) { return reinterpret_cast<const Index*>(h)->list_len; }
int index_device(const knnj_index* h) { return reinterpret_cast<const Index*>(h)->device; }
}  // namespace knnj

// The public handle is the internal Index itself, seen through an opaque type.
static Index* impl(const knnj_index* h) { return reinterpret_cast<Index*>(const_cast<knnj_index*>(h)); }

extern "C" {

const char* knnj_last_error(void) { return g_last_error.c_str(); }

knnj_status knnj_build_index(const knnj_csr* S, const knnj_index_opts* opt, void* stream, knnj_index** out) {
  g_last_error.clear();
  if (!out) return fail(KNNJ_EINVAL, "out is NULL");
  *out = nullptr;
  knnj_status rc = check_csr_host(S, "S");
  if (rc != KNNJ_OK) return rc;
  int tile = opt && opt->tile_width ? opt->tile_width : 4096;
  if (tile < 256 || tile > 65536 || (tile & (tile - 1)))
    return fail(KNNJ_EINVAL, "tile_width must be a power of two in [256, 65536]");
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  KNNJ_HIP(hipGetDevice(&dev));
  const int max_smem = device_max_smem(dev);
  if (tile_smem_bytes(tile, kMaxK, acc_bytes(S->dtype)) > size_t(max_smem))
    return fail(KNNJ_EUNSUPPORTED, "tile_width too large for this device's local memory (" +
                                       std::to_string(max_smem) + " bytes per workgroup)");
  const int head = opt ? opt->dense_head : 0;
  if (head != 0) {
    if (head < 64 || head > 256 || (head % 64)) return fail(KNNJ_EINVAL, "dense_head must be 64, 128, 192 or 256");
    if (head_smem_bytes(tile, 1, head, S->dtype) > size_t(max_smem))
      return fail(KNNJ_EUNSUPPORTED, "tile_width too large for the dense-head join's local memory");
  }
  Index* ix = new Index();
  ix->device = dev;
  ix->n_rows = S->n_rows;
  ix->n_dims = S->n_dims;
  ix->dtype = S->dtype;
  ix->nnz = S->nnz;
  ix->tile = tile;
  ix->log2_tile = 0;
  while ((1 << ix->log2_tile) < tile) ++ix->log2_tile;
  ix->n_tiles = int32_t((S->n_rows + tile - 1) / tile);
  if (ix->n_tiles < 1) ix->n_tiles = 1;
  const size_t vbytes = S->dtype == KNNJ_U8 ? 1 : 4;
  const size_t nnz1 = size_t(S->nnz > 0 ? S->nnz : 1);
  if (hipMalloc(&ix->dev_err, 4 * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&ix->stat_slots, sizeof(uint64_t) * 256 * KNNJ_STAT_COUNT) != hipSuccess) {
    free_index(ix);
    return fail(KNNJ_ENOMEM, "device allocation failed");
  }
  int32_t max_row = 0;
  if ((rc = validate_csr(S, ix->dev_err, st, &max_row)) != KNNJ_OK) {
    free_index(ix);
    return rc;
  }
  ix->max_row_nnz = max_row;
  if (hipMalloc(&ix->s_indptr, sizeof(int64_t) * (S->n_rows + 1)) != hipSuccess ||
      hipMalloc(&ix->s_indices, sizeof(int32_t) * nnz1) != hipSuccess ||
      hipMalloc(&ix->s_values, vbytes * nnz1) != hipSuccess ||
      (S->dtype == KNNJ_U8 ? hipMalloc(&ix->post_u8, sizeof(uint32_t) * (nnz1 + kPostPad))
                           : (hipMalloc(&ix->post_s, sizeof(uint16_t) * (nnz1 + kPostPad)) == hipSuccess
                                  ? hipMalloc(&ix->post_w, sizeof(float) * (nnz1 + kPostPad))
                                  : hipErrorOutOfMemory)) != hipSuccess) {
    free_index(ix);
    return fail(KNNJ_ENOMEM, "device allocation for the index failed");
  }
  if ((S->dtype == KNNJ_U8 ? hipMemsetAsync(ix->post_u8 + nnz1, 0, sizeof(uint32_t) * kPostPad, st)
                           : hipMemsetAsync(ix->post_s + nnz1, 0, sizeof(uint16_t) * kPostPad, st)) != hipSuccess ||
      (S->dtype == KNNJ_F32 && hipMemsetAsync(ix->post_w + nnz1, 0, sizeof(float) * kPostPad, st) != hipSuccess)) {
    free_index(ix);
    return fail(KNNJ_EDEVICE, "hipMemsetAsync failed");
  }
  if (hipMemcpyAsync(ix->s_indptr, S->indptr, sizeof(int64_t) * (S->n_rows + 1), hipMemcpyDeviceToDevice, st) !=
          hipSuccess ||
      (S->nnz > 0 &&
       (hipMemcpyAsync(ix->s_indices, S->indices, sizeof(int32_t) * S->nnz, hipMemcpyDeviceToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(ix->s_values, S->values, vbytes * S->nnz, hipMemcpyDeviceToDevice, st) != hipSuccess))) {
    free_index(ix);
    return fail(KNNJ_EDEVICE, "copy of S into the index failed");
  }
  if ((rc = build_postings(ix, ix->s_indptr, ix->s_indices, ix->s_values, st)) != KNNJ_OK) {
    free_index(ix);
    return rc;
  }
  if (head > 0) {
    ix->head_h = head;
    if ((rc = build_head(ix, st)) != KNNJ_OK) {
      free_index(ix);
      return rc;
    }
  }
  *out = reinterpret_cast<knnj_index*>(ix);
  return KNNJ_OK;
}

knnj_status knnj_index_info_get(const knnj_index* h, knnj_index_info* out) {
  if (!h || !out) return fail(KNNJ_EINVAL, "NULL argument");
  const Index* ix = impl(h);
  memset(out, 0, sizeof(*out));
  out->n_rows = ix->n_rows;
  out->n_dims = ix->n_dims;
  out->dtype = ix->dtype;
  out->nnz = ix->nnz;
  out->tile_width = ix->tile;
  out->n_tiles = ix->n_tiles;
  out->max_row_nnz = ix->max_row_nnz;
  out->dense_head = ix->head_h;
  return KNNJ_OK;
}

knnj_status knnj_index_list_lengths(const knnj_index* h, uint32_t* out, void* stream) {
  if (!h || !out) return fail(KNNJ_EINVAL, "NULL argument");
  const Index* ix = impl(h);
  const knnj_status rc = check_device(ix->device, "the index");
  if (rc != KNNJ_OK) return rc;
  KNNJ_HIP(hipMemcpyAsync(out, ix->list_len, sizeof(uint32_t) * ix->n_dims, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
  return KNNJ_OK;
}

void knnj_index_free(knnj_index* h) {
  if (!h) return;
  // wait for and free on the index's own device, whichever device is current
  int cur = -1;
  const bool other = hipGetDevice(&cur) == hipSuccess && cur != impl(h)->device &&
                     hipSetDevice(impl(h)->device) == hipSuccess;
  (void)hipDeviceSynchronize();
  free_index(impl(h));
  if (other) (void)hipSetDevice(cur);
}

static knnj_status check_join_args(const knnj_csr* R, int32_t k, int32_t* ids, void* sc, int32_t n_dims,
                                   int32_t dtype) {
  knnj_status rc = check_csr_host(R, "R");
  if (rc != KNNJ_OK) return rc;
  if (R->n_dims != n_dims) return fail(KNNJ_EINVAL, "R.n_dims differs from S.n_dims");
  if (R->dtype != dtype) return fail(KNNJ_EINVAL, "R.dtype differs from S.dtype");
  if (k < 1 || k > kMaxK) return fail(KNNJ_EINVAL, "k must be in [1, 1024]");
  if (R->n_rows > 0 && (!ids || !sc)) return fail(KNNJ_EINVAL, "output buffers are NULL");
  return KNNJ_OK;
}

static knnj_status overflow_check(int32_t dtype, int64_t max_r, int64_t max_s) {
  if (dtype != KNNJ_U8) return KNNJ_OK;
  const int64_t m = max_r < max_s ? max_r : max_s;
  if (m * 65025ll > 0x7fffffffll) return fail(KNNJ_EOVERFLOW, "u8 scores could exceed 2^31-1");
  return KNNJ_OK;
}

// Grow-only device buffer of at least `bytes` on the current device, one per
// (calling thread, device, use): the count buffer of joins called with
// out_count = NULL, and the error words of the brute-force join's validation.
enum ThreadBuffer { kCountBuffer = 0, kBfErrBuffer = 1 };

static void* thread_buffer(ThreadBuffer use, size_t bytes) {
  constexpr int kMaxDevices = 64;
  struct Buf {
    void* p = nullptr;
    size_t cap = 0;
  };
  static thread_local Buf bufs[2][kMaxDevices];
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  Buf& b = bufs[use][dev];
  if (bytes > b.cap) {
    if (b.p) {
      (void)hipDeviceSynchronize();
      (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.cap = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) return nullptr;
    b.cap = bytes;
  }
  return b.p;
}

static int32_t* scratch_count(int64_t n) {
  return static_cast<int32_t*>(thread_buffer(kCountBuffer, sizeof(int32_t) * size_t(n)));
}

// Grow the persistent-schedule scratch to n queries (the only allocation of an
// IIB join; skipped when an earlier join was at least as large).
static knnj_status ensure_join_scratch(Index* ix, int64_t n) {
  // both small buffers or neither: a failed pair is released so a later call retries
  if (ix->js_small == nullptr || ix->js_heads == nullptr) {
    (void)hipFree(ix->js_small);
    (void)hipFree(ix->js_heads);
    ix->js_small = nullptr;
    ix->js_heads = nullptr;
    if (hipMalloc(&ix->js_small, sizeof(uint32_t) * 64) != hipSuccess ||
        hipMalloc(&ix->js_heads, sizeof(uint32_t) * 2 * size_t(ix->n_tiles)) != hipSuccess) {
      (void)hipFree(ix->js_small);
      (void)hipFree(ix->js_heads);
      ix->js_small = nullptr;
      ix->js_heads = nullptr;
      return fail(KNNJ_ENOMEM, "join scratch allocation failed");
    }
  }
  if (n <= ix->js_cap) return KNNJ_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(ix->js_order);
  (void)hipFree(ix->js_bucket);
  ix->js_order = nullptr;
  ix->js_bucket = nullptr;
  ix->js_cap = 0;
  if (hipMalloc(&ix->js_order, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&ix->js_bucket, sizeof(uint32_t) * n) != hipSuccess)
    return fail(KNNJ_ENOMEM, "join scratch allocation failed");
  ix->js_cap = n;
  return KNNJ_OK;
}

// Schedule over `n` positions of `order` (or a device count when count != nullptr),
// using per-tile counter bank `bank` (0 or 1).
Sched make_sched(Index* ix, int64_t n, const int32_t* order, const uint32_t* count, int bank) {
  Sched s;
  s.head = ix->js_heads + size_t(bank) * ix->n_tiles;
  s.order = order;
  s.count = count;
  s.n = n;
  return s;
}

knnj_status reset_sched(Index* ix, int bank, hipStream_t st) {
  return launch_fill_u32(ix->js_heads + size_t(bank) * ix->n_tiles, ix->n_tiles, 0u, st);
}

}  // extern "C"

namespace knnj {

// knnj_join, and the blocked join's per-block join: with init_out false the
// outputs already hold each query's list (ids below this index's rows) and the
// join merges into it, starting from its k-th score.
knnj_status join_impl(const knnj_index* h, const knnj_csr* R, int32_t k, const knnj_join_opts* opt, int32_t* ids,
                      void* sc, int32_t* cnt, void* stream, bool init_out) {
  if (!h) return fail(KNNJ_EINVAL, "index is NULL");
  Index* ix = impl(h);
  knnj_status rc = check_device(ix->device, "the index");
  if (rc != KNNJ_OK) return rc;
  if ((rc = check_join_args(R, k, ids, sc, ix->n_dims, ix->dtype)) != KNNJ_OK) return rc;
  knnj_join_opts o;
  memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.algo != KNNJ_IIB && o.algo != KNNJ_IIIB) return fail(KNNJ_EINVAL, "unknown algo");
  if (o.r_block_rows < 0) return fail(KNNJ_EINVAL, "r_block_rows must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  if (o.r_max_row_nnz < 0 || o.r_max_row_nnz > kMaxRowNnz) return fail(KNNJ_EINVAL, "r_max_row_nnz out of range");
  if (o.tiles_per_launch < 0) return fail(KNNJ_EINVAL, "tiles_per_launch must be >= 0");
  int32_t max_r = o.r_max_row_nnz > 0 ? o.r_max_row_nnz : kMaxRowNnz;
  if (!(o.flags & KNNJ_FLAG_NO_VALIDATE)) {
    if ((rc = validate_csr(R, ix->dev_err, st, &max_r)) != KNNJ_OK) return rc;
  }
  if ((rc = overflow_check(ix->dtype, max_r, ix->max_row_nnz)) != KNNJ_OK) return rc;
  if (R->n_rows == 0) return KNNJ_OK;
  if (!init_out && !cnt) return fail(KNNJ_EINVAL, "a continued join needs out_count");
  if (!cnt && !(cnt = scratch_count(R->n_rows))) return fail(KNNJ_ENOMEM, "count buffer allocation failed");
  if (init_out && (rc = launch_init_out(R->n_rows, k, ids, sc, cnt, st)) != KNNJ_OK) return rc;
  uint64_t* slots = nullptr;
  if (o.stats) {
    slots = ix->stat_slots;
    if ((rc = launch_fill_u32(reinterpret_cast<uint32_t*>(slots), 2 * 256 * KNNJ_STAT_COUNT, 0u, st)) != KNNJ_OK)
      return rc;
  }
  // longest-first query order (cost = the query's IIB postings), used by every schedule
  if ((rc = ensure_join_scratch(ix, R->n_rows)) != KNNJ_OK) return rc;
  if ((rc = launch_lpt_order(R->n_rows, R->indptr, R->indices, ix->list_len, ix->js_bucket, ix->js_small,
                             ix->js_order, st)) != KNNJ_OK)
    return rc;
  if (o.algo == KNNJ_IIB) {
    if (o.flags & KNNJ_FLAG_PERSISTENT) {
      if ((rc = reset_sched(ix, 0, st)) != KNNJ_OK) return rc;
      rc = launch_iib_persistent(ix, R, k, make_sched(ix, R->n_rows, ix->js_order, nullptr, 0), ids, sc, cnt, slots,
                                 st);
    } else if (ix->head_h > 0 && !(o.flags & KNNJ_FLAG_NO_DENSE_HEAD) &&
               head_smem_bytes(ix->tile, k, ix->head_h, ix->dtype) <= size_t(device_max_smem(ix->device))) {
      // (a k too large for the dense-head kernel's local memory takes the plain walk)
      rc = launch_iib_head(ix, R, k, ix->js_order, o.tiles_per_launch, ids, sc, cnt, slots, st);
    } else {
      rc = launch_iib(ix, R, k, ix->js_order, ids, sc, cnt, slots, st);
    }
  } else {
    rc = launch_iiib(ix, R, k, &o, ix->js_order, max_r, ids, sc, cnt, slots, st);
  }
  if (rc != KNNJ_OK) return rc;
  if (o.stats && (rc = launch_reduce_stats(slots, o.stats, st)) != KNNJ_OK) return rc;
  return KNNJ_OK;
}

}  // namespace knnj

extern "C" {

knnj_status knnj_join(const knnj_index* h, const knnj_csr* R, int32_t k, const knnj_join_opts* opt, int32_t* ids,
                      void* sc, int32_t* cnt, void* stream) {
  g_last_error.clear();
  return join_impl(h, R, k, opt, ids, sc, cnt, stream, true);
}

knnj_status knnj_join_bf(const knnj_csr* S, const knnj_csr* R, int32_t k, int32_t* ids, void* sc, int32_t* cnt,
                         void* stream) {
  g_last_error.clear();
  knnj_status rc = check_csr_host(S, "S");
  if (rc != KNNJ_OK) return rc;
  if ((rc = check_join_args(R, k, ids, sc, S->n_dims, S->dtype)) != KNNJ_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  int32_t* err = static_cast<int32_t*>(thread_buffer(kBfErrBuffer, 4 * sizeof(int32_t)));
  if (!err) return fail(KNNJ_ENOMEM, "allocation failed");
  int32_t max_s = 0, max_r = 0;
  if ((rc = validate_csr(S, err, st, &max_s)) != KNNJ_OK) return rc;
  if ((rc = validate_csr(R, err, st, &max_r)) != KNNJ_OK) return rc;
  if ((rc = overflow_check(S->dtype, max_r, max_s)) != KNNJ_OK) return rc;
  if (R->n_rows == 0) return KNNJ_OK;
  if (!cnt && !(cnt = scratch_count(R->n_rows))) return fail(KNNJ_ENOMEM, "count buffer allocation failed");
  if ((rc = launch_init_out(R->n_rows, k, ids, sc, cnt, st)) != KNNJ_OK) return rc;
  return launch_bf(S, R, k, ids, sc, cnt, st);
}

}  // extern "C"
