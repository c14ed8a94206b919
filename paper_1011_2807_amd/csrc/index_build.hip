// Inverted-index construction on the device (Algorithm 3,
// Create_Inverted_List_IIB), generalised to one list per (S tile, dimension).
//
//   count    : entries per key (tile, d), key = tile * n_dims + d
//   scan     : exclusive prefix -> offsets
//   scatter  : place (s_local, w) records at offsets[key] + atomic cursor
//   sort     : restore ascending s_local inside each list (three size classes)
//   finalize : pack records into the compact layout the join walks
//
// Also holds the CSR validator shared by the build and the join.
#include "common.hpp"

namespace knnj {

// ---------------------------------------------------------------- validation
// err[0]: bit flags (1 indptr, 2 index order/range, 4 value, 8 row too long)
// err[1]: longest row
template <typename V>
__global__ void k_validate(int64_t n_rows, int32_t n_dims, int64_t nnz, const int64_t* __restrict__ indptr,
                           const int32_t* __restrict__ indices, const V* __restrict__ values, int32_t* err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t n_waves = int64_t(gridDim.x) * blockDim.x / kWave;
  if (wave == 0 && lane == 0) {
    if (indptr[0] != 0 || indptr[n_rows] != nnz) atomicOr(&err[0], 1);
  }
  for (int64_t r = wave; r < n_rows; r += n_waves) {
    const int64_t b = indptr[r], e = indptr[r + 1];
    if (b < 0 || e < b || e > nnz) {
      if (lane == 0) atomicOr(&err[0], 1);
      continue;
    }
    const int64_t len = e - b;
    if (lane == 0) atomicMax(&err[1], (int32_t)(len > 0x7fffffff ? 0x7fffffff : len));
    if (len > kMaxRowNnz) {
      if (lane == 0) atomicOr(&err[0], 8);
      continue;
    }
    int bad = 0;
    for (int64_t j = b + lane; j < e; j += kWave) {
      const int32_t d = indices[j];
      if (d < 0 || d >= n_dims) bad |= 2;
      if (j + 1 < e && indices[j + 1] <= d) bad |= 2;
      const V w = values[j];
      if constexpr (sizeof(V) == 1) {
        if (w == 0) bad |= 4;
      } else {
        if (!(w > 0.0f) || !(w < INFINITY)) bad |= 4;
      }
    }
    if (bad) atomicOr(&err[0], bad);
  }
}

template __global__ void k_validate<uint8_t>(int64_t, int32_t, int64_t, const int64_t*, const int32_t*,
                                             const uint8_t*, int32_t*);
template __global__ void k_validate<float>(int64_t, int32_t, int64_t, const int64_t*, const int32_t*,
                                           const float*, int32_t*);

// ---------------------------------------------------------------- counting
__global__ void k_count_keys(int64_t n_rows, int32_t n_dims, int32_t log2_tile, const int64_t* __restrict__ indptr,
                             const int32_t* __restrict__ indices, uint32_t* __restrict__ cnt) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t n_waves = int64_t(gridDim.x) * blockDim.x / kWave;
  for (int64_t r = wave; r < n_rows; r += n_waves) {
    const int64_t base = (r >> log2_tile) * int64_t(n_dims);
    for (int64_t j = indptr[r] + lane; j < indptr[r + 1]; j += kWave) atomicAdd(&cnt[base + indices[j]], 1u);
  }
}

// ---------------------------------------------------------------- scan (u32 -> i64 exclusive)
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__global__ void k_scan_partials(const uint32_t* __restrict__ in, int64_t n, int64_t* __restrict__ partial) {
  // a list holds at most T <= 65536 entries, so a workgroup's sum (2048 lists) fits 32 bits
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  const int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  const uint32_t total = block_sum(s, tmp);
  if (threadIdx.x == 0) partial[blockIdx.x] = int64_t(total);
}

// single workgroup: exclusive scan of partial[0..n) in place, total to *total
__global__ void k_scan_top(int64_t* partial, int64_t n, int64_t* total) {
  __shared__ int64_t buf[kBlock];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b = 0; b < n; b += kBlock) {
    const int64_t i = b + threadIdx.x;
    int64_t v = i < n ? partial[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
      int64_t y = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < n) partial[i] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += buf[kBlock - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_final(const uint32_t* __restrict__ in, int64_t n, const int64_t* __restrict__ partial,
                             int64_t* __restrict__ out) {
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  const int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_scan(s, tmp, &total);
  int64_t run = partial[blockIdx.x] + ex;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

// ---------------------------------------------------------------- scatter
template <typename V>
__global__ void k_scatter(int64_t n_rows, int32_t n_dims, int32_t log2_tile, const int64_t* __restrict__ indptr,
                          const int32_t* __restrict__ indices, const V* __restrict__ values,
                          const int64_t* __restrict__ offsets, uint32_t* __restrict__ cursor,
                          uint64_t* __restrict__ rec) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t n_waves = int64_t(gridDim.x) * blockDim.x / kWave;
  const uint32_t tmask = (1u << log2_tile) - 1u;
  for (int64_t r = wave; r < n_rows; r += n_waves) {
    const int64_t base = (r >> log2_tile) * int64_t(n_dims);
    const uint64_t s_local = uint64_t(uint32_t(r) & tmask);
    for (int64_t j = indptr[r] + lane; j < indptr[r + 1]; j += kWave) {
      const int64_t key = base + indices[j];
      const uint32_t pos = atomicAdd(&cursor[key], 1u);
      uint32_t payload;
      if constexpr (sizeof(V) == 1) payload = values[j];
      else payload = __float_as_uint(values[j]);
      rec[offsets[key] + pos] = (s_local << 32) | payload;
    }
  }
}

template __global__ void k_scatter<uint8_t>(int64_t, int32_t, int32_t, const int64_t*, const int32_t*,
                                            const uint8_t*, const int64_t*, uint32_t*, uint64_t*);
template __global__ void k_scatter<float>(int64_t, int32_t, int32_t, const int64_t*, const int32_t*, const float*,
                                          const int64_t*, uint32_t*, uint64_t*);

// ---------------------------------------------------------------- per-list sort by s_local
constexpr int kSmallSort = 16;
constexpr int kMidSort = 2048;
constexpr int kSlotPass = 8192;

// Lists of <= 16 entries: insertion sort in one thread; longer ones are queued.
__global__ void k_sort_small(const int64_t* __restrict__ offsets, int64_t n_keys, uint64_t* __restrict__ rec,
                             int64_t* __restrict__ big, uint32_t* __restrict__ n_big) {
  const int64_t key = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (key >= n_keys) return;
  const int64_t b = offsets[key], e = offsets[key + 1];
  const int64_t len = e - b;
  if (len < 2) return;
  if (len > kSmallSort) {
    big[atomicAdd(n_big, 1u)] = key;
    return;
  }
  uint64_t a[kSmallSort];
  for (int i = 0; i < len; ++i) a[i] = rec[b + i];
  for (int i = 1; i < len; ++i) {
    uint64_t x = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
  for (int i = 0; i < len; ++i) rec[b + i] = a[i];
}

// Lists of 17..2048 entries: bitonic sort in local memory (ascending).  The
// grid strides over the queued lists (count on the device).
__global__ void k_sort_mid(const int64_t* __restrict__ offsets, const int64_t* __restrict__ big,
                           const uint32_t* __restrict__ n_big, uint64_t* __restrict__ rec) {
  __shared__ uint64_t buf[kMidSort];
  const uint32_t nb = *n_big;
  for (uint32_t item = blockIdx.x; item < nb; item += gridDim.x) {
    const int64_t key = big[item];
    const int64_t b = offsets[key], e = offsets[key + 1];
    const int len = int(e - b);
    if (len > kMidSort) continue;
    int p = 1;
    while (p < len) p <<= 1;
    for (int i = threadIdx.x; i < p; i += blockDim.x) buf[i] = i < len ? rec[b + i] : ~0ull;
    __syncthreads();
    for (int size = 2; size <= p; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < (p >> 1); i += blockDim.x) {
          const int lo = 2 * i - (i & (stride - 1));
          const int hi = lo + stride;
          const bool up = ((lo & size) == 0);
          const uint64_t x = buf[lo], y = buf[hi];
          if ((x > y) == up) {
            buf[lo] = y;
            buf[hi] = x;
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < len; i += blockDim.x) rec[b + i] = buf[i];
    __syncthreads();
  }
}

// Lists longer than 2048: s_local values of one list are distinct and below T,
// so place each payload in slot s_local of a local array and read the slots
// back in order (one pass per 16384 slots).  Payloads are never 0 (w > 0).
__global__ void k_sort_large(const int64_t* __restrict__ offsets, const int64_t* __restrict__ big,
                             uint64_t* __restrict__ rec, uint64_t* __restrict__ out_tmp, int32_t tile) {
  extern __shared__ uint32_t slots[];  // kSlotPass
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  __shared__ uint32_t written;
  const int64_t key = big[blockIdx.x];
  const int64_t b = offsets[key], e = offsets[key + 1];
  const int64_t len = e - b;
  if (len <= kMidSort) return;
  if (threadIdx.x == 0) written = 0;
  for (int32_t lo = 0; lo < tile; lo += kSlotPass) {
    for (int i = threadIdx.x; i < kSlotPass; i += blockDim.x) slots[i] = 0u;
    __syncthreads();
    for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) {
      const uint64_t x = rec[j];
      const int32_t s = int32_t(x >> 32);
      if (s >= lo && s < lo + kSlotPass) slots[s - lo] = uint32_t(x);
    }
    __syncthreads();
    constexpr int per = kSlotPass / kBlock;
    const int t0 = threadIdx.x * per;
    uint32_t c = 0;
    for (int i = 0; i < per; ++i) c += slots[t0 + i] != 0u;
    uint32_t total;
    uint32_t ex = block_exclusive_scan(c, tmp, &total);
    uint32_t w0 = written;
    for (int i = 0; i < per; ++i) {
      const uint32_t v = slots[t0 + i];
      if (v != 0u) out_tmp[b + w0 + ex++] = (uint64_t(uint32_t(lo + t0 + i)) << 32) | v;
    }
    __syncthreads();
    if (threadIdx.x == 0) written = w0 + total;
    __syncthreads();
  }
  __syncthreads();
  for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) rec[j] = out_tmp[j];
}

// ---------------------------------------------------------------- finalize
// Packed entries keep the row's score slot swz(s_local) (the swizzled local-memory
// slot the join accumulates into), so the walk adds at the stored slot directly.
// Grid-stride (capped grid: a dispatch counts its work-items in 32 bits).
__global__ void k_finalize_u8(const uint64_t* __restrict__ rec, int64_t n, uint32_t* __restrict__ post) {
  const int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) {
    const uint64_t x = rec[i];
    post[i] = (swz(uint32_t(x >> 32)) << 16) | ((uint32_t(x) & 0xffu) << 8);
  }
}

__global__ void k_finalize_f32(const uint64_t* __restrict__ rec, int64_t n, uint16_t* __restrict__ ps,
                               float* __restrict__ pw) {
  const int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) {
    const uint64_t x = rec[i];
    ps[i] = uint16_t(swz(uint32_t(x >> 32)));
    pw[i] = __uint_as_float(uint32_t(x));
  }
}

__global__ void k_list_lengths(const uint32_t* __restrict__ cnt, int32_t n_dims, int32_t n_tiles,
                               uint32_t* __restrict__ len) {
  const int32_t d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n_dims) return;
  uint32_t s = 0;
  for (int32_t t = 0; t < n_tiles; ++t) s += cnt[int64_t(t) * n_dims + d];
  len[d] = s;
}

// ---------------------------------------------------------------- host drivers
static unsigned grid_for(int64_t n, int per_block, unsigned cap = 1u << 20) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

knnj_status validate_csr(const knnj_csr* m, int32_t* dev_err, hipStream_t st, int32_t* max_row) {
  KNNJ_HIP(hipMemsetAsync(dev_err, 0, 2 * sizeof(int32_t), st));
  if (m->n_rows > 0) {
    const unsigned g = grid_for(m->n_rows, kBlock / kWave, 65536);
    if (m->dtype == KNNJ_U8)
      k_validate<uint8_t><<<g, kBlock, 0, st>>>(m->n_rows, m->n_dims, m->nnz, m->indptr, m->indices,
                                                (const uint8_t*)m->values, dev_err);
    else
      k_validate<float><<<g, kBlock, 0, st>>>(m->n_rows, m->n_dims, m->nnz, m->indptr, m->indices,
                                              (const float*)m->values, dev_err);
    KNNJ_HIP(hipGetLastError());
  }
  int32_t h[2] = {0, 0};
  KNNJ_HIP(hipMemcpyAsync(h, dev_err, sizeof(h), hipMemcpyDeviceToHost, st));
  KNNJ_HIP(hipStreamSynchronize(st));
  if (h[0] & 1) return fail(KNNJ_EINVAL, "CSR indptr is not a valid row pointer array");
  if (h[0] & 8) return fail(KNNJ_EINVAL, "a row has more than 4096 features");
  if (h[0] & 2) return fail(KNNJ_EINVAL, "CSR indices must be strictly ascending within a row and in [0, n_dims)");
  if (h[0] & 4) return fail(KNNJ_EINVAL, "CSR values must be > 0 (and finite for float32)");
  if (max_row) *max_row = h[1];
  return KNNJ_OK;
}

knnj_status exclusive_scan_u32(const uint32_t* in, int64_t n, int64_t* out, int64_t* partial, hipStream_t st) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  k_scan_partials<<<unsigned(nb), kBlock, 0, st>>>(in, n, partial);
  k_scan_top<<<1, kBlock, 0, st>>>(partial, nb, out + n);
  k_scan_final<<<unsigned(nb), kBlock, 0, st>>>(in, n, partial, out);
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

// Builds offsets + postings of `ix` from CSR arrays already resident on the device.
knnj_status build_postings(Index* ix, const int64_t* indptr, const int32_t* indices, const void* values,
                           hipStream_t st) {
  const int64_t n_keys = int64_t(ix->n_tiles) * ix->n_dims;
  uint32_t* cnt = nullptr;
  uint32_t* cursor = nullptr;
  int64_t* partial = nullptr;
  int64_t* big = nullptr;
  uint32_t* n_big = nullptr;
  uint64_t* tmp2 = nullptr;
  knnj_status rc = KNNJ_OK;
  const int64_t nb = (n_keys + kScanTile - 1) / kScanTile;
  auto cleanup = [&]() {
    (void)hipFree(cnt);
    (void)hipFree(cursor);
    (void)hipFree(partial);
    (void)hipFree(big);
    (void)hipFree(n_big);
    (void)hipFree(tmp2);
  };
  if (hipMalloc(&cnt, sizeof(uint32_t) * n_keys) != hipSuccess ||
      hipMalloc(&cursor, sizeof(uint32_t) * n_keys) != hipSuccess ||
      hipMalloc(&partial, sizeof(int64_t) * (nb + 1)) != hipSuccess ||
      hipMalloc(&big, sizeof(int64_t) * n_keys) != hipSuccess || hipMalloc(&n_big, sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&ix->offsets, sizeof(int64_t) * (n_keys + 1)) != hipSuccess ||
      hipMalloc(&ix->list_len, sizeof(uint32_t) * ix->n_dims) != hipSuccess ||
      hipMalloc(&ix->rec_tmp, sizeof(uint64_t) * (ix->nnz > 0 ? ix->nnz : 1)) != hipSuccess ||
      hipMalloc(&tmp2, sizeof(uint64_t) * (ix->nnz > 0 ? ix->nnz : 1)) != hipSuccess) {
    cleanup();
    return fail(KNNJ_ENOMEM, "device allocation for the index failed");
  }
  do {
    if (hipMemsetAsync(cnt, 0, sizeof(uint32_t) * n_keys, st) != hipSuccess ||
        hipMemsetAsync(cursor, 0, sizeof(uint32_t) * n_keys, st) != hipSuccess ||
        hipMemsetAsync(n_big, 0, sizeof(uint32_t), st) != hipSuccess) {
      rc = fail(KNNJ_EDEVICE, "hipMemsetAsync failed");
      break;
    }
    const unsigned gr = grid_for(ix->n_rows, kBlock / kWave, 65536);
    if (ix->n_rows > 0)
      k_count_keys<<<gr, kBlock, 0, st>>>(ix->n_rows, ix->n_dims, ix->log2_tile, indptr, indices, cnt);
    if ((rc = exclusive_scan_u32(cnt, n_keys, ix->offsets, partial, st)) != KNNJ_OK) break;
    k_list_lengths<<<grid_for(ix->n_dims, kBlock), kBlock, 0, st>>>(cnt, ix->n_dims, ix->n_tiles, ix->list_len);
    if (ix->n_rows > 0) {
      if (ix->dtype == KNNJ_U8)
        k_scatter<uint8_t><<<gr, kBlock, 0, st>>>(ix->n_rows, ix->n_dims, ix->log2_tile, indptr, indices,
                                                  (const uint8_t*)values, ix->offsets, cursor, ix->rec_tmp);
      else
        k_scatter<float><<<gr, kBlock, 0, st>>>(ix->n_rows, ix->n_dims, ix->log2_tile, indptr, indices,
                                                (const float*)values, ix->offsets, cursor, ix->rec_tmp);
    }
    k_sort_small<<<grid_for(n_keys, kBlock, 1u << 30), kBlock, 0, st>>>(ix->offsets, n_keys, ix->rec_tmp, big, n_big);
    uint32_t h_big = 0;
    if (hipMemcpyAsync(&h_big, n_big, sizeof(uint32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(KNNJ_EDEVICE, "index build: kernel failure before the list sort");
      break;
    }
    if (h_big > 0) {
      k_sort_mid<<<h_big, kBlock, 0, st>>>(ix->offsets, big, n_big, ix->rec_tmp);
      k_sort_large<<<h_big, kBlock, kSlotPass * sizeof(uint32_t), st>>>(ix->offsets, big, ix->rec_tmp, tmp2,
                                                                         ix->tile);
    }
    if (ix->nnz > 0) {
      const unsigned gf = grid_for(ix->nnz, kBlock);
      if (ix->dtype == KNNJ_U8) k_finalize_u8<<<gf, kBlock, 0, st>>>(ix->rec_tmp, ix->nnz, ix->post_u8);
      else k_finalize_f32<<<gf, kBlock, 0, st>>>(ix->rec_tmp, ix->nnz, ix->post_s, ix->post_w);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(KNNJ_EDEVICE, "index build kernels failed");
      break;
    }
  } while (0);
  cleanup();
  return rc;
}

}  // namespace knnj
