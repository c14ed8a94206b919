// IIB join (Algorithm 3, Find_Matches_IIB) and the brute-force join
// (Algorithm 2) on one S tile at a time.
//
// One workgroup owns one query r for one tile t.  Its score map A (the map of
// Algorithm 3) is a dense array acc[T] in local memory indexed by s_local; the
// postings walk adds r[d] * w to acc[s_local] with local-memory atomics, which
// are exact for integer scores.  The lists (t, d) of all features of r are
// walked as one concatenated sequence of 16-byte groups shared out over teams of
// lanes (see walk_lists), so lanes stay busy even when most lists are short.
#include "sched.hpp"
#include "walk.hpp"

namespace knnj {

// local memory of the IIB tile kernels: score map (acc_b bytes per row) + stage
size_t tile_smem_bytes(int tile, int k, size_t acc_b) { return size_t(tile) * acc_b + stage_bytes(k); }

__global__ void k_init_out(int64_t n, int32_t* ids, uint32_t* sc, int64_t n_rows, int32_t* cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    ids[i] = -1;
    sc[i] = 0u;
  }
  if (i < n_rows) cnt[i] = 0;
}

__global__ void k_reduce_stats(const uint64_t* slots, int n_slots, uint64_t* out) {
  // one workgroup per counter; slots laid out [counter][n_slots]
  __shared__ uint64_t part[kBlock];
  uint64_t s = 0;
  for (int i = threadIdx.x; i < n_slots; i += kBlock) s += slots[int64_t(blockIdx.x) * n_slots + i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && part[0] != 0) atomicAdd((unsigned long long*)&out[blockIdx.x], (unsigned long long)part[0]);
}

// IIB for query q on tile `tile` (one workgroup).  acc: T scores in local
// memory; stage: the list table / selection workspace; tmp: scan scratch.
template <typename V>
__device__ __forceinline__ uint64_t iib_item(int32_t tile, int64_t q, int32_t log2_tile, int32_t n_dims, int32_t k,
                                             const int64_t* __restrict__ r_ptr, const int32_t* __restrict__ r_idx,
                                             const V* __restrict__ r_val, const int64_t* __restrict__ offsets,
                                             Postings<V> P, int32_t* __restrict__ out_ids,
                                             typename ScoreOf<V>::T* __restrict__ out_sc, int32_t* __restrict__ out_cnt,
                                             bool count, typename AccOf<V>::T* acc, char* stage, uint32_t* tmp) {
  using S = typename ScoreOf<V>::T;
  using A = typename AccOf<V>::T;
  const int T = 1 << log2_tile;
  const int64_t s_base = int64_t(tile) << log2_tile;
  // rows past the end of S have no postings, so their slots stay 0
  for (int i = threadIdx.x; i < int(T * sizeof(A) / 16); i += kBlock)
    reinterpret_cast<uint4*>(acc)[i] = make_uint4(0, 0, 0, 0);
  const int64_t rb = r_ptr[q], re = r_ptr[q + 1];
  const int64_t key0 = int64_t(tile) * n_dims;
  uint64_t walked = 0;
  for (int64_t cb = rb; cb < re; cb += kSegChunk) {
    const int n = int(re - cb < kSegChunk ? re - cb : kSegChunk);
    const uint32_t total = stage_lists<V, S>(stage, tmp, key0, r_idx, r_val, cb, n, offsets);
    walk_lists<V, S, false, A>(acc, stage, n, total, P);
    if (count) {
      // exact entries walked: sum of list lengths of this pass
      uint32_t l = threadIdx.x < n ? reinterpret_cast<const uint32_t*>(stage + kMetaOff)[threadIdx.x] >> 2 : 0u;
      walked += block_sum(l, tmp);
    }
    __syncthreads();
  }
  tile_select<S, true, A>(acc, T, s_base, k, out_ids + q * k, out_sc + q * k, out_cnt + q,
                          select_smem(stage, k, tmp));
  return walked;
}

// One launch per tile: workgroup b joins query order[q0 + b] (or q0 + b).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_iib_tile(int32_t tile, int32_t log2_tile, int64_t n_s, int32_t n_dims,
                                                     int32_t k, int64_t q0, const int32_t* __restrict__ order,
                                                     const int64_t* __restrict__ r_ptr,
                                                     const int32_t* __restrict__ r_idx, const V* __restrict__ r_val,
                                                     const int64_t* __restrict__ offsets, Postings<V> P,
                                                     int32_t* __restrict__ out_ids,
                                                     typename ScoreOf<V>::T* __restrict__ out_sc,
                                                     int32_t* __restrict__ out_cnt, uint64_t* __restrict__ slots) {
  using A = typename AccOf<V>::T;
  extern __shared__ __align__(16) char smem[];
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  (void)n_s;
  A* acc = reinterpret_cast<A*>(smem);
  char* stage = smem + (sizeof(A) << log2_tile);
  const int64_t q = order ? int64_t(order[q0 + blockIdx.x]) : q0 + blockIdx.x;
  const uint64_t walked = iib_item<V>(tile, q, log2_tile, n_dims, k, r_ptr, r_idx, r_val, offsets, P,
                                      out_ids, out_sc, out_cnt, slots != nullptr, acc, stage, tmp);
  if (threadIdx.x == 0 && slots) atomicAdd((unsigned long long*)&slots[KNNJ_STAT_POSTINGS * 256 + (blockIdx.x & 255)],
                                           (unsigned long long)walked);
}

// Persistent launch for tile `tile` (see sched.hpp).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_iib_persistent(Sched sch, int32_t tile, int32_t log2_tile, int32_t n_dims,
                                                           int32_t k, const int64_t* __restrict__ r_ptr,
                                                           const int32_t* __restrict__ r_idx,
                                                           const V* __restrict__ r_val,
                                                           const int64_t* __restrict__ offsets, Postings<V> P,
                                                           int32_t* __restrict__ out_ids,
                                                           typename ScoreOf<V>::T* __restrict__ out_sc,
                                                           int32_t* __restrict__ out_cnt, uint64_t* __restrict__ slots) {
  using A = typename AccOf<V>::T;
  extern __shared__ __align__(16) char smem[];
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  __shared__ uint32_t slot[1];
  A* acc = reinterpret_cast<A*>(smem);
  char* stage = smem + (sizeof(A) << log2_tile);
  uint64_t walked = 0;
  int64_t first, n;
  while (sched_chunk(sch, tile, &first, &n, slot)) {
    for (int64_t p = first; p < first + kChunk && p < n; ++p)
      walked += iib_item<V>(tile, sched_query(sch, p), log2_tile, n_dims, k, r_ptr, r_idx, r_val, offsets, P, out_ids,
                            out_sc, out_cnt, slots != nullptr, acc, stage, tmp);
  }
  if (threadIdx.x == 0 && slots) atomicAdd((unsigned long long*)&slots[KNNJ_STAT_POSTINGS * 256 + (blockIdx.x & 255)],
                                           (unsigned long long)walked);
}

// Brute force (Algorithm 2): scores of rows [s0, s0 + T) of S by a two-pointer
// merge of r (staged in local memory) with each s; one thread per s.  The sum
// runs in the score map type of the tile kernels (fp64 for float32 data, where
// each product is exact) and is stored rounded to the output type.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_bf(int32_t log2_tile, int64_t n_s, int32_t k, int64_t q0,
                                               const int64_t* __restrict__ r_ptr, const int32_t* __restrict__ r_idx,
                                               const V* __restrict__ r_val, const int64_t* __restrict__ s_ptr,
                                               const int32_t* __restrict__ s_idx, const V* __restrict__ s_val,
                                               int32_t* __restrict__ out_ids,
                                               typename ScoreOf<V>::T* __restrict__ out_sc,
                                               int32_t* __restrict__ out_cnt) {
  using S = typename ScoreOf<V>::T;
  using A = typename AccOf<V>::T;
  extern __shared__ __align__(16) char smem[];
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  __shared__ int32_t rd[kMaxRowNnz];
  __shared__ S rw[kMaxRowNnz];
  const int T = 1 << log2_tile;
  S* acc = reinterpret_cast<S*>(smem);
  char* stage = smem + size_t(T) * 4;
  const int64_t q = q0 + blockIdx.x;
  const int64_t rb = r_ptr[q];
  const int nr = int(r_ptr[q + 1] - rb);
  for (int i = threadIdx.x; i < nr; i += kBlock) {
    rd[i] = r_idx[rb + i];
    rw[i] = S(r_val[rb + i]);
  }
  __syncthreads();
  const SelectSmem sm = select_smem(stage, k, tmp);
  for (int64_t s0 = 0; s0 < n_s; s0 += T) {
    const int n_valid = int(n_s - s0 < T ? n_s - s0 : T);
    for (int i = threadIdx.x; i < n_valid; i += kBlock) {
      const int64_t sb = s_ptr[s0 + i], se = s_ptr[s0 + i + 1];
      A ret = A(0);
      int a = 0;
      int64_t b = sb;
      while (a < nr && b < se) {
        const int32_t dr = rd[a], ds = s_idx[b];
        if (dr == ds) {
          ret += A(rw[a]) * A(s_val[b]);
          ++a;
          ++b;
        } else if (dr > ds) {
          ++b;
        } else {
          ++a;
        }
      }
      acc[i] = S(ret);
    }
    __syncthreads();
    tile_select<S, false>(acc, n_valid, s0, k, out_ids + q * k, out_sc + q * k, out_cnt + q, sm);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- host launchers
knnj_status launch_init_out(int64_t n_rows, int32_t k, int32_t* ids, void* sc, int32_t* cnt, hipStream_t st) {
  const int64_t n = n_rows * int64_t(k);
  const int64_t m = n > n_rows ? n : n_rows;
  if (m > 0) k_init_out<<<unsigned((m + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, ids, (uint32_t*)sc, n_rows, cnt);
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

knnj_status launch_reduce_stats(const uint64_t* slots, uint64_t* out, hipStream_t st) {
  k_reduce_stats<<<KNNJ_STAT_COUNT, kBlock, 0, st>>>(slots, 256, out);
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

static const int64_t kMaxGrid = 1ll << 30;

knnj_status launch_iib(const Index* ix, const knnj_csr* R, int32_t k, const int32_t* order, int32_t* ids, void* sc,
                       int32_t* cnt, uint64_t* slots, hipStream_t st) {
  const size_t smem = tile_smem_bytes(ix->tile, k, acc_bytes(ix->dtype));
  for (int32_t t = 0; t < ix->n_tiles; ++t) {
    for (int64_t q0 = 0; q0 < R->n_rows; q0 += kMaxGrid) {
      const unsigned g = unsigned(R->n_rows - q0 < kMaxGrid ? R->n_rows - q0 : kMaxGrid);
      if (ix->dtype == KNNJ_U8) {
        Postings<uint8_t> P{reinterpret_cast<const uint4*>(ix->post_u8)};
        k_iib_tile<uint8_t><<<g, kBlock, smem, st>>>(t, ix->log2_tile, ix->n_rows, ix->n_dims, k, q0, order, R->indptr,
                                                     R->indices, (const uint8_t*)R->values, ix->offsets, P, ids,
                                                     (uint32_t*)sc, cnt, slots);
      } else {
        Postings<float> P{reinterpret_cast<const uint2*>(ix->post_s), reinterpret_cast<const float4*>(ix->post_w)};
        k_iib_tile<float><<<g, kBlock, smem, st>>>(t, ix->log2_tile, ix->n_rows, ix->n_dims, k, q0, order, R->indptr,
                                                   R->indices, (const float*)R->values, ix->offsets, P, ids,
                                                   (float*)sc, cnt, slots);
      }
    }
  }
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

// Workgroups of the persistent launch: every CU filled to its occupancy.
template <typename K>
static unsigned persistent_grid(K kernel, size_t smem, int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, smem) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  return unsigned(per_cu * cus);
}

knnj_status launch_iib_persistent(const Index* ix, const knnj_csr* R, int32_t k, const Sched& sch, int32_t* ids,
                                  void* sc, int32_t* cnt, uint64_t* slots, hipStream_t st) {
  const size_t smem = tile_smem_bytes(ix->tile, k, acc_bytes(ix->dtype));
  if (ix->dtype == KNNJ_U8) {
    Postings<uint8_t> P{reinterpret_cast<const uint4*>(ix->post_u8)};
    const unsigned g = persistent_grid(k_iib_persistent<uint8_t>, smem, ix->device);
    for (int32_t t = 0; t < ix->n_tiles; ++t)
      k_iib_persistent<uint8_t><<<g, kBlock, smem, st>>>(sch, t, ix->log2_tile, ix->n_dims, k, R->indptr, R->indices,
                                                         (const uint8_t*)R->values, ix->offsets, P, ids,
                                                         (uint32_t*)sc, cnt, slots);
  } else {
    Postings<float> P{reinterpret_cast<const uint2*>(ix->post_s), reinterpret_cast<const float4*>(ix->post_w)};
    const unsigned g = persistent_grid(k_iib_persistent<float>, smem, ix->device);
    for (int32_t t = 0; t < ix->n_tiles; ++t)
      k_iib_persistent<float><<<g, kBlock, smem, st>>>(sch, t, ix->log2_tile, ix->n_dims, k, R->indptr, R->indices,
                                                       (const float*)R->values, ix->offsets, P, ids, (float*)sc, cnt,
                                                       slots);
  }
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

knnj_status launch_bf(const knnj_csr* S, const knnj_csr* R, int32_t k, int32_t* ids, void* sc, int32_t* cnt,
                      hipStream_t st) {
  const int log2_tile = 11;
  const size_t smem = tile_smem_bytes(1 << log2_tile, k, 4);
  for (int64_t q0 = 0; q0 < R->n_rows; q0 += kMaxGrid) {
    const unsigned g = unsigned(R->n_rows - q0 < kMaxGrid ? R->n_rows - q0 : kMaxGrid);
    if (S->dtype == KNNJ_U8)
      k_bf<uint8_t><<<g, kBlock, smem, st>>>(log2_tile, S->n_rows, k, q0, R->indptr, R->indices,
                                             (const uint8_t*)R->values, S->indptr, S->indices,
                                             (const uint8_t*)S->values, ids, (uint32_t*)sc, cnt);
    else
      k_bf<float><<<g, kBlock, smem, st>>>(log2_tile, S->n_rows, k, q0, R->indptr, R->indices,
                                           (const float*)R->values, S->indptr, S->indices, (const float*)S->values,
                                           ids, (float*)sc, cnt);
  }
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

}  // namespace knnj
