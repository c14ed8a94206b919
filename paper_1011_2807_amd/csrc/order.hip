// Query order for the persistent schedule: longest processing time first.
// The cost of a query is sum over its features of |I_d| (its share of the
// second term of Eq. 4, the postings IIB walks); queries are bucketed by
// floor(log2(cost + 1)) and placed in descending bucket order (counting sort;
// order inside a bucket is arbitrary).
#include "common.hpp"

namespace knnj {

constexpr int kCostBuckets = 64;

// Grid-stride fill: a dispatch counts its work-items in 32 bits, so the grid is
// capped and each thread covers every (grid size)-th word (the IIIB cut table
// alone exceeds 2^32 words at 10M rows x 100K dimensions).
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) p[i] = v;
}

__device__ __forceinline__ uint32_t cost_bucket(uint64_t c) {
  const uint32_t lg = 63u - uint32_t(__clzll(c + 1ull));  // floor(log2(c + 1))
  return uint32_t(kCostBuckets - 1) - lg;                 // descending cost
}

__device__ __forceinline__ uint64_t query_cost(int64_t q, const int64_t* r_ptr, const int32_t* r_idx,
                                               const uint32_t* list_len) {
  uint64_t c = 0;
  for (int64_t j = r_ptr[q]; j < r_ptr[q + 1]; ++j) c += list_len[r_idx[j]];
  return c;
}

// hist[kCostBuckets] must be 0
__global__ void k_cost_hist(int64_t n, const int64_t* __restrict__ r_ptr, const int32_t* __restrict__ r_idx,
                            const uint32_t* __restrict__ list_len, uint32_t* __restrict__ bucket,
                            uint32_t* __restrict__ hist) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const uint32_t b = cost_bucket(query_cost(q, r_ptr, r_idx, list_len));
  bucket[q] = b;
  atomicAdd(&hist[b], 1u);
}

__global__ void k_cost_scan(uint32_t* hist) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int b = 0; b < kCostBuckets; ++b) {
    const uint32_t v = hist[b];
    hist[b] = run;
    run += v;
  }
}

__global__ void k_cost_scatter(int64_t n, const uint32_t* __restrict__ bucket, uint32_t* __restrict__ cursor,
                               int32_t* __restrict__ order) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  order[atomicAdd(&cursor[bucket[q]], 1u)] = int32_t(q);
}

knnj_status launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  constexpr int64_t kMaxFillBlocks = int64_t(1) << 20;
  const int64_t nb = (n + kBlock - 1) / kBlock;
  if (n > 0) k_fill_u32<<<unsigned(nb < kMaxFillBlocks ? nb : kMaxFillBlocks), kBlock, 0, st>>>(p, n, v);
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

// order[0..n) = queries by descending cost; scratch: bucket uint32[n], hist uint32[64]
knnj_status launch_lpt_order(int64_t n, const int64_t* r_ptr, const int32_t* r_idx, const uint32_t* list_len,
                             uint32_t* bucket, uint32_t* hist, int32_t* order, hipStream_t st) {
  if (n <= 0) return KNNJ_OK;
  knnj_status rc = launch_fill_u32(hist, kCostBuckets, 0u, st);
  if (rc != KNNJ_OK) return rc;
  const unsigned g = unsigned((n + kBlock - 1) / kBlock);
  k_cost_hist<<<g, kBlock, 0, st>>>(n, r_ptr, r_idx, list_len, bucket, hist);
  k_cost_scan<<<1, 64, 0, st>>>(hist);
  k_cost_scatter<<<g, kBlock, 0, st>>>(n, bucket, hist, order);
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

}  // namespace knnj
