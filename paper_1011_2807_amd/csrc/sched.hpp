// Persistent schedule of one S tile of a join (one step of Algorithm 1's inner
// loop).  The launch holds as many workgroups as the device keeps resident; they
// take queries from a device counter in chunks of kChunk positions of a query
// order (longest first), so queries of very different lengths still balance.
// Every query appears once per tile, so items of one launch are independent;
// consecutive tiles are ordered by the launches themselves.
#pragma once

#include "common.hpp"

namespace knnj {

constexpr uint32_t kChunk = 1;

struct Sched {
  uint32_t* head;         // per-tile counters, 0 before the join
  const int32_t* order;   // query at position i, or nullptr for the identity
  const uint32_t* count;  // number of positions (device), or nullptr: use n
  int64_t n;              // number of positions when count is nullptr
};

// Positions [*first, *first + kChunk) for the whole workgroup; false when none
// is left.  `slot` is one word of shared memory.
__device__ __forceinline__ bool sched_chunk(const Sched& s, int32_t tile, int64_t* first, int64_t* n_out,
                                            uint32_t* slot) {
  const int64_t n = s.count ? int64_t(*s.count) : s.n;
  if (threadIdx.x == 0) slot[0] = atomicAdd(&s.head[tile], kChunk);
  __syncthreads();
  const int64_t f = int64_t(slot[0]);
  __syncthreads();
  *first = f;
  *n_out = n;
  return f < n;
}

__device__ __forceinline__ int64_t sched_query(const Sched& s, int64_t pos) {
  return s.order ? int64_t(s.order[pos]) : pos;
}

}  // namespace knnj
