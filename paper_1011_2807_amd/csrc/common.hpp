// Shared device helpers and the library's internal types.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/knnj.h"

namespace knnj {

constexpr int kWave = 64;
constexpr int kBlock = 256;           // threads per workgroup for most kernels
constexpr int kMaxK = 1024;           // largest k accepted by the join
constexpr int kSegChunk = kBlock;     // query features staged per pass of the postings walk
constexpr int kPostPad = 8;           // zeroed entries after the postings (vector loads past the end)
constexpr int kMaxRowNnz = 4096;      // longest row accepted
constexpr int kLevels = 64;           // IIIB threshold levels

// Status helper: record a message for knnj_last_error and return the code.
knnj_status fail(knnj_status code, const std::string& msg);

#define KNNJ_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::knnj::fail(KNNJ_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// The opaque index (Algorithm 3's inverted lists split by S tile).
struct Index {
  int64_t n_rows = 0;
  int32_t n_dims = 0;
  int32_t dtype = KNNJ_U8;
  int64_t nnz = 0;
  int32_t tile = 0;      // T
  int32_t log2_tile = 0;
  int32_t n_tiles = 0;
  int32_t max_row_nnz = 0;
  int device = 0;
  // offsets[t * n_dims + d] .. offsets[t * n_dims + d + 1] is list (t, d)
  int64_t* offsets = nullptr;
  // u8: one uint32 per entry, (s_local << 16) | (w << 8); f32: s_local uint16 + weight float
  uint32_t* post_u8 = nullptr;
  uint16_t* post_s = nullptr;
  float* post_w = nullptr;
  uint32_t* list_len = nullptr;  // |I_d| over all of S
  // dense head (optional): the head_h dimensions with the longest lists, per tile
  // as [head_h / E][T][E] weights of the index's value type, E = 16 bytes / weight size
  int32_t head_h = 0;
  int32_t* head_pos = nullptr;   // rank of d among the head dimensions, or -1
  uint8_t* head_blk = nullptr;
  // join scratch of the dense-head join (grow-only): per query, its tail
  // features moved to the front of its CSR row (d, w) and their count, and its
  // head weights as a dense row of head_h weights (uint8 or float32 buffers)
  int64_t hj_cap_q = 0, hj_cap_nnz = 0;
  uint32_t* hj_cnt = nullptr;
  int32_t* hj_d = nullptr;
  uint8_t* hj_w = nullptr;
  uint8_t* hj_rh = nullptr;
  // private copy of S (forward lists), used by the IIIB refinement
  int64_t* s_indptr = nullptr;
  int32_t* s_indices = nullptr;
  void* s_values = nullptr;
  // IIIB index of the current R block (rebuilt per block, allocated on first use)
  uint32_t* iiib_post = nullptr;     // u8 entries (s_local << 16) | (w << 8) | level, lists in level-desc order
  uint16_t* iiib_post_s = nullptr;   // f32 s_local, same order
  float* iiib_post_w = nullptr;      // f32 weights, same order
  uint32_t* iiib_fwd = nullptr;      // each S row in the block's dimension order (see iiib.hip)
  float* iiib_fwd_w = nullptr;       // f32 weights of iiib_fwd
  uint32_t* iiib_cut = nullptr;      // [(tile, d), level]: entries of list (tile, d) with level >= that level
  uint32_t* iiib_freq = nullptr;     // freq_d(B_r)
  uint32_t* iiib_maxw = nullptr;     // maxWeight_d(B_r) (value bits)
  int64_t* iiib_big = nullptr;       // lists queued for the long-list sorts
  uint32_t* iiib_small = nullptr;    // [0] queued long lists, [1] fallback queue length
  uint64_t* iiib_out_tmp = nullptr;  // sort scratch (8 bytes per entry)
  int32_t* iiib_qlist = nullptr;     // fallback queue
  float* iiib_seed2 = nullptr;       // fallback seeds (proven lower bounds)
  int64_t iiib_qcap = 0;
  uint64_t* rec_tmp = nullptr;       // build scratch (8 bytes per entry)
  // join scratch of the persistent schedule (grow-only: allocated when a join has
  // more queries than any earlier one)
  int64_t js_cap = 0;
  int32_t* js_order = nullptr;       // query order (longest first)
  uint32_t* js_bucket = nullptr;     // cost bucket per query
  uint32_t* js_heads = nullptr;      // per-tile queue counters [n_tiles]
  uint32_t* js_small = nullptr;      // [0, 64) cost histogram
  // small persistent scratch
  int32_t* dev_err = nullptr;        // validation result
  uint64_t* stat_slots = nullptr;    // spread counters, reduced into caller stats
};

// Element-type traits for the value arrays.
template <typename V>
struct ScoreOf;
template <>
struct ScoreOf<uint8_t> {
  using T = uint32_t;
};
template <>
struct ScoreOf<float> {
  using T = float;
};
// Type of the local-memory score map of the IIB / IIIB tile kernels: exact
// uint32 sums for uint8 data; fp64 for float32 data (a product of two floats is
// exact in fp64, and fp64 local-memory atomics run far faster on gfx950 than
// fp32 ones).  Selection and outputs use the fp32 rounding of each fp64 sum.
template <typename V>
struct AccOf;
template <>
struct AccOf<uint8_t> {
  using T = uint32_t;
};
template <>
struct AccOf<float> {
  using T = double;
};
inline size_t acc_bytes(int dtype) { return dtype == KNNJ_U8 ? 4 : 8; }

__device__ __forceinline__ uint32_t score_bits(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t score_bits(float v) { return __float_as_uint(v); }

// Slot of row s_local in a swizzled score array: the low five address bits are
// XORed with the next five, so lanes that touch rows a fixed stride apart (4 to
// 32 rows) land in different LDS banks.  The map is its own inverse.  IIB and
// IIIB postings store this slot for their row.
__device__ __forceinline__ uint32_t swz(uint32_t s) { return s ^ ((s >> 5) & 31u); }

// Block-wide exclusive scan of one uint32 per thread (kBlock threads).
// `tmp` needs kBlock / kWave + 1 words of shared memory.  Returns the exclusive
// prefix; *total gets the block sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) tmp[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      uint32_t t = tmp[w];
      tmp[w] = s;
      s += t;
    }
    tmp[kBlock / kWave] = s;
  }
  __syncthreads();
  uint32_t r = tmp[wid] + x - v;
  *total = tmp[kBlock / kWave];
  __syncthreads();
  return r;
}

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* tmp) {
  uint32_t total;
  (void)block_exclusive_scan(v, tmp, &total);
  return total;
}

}  // namespace knnj
