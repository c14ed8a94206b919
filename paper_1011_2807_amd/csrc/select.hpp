// Per-query top-k selection over one S tile's score array held in local
// memory, merged into the query's running list (the candidate step of
// Algorithms 2, 3 and 4).
//
// Keys: (score bits << 32) | ~id.  For int scores and for positive floats the
// bit pattern orders like the value, and ~id puts the lower id first among
// equal scores, so "larger key" is "better neighbour" under the total order
// (score desc, id asc).
//
// A tile entry can enter the list only if its score is strictly above the
// running pruneScore (the k-th score once k are held, else 0): every id of
// this tile is larger than every id already held, so an equal score loses.
#pragma once

#include "common.hpp"

namespace knnj {

// Local-memory workspace of the selection (reuses the walk's staging area).
struct SelectSmem {
  uint64_t* keys;  // cap entries
  uint32_t cap;    // power of two >= 2k
  uint32_t* hist;  // 256
  uint32_t* scal;  // 8
  uint32_t* tmp;   // kBlock / kWave + 1
};

// Selection buffer entries for a given k: a power of two >= max(256, 2k).
__host__ __device__ inline uint32_t select_cap(int k) {
  uint32_t c = 256;
  while (c < uint32_t(2 * k)) c <<= 1;
  return c;
}
__host__ __device__ inline uint32_t select_bytes(int k) { return select_cap(k) * 8u + 256u * 4u + 8u * 4u; }

__device__ __forceinline__ uint32_t to_bits(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t to_bits(float v) { return __float_as_uint(v); }
// fp64 sums select by their fp32 rounding (round to nearest: order-preserving)
__device__ __forceinline__ uint32_t to_bits(double v) { return __float_as_uint(float(v)); }
template <typename S>
__device__ __forceinline__ S from_bits(uint32_t b);
template <>
__device__ __forceinline__ uint32_t from_bits<uint32_t>(uint32_t b) {
  return b;
}
template <>
__device__ __forceinline__ float from_bits<float>(uint32_t b) {
  return __uint_as_float(b);
}

// Descending bitonic sort of keys[0..p), p a power of two, whole workgroup.
__device__ __forceinline__ void bitonic_desc(uint64_t* keys, int p) {
  for (int size = 2; size <= p; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (p >> 1); i += kBlock) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t x = keys[lo], y = keys[hi];
        if ((x < y) == up) {
          keys[lo] = y;
          keys[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Radix select (8 bits per pass, most significant digit first) over the values
// val(i) of the items with pred(i) true.  Returns the value of rank `want`
// (1-based) counting from the largest (desc=true) or the smallest (desc=false).
template <int BITS, typename ValF, typename PredF>
__device__ uint32_t radix_select(int n, uint32_t want, bool desc, ValF val, PredF pred, const SelectSmem& sm) {
  uint32_t prefix = 0, mask = 0;
  for (int shift = BITS - 8; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += kBlock) sm.hist[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kBlock) {
      if (!pred(i)) continue;
      const uint32_t b = val(i);
      if ((b & mask) == prefix) atomicAdd(&sm.hist[(b >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t run = 0, sel = 0;
      for (int t = 0; t < 256; ++t) {
        const int dg = desc ? 255 - t : t;
        const uint32_t h = sm.hist[dg];
        if (run + h >= want) {
          sel = uint32_t(dg);
          break;
        }
        run += h;
      }
      sm.scal[0] = sel;
      sm.scal[1] = want - run;
    }
    __syncthreads();
    prefix |= sm.scal[0] << shift;
    mask |= 255u << shift;
    want = sm.scal[1];
    __syncthreads();
  }
  return prefix;
}

// acc[0..n): scores; slot i holds row s_base + (SWZ ? swz(i) : i), rows past the
// tile's end hold 0.  The running list of this query lives in o_ids / o_sc
// (k slots) and *o_cnt.
template <typename S, bool SWZ, typename A = S>
__device__ void tile_select(const A* acc, int n_valid, int64_t s_base, int k, int32_t* __restrict__ o_ids,
                            S* __restrict__ o_sc, int32_t* __restrict__ o_cnt, const SelectSmem& sm) {
  const int cnt = *o_cnt;
  const uint32_t theta = cnt == k ? to_bits(o_sc[k - 1]) : 0u;
  uint32_t c = 0;
  for (int i = threadIdx.x; i < n_valid; i += kBlock) c += to_bits(acc[i]) > theta;
  const uint32_t n = block_sum(c, sm.tmp);
  if (n == 0) return;

  // candidate rule: bits > lo_bits, or (with ties) bits > tie_v || (bits == tie_v && i <= tie_u)
  uint32_t lo_bits = theta, tie_v = 0, tie_u = 0;
  bool use_tie = false;
  if (n + uint32_t(cnt) > sm.cap) {
    auto val = [&](int i) { return to_bits(acc[i]); };
    auto pred = [&](int i) { return to_bits(acc[i]) > theta; };
    const uint32_t v = radix_select<32>(n_valid, uint32_t(k), true, val, pred, sm);
    uint32_t g = 0, e = 0;
    for (int i = threadIdx.x; i < n_valid; i += kBlock) {
      const uint32_t b = to_bits(acc[i]);
      g += b > v;
      e += b == v;
    }
    g = block_sum(g, sm.tmp);
    e = block_sum(e, sm.tmp);
    if (g + e + uint32_t(cnt) <= sm.cap) {
      lo_bits = v - 1u;  // v > theta >= 0
    } else {
      // too many equal scores: keep the (k - g) lowest ids among them
      auto ival = [&](int i) { return SWZ ? swz(uint32_t(i)) : uint32_t(i); };
      auto ipred = [&](int i) { return to_bits(acc[i]) == v; };
      tie_u = radix_select<16>(n_valid, uint32_t(k) - g, false, ival, ipred, sm);
      tie_v = v;
      use_tie = true;
    }
  }
  for (int i = threadIdx.x; i < cnt; i += kBlock)
    sm.keys[i] = (uint64_t(to_bits(o_sc[i])) << 32) | uint32_t(~uint32_t(o_ids[i]));
  if (threadIdx.x == 0) sm.scal[2] = uint32_t(cnt);
  __syncthreads();
  for (int i = threadIdx.x; i < n_valid; i += kBlock) {
    const uint32_t b = to_bits(acc[i]);
    const uint32_t sl = SWZ ? swz(uint32_t(i)) : uint32_t(i);
    const bool take = use_tie ? (b > tie_v || (b == tie_v && sl <= tie_u)) : (b > lo_bits);
    if (take) {
      const uint32_t pos = atomicAdd(&sm.scal[2], 1u);
      sm.keys[pos] = (uint64_t(b) << 32) | uint32_t(~uint32_t(s_base + sl));
    }
  }
  __syncthreads();
  const int m = int(sm.scal[2]);
  int p = 1;
  while (p < m) p <<= 1;
  for (int i = m + threadIdx.x; i < p; i += kBlock) sm.keys[i] = 0ull;
  __syncthreads();
  bitonic_desc(sm.keys, p);
  const int keep = m < k ? m : k;
  for (int i = threadIdx.x; i < k; i += kBlock) {
    if (i < keep) {
      const uint64_t key = sm.keys[i];
      o_ids[i] = int32_t(~uint32_t(key));
      o_sc[i] = from_bits<S>(uint32_t(key >> 32));
    } else {
      o_ids[i] = -1;
      o_sc[i] = S(0);
    }
  }
  if (threadIdx.x == 0) *o_cnt = keep;
  __syncthreads();
}

}  // namespace knnj
