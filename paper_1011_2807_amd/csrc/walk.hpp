// Postings walk shared by the IIB and IIIB tile kernels: staging of a query's
// lists for one S tile and the team-split walk that adds r[d] * w into the
// tile's local-memory score array.
#pragma once

#include "select.hpp"

namespace knnj {

// Dynamic local memory of the tile kernels: [acc: T scores][stage], where the
// stage holds either the walk's list table or the selection workspace.
//   list table (kSegChunk lists): pre uint32[kSegChunk + 2] | cbase int64[kSegChunk]
//                                 | meta uint32[kSegChunk] | w 4-byte[kSegChunk]
constexpr int kPreOff = 0;
constexpr int kCbOff = 4 * (kSegChunk + 2);
constexpr int kMetaOff = kCbOff + 8 * kSegChunk;
constexpr int kWOff = kMetaOff + 4 * kSegChunk;
constexpr int kWalkBytes = kWOff + 4 * kSegChunk;

inline size_t stage_bytes(int k) {
  const size_t sel = select_bytes(k);
  return sel > size_t(kWalkBytes) ? sel : size_t(kWalkBytes);
}

__device__ __forceinline__ SelectSmem select_smem(char* stage, int k, uint32_t* tmp) {
  const uint32_t cap = select_cap(k);
  return SelectSmem{reinterpret_cast<uint64_t*>(stage), cap, reinterpret_cast<uint32_t*>(stage + 8 * cap),
                    reinterpret_cast<uint32_t*>(stage + 8 * cap + 1024), tmp};
}

template <typename V>
struct Postings;
// u8: entries (s_local << 16) | (w << 8), read four at a time (16-byte aligned groups)
template <>
struct Postings<uint8_t> {
  const uint4* e;
};
// f32: s_local uint16 and weight float arrays, four at a time
template <>
struct Postings<float> {
  const uint2* s;
  const float4* w;
};

// Write the list table of n lists (thread j < n describes list j: first entry
// `beg`, `len` entries, weight w, and for float lists of several queries the
// query's score row `row` in the top bits of its meta word) and return the
// number of 4-entry groups in the lists' concatenation.  Ends with a barrier.
constexpr int kRowShift = 28;
template <typename S>
__device__ __forceinline__ uint32_t stage_write(char* stage, uint32_t* tmp, int n, int64_t beg, uint32_t len, S w,
                                                uint32_t row = 0) {
  uint32_t* pre = reinterpret_cast<uint32_t*>(stage + kPreOff);
  int64_t* cbase = reinterpret_cast<int64_t*>(stage + kCbOff);
  uint32_t* meta = reinterpret_cast<uint32_t*>(stage + kMetaOff);
  S* w_of = reinterpret_cast<S*>(stage + kWOff);
  const int j = threadIdx.x;
  const uint32_t off = uint32_t(beg & 3);
  const uint32_t groups = len ? uint32_t(((beg + len + 3) >> 2) - (beg >> 2)) : 0u;
  uint32_t total;
  const uint32_t ex = block_exclusive_scan(groups, tmp, &total);
  if (j < n) {
    pre[j] = ex;
    cbase[j] = (beg >> 2) - int64_t(ex);
    meta[j] = (row << kRowShift) | (len << 2) | off;
    w_of[j] = w;
  }
  if (j == 0) pre[n] = total;
  __syncthreads();
  return total;
}

// Stage the lists (tile, d) of features [cb, cb + n) of one query; returns the
// number of 4-entry groups in their concatenation.  Thread t stages list t.
// With a cut table (IIIB) only the first cut[key * kLevels + lambda] entries of
// list `key` are staged: the entries whose level is >= lambda.
template <typename V, typename S>
__device__ __forceinline__ uint32_t stage_lists(char* stage, uint32_t* tmp, int64_t key0, const int32_t* r_idx,
                                                const V* r_val, int64_t cb, int n, const int64_t* offsets,
                                                const uint32_t* cut = nullptr, uint32_t lambda = 0) {
  const int j = threadIdx.x;
  uint32_t len = 0;
  int64_t beg = 0;
  S w = S(0);
  if (j < n) {
    const int64_t key = key0 + r_idx[cb + j];
    beg = offsets[key];
    len = cut ? cut[key * kLevels + lambda] : uint32_t(offsets[key + 1] - beg);
    w = S(r_val[cb + j]);
  }
  return stage_write<S>(stage, tmp, n, beg, len, w);
}

// Walk the staged concatenation.  The workgroup is split into teams of 8 lanes;
// team t takes the t-th of 32 contiguous ranges of groups and its lanes take
// groups start + i, start + i + 8, ...  A group is one aligned 16-byte load of
// four entries, so one team load is one 128-byte line.  Entries inside the
// list's range are added into acc at the slot they carry (the swizzled slot of
// their row, stored by the index build) with local-memory atomics.
// A lane only steps over the lists inside its team's range.
// kMulti: the lists belong to several queries.  uint8: a list's weight word is
// (base << 8) | w and its scores go to acc + base (the query's score row);
// float: the query's row index sits in the meta word's top bits and its scores
// go to acc + row * stride.
constexpr int kTeam = 8;
// A: type of the score map (the staged weights are S; float lists accumulate
// into fp64).
template <typename V, typename S, bool kMulti = false, typename A = S>
__device__ __forceinline__ void walk_lists(A* acc, const char* stage, int n_lists, uint32_t total, Postings<V> P,
                                           int stride = 0) {
  constexpr int U = 4;
  const uint32_t* pre = reinterpret_cast<const uint32_t*>(stage + kPreOff);
  const int64_t* cbase = reinterpret_cast<const int64_t*>(stage + kCbOff);
  const uint32_t* meta = reinterpret_cast<const uint32_t*>(stage + kMetaOff);
  const S* w_of = reinterpret_cast<const S*>(stage + kWOff);
  constexpr int kTeams = kBlock / kTeam;
  const int li = threadIdx.x % kTeam;
  const int team = threadIdx.x / kTeam;
  const uint32_t per = (total + kTeams - 1) / kTeams;
  const uint32_t start = per * team;
  const uint32_t stop = start + per < total ? start + per : total;
  if (start >= stop) return;
  // list holding the lane's first group (binary search; later steps advance linearly)
  const uint32_t g_first = start + li < stop ? start + li : stop - 1;
  int lo = 0, hi = n_lists - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= g_first) lo = mid; else hi = mid - 1;
  }
  int j = lo;
  uint32_t cur = pre[j], nxt = pre[j + 1];
  int64_t cb = cbase[j];
  uint32_t mt = meta[j];
  S w = w_of[j];
  for (uint32_t g0 = start + li; g0 < stop; g0 += kTeam * U) {
    uint4 e[U];
    uint2 es[U];
    float4 ew[U];
    uint32_t rel[U], len[U];
    S ww[U];
    [[maybe_unused]] uint32_t rw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t g = g0 + u * kTeam;
      len[u] = 0;
      if (g < stop) {
        if (g >= nxt) {
          do {
            ++j;
            nxt = pre[j + 1];
          } while (g >= nxt);
          cur = pre[j];
          cb = cbase[j];
          mt = meta[j];
          w = w_of[j];
        }
        if constexpr (sizeof(V) == 1) {
          e[u] = P.e[cb + g];
        } else {
          es[u] = P.s[cb + g];
          ew[u] = P.w[cb + g];
        }
        rel[u] = 4u * (g - cur) - (mt & 3u);
        if constexpr (kMulti && sizeof(V) == 4) {
          len[u] = (mt >> 2) & ((1u << (kRowShift - 2)) - 1u);
          rw[u] = mt >> kRowShift;
        } else {
          len[u] = mt >> 2;
        }
        ww[u] = w;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (sizeof(V) == 1) {
        const uint32_t x[4] = {e[u].x, e[u].y, e[u].z, e[u].w};
        if constexpr (kMulti) {
          A* a = acc + (ww[u] >> 8);
          const uint32_t wq = ww[u] & 0xffu;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (rel[u] + uint32_t(i) < len[u]) atomicAdd(&a[x[i] >> 16], wq * ((x[i] >> 8) & 0xffu));
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (rel[u] + uint32_t(i) < len[u]) atomicAdd(&acc[x[i] >> 16], ww[u] * ((x[i] >> 8) & 0xffu));
        }
      } else {
        const uint32_t sx[4] = {es[u].x & 0xffffu, es[u].x >> 16, es[u].y & 0xffffu, es[u].y >> 16};
        const float wx[4] = {ew[u].x, ew[u].y, ew[u].z, ew[u].w};
        A* a = acc;
        if constexpr (kMulti) a = acc + size_t(rw[u]) * stride;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (rel[u] + uint32_t(i) < len[u]) atomicAdd(&a[sx[i]], A(ww[u]) * A(wx[i]));
      }
    }
  }
}

}  // namespace knnj
