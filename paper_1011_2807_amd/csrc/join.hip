// IIB join (Algorithm 3, Find_Matches_IIB) and the brute-force join
// (Algorithm 2) on one S tile at a time.
//
// One workgroup owns one query r for one tile t.  Its score map A (Algorithm 3
// line 10) is a dense array acc[T] in local memory indexed by s_local; the
// postings walk adds r[d] * w to acc[s_local] with local-memory atomics, which
// are exact for integer scores.  The lists (t, d) of all features of r are
// walked as one concatenated sequence so that every lane of the workgroup has
// work even when the lists are short: lane i handles positions
// i, i + 256, i + 512, ... of the concatenation and carries the index of the
// list it is in, so each position costs one compare and one load.
#include "select.hpp"

namespace knnj {

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

// Dynamic local memory of the tile kernels: [acc: T scores][stage], where the
// stage holds either the walk's list table or the selection workspace.
//   list table (kSegChunk lists): pre uint32[kSegChunk + 2] | cbase int64[kSegChunk]
//                                 | meta uint32[kSegChunk] | w 4-byte[kSegChunk]
constexpr int kPreOff = 0;
constexpr int kCbOff = 4 * (kSegChunk + 2);
constexpr int kMetaOff = kCbOff + 8 * kSegChunk;
constexpr int kWOff = kMetaOff + 4 * kSegChunk;
constexpr int kWalkBytes = kWOff + 4 * kSegChunk;

size_t stage_bytes(int k) {
  const size_t sel = select_bytes(k);
  return sel > size_t(kWalkBytes) ? sel : size_t(kWalkBytes);
}
size_t tile_smem_bytes(int tile, int k) { return size_t(tile) * 4 + stage_bytes(k); }
size_t tile_smem_bytes(int tile) { return tile_smem_bytes(tile, kMaxK); }

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

// Stage the lists (tile, d) of features [cb, cb + n) of one query; returns the
// number of 4-entry groups in their concatenation.  Thread t stages list t.
template <typename V, typename S>
__device__ __forceinline__ uint32_t stage_lists(char* stage, uint32_t* tmp, int64_t key0, const int32_t* r_idx,
                                                const V* r_val, int64_t cb, int n, const int64_t* offsets) {
  uint32_t* pre = reinterpret_cast<uint32_t*>(stage + kPreOff);
  int64_t* cbase = reinterpret_cast<int64_t*>(stage + kCbOff);
  uint32_t* meta = reinterpret_cast<uint32_t*>(stage + kMetaOff);
  S* w_of = reinterpret_cast<S*>(stage + kWOff);
  const int j = threadIdx.x;
  uint32_t groups = 0, len = 0, off = 0;
  int64_t beg = 0;
  S w = S(0);
  if (j < n) {
    const int64_t key = key0 + r_idx[cb + j];
    beg = offsets[key];
    len = uint32_t(offsets[key + 1] - beg);
    off = uint32_t(beg & 3);
    groups = len ? uint32_t(((beg + len + 3) >> 2) - (beg >> 2)) : 0u;
    w = S(r_val[cb + j]);
  }
  uint32_t total;
  const uint32_t ex = block_exclusive_scan(groups, tmp, &total);
  if (j < n) {
    pre[j] = ex;
    cbase[j] = (beg >> 2) - int64_t(ex);
    meta[j] = (len << 2) | off;
    w_of[j] = w;
  }
  if (j == 0) pre[n] = total;
  __syncthreads();
  return total;
}

// Walk the staged concatenation: lane i takes groups i, i + 256, ...; a group
// is one aligned 16-byte load of four entries, of which those inside the
// list's range are added into acc with local-memory atomics.
template <typename V, typename S>
__device__ __forceinline__ void walk_lists(S* acc, const char* stage, uint32_t total, Postings<V> P) {
  constexpr int U = 4;
  const uint32_t* pre = reinterpret_cast<const uint32_t*>(stage + kPreOff);
  const int64_t* cbase = reinterpret_cast<const int64_t*>(stage + kCbOff);
  const uint32_t* meta = reinterpret_cast<const uint32_t*>(stage + kMetaOff);
  const S* w_of = reinterpret_cast<const S*>(stage + kWOff);
  int j = 0;
  uint32_t cur = 0, nxt = pre[1];
  int64_t cb = cbase[0];
  uint32_t mt = meta[0];
  S w = w_of[0];
  for (uint32_t g0 = threadIdx.x; g0 < total; g0 += kBlock * U) {
    uint4 e[U];
    uint2 es[U];
    float4 ew[U];
    uint32_t rel[U], len[U];
    S ww[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t g = g0 + u * kBlock;
      len[u] = 0;
      if (g < total) {
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
        len[u] = mt >> 2;
        ww[u] = w;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (sizeof(V) == 1) {
        const uint32_t x[4] = {e[u].x, e[u].y, e[u].z, e[u].w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (rel[u] + uint32_t(i) < len[u]) atomicAdd(&acc[x[i] >> 16], ww[u] * ((x[i] >> 8) & 0xffu));
      } else {
        const uint32_t sx[4] = {es[u].x & 0xffffu, es[u].x >> 16, es[u].y & 0xffffu, es[u].y >> 16};
        const float wx[4] = {ew[u].x, ew[u].y, ew[u].z, ew[u].w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (rel[u] + uint32_t(i) < len[u]) atomicAdd(&acc[sx[i]], ww[u] * wx[i]);
      }
    }
  }
}

// IIB on tile `tile` for queries q0 + blockIdx.x.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_iib_tile(int32_t tile, int32_t log2_tile, int64_t n_s, int32_t n_dims,
                                                     int32_t k, int64_t q0, const int64_t* __restrict__ r_ptr,
                                                     const int32_t* __restrict__ r_idx, const V* __restrict__ r_val,
                                                     const int64_t* __restrict__ offsets, Postings<V> P,
                                                     int32_t* __restrict__ out_ids,
                                                     typename ScoreOf<V>::T* __restrict__ out_sc,
                                                     int32_t* __restrict__ out_cnt, uint64_t* __restrict__ slots) {
  using S = typename ScoreOf<V>::T;
  extern __shared__ __align__(16) char smem[];
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  const int T = 1 << log2_tile;
  S* acc = reinterpret_cast<S*>(smem);
  char* stage = smem + size_t(T) * 4;

  const int64_t q = q0 + blockIdx.x;
  const int64_t s_base = int64_t(tile) << log2_tile;
  const int n_valid = int(n_s - s_base < T ? n_s - s_base : T);
  for (int i = threadIdx.x; i < T / 4; i += kBlock) reinterpret_cast<uint4*>(acc)[i] = make_uint4(0, 0, 0, 0);

  const int64_t rb = r_ptr[q], re = r_ptr[q + 1];
  const int64_t key0 = int64_t(tile) * n_dims;
  uint64_t walked = 0;
  for (int64_t cb = rb; cb < re; cb += kSegChunk) {
    const int n = int(re - cb < kSegChunk ? re - cb : kSegChunk);
    const uint32_t total = stage_lists<V, S>(stage, tmp, key0, r_idx, r_val, cb, n, offsets);
    walk_lists<V, S>(acc, stage, total, P);
    if (slots) {
      // exact entries walked: sum of list lengths of this pass
      uint32_t l = threadIdx.x < n ? reinterpret_cast<const uint32_t*>(stage + kMetaOff)[threadIdx.x] >> 2 : 0u;
      walked += block_sum(l, tmp);
    }
    __syncthreads();
  }
  tile_select<S>(acc, n_valid, s_base, k, out_ids + q * k, out_sc + q * k, out_cnt + q, select_smem(stage, k, tmp));
  if (threadIdx.x == 0 && slots) atomicAdd((unsigned long long*)&slots[KNNJ_STAT_POSTINGS * 256 + (blockIdx.x & 255)],
                                           (unsigned long long)walked);
}

// Brute force (Algorithm 2): scores of rows [s0, s0 + T) of S by a two-pointer
// merge of r (staged in local memory) with each s; one thread per s.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_bf(int32_t log2_tile, int64_t n_s, int32_t k, int64_t q0,
                                               const int64_t* __restrict__ r_ptr, const int32_t* __restrict__ r_idx,
                                               const V* __restrict__ r_val, const int64_t* __restrict__ s_ptr,
                                               const int32_t* __restrict__ s_idx, const V* __restrict__ s_val,
                                               int32_t* __restrict__ out_ids,
                                               typename ScoreOf<V>::T* __restrict__ out_sc,
                                               int32_t* __restrict__ out_cnt) {
  using S = typename ScoreOf<V>::T;
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
      S ret = S(0);
      int a = 0;
      int64_t b = sb;
      while (a < nr && b < se) {
        const int32_t dr = rd[a], ds = s_idx[b];
        if (dr == ds) {
          ret += rw[a] * S(s_val[b]);
          ++a;
          ++b;
        } else if (dr > ds) {
          ++b;
        } else {
          ++a;
        }
      }
      acc[i] = ret;
    }
    __syncthreads();
    tile_select<S>(acc, n_valid, s0, k, out_ids + q * k, out_sc + q * k, out_cnt + q, sm);
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

knnj_status launch_iib(const Index* ix, const knnj_csr* R, int32_t k, int32_t* ids, void* sc, int32_t* cnt,
                       uint64_t* slots, hipStream_t st) {
  const size_t smem = tile_smem_bytes(ix->tile, k);
  for (int32_t t = 0; t < ix->n_tiles; ++t) {
    for (int64_t q0 = 0; q0 < R->n_rows; q0 += kMaxGrid) {
      const unsigned g = unsigned(R->n_rows - q0 < kMaxGrid ? R->n_rows - q0 : kMaxGrid);
      if (ix->dtype == KNNJ_U8) {
        Postings<uint8_t> P{reinterpret_cast<const uint4*>(ix->post_u8)};
        k_iib_tile<uint8_t><<<g, kBlock, smem, st>>>(t, ix->log2_tile, ix->n_rows, ix->n_dims, k, q0, R->indptr,
                                                     R->indices, (const uint8_t*)R->values, ix->offsets, P, ids,
                                                     (uint32_t*)sc, cnt, slots);
      } else {
        Postings<float> P{reinterpret_cast<const uint2*>(ix->post_s), reinterpret_cast<const float4*>(ix->post_w)};
        k_iib_tile<float><<<g, kBlock, smem, st>>>(t, ix->log2_tile, ix->n_rows, ix->n_dims, k, q0, R->indptr,
                                                   R->indices, (const float*)R->values, ix->offsets, P, ids,
                                                   (float*)sc, cnt, slots);
      }
    }
  }
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

knnj_status launch_bf(const knnj_csr* S, const knnj_csr* R, int32_t k, int32_t* ids, void* sc, int32_t* cnt,
                      hipStream_t st) {
  const int log2_tile = 11;
  const size_t smem = tile_smem_bytes(1 << log2_tile, k);
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
