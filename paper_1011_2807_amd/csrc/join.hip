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

// Layout of the dynamic local memory of the tile kernels:
//   [acc: T scores][stage: max(walk staging, selection workspace)]
struct StageLayout {
  static constexpr int kPreOff = 0;                                    // uint32[kSegChunk + 1]
  static constexpr int kBaseOff = 4 * (kSegChunk + 2);                 // int64[kSegChunk]
  static constexpr int kWOff = kBaseOff + 8 * kSegChunk;               // 4-byte weight[kSegChunk]
  static constexpr int kWalkBytes = kWOff + 4 * kSegChunk;
  static constexpr int kKeysOff = 0;                                   // uint64[kSortBuf]
  static constexpr int kHistOff = 8 * kSortBuf;                        // uint32[256]
  static constexpr int kScalOff = kHistOff + 4 * 256;                  // uint32[8]
  static constexpr int kSelBytes = kScalOff + 4 * 8;
  static constexpr int kBytes = kWalkBytes > kSelBytes ? kWalkBytes : kSelBytes;
};

size_t tile_smem_bytes(int tile) { return size_t(tile) * 4 + StageLayout::kBytes; }

template <typename V>
struct Postings;
template <>
struct Postings<uint8_t> {
  const uint32_t* e;
};
template <>
struct Postings<float> {
  const uint16_t* s;
  const float* w;
};

// Walk the concatenation of lists staged in (pre, base, w); add into acc.
template <typename V, typename S>
__device__ __forceinline__ void walk_lists(S* acc, const uint32_t* pre, const int64_t* base_of, const S* w_of,
                                           uint32_t total, Postings<V> P) {
  constexpr int U = 4;
  int j = 0;
  uint32_t nxt = pre[1];
  int64_t base = base_of[0];
  S w = w_of[0];
  for (uint32_t p0 = threadIdx.x; p0 < total; p0 += kBlock * U) {
    uint32_t e[U];
    float ew[U];
    S ww[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t p = p0 + u * kBlock;
      if (p < total) {
        if (p >= nxt) {
          do {
            ++j;
            nxt = pre[j + 1];
          } while (p >= nxt);
          base = base_of[j];
          w = w_of[j];
        }
        if constexpr (sizeof(V) == 1) {
          e[u] = P.e[base + p];
        } else {
          e[u] = P.s[base + p];
          ew[u] = P.w[base + p];
        }
        ww[u] = w;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (p0 + u * kBlock < total) {
        if constexpr (sizeof(V) == 1) atomicAdd(&acc[e[u] >> 16], ww[u] * ((e[u] >> 8) & 0xffu));
        else atomicAdd(&acc[e[u]], ww[u] * ew[u]);
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
  uint32_t* pre = reinterpret_cast<uint32_t*>(stage + StageLayout::kPreOff);
  int64_t* base_of = reinterpret_cast<int64_t*>(stage + StageLayout::kBaseOff);
  S* w_of = reinterpret_cast<S*>(stage + StageLayout::kWOff);

  const int64_t q = q0 + blockIdx.x;
  const int64_t s_base = int64_t(tile) << log2_tile;
  const int n_valid = int(n_s - s_base < T ? n_s - s_base : T);
  for (int i = threadIdx.x; i < T; i += kBlock) acc[i] = S(0);

  const int64_t rb = r_ptr[q], re = r_ptr[q + 1];
  const int64_t key0 = int64_t(tile) * n_dims;
  uint64_t walked = 0;
  for (int64_t cb = rb; cb < re; cb += kSegChunk) {
    const int n = int(re - cb < kSegChunk ? re - cb : kSegChunk);
    // two staged features per thread, contiguous (2t, 2t+1) so the scan order is the list order
    uint32_t len[2];
    int64_t beg[2];
    S wv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * threadIdx.x + h;
      len[h] = 0;
      beg[h] = 0;
      wv[h] = S(0);
      if (j < n) {
        const int64_t key = key0 + r_idx[cb + j];
        beg[h] = offsets[key];
        len[h] = uint32_t(offsets[key + 1] - beg[h]);
        wv[h] = S(r_val[cb + j]);
      }
    }
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(len[0] + len[1], tmp, &total);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * threadIdx.x + h;
      const uint32_t pj = ex + (h ? len[0] : 0u);
      if (j < n) {
        pre[j] = pj;
        base_of[j] = beg[h] - int64_t(pj);
        w_of[j] = wv[h];
      }
    }
    if (threadIdx.x == 0) pre[n] = total;
    __syncthreads();
    walk_lists<V, S>(acc, pre, base_of, w_of, total, P);
    walked += total;
    __syncthreads();
  }

  SelectSmem sm{reinterpret_cast<uint64_t*>(stage + StageLayout::kKeysOff),
                reinterpret_cast<uint32_t*>(stage + StageLayout::kHistOff),
                reinterpret_cast<uint32_t*>(stage + StageLayout::kScalOff), tmp};
  tile_select<S>(acc, n_valid, s_base, k, out_ids + q * k, out_sc + q * k, out_cnt + q, sm);
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
  SelectSmem sm{reinterpret_cast<uint64_t*>(stage + StageLayout::kKeysOff),
                reinterpret_cast<uint32_t*>(stage + StageLayout::kHistOff),
                reinterpret_cast<uint32_t*>(stage + StageLayout::kScalOff), tmp};
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
  const size_t smem = tile_smem_bytes(ix->tile);
  for (int32_t t = 0; t < ix->n_tiles; ++t) {
    for (int64_t q0 = 0; q0 < R->n_rows; q0 += kMaxGrid) {
      const unsigned g = unsigned(R->n_rows - q0 < kMaxGrid ? R->n_rows - q0 : kMaxGrid);
      if (ix->dtype == KNNJ_U8) {
        Postings<uint8_t> P{ix->post_u8};
        k_iib_tile<uint8_t><<<g, kBlock, smem, st>>>(t, ix->log2_tile, ix->n_rows, ix->n_dims, k, q0, R->indptr,
                                                     R->indices, (const uint8_t*)R->values, ix->offsets, P, ids,
                                                     (uint32_t*)sc, cnt, slots);
      } else {
        Postings<float> P{ix->post_s, ix->post_w};
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
  const size_t smem = tile_smem_bytes(1 << log2_tile);
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
