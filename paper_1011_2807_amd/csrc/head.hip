// Dense head for the IIB join on skewed data (opt-in; same exact result).
//
// Sec. 4.3's accumulation walks I_d for every feature d of r.  On Zipf-like
// data a few dimensions hold most postings, and within an S tile their lists
// are nearly dense.  For the H dimensions with the longest lists the index also
// keeps, per tile, the weights as a dense block, and the join computes their
// part of A[s] = sum_d r[d] * s[d] as byte dot products (v_dot4_u32_u8) instead
// of one local-memory atomic per posting; only the other ("tail") lists are
// walked.  Integer sums, so the scores are bit-identical to the plain walk.
//
// Layout of the block of tile t: [H / 16 chunks][T rows][16 bytes]; byte j of
// chunk c of row s is the weight of head dimension 16 c + j.  Lanes handling
// consecutive rows read consecutive 16-byte chunks.
//
// The join kernel takes Q = 4 queries per workgroup: each head chunk is loaded
// once and feeds the dot products of all four queries.
#include "sched.hpp"
#include "walk.hpp"

namespace knnj {

constexpr int kHeadQ = 2;

// head_pos[d] = rank of d among the H longest lists (ties: smaller d first), or -1.
// One workgroup; `taken` is a bitmap of n_dims bits in global memory (zeroed).
__global__ void k_head_select(int32_t n_dims, int32_t H, const uint32_t* __restrict__ list_len,
                              uint32_t* __restrict__ taken, int32_t* __restrict__ head_pos) {
  __shared__ uint64_t best[kBlock];
  for (int d = threadIdx.x; d < n_dims; d += kBlock) head_pos[d] = -1;
  __syncthreads();
  for (int h = 0; h < H; ++h) {
    // key: length high, then smaller d first
    uint64_t b = 0;
    for (int d = threadIdx.x; d < n_dims; d += kBlock) {
      if (taken[d >> 5] & (1u << (d & 31))) continue;
      const uint64_t key = (uint64_t(list_len[d]) << 32) | uint32_t(0x7fffffff - d);
      if (key > b) b = key;
    }
    best[threadIdx.x] = b;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o && best[threadIdx.x + o] > best[threadIdx.x]) best[threadIdx.x] = best[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0 && best[0] != 0) {
      const int d = 0x7fffffff - int(uint32_t(best[0]));
      taken[d >> 5] |= 1u << (d & 31);
      head_pos[d] = h;
    }
    __syncthreads();
  }
}

// Scatter the head weights of every S row into the dense blocks (zeroed).
__global__ void k_head_fill(int64_t n_rows, int32_t log2_tile, int32_t H, const int64_t* __restrict__ s_ptr,
                            const int32_t* __restrict__ s_idx, const uint8_t* __restrict__ s_val,
                            const int32_t* __restrict__ head_pos, uint8_t* __restrict__ head) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t n_waves = int64_t(gridDim.x) * blockDim.x / kWave;
  const int64_t T = int64_t(1) << log2_tile;
  for (int64_t r = wave; r < n_rows; r += n_waves) {
    const int64_t t = r >> log2_tile, s = r & (T - 1);
    for (int64_t j = s_ptr[r] + lane; j < s_ptr[r + 1]; j += kWave) {
      const int32_t h = head_pos[s_idx[j]];
      if (h < 0) continue;
      head[((t * (H / 16) + h / 16) * T + s) * 16 + (h & 15)] = s_val[j];
    }
  }
}

// Per join, once: for every query q, its tail features (d, w) moved to the
// front of its own CSR row (hj_d / hj_w at r_ptr[q] ..), their count hj_cnt[q],
// and its head weights as a dense row rh[q][H] (zeroed beforehand).  One wave
// per query; the compaction keeps the row's order.
__global__ void k_head_prep(int64_t n_q, int32_t H, const int64_t* __restrict__ r_ptr,
                            const int32_t* __restrict__ r_idx, const uint8_t* __restrict__ r_val,
                            const int32_t* __restrict__ head_pos, int32_t* __restrict__ hj_d,
                            uint8_t* __restrict__ hj_w, uint32_t* __restrict__ hj_cnt, uint8_t* __restrict__ rh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t q = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  if (q >= n_q) return;
  const int64_t rb = r_ptr[q], re = r_ptr[q + 1];
  const uint64_t below = (uint64_t(1) << lane) - 1u;
  uint32_t n_tail = 0;
  for (int64_t j0 = rb; j0 < re; j0 += kWave) {
    const int64_t j = j0 + lane;
    int32_t d = 0, h = 0;
    uint8_t w = 0;
    if (j < re) {
      d = r_idx[j];
      w = r_val[j];
      h = head_pos[d];
    }
    const bool tail = j < re && h < 0;
    const uint64_t m = __ballot(tail);
    if (tail) {
      const int64_t at = rb + n_tail + __popcll(m & below);
      hj_d[at] = d;
      hj_w[at] = w;
    } else if (j < re) {
      rh[q * H + h] = w;
    }
    n_tail += uint32_t(__popcll(m));
  }
  if (lane == 0) hj_cnt[q] = n_tail;
}

// IIB with the dense head for the queries at positions Q b .. Q b + Q - 1 of
// `order`, on tile t.  Local memory: acc[Q][T] | head weights [Q][H] bytes | stage.
// The tail lists of the Q queries are staged and walked together (chunks of
// kSegChunk lists); the first chunk's list lookups are issued before the head
// dot products, so their latency overlaps that work.
template <int Q>
__global__ __launch_bounds__(kBlock) void k_iibh_tile(int32_t tile, int32_t log2_tile, int32_t n_dims, int32_t k,
                                                      int32_t H, int64_t n_q, const int32_t* __restrict__ order,
                                                      const int64_t* __restrict__ r_ptr,
                                                      const int32_t* __restrict__ hj_d,
                                                      const uint8_t* __restrict__ hj_w,
                                                      const uint32_t* __restrict__ hj_cnt,
                                                      const uint4* __restrict__ rh_g,
                                                      const int64_t* __restrict__ offsets, Postings<uint8_t> P,
                                                      const uint4* __restrict__ head, int32_t* __restrict__ out_ids,
                                                      uint32_t* __restrict__ out_sc, int32_t* __restrict__ out_cnt,
                                                      uint64_t* __restrict__ slots) {
  extern __shared__ __align__(16) char smem[];
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  const int T = 1 << log2_tile;
  uint32_t* acc = reinterpret_cast<uint32_t*>(smem);                    // [Q][T]
  uint4* rh = reinterpret_cast<uint4*>(smem + size_t(Q) * T * 4);       // [Q][H / 16]
  char* stage = smem + size_t(Q) * T * 4 + size_t(Q) * H;
  const int64_t s_base = int64_t(tile) << log2_tile;
  const int64_t key0 = int64_t(tile) * n_dims;
  const int HC = H / 16;
  int64_t qs[Q], tb[Q];
  uint32_t pre[Q + 1];
  pre[0] = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int64_t p = int64_t(blockIdx.x) * Q + i;
    qs[i] = p < n_q ? (order ? int64_t(order[p]) : p) : -1;
    tb[i] = qs[i] >= 0 ? r_ptr[qs[i]] : 0;
    pre[i + 1] = pre[i] + (qs[i] >= 0 ? hj_cnt[qs[i]] : 0u);
  }
  const uint32_t n_tail = pre[Q];
  // list lookup of tail list g (< n_tail) of the group
  auto lookup = [&](uint32_t g, int64_t* beg, uint32_t* len, uint32_t* w) {
    int i = 0;
#pragma unroll
    for (int x = 1; x < Q; ++x) i += g >= pre[x];
    const int64_t at = tb[i] + (g - pre[i]);
    const int64_t key = key0 + hj_d[at];
    *beg = offsets[key];
    *len = uint32_t(offsets[key + 1] - *beg);
    *w = (uint32_t(i) << 8) | hj_w[at];
  };
  int64_t beg = 0;
  uint32_t len = 0, w = 0;
  if (threadIdx.x < n_tail) lookup(threadIdx.x, &beg, &len, &w);
  for (int x = threadIdx.x; x < Q * HC; x += kBlock) {
    const int i = x / HC;
    rh[x] = qs[i] >= 0 ? rh_g[qs[i] * HC + (x - i * HC)] : make_uint4(0u, 0u, 0u, 0u);
  }
  __syncthreads();
  // head part: a thread takes rows s0 + 256 j (j < RB) at a time; each 16-byte
  // chunk of a row feeds the dot products of all Q queries, and each chunk of
  // the queries' weights (one local-memory broadcast) feeds RB rows
  constexpr int RB = 4;
  const uint4* blk = head + size_t(tile) * HC * T;
  for (int s0 = threadIdx.x; s0 < T; s0 += RB * kBlock) {
    uint32_t a[Q][RB];
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int j = 0; j < RB; ++j) a[i][j] = 0u;
    for (int c = 0; c < HC; ++c) {
      uint4 v[RB];
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        const int s = s0 + j * kBlock;
        v[j] = s < T ? blk[size_t(c) * T + s] : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const uint4 wq = rh[i * HC + c];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
          a[i][j] = __builtin_amdgcn_udot4(v[j].x, wq.x, a[i][j], false);
          a[i][j] = __builtin_amdgcn_udot4(v[j].y, wq.y, a[i][j], false);
          a[i][j] = __builtin_amdgcn_udot4(v[j].z, wq.z, a[i][j], false);
          a[i][j] = __builtin_amdgcn_udot4(v[j].w, wq.w, a[i][j], false);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int s = s0 + j * kBlock;
      if (s < T) {
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i * T + swz(uint32_t(s))] = a[i][j];
      }
    }
  }
  // tail lists of all Q queries (stage_write's scan orders the head stores
  // before the walk's atomics)
  uint64_t walked = 0;
  for (uint32_t c0 = 0; c0 < n_tail; c0 += kSegChunk) {
    const int n = int(n_tail - c0 < uint32_t(kSegChunk) ? n_tail - c0 : uint32_t(kSegChunk));
    if (c0 > 0) {
      beg = 0;
      len = 0;
      w = 0;
      if (threadIdx.x < n) lookup(c0 + threadIdx.x, &beg, &len, &w);
    }
    const uint32_t total = stage_write<uint32_t>(stage, tmp, n, beg, len, w);
    walk_lists<uint8_t, uint32_t, true>(acc, stage, n, total, P, log2_tile);
    if (slots) walked += block_sum(threadIdx.x < n ? len : 0u, tmp);
    __syncthreads();
  }
  if (n_tail == 0) __syncthreads();
  for (int i = 0; i < Q; ++i) {
    if (qs[i] < 0) continue;
    const int64_t q = qs[i];
    tile_select<uint32_t, true>(acc + size_t(i) * T, T, s_base, k, out_ids + q * k, out_sc + q * k, out_cnt + q,
                                select_smem(stage, k, tmp));
  }
  if (threadIdx.x == 0 && slots)
    atomicAdd((unsigned long long*)&slots[KNNJ_STAT_POSTINGS * 256 + (blockIdx.x & 255)], (unsigned long long)walked);
}

size_t tile_smem_bytes(int tile, int k);

size_t head_smem_bytes(int tile, int k, int H) {
  return size_t(kHeadQ) * tile * 4 + size_t(kHeadQ) * H + stage_bytes(k);
}

knnj_status launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

knnj_status build_head(Index* ix, hipStream_t st) {
  const int H = ix->head_h;
  const size_t bytes = size_t(ix->n_tiles) * size_t(ix->tile) * H;
  uint32_t* taken = nullptr;
  if (hipMalloc(&ix->head_pos, sizeof(int32_t) * ix->n_dims) != hipSuccess ||
      hipMalloc(&ix->head_blk, bytes) != hipSuccess ||
      hipMalloc(&taken, sizeof(uint32_t) * ((ix->n_dims + 31) / 32)) != hipSuccess) {
    (void)hipFree(taken);
    return fail(KNNJ_ENOMEM, "device allocation for the dense head failed");
  }
  knnj_status rc = launch_fill_u32(taken, (ix->n_dims + 31) / 32, 0u, st);
  if (rc == KNNJ_OK) rc = launch_fill_u32(reinterpret_cast<uint32_t*>(ix->head_blk), int64_t(bytes / 4), 0u, st);
  if (rc == KNNJ_OK) {
    k_head_select<<<1, kBlock, 0, st>>>(ix->n_dims, H, ix->list_len, taken, ix->head_pos);
    if (ix->n_rows > 0)
      k_head_fill<<<unsigned((ix->n_rows + 3) / 4 < 65536 ? (ix->n_rows + 3) / 4 : 65536), kBlock, 0, st>>>(
          ix->n_rows, ix->log2_tile, H, ix->s_indptr, ix->s_indices, (const uint8_t*)ix->s_values, ix->head_pos,
          ix->head_blk);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      rc = fail(KNNJ_EDEVICE, "dense head build failed");
  }
  (void)hipFree(taken);
  return rc;
}

// Grow the dense-head join scratch to n queries / nnz features (the only
// allocation of such a join; skipped when an earlier join was at least as large).
static knnj_status ensure_head_scratch(Index* ix, int64_t n, int64_t nnz) {
  if (n <= ix->hj_cap_q && nnz <= ix->hj_cap_nnz) return KNNJ_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(ix->hj_cnt);
  (void)hipFree(ix->hj_d);
  (void)hipFree(ix->hj_w);
  (void)hipFree(ix->hj_rh);
  ix->hj_cnt = nullptr;
  ix->hj_d = nullptr;
  ix->hj_w = nullptr;
  ix->hj_rh = nullptr;
  ix->hj_cap_q = ix->hj_cap_nnz = 0;
  const int64_t cq = n > ix->hj_cap_q ? n : ix->hj_cap_q;
  const int64_t cz = (nnz > ix->hj_cap_nnz ? nnz : ix->hj_cap_nnz) + 1;
  if (hipMalloc(&ix->hj_cnt, sizeof(uint32_t) * cq) != hipSuccess ||
      hipMalloc(&ix->hj_d, sizeof(int32_t) * cz) != hipSuccess || hipMalloc(&ix->hj_w, cz) != hipSuccess ||
      hipMalloc(&ix->hj_rh, size_t(cq) * ix->head_h) != hipSuccess)
    return fail(KNNJ_ENOMEM, "dense-head join scratch allocation failed");
  ix->hj_cap_q = cq;
  ix->hj_cap_nnz = cz;
  return KNNJ_OK;
}

knnj_status launch_iib_head(Index* ix, const knnj_csr* R, int32_t k, const int32_t* order, int32_t* ids,
                            void* sc, int32_t* cnt, uint64_t* slots, hipStream_t st) {
  const int64_t n = R->n_rows;
  if (n == 0) return KNNJ_OK;
  const int H = ix->head_h;
  knnj_status rc = ensure_head_scratch(ix, n, R->nnz);
  if (rc != KNNJ_OK) return rc;
  if ((rc = launch_fill_u32(reinterpret_cast<uint32_t*>(ix->hj_rh), n * H / 4, 0u, st)) != KNNJ_OK) return rc;
  k_head_prep<<<unsigned((n + 3) / 4), kBlock, 0, st>>>(n, H, R->indptr, R->indices, (const uint8_t*)R->values,
                                                       ix->head_pos, ix->hj_d, ix->hj_w, ix->hj_cnt, ix->hj_rh);
  const size_t smem = head_smem_bytes(ix->tile, k, H);
  const unsigned g = unsigned((n + kHeadQ - 1) / kHeadQ);
  Postings<uint8_t> P{reinterpret_cast<const uint4*>(ix->post_u8)};
  for (int32_t t = 0; t < ix->n_tiles; ++t)
    k_iibh_tile<kHeadQ><<<g, kBlock, smem, st>>>(t, ix->log2_tile, ix->n_dims, k, H, n, order, R->indptr, ix->hj_d,
                                                 ix->hj_w, ix->hj_cnt, reinterpret_cast<const uint4*>(ix->hj_rh),
                                                 ix->offsets, P, reinterpret_cast<const uint4*>(ix->head_blk), ids,
                                                 (uint32_t*)sc, cnt, slots);
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

}  // namespace knnj
