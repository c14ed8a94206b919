// Dense head for the IIB join on skewed data (opt-in; same exact result).
//
// Sec. 4.3's accumulation walks I_d for every feature d of r.  On Zipf-like
// data a few dimensions hold most postings, and within an S tile their lists
// are nearly dense.  For the H dimensions with the longest lists the index also
// keeps, per tile, the weights as a dense block, and the join computes their
// part of A[s] = sum_d r[d] * s[d] as a dense product instead of one
// local-memory atomic per posting; only the other ("tail") lists are walked.
// Integer sums, so the scores are bit-identical to the plain walk.
//
// Layout of the block of tile t: [H / 16 chunks][T rows][16 bytes]; byte j of
// chunk c of row s is the weight of head dimension 16 c + j.  Lanes handling
// consecutive rows read consecutive 16-byte chunks.
//
// A workgroup of the join takes Q queries (the same group for a run of tiles):
// each head chunk it loads feeds the products of all Q queries, and their tail
// lists are staged and walked together.  The product runs on the vector units
// (v_dot4_u32_u8): with Q = 4 query columns it is narrower than the smallest
// byte matrix-core shape (16 columns), and a wider Q needs more local memory
// for the score rows than leaves room for enough resident workgroups.
#include "walk.hpp"

namespace knnj {

// defaults: queries per workgroup, S tiles per launch
constexpr int kHeadQ = 4;
constexpr int kHeadTiles = 4;

// score rows of the Q queries lie T + kAccPad words apart: the same row slot of
// different queries falls in different local-memory banks
constexpr int kAccPad = 4;

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

// Scatter the head weights of every S row into the dense blocks (zeroed): per
// tile [H / E][T][E] weights, E = 16 bytes / weight size.  One wave per row.
template <typename V>
__global__ void k_head_fill(int64_t n_rows, int32_t log2_tile, int32_t H, const int64_t* __restrict__ s_ptr,
                            const int32_t* __restrict__ s_idx, const V* __restrict__ s_val,
                            const int32_t* __restrict__ head_pos, V* __restrict__ head) {
  constexpr int E = 16 / int(sizeof(V));
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t n_waves = int64_t(gridDim.x) * blockDim.x / kWave;
  const int64_t T = int64_t(1) << log2_tile;
  for (int64_t r = wave; r < n_rows; r += n_waves) {
    const int64_t t = r >> log2_tile, s = r & (T - 1);
    for (int64_t j = s_ptr[r] + lane; j < s_ptr[r + 1]; j += kWave) {
      const int32_t h = head_pos[s_idx[j]];
      if (h >= 0) head[((t * (H / E) + h / E) * T + s) * E + (h % E)] = s_val[j];
    }
  }
}

// Per join, once: for every query q, its tail features (d, w) moved to the
// front of its own CSR row (hj_d / hj_w at r_ptr[q] ..), their count hj_cnt[q],
// and its head weights as a dense row rh[q][H] (zeroed beforehand).  One wave
// per query; the compaction keeps the row's order.
template <typename V>
__global__ void k_head_prep(int64_t n_q, int32_t H, const int64_t* __restrict__ r_ptr,
                            const int32_t* __restrict__ r_idx, const V* __restrict__ r_val,
                            const int32_t* __restrict__ head_pos, int32_t* __restrict__ hj_d,
                            V* __restrict__ hj_w, uint32_t* __restrict__ hj_cnt, V* __restrict__ rh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t q = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  if (q >= n_q) return;
  const int64_t rb = r_ptr[q], re = r_ptr[q + 1];
  const uint64_t below = (uint64_t(1) << lane) - 1u;
  uint32_t n_tail = 0;
  for (int64_t j0 = rb; j0 < re; j0 += kWave) {
    const int64_t j = j0 + lane;
    int32_t d = 0, h = 0;
    V w = V(0);
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

// Top-k update of the Q queries of a workgroup after one tile (Algorithm 3's
// candidate step for each of them).  th / cn: the queries' running k-th scores
// and list sizes, kept in local memory by the workgroup that owns the queries.
// One pass counts, for every query at once, the scores above its running k-th
// score, with a single workgroup reduction.  A query with such scores is then
// merged by one wave (wave i % 4 takes query i) when its list and the new
// candidates fit in 64 lanes: the candidates are compacted into a per-wave
// buffer, sorted with the list by a wave-wide bitonic sort on the key (score
// desc, id asc), and the first k written back.  Larger merges (early tiles with
// a large k) take the workgroup selection.  red: 4 * Q words, hard: Q words;
// stage: at least 2 KiB.
template <int Q, typename A, typename S>
__device__ __forceinline__ void group_select(const A* acc, int stride, int T, int64_t s_base, int k,
                                             const int64_t* qs, int32_t* __restrict__ out_ids,
                                             S* __restrict__ out_sc, int32_t* __restrict__ out_cnt,
                                             char* stage, uint32_t* tmp, uint32_t* red, uint32_t* hard, uint32_t* th,
                                             int32_t* cn) {
  uint32_t c[Q], thv[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    c[i] = 0u;
    thv[i] = th[i];
  }
  for (int x = threadIdx.x; x < T; x += kBlock) {
#pragma unroll
    for (int i = 0; i < Q; ++i) c[i] += to_bits(acc[i * stride + x]) > thv[i] ? 1u : 0u;
  }
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) c[i] += __shfl_xor(c[i], o, kWave);
    if (lane == 0) red[wv * Q + i] = c[i];
  }
  __syncthreads();
  uint64_t* kb = reinterpret_cast<uint64_t*>(stage) + wv * kWave;
  const uint64_t below = (uint64_t(1) << lane) - 1u;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if ((i & 3) != wv) continue;
    uint32_t n = 0;
#pragma unroll
    for (int x = 0; x < kBlock / kWave; ++x) n += red[x * Q + i];
    const int cnt = cn[i];
    const bool big = n > 0 && qs[i] >= 0 && n + uint32_t(cnt) > uint32_t(kWave);
    if (lane == 0) hard[i] = big ? 1u : 0u;
    if (n == 0 || qs[i] < 0 || big) continue;
    const int64_t q = qs[i];
    int32_t* o_ids = out_ids + q * k;
    S* o_sc = out_sc + q * k;
    const A* a = acc + size_t(i) * stride;
    // the list, then the candidates in slot order
    if (lane < cnt) kb[lane] = (uint64_t(to_bits(o_sc[lane])) << 32) | uint32_t(~uint32_t(o_ids[lane]));
    uint32_t m = uint32_t(cnt);
    for (int x0 = 0; x0 < T; x0 += kWave) {
      const uint32_t v = to_bits(a[x0 + lane]);
      const bool take = v > thv[i];
      const uint64_t bal = __ballot(take);
      if (take)
        kb[m + __popcll(bal & below)] =
            (uint64_t(v) << 32) | uint32_t(~uint32_t(s_base + swz(uint32_t(x0 + lane))));
      m += uint32_t(__popcll(bal));
    }
    __builtin_amdgcn_wave_barrier();
    uint64_t key = uint64_t(lane) < m ? kb[lane] : 0ull;
    // bitonic sort of the 64 lanes' keys, descending
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
      for (int st = size >> 1; st > 0; st >>= 1) {
        const uint32_t lo = __shfl_xor(uint32_t(key), st, kWave);
        const uint32_t hi = __shfl_xor(uint32_t(key >> 32), st, kWave);
        const uint64_t other = (uint64_t(hi) << 32) | lo;
        const bool desc = (lane & size) == 0 || size == kWave;
        const bool lower = (lane & st) == 0;
        const uint64_t mx = key > other ? key : other, mn = key > other ? other : key;
        key = lower == desc ? mx : mn;
      }
    }
    const int keep = int(m) < k ? int(m) : k;
    if (lane < keep) {
      o_ids[lane] = int32_t(~uint32_t(key));
      o_sc[lane] = from_bits<S>(uint32_t(key >> 32));
    }
    if (lane == 0) {
      out_cnt[q] = keep;
      cn[i] = keep;
    }
    if (keep == k && lane == k - 1) th[i] = uint32_t(key >> 32);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (!hard[i]) continue;
    const int64_t q = qs[i];
    tile_select<S, true, A>(acc + size_t(i) * stride, T, s_base, k, out_ids + q * k, out_sc + q * k, out_cnt + q,
                            select_smem(stage, k, tmp));
    // the running state from the list the selection wrote (it ends with a barrier)
    if (threadIdx.x == 0) {
      const int keep = out_cnt[q];
      cn[i] = keep;
      th[i] = keep == k ? to_bits(out_sc[q * k + k - 1]) : 0u;
    }
    __syncthreads();
  }
}

// Head part of one tile on the vector units: thread rows s0 + 256 j (j < RB);
// each 16-byte chunk of a row feeds the byte dot products (v_dot4_u32_u8) of
// all Q queries, and each chunk of the queries' weights (one local-memory
// broadcast) feeds RB rows.
template <int Q, int HC>
__device__ __forceinline__ void head_dot4(uint32_t* acc, int stride, int T, const uint4* blk, const uint4* rh) {
  constexpr int RB = 4;
  for (int s0 = threadIdx.x; s0 < T; s0 += RB * kBlock) {
    uint32_t a[Q][RB];
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int j = 0; j < RB; ++j) a[i][j] = 0u;
#pragma unroll 1
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
        for (int i = 0; i < Q; ++i) acc[i * stride + swz(uint32_t(s))] = a[i][j];
      }
    }
  }
}

// Head part of one tile for float32 weights: thread rows s0 + 256 j (j < RB);
// each 16-byte chunk of a row (four weights, widened to fp64) feeds the fused
// multiply-adds of all Q queries, whose weights sit in local memory as fp64.
// A product of two floats is exact in fp64, so each step adds the exact
// product with one rounding, as the list walk's fp64 atomics do.
template <int Q, int HC>
__device__ __forceinline__ void head_dot_f64(double* acc, int stride, int T, const float4* blk, const double* rq) {
  constexpr int RB = 2;
  constexpr int H = 4 * HC;
  for (int s0 = threadIdx.x; s0 < T; s0 += RB * kBlock) {
    double a[Q][RB];
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int j = 0; j < RB; ++j) a[i][j] = 0.0;
#pragma unroll 1
    for (int c = 0; c < HC; ++c) {
      double v[RB][4];
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        const int s = s0 + j * kBlock;
        const float4 x = s < T ? blk[size_t(c) * T + s] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        v[j][0] = double(x.x);
        v[j][1] = double(x.y);
        v[j][2] = double(x.z);
        v[j][3] = double(x.w);
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double* w = rq + i * H + 4 * c;
        const double w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
          a[i][j] = fma(v[j][0], w0, a[i][j]);
          a[i][j] = fma(v[j][1], w1, a[i][j]);
          a[i][j] = fma(v[j][2], w2, a[i][j]);
          a[i][j] = fma(v[j][3], w3, a[i][j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int s = s0 + j * kBlock;
      if (s < T) {
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i * stride + swz(uint32_t(s))] = a[i][j];
      }
    }
  }
}

// Per-workgroup state of the join kept in local memory for the whole launch
// (registers stay free for the walk and the selection).
template <int Q>
struct GroupState {
  int64_t qs[Q];        // query ids (-1: none)
  int64_t tb[Q];        // first CSR position of each query
  uint32_t pre[Q + 1];  // prefix of the queries' tail-feature counts
  uint32_t th[Q];       // running k-th score (0 until k are held)
  int32_t cn[Q];        // running list size
  uint32_t red[4 * Q];  // selection scratch
  uint32_t hard[Q];
};

// IIB with the dense head for the queries at positions Q b .. Q b + Q - 1 of
// `order`, on tiles t0 .. t1 - 1 in ascending order (each tile is one step of
// Algorithm 1's inner loop for these queries).  Local memory: acc[Q][T +
// kAccPad] score maps | head weights of the Q queries (uint8: H bytes each;
// float32: H fp64 values each) | stage.  What does not depend on the tile
// (the queries, their tail features, their head weights, their running k-th
// scores) is loaded once; the list bounds of the next tile are loaded while
// the current tile is processed.
template <int Q, int HK, typename V>
__global__ __launch_bounds__(kBlock) void k_iibh_tiles(int32_t t0, int32_t t1, int32_t log2_tile, int32_t n_dims,
                                                       int32_t k, int64_t n_q, const int32_t* __restrict__ order,
                                                       const int64_t* __restrict__ r_ptr,
                                                       const int32_t* __restrict__ hj_d,
                                                       const V* __restrict__ hj_w,
                                                       const uint32_t* __restrict__ hj_cnt,
                                                       const void* __restrict__ rh_g,
                                                       const int64_t* __restrict__ offsets, Postings<V> P,
                                                       const void* __restrict__ head, int32_t* __restrict__ out_ids,
                                                       typename ScoreOf<V>::T* __restrict__ out_sc,
                                                       int32_t* __restrict__ out_cnt, uint64_t* __restrict__ slots) {
  using A = typename AccOf<V>::T;
  using S = typename ScoreOf<V>::T;  // also the staged list weight
  constexpr bool kU8 = sizeof(V) == 1;
  constexpr int H = 64 * HK, HC = 4 * HK;
  constexpr int RHB = kU8 ? H : 8 * H;  // bytes of one query's head weights in local memory
  extern __shared__ __align__(16) char smem[];
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  __shared__ GroupState<Q> gs;
  const int T = 1 << log2_tile;
  const int stride = T + kAccPad;
  A* acc = reinterpret_cast<A*>(smem);                                     // [Q][stride]
  char* rhp = smem + size_t(Q) * stride * sizeof(A);                       // [Q][RHB]
  char* stage = rhp + size_t(Q) * RHB;
  // thread i loads query i's state (the loads of the Q queries overlap), then
  // thread 0 turns the tail counts into their prefix
  if (threadIdx.x < Q) {
    const int i = threadIdx.x;
    const int64_t p = int64_t(blockIdx.x) * Q + i;
    const int64_t q = p < n_q ? (order ? int64_t(order[p]) : p) : -1;
    gs.qs[i] = q;
    gs.tb[i] = q >= 0 ? r_ptr[q] : 0;
    gs.pre[i + 1] = q >= 0 ? hj_cnt[q] : 0u;
    const int32_t c = q >= 0 ? out_cnt[q] : 0;
    gs.cn[i] = c;
    gs.th[i] = c == k ? to_bits(out_sc[q * k + k - 1]) : 0u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    gs.pre[0] = 0;
    for (int i = 0; i < Q; ++i) gs.pre[i + 1] += gs.pre[i];
  }
  __syncthreads();
  const uint32_t n_tail = gs.pre[Q];
  // tail list g (< n_tail) of the group: dimension, weight and score row
  // (uint8: the weight word carries the row's offset, (offset << 8) | weight)
  auto tail_list = [&](uint32_t g, int32_t* d, S* w, uint32_t* row) {
    int i = 0;
#pragma unroll
    for (int x = 1; x < Q; ++x) i += g >= gs.pre[x];
    const int64_t at = gs.tb[i] + (g - gs.pre[i]);
    *d = hj_d[at];
    if constexpr (kU8) {
      *w = (uint32_t(i * stride) << 8) | hj_w[at];
      *row = 0u;
    } else {
      *w = hj_w[at];
      *row = uint32_t(i);
    }
  };
  // the first kSegChunk tail lists stay in registers for all tiles
  int32_t d0 = 0;
  S w0 = S(0);
  uint32_t row0 = 0;
  if (threadIdx.x < n_tail) tail_list(threadIdx.x, &d0, &w0, &row0);
  if constexpr (kU8) {
    const uint4* rg = reinterpret_cast<const uint4*>(rh_g);
    uint4* rh = reinterpret_cast<uint4*>(rhp);
    for (int x = threadIdx.x; x < Q * HC; x += kBlock) {
      const int i = x / HC;
      const int64_t q = gs.qs[i];
      rh[x] = q >= 0 ? rg[q * HC + (x - i * HC)] : make_uint4(0u, 0u, 0u, 0u);
    }
  } else {
    const float* rg = reinterpret_cast<const float*>(rh_g);
    double* rq = reinterpret_cast<double*>(rhp);
    for (int x = threadIdx.x; x < Q * H; x += kBlock) {
      const int i = x / H;
      const int64_t q = gs.qs[i];
      rq[x] = q >= 0 ? double(rg[q * H + (x - i * H)]) : 0.0;
    }
  }
  int64_t nb = 0, ne = 0;  // bounds of list (tile, d0)
  if (threadIdx.x < n_tail) {
    nb = offsets[int64_t(t0) * n_dims + d0];
    ne = offsets[int64_t(t0) * n_dims + d0 + 1];
  }
  uint64_t walked = 0;
  for (int32_t tile = t0; tile < t1; ++tile) {
    const int64_t s_base = int64_t(tile) << log2_tile;
    const int64_t key0 = int64_t(tile) * n_dims;
    const int64_t beg = nb;
    const uint32_t len = uint32_t(ne - nb);
    if (tile + 1 < t1 && threadIdx.x < n_tail) {
      nb = offsets[key0 + n_dims + d0];
      ne = offsets[key0 + n_dims + d0 + 1];
    }
    __syncthreads();  // the head weights are in place; the previous tile's selection is done with acc and stage
    if constexpr (kU8)
      head_dot4<Q, HC>(acc, stride, T, reinterpret_cast<const uint4*>(head) + size_t(tile) * HC * T,
                       reinterpret_cast<const uint4*>(rhp));
    else
      head_dot_f64<Q, H / 4>(acc, stride, T, reinterpret_cast<const float4*>(head) + size_t(tile) * (H / 4) * T,
                             reinterpret_cast<const double*>(rhp));
    // tail lists of all Q queries (stage_write's scan orders the head stores
    // before the walk's atomics)
    for (uint32_t c0 = 0; c0 < n_tail; c0 += kSegChunk) {
      const int n = int(n_tail - c0 < uint32_t(kSegChunk) ? n_tail - c0 : uint32_t(kSegChunk));
      int64_t b = beg;
      uint32_t l = len, rw = row0;
      S w = w0;
      if (c0 > 0) {
        b = 0;
        l = 0;
        w = S(0);
        rw = 0;
        if (threadIdx.x < n) {
          int32_t d;
          tail_list(c0 + threadIdx.x, &d, &w, &rw);
          b = offsets[key0 + d];
          l = uint32_t(offsets[key0 + d + 1] - b);
        }
      } else if (threadIdx.x >= n) {
        l = 0;
      }
      const uint32_t total = stage_write<S>(stage, tmp, n, b, l, w, rw);
      if constexpr (kU8)
        walk_lists<uint8_t, uint32_t, true>(acc, stage, n, total, P);
      else
        walk_lists<float, float, true, double>(acc, stage, n, total, P, stride);
      if (slots) walked += block_sum(threadIdx.x < n ? l : 0u, tmp);
      __syncthreads();
    }
    if (n_tail == 0) __syncthreads();
    group_select<Q, A, S>(acc, stride, T, s_base, k, gs.qs, out_ids, out_sc, out_cnt, stage, tmp, gs.red, gs.hard,
                          gs.th, gs.cn);
  }
  if (threadIdx.x == 0 && slots)
    atomicAdd((unsigned long long*)&slots[KNNJ_STAT_POSTINGS * 256 + (blockIdx.x & 255)], (unsigned long long)walked);
}

// Head weights are uint8 or float32, like the index's values.
static size_t weight_bytes(int dtype) { return dtype == KNNJ_U8 ? 1 : 4; }

size_t head_smem_bytes(int tile, int k, int H, int dtype) {
  return size_t(kHeadQ) * (tile + kAccPad) * acc_bytes(dtype) + size_t(kHeadQ) * H * (dtype == KNNJ_U8 ? 1 : 8) +
         stage_bytes(k);
}

knnj_status launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

knnj_status build_head(Index* ix, hipStream_t st) {
  const int H = ix->head_h;
  const size_t bytes = size_t(ix->n_tiles) * size_t(ix->tile) * H * weight_bytes(ix->dtype);
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
    if (ix->n_rows > 0) {
      const unsigned g = unsigned((ix->n_rows + 3) / 4 < 65536 ? (ix->n_rows + 3) / 4 : 65536);
      if (ix->dtype == KNNJ_U8)
        k_head_fill<uint8_t><<<g, kBlock, 0, st>>>(ix->n_rows, ix->log2_tile, H, ix->s_indptr, ix->s_indices,
                                                   (const uint8_t*)ix->s_values, ix->head_pos, ix->head_blk);
      else
        k_head_fill<float><<<g, kBlock, 0, st>>>(ix->n_rows, ix->log2_tile, H, ix->s_indptr, ix->s_indices,
                                                 (const float*)ix->s_values, ix->head_pos,
                                                 reinterpret_cast<float*>(ix->head_blk));
    }
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
  const size_t wb = weight_bytes(ix->dtype);
  const int64_t cq = n > ix->hj_cap_q ? n : ix->hj_cap_q;
  const int64_t cz = (nnz > ix->hj_cap_nnz ? nnz : ix->hj_cap_nnz) + 1;
  if (hipMalloc(&ix->hj_cnt, sizeof(uint32_t) * cq) != hipSuccess ||
      hipMalloc(&ix->hj_d, sizeof(int32_t) * cz) != hipSuccess || hipMalloc(&ix->hj_w, wb * cz) != hipSuccess ||
      hipMalloc(&ix->hj_rh, size_t(cq) * ix->head_h * wb) != hipSuccess)
    return fail(KNNJ_ENOMEM, "dense-head join scratch allocation failed");
  ix->hj_cap_q = cq;
  ix->hj_cap_nnz = cz;
  return KNNJ_OK;
}

template <typename V>
static knnj_status launch_head_tiles(Index* ix, const knnj_csr* R, int32_t k, const int32_t* order, int32_t G,
                                     int32_t* ids, typename ScoreOf<V>::T* sc, int32_t* cnt, uint64_t* slots,
                                     Postings<V> P, hipStream_t st) {
  const int64_t n = R->n_rows;
  const int H = ix->head_h;
  k_head_prep<V><<<unsigned((n + 3) / 4), kBlock, 0, st>>>(n, H, R->indptr, R->indices, (const V*)R->values,
                                                          ix->head_pos, ix->hj_d, reinterpret_cast<V*>(ix->hj_w),
                                                          ix->hj_cnt, reinterpret_cast<V*>(ix->hj_rh));
  const size_t smem = head_smem_bytes(ix->tile, k, H, ix->dtype);
  const unsigned g = unsigned((n + kHeadQ - 1) / kHeadQ);
  for (int32_t t = 0; t < ix->n_tiles; t += G) {
    const int32_t t1 = t + G < ix->n_tiles ? t + G : ix->n_tiles;
#define KNNJ_IIBH(HK)                                                                                              \
  k_iibh_tiles<kHeadQ, HK, V><<<g, kBlock, smem, st>>>(t, t1, ix->log2_tile, ix->n_dims, k, n, order, R->indptr,   \
                                                      ix->hj_d, reinterpret_cast<const V*>(ix->hj_w), ix->hj_cnt,  \
                                                      ix->hj_rh, ix->offsets, P, ix->head_blk, ids, sc, cnt, slots);
    switch (H / 64) {
      case 1: KNNJ_IIBH(1) break;
      case 2: KNNJ_IIBH(2) break;
      case 3: KNNJ_IIBH(3) break;
      default: KNNJ_IIBH(4) break;
    }
#undef KNNJ_IIBH
  }
  return KNNJ_OK;
}

knnj_status launch_iib_head(Index* ix, const knnj_csr* R, int32_t k, const int32_t* order, int32_t tiles_per_launch,
                            int32_t* ids, void* sc, int32_t* cnt, uint64_t* slots, hipStream_t st) {
  const int64_t n = R->n_rows;
  if (n == 0) return KNNJ_OK;
  const int H = ix->head_h;
  knnj_status rc = ensure_head_scratch(ix, n, R->nnz);
  if (rc != KNNJ_OK) return rc;
  const int64_t rh_words = n * H * int64_t(weight_bytes(ix->dtype)) / 4;
  if ((rc = launch_fill_u32(reinterpret_cast<uint32_t*>(ix->hj_rh), rh_words, 0u, st)) != KNNJ_OK) return rc;
  const int32_t G = tiles_per_launch > 0 ? tiles_per_launch : kHeadTiles;
  if (ix->dtype == KNNJ_U8)
    rc = launch_head_tiles<uint8_t>(ix, R, k, order, G, ids, (uint32_t*)sc, cnt, slots,
                                    Postings<uint8_t>{reinterpret_cast<const uint4*>(ix->post_u8)}, st);
  else
    rc = launch_head_tiles<float>(ix, R, k, order, G, ids, (float*)sc, cnt, slots,
                                  Postings<float>{reinterpret_cast<const uint2*>(ix->post_s),
                                                  reinterpret_cast<const float4*>(ix->post_w)},
                                  st);
  if (rc != KNNJ_OK) return rc;
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

}  // namespace knnj
