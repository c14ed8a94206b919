// IIIB: threshold-refined inverted index (Algorithm 4) on the GPU.
//
// Per block of R rows (the B_r of Algorithm 1):
//   k_block_stats   freq_d(B_r) and maxWeight_d(B_r) (Algorithm 4's block statistics)
//   k_split_rows    for every s: its features in the block's dimension order
//                   (frequency in B_r descending, then d ascending), the running
//                   bound t = sum maxWeight_d * w over that order (Algorithm 4's split),
//                   and the level of t on a fixed geometric ladder tau_1 < tau_2 < ...
//                   (a feature is indexed for a threshold tau_l iff its t >= tau_l).
//                   Writes the row in that order ("fwd") and counts entries per
//                   (tile, d, level).
//   k_bucket_starts per list (tile, d): bucket starts in level-descending order
//   k_split_scatter place every entry in its list at its level bucket
//   list sort       ascending s inside every level bucket
// Join, per S tile (one workgroup per query; k_iiib_tile):
//   theta = the query's running pruneScore (or its seed); lambda = level(theta):
//   walk only the prefix of each list with level >= lambda (the indexed part,
//   Algorithm 4's accumulation); then for every s with A[s] != 0 add dot(r, s')
//   over the row's leading features with level < lambda (the unindexed part,
//   Algorithm 4's completion); select.
//
// The split rule is "index once t >= tau" with tau <= theta, so every s whose
// score reaches theta shares an indexed feature with r (Theorem 1's argument
// with >= in place of >): exact for running and for seeded thresholds.
#include <mutex>
#include <type_traits>

#include "walk.hpp"

namespace knnj {

// ---------------------------------------------------------------- level ladder
// tau[0] = 0 (level 0: every feature), tau[l] = 2^(b + (l - 1) / 4) for l >= 1,
// b = 8 for u8 scores and b = -12 for float scores.
__constant__ uint32_t c_tau_u8[kLevels];
__constant__ float c_tau_f32[kLevels];

// The ladder lives in each device's constant memory: uploaded once per device.
static std::mutex g_tau_mu;
static bool g_tau_ready[64] = {};
static knnj_status upload_tau() {
  int dev = -1;
  KNNJ_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_tau_mu);
  if (dev >= 0 && dev < 64 && g_tau_ready[dev]) return KNNJ_OK;
  uint32_t tu[kLevels];
  float tf[kLevels];
  tu[0] = 0;
  tf[0] = 0.0f;
  for (int l = 1; l < kLevels; ++l) {
    tu[l] = uint32_t(ceil(ldexp(1.0, 8) * pow(2.0, (l - 1) / 4.0)));
    tf[l] = float(ldexp(1.0, -12) * pow(2.0, (l - 1) / 4.0));
  }
  KNNJ_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tau_u8), tu, sizeof(tu)));
  KNNJ_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tau_f32), tf, sizeof(tf)));
  if (dev >= 0 && dev < 64) g_tau_ready[dev] = true;
  return KNNJ_OK;
}

// largest l with tau[l] <= t
__device__ __forceinline__ uint32_t level_of(uint32_t t) {
  int lo = 0, hi = kLevels - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (c_tau_u8[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return uint32_t(lo);
}
__device__ __forceinline__ uint32_t level_of(float t) {
  int lo = 0, hi = kLevels - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (c_tau_f32[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return uint32_t(lo);
}
__device__ __forceinline__ uint32_t tau_of(uint32_t l, uint32_t) { return c_tau_u8[l]; }
__device__ __forceinline__ float tau_of(uint32_t l, float) { return c_tau_f32[l]; }

// fwd entry: u8 (d << 14) | (w << 6) | level, d < 2^18; f32 (d << 6) | level + weight array
constexpr int kFwdMaxDimsU8 = 1 << 18;

// ---------------------------------------------------------------- statistics
template <typename V>
__global__ void k_block_stats(int64_t r0, int64_t r1, const int64_t* __restrict__ r_ptr,
                              const int32_t* __restrict__ r_idx, const V* __restrict__ r_val,
                              uint32_t* __restrict__ freq, uint32_t* __restrict__ maxw) {
  const int64_t b = r_ptr[r0], e = r_ptr[r1];
  for (int64_t j = b + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < e; j += int64_t(gridDim.x) * blockDim.x) {
    const int32_t d = r_idx[j];
    atomicAdd(&freq[d], 1u);
    uint32_t bits;
    if constexpr (sizeof(V) == 1) bits = r_val[j];
    else bits = __float_as_uint(r_val[j]);  // positive floats order like their bits
    atomicMax(&maxw[d], bits);
  }
}

// ---------------------------------------------------------------- split
// One workgroup of 64 threads per S row.  Local memory: p 64-bit keys, p = the
// next power of two >= the longest row.
template <typename V>
__global__ __launch_bounds__(kWave) void k_split_rows(int64_t n_s, int32_t n_dims, int32_t log2_tile, int32_t p,
                                                      const int64_t* __restrict__ s_ptr,
                                                      const int32_t* __restrict__ s_idx,
                                                      const V* __restrict__ s_val, const uint32_t* __restrict__ freq,
                                                      const uint32_t* __restrict__ maxw,
                                                      uint32_t* __restrict__ fwd, float* __restrict__ fwd_w,
                                                      uint32_t* __restrict__ cnt3) {
  extern __shared__ __align__(16) char smem[];
  uint64_t* key = reinterpret_cast<uint64_t*>(smem);
  const int64_t row = blockIdx.x;
  const int64_t b = s_ptr[row];
  const int len = int(s_ptr[row + 1] - b);
  if (len == 0) return;
  int pp = 1;
  while (pp < len) pp <<= 1;
  (void)p;
  // key: frequency descending, then d ascending; low 12 bits keep the position
  for (int j = threadIdx.x; j < pp; j += kWave) {
    if (j < len) {
      const uint32_t d = uint32_t(s_idx[b + j]);
      key[j] = (uint64_t(0xffffffffu - freq[d]) << 32) | (uint64_t(d) << 12) | uint64_t(j);
    } else {
      key[j] = ~0ull;
    }
  }
  __syncthreads();
  for (int size = 2; size <= pp; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (pp >> 1); i += kWave) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t x = key[lo], y = key[hi];
        if ((x > y) == up) {
          key[lo] = y;
          key[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  // running bound over the sorted order: each thread takes a contiguous run
  const int per = (len + kWave - 1) / kWave;
  const int j0 = threadIdx.x * per;
  const int j1 = j0 + per < len ? j0 + per : len;
  using Acc = typename std::conditional<sizeof(V) == 1, uint32_t, double>::type;
  Acc part = Acc(0);
  for (int j = j0; j < j1; ++j) {
    const uint64_t kk = key[j];
    const uint32_t d = uint32_t(kk >> 12) & 0xfffffu;
    const int pos = int(kk & 0xfffu);
    if constexpr (sizeof(V) == 1) part += maxw[d] * uint32_t(s_val[b + pos]);
    else part += double(__uint_as_float(maxw[d])) * double(s_val[b + pos]);
  }
  // exclusive scan of the parts across the wave
  Acc x = part;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const Acc y = __shfl_up(x, o, kWave);
    if (int(threadIdx.x) >= o) x += y;
  }
  Acc run = x - part;
  const int64_t tile_key = (row >> log2_tile) * int64_t(n_dims);
  for (int j = j0; j < j1; ++j) {
    const uint64_t kk = key[j];
    const uint32_t d = uint32_t(kk >> 12) & 0xfffffu;
    const int pos = int(kk & 0xfffu);
    uint32_t lvl;
    if constexpr (sizeof(V) == 1) {
      const uint32_t w = s_val[b + pos];
      run += maxw[d] * w;
      lvl = level_of(run);
      fwd[b + j] = (d << 14) | (w << 6) | lvl;
    } else {
      const float w = s_val[b + pos];
      run += double(__uint_as_float(maxw[d])) * double(w);
      // round the bound up so a float compare never understates it
      const float tf = __double2float_ru(run);
      lvl = level_of(tf);
      fwd[b + j] = (d << 6) | lvl;
      fwd_w[b + j] = w;
    }
    atomicAdd(&cnt3[(tile_key + d) * kLevels + lvl], 1u);
  }
}

// Per list: turn level counts into bucket starts (level 63 first).  After the
// scatter each slot holds the end of its bucket, i.e. the number of entries of
// the list with level >= l: that is the cut table the join reads.
__global__ void k_bucket_starts(int64_t n_keys, uint32_t* __restrict__ cnt3) {
  const int64_t key = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (key >= n_keys) return;
  uint32_t* c = cnt3 + key * kLevels;
  uint32_t run = 0;
  for (int l = kLevels - 1; l >= 0; --l) {
    const uint32_t v = c[l];
    c[l] = run;
    run += v;
  }
}

template <typename V>
__global__ __launch_bounds__(kWave) void k_split_scatter(int64_t n_s, int32_t n_dims, int32_t log2_tile,
                                                         const int64_t* __restrict__ s_ptr,
                                                         const uint32_t* __restrict__ fwd,
                                                         const float* __restrict__ fwd_w,
                                                         const int64_t* __restrict__ offsets,
                                                         uint32_t* __restrict__ cnt3, uint64_t* __restrict__ rec) {
  const int64_t row = blockIdx.x;
  const int64_t b = s_ptr[row], e = s_ptr[row + 1];
  const int64_t tile_key = (row >> log2_tile) * int64_t(n_dims);
  const uint32_t s_local = uint32_t(row) & ((1u << log2_tile) - 1u);
  for (int64_t j = b + threadIdx.x; j < e; j += kWave) {
    const uint32_t f = fwd[j];
    uint32_t d, lvl, payload;
    if constexpr (sizeof(V) == 1) {
      d = f >> 14;
      lvl = f & 63u;
      payload = (swz(s_local) << 16) | (((f >> 6) & 0xffu) << 8) | lvl;
    } else {
      d = f >> 6;
      lvl = f & 63u;
      payload = __float_as_uint(fwd_w[j]);
    }
    const int64_t key = tile_key + d;
    const uint32_t pos = atomicAdd(&cnt3[key * kLevels + lvl], 1u);
    rec[offsets[key] + pos] = (uint64_t((uint32_t(kLevels - 1 - lvl) << 16) | s_local) << 32) | payload;
  }
}

// Lists longer than 2048 entries arrive grouped by level (the scatter put each
// entry in its level bucket); sort every bucket by s_local.  s_local values of
// one list are distinct, so each pass drops payloads into slot s_local of a
// local array and reads the slots back in order (payloads are never 0 bits).
constexpr int kBucketSlots = 8192;
__global__ void k_sort_buckets(const int64_t* __restrict__ offsets, const int64_t* __restrict__ big,
                               const uint32_t* __restrict__ n_big, const uint32_t* __restrict__ cut,
                               uint64_t* __restrict__ rec, uint64_t* __restrict__ out_tmp, int32_t tile) {
  extern __shared__ uint32_t slots[];  // kBucketSlots
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  __shared__ uint32_t written;
  const uint32_t nb = *n_big;
  for (uint32_t item = blockIdx.x; item < nb; item += gridDim.x) {
  const int64_t key = big[item];
  const int64_t b = offsets[key], e = offsets[key + 1];
  if (e - b <= 2048) continue;
  const uint32_t* c = cut + key * kLevels;
  uint32_t beg = 0;
  for (int l = kLevels - 1; l >= 0; --l) {
    const uint32_t end = c[l];  // entries with level >= l
    if (end - beg > 1) {
      const uint64_t hw = uint64_t(kLevels - 1 - l) << 16;
      if (threadIdx.x == 0) written = 0;
      for (int32_t lo = 0; lo < tile; lo += kBucketSlots) {
        for (int i = threadIdx.x; i < kBucketSlots; i += kBlock) slots[i] = 0u;
        __syncthreads();
        for (uint32_t j = beg + threadIdx.x; j < end; j += kBlock) {
          const uint64_t x = rec[b + j];
          const int32_t s = int32_t((x >> 32) & 0xffffu);
          if (s >= lo && s < lo + kBucketSlots) slots[s - lo] = uint32_t(x);
        }
        __syncthreads();
        constexpr int per = kBucketSlots / kBlock;
        const int t0 = threadIdx.x * per;
        uint32_t cn = 0;
        for (int i = 0; i < per; ++i) cn += slots[t0 + i] != 0u;
        uint32_t total;
        uint32_t ex = block_exclusive_scan(cn, tmp, &total);
        const uint32_t w0 = written;
        for (int i = 0; i < per; ++i) {
          const uint32_t v = slots[t0 + i];
          if (v != 0u) out_tmp[b + beg + w0 + ex++] = ((hw | uint64_t(lo + t0 + i)) << 32) | v;
        }
        __syncthreads();
        if (threadIdx.x == 0) written = w0 + total;
        __syncthreads();
      }
      for (uint32_t j = beg + threadIdx.x; j < end; j += kBlock) rec[b + j] = out_tmp[b + j];
      __syncthreads();
    }
    beg = end;
  }
  }
}

// grid-stride (capped grid: a dispatch counts its work-items in 32 bits)
__global__ void k_finalize_iiib_u8(const uint64_t* __restrict__ rec, int64_t n, uint32_t* __restrict__ post) {
  const int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) post[i] = uint32_t(rec[i]);
}
__global__ void k_finalize_iiib_f32(const uint64_t* __restrict__ rec, int64_t n, uint16_t* __restrict__ ps,
                                    float* __restrict__ pw) {
  const int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) {
    const uint64_t x = rec[i];
    ps[i] = uint16_t(swz(uint32_t(x >> 32) & 0xffffu));
    pw[i] = __uint_as_float(uint32_t(x));
  }
}

// ---------------------------------------------------------------- join
// r as an open-addressing table in local memory: 2^lg slots of (d, weight),
// empty slots hold d = -1; multiplicative hashing, linear probing.  The table
// has at least twice as many slots as r has features, so probes stay short.
template <typename RW>
struct RHash {
  int32_t* key;
  RW* val;
  int32_t lg;
  __device__ __forceinline__ uint32_t slot(int32_t d) const { return (uint32_t(d) * 0x9e3779b1u) >> (32 - lg); }
  __device__ __forceinline__ void insert(int32_t d, RW w) {
    const uint32_t mask = (1u << lg) - 1u;
    for (uint32_t h = slot(d);; h = (h + 1u) & mask) {
      const int32_t prev = atomicCAS(&key[h], -1, d);
      if (prev == -1 || prev == d) {
        val[h] = w;
        return;
      }
    }
  }
  __device__ __forceinline__ RW find(int32_t d) const {
    const uint32_t mask = (1u << lg) - 1u;
    for (uint32_t h = slot(d);; h = (h + 1u) & mask) {
      const int32_t kk = key[h];
      if (kk == d) return val[h];
      if (kk == -1) return RW(0);
    }
  }
};

__host__ __device__ inline size_t r_region_bytes(int32_t n_dims, size_t wbytes, int32_t hash_log2) {
  if (hash_log2 > 0) return (size_t(4) + (wbytes < 4 ? 4 : wbytes)) << hash_log2;
  return (size_t(n_dims) * wbytes + 15) & ~size_t(15);
}

// IIIB on tile `tile`.  Queries: q0 + blockIdx.x, or (fallback pass) qlist[blockIdx.x]
// for blockIdx.x < *qcount.  Local memory: acc[T] | r as a dense array over the
// dimensions | stage.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_iiib_tile(
    int32_t tile, int32_t log2_tile, int32_t n_dims, int32_t k, int64_t q0, const int32_t* __restrict__ order,
    const int32_t* __restrict__ qlist, const uint32_t* __restrict__ qcount, const int64_t* __restrict__ r_ptr, const int32_t* __restrict__ r_idx,
    const V* __restrict__ r_val, const int64_t* __restrict__ offsets, const uint32_t* __restrict__ cut,
    Postings<V> P, const int64_t* __restrict__ s_ptr, const uint32_t* __restrict__ fwd,
    const float* __restrict__ fwd_w, const float* __restrict__ seed, int32_t level_drop, int32_t bound_filter,
    int32_t r_hash_log2, int32_t* __restrict__ out_ids, typename ScoreOf<V>::T* __restrict__ out_sc,
    int32_t* __restrict__ out_cnt, uint64_t* __restrict__ slots) {
  using S = typename ScoreOf<V>::T;
  using A = typename AccOf<V>::T;
  extern __shared__ __align__(16) char smem[];
  __shared__ uint32_t tmp[kBlock / kWave + 1];
  int64_t q;
  if (qlist) {
    if (blockIdx.x >= *qcount) return;
    q = qlist[blockIdx.x];
  } else {
    q = order ? int64_t(order[q0 + blockIdx.x]) : q0 + blockIdx.x;
  }
  const int T = 1 << log2_tile;
  A* acc = reinterpret_cast<A*>(smem);
  // r for the completion: a dense array over the dimensions, or (large n_dims,
  // r_hash_log2 > 0) an open-addressing table keyed by d in local memory
  using RW = typename std::conditional<sizeof(V) == 1, uint8_t, float>::type;
  const size_t rbytes = r_region_bytes(n_dims, sizeof(RW), r_hash_log2);
  const size_t abytes = size_t(T) * sizeof(A);
  RW* rdense = reinterpret_cast<RW*>(smem + abytes);
  RHash<RW> rh{reinterpret_cast<int32_t*>(smem + abytes),
               reinterpret_cast<RW*>(smem + abytes + (size_t(4) << (r_hash_log2 > 0 ? r_hash_log2 : 0))),
               r_hash_log2};
  char* stage = smem + abytes + rbytes;
  const int64_t s_base = int64_t(tile) << log2_tile;

  for (int i = threadIdx.x; i < int(abytes / 16); i += kBlock)
    reinterpret_cast<uint4*>(acc)[i] = make_uint4(0, 0, 0, 0);
  if (r_hash_log2 > 0) {
    for (int i = threadIdx.x; i < (1 << r_hash_log2); i += kBlock) rh.key[i] = -1;
  } else {
    for (size_t i = threadIdx.x; i < rbytes / 16; i += kBlock) reinterpret_cast<uint4*>(rdense)[i] = make_uint4(0, 0, 0, 0);
  }
  __syncthreads();
  const int64_t rb = r_ptr[q], re = r_ptr[q + 1];
  for (int64_t j = rb + threadIdx.x; j < re; j += kBlock) {
    if (r_hash_log2 > 0) rh.insert(r_idx[j], RW(r_val[j]));
    else rdense[r_idx[j]] = r_val[j];
  }

  // threshold: the running pruneScore, raised by the seed if one is given
  const int cnt = out_cnt[q];
  S theta = cnt == k ? out_sc[q * k + k - 1] : S(0);
  if (seed) {
    const float sd = seed[q];
    if constexpr (sizeof(V) == 1) {
      // integer scores: a seed x means "score >= ceil(x)"
      const float c = ceilf(sd);
      const S si = c >= 4294967040.0f ? S(0xffffff00u) : (c > 0.0f ? S(c) : S(0));
      theta = si > theta ? si : theta;
    } else {
      theta = sd > theta ? sd : theta;
    }
  }
  int lam = int(level_of(theta)) - level_drop;
  if (lam < 0) lam = 0;
  const uint32_t lambda = uint32_t(lam);

  const int64_t key0 = int64_t(tile) * n_dims;
  uint64_t walked = 0;
  for (int64_t cb = rb; cb < re; cb += kSegChunk) {
    const int n = int(re - cb < kSegChunk ? re - cb : kSegChunk);
    const uint32_t total = stage_lists<V, S>(stage, tmp, key0, r_idx, r_val, cb, n, offsets, cut, lambda);
    walk_lists<V, S, false, A>(acc, stage, n, total, P);
    if (slots) {
      uint32_t l = threadIdx.x < n ? reinterpret_cast<const uint32_t*>(stage + kMetaOff)[threadIdx.x] >> 2 : 0u;
      walked += block_sum(l, tmp);
    }
    __syncthreads();
  }

  // completion (Algorithm 4): every s with A[s] != 0 gets dot(r, s') over
  // the leading features of its row whose level is below lambda
  uint32_t n_cand = 0, n_compl = 0;
  if (lambda > 0) {
    const S tau = tau_of(lambda, S(0));
    for (int a = threadIdx.x; a < T; a += kBlock) {
      const A v = acc[a];
      if (v == A(0)) continue;
      if (bound_filter && v + A(tau) <= A(theta)) {
        // A[s] + (bound of the unindexed part, < tau) < theta: s cannot reach theta
        acc[a] = A(0);
        continue;
      }
      const int64_t row = s_base + int64_t(swz(uint32_t(a)));
      const int64_t e1 = s_ptr[row + 1];
      A sum = A(0);
      int64_t e = s_ptr[row];
      for (; e < e1; ++e) {
        const uint32_t f = fwd[e];
        if ((f & 63u) >= lambda) break;
        if constexpr (sizeof(V) == 1) {
          const uint32_t d = f >> 14;
          sum += uint32_t(r_hash_log2 > 0 ? rh.find(int32_t(d)) : rdense[d]) * ((f >> 6) & 0xffu);
        } else {
          const uint32_t d = f >> 6;
          sum += A(r_hash_log2 > 0 ? rh.find(int32_t(d)) : rdense[d]) * A(fwd_w[e]);
        }
      }
      acc[a] = v + sum;
      ++n_cand;
      n_compl += uint32_t(e - s_ptr[row]);
    }
    __syncthreads();
  }
  tile_select<S, true, A>(acc, T, s_base, k, out_ids + q * k, out_sc + q * k, out_cnt + q,
                          select_smem(stage, k, tmp));
  if (slots) {
    const uint32_t c1 = block_sum(n_cand, tmp);
    const uint32_t c2 = block_sum(n_compl, tmp);
    if (threadIdx.x == 0) {
      atomicAdd((unsigned long long*)&slots[KNNJ_STAT_POSTINGS * 256 + (blockIdx.x & 255)], (unsigned long long)walked);
      atomicAdd((unsigned long long*)&slots[KNNJ_STAT_CANDIDATES * 256 + (blockIdx.x & 255)], (unsigned long long)c1);
      atomicAdd((unsigned long long*)&slots[KNNJ_STAT_COMPLETION * 256 + (blockIdx.x & 255)], (unsigned long long)c2);
    }
  }
}

// Survivor check of a seeded pass: the result of q is exact iff it holds k
// neighbours whose k-th score reaches the seed (every s scoring >= the seed was
// found).  Other queries are reset and queued for a second pass.  A queued query
// that held k neighbours keeps their k-th score as its new seed: k real vectors
// score at least that much, so it never exceeds the true k-th score and the
// second pass needs no check.
template <typename S>
__global__ void k_survivors(int64_t q0, int64_t n, int32_t k, const float* __restrict__ seed,
                            float* __restrict__ seed2, int32_t* __restrict__ ids, S* __restrict__ sc,
                            int32_t* __restrict__ cnt, int32_t* __restrict__ qlist, uint32_t* __restrict__ qcount,
                            uint8_t* __restrict__ fb_out, uint64_t* __restrict__ slots) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t q = q0 + i;
  const float sd = seed[q];
  const int c = cnt[q];
  bool fb = false;
  if (sd > 0.0f) {
    if constexpr (std::is_integral<S>::value) {
      // integer scores: the threshold used was ceil(seed)
      fb = !(c == k && double(sc[q * k + k - 1]) >= ceil(double(sd)));
    } else {
      fb = !(c == k && sc[q * k + k - 1] >= sd);
    }
  }
  if (fb_out) fb_out[q] = fb ? 1 : 0;
  if (!fb) return;
  // a float lower bound of the k-th score, rounded down
  float lb = 0.0f;
  if (c == k) {
    if constexpr (std::is_integral<S>::value) lb = __uint2float_rd(uint32_t(sc[q * k + k - 1]));
    else lb = float(sc[q * k + k - 1]);
  }
  seed2[q] = lb;
  qlist[atomicAdd(qcount, 1u)] = int32_t(q);
  for (int j = 0; j < k; ++j) {
    ids[q * k + j] = -1;
    sc[q * k + j] = S(0);
  }
  cnt[q] = 0;
  if (slots) atomicAdd((unsigned long long*)&slots[KNNJ_STAT_FALLBACKS * 256 + (i & 255)], 1ull);
}

// ---------------------------------------------------------------- host driver
knnj_status launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
__global__ void k_sort_small(const int64_t* __restrict__ offsets, int64_t n_keys, uint64_t* __restrict__ rec,
                             int64_t* __restrict__ big, uint32_t* __restrict__ n_big);
__global__ void k_sort_mid(const int64_t* __restrict__ offsets, const int64_t* __restrict__ big,
                           const uint32_t* __restrict__ n_big, uint64_t* __restrict__ rec);
size_t tile_smem_bytes(int tile, int k, size_t acc_b);

constexpr unsigned kSortGrid = 4096;  // workgroups striding over the queued long lists

// Index-level IIIB buffers (first use) and per-query ones (grow-only).  The only
// allocations of an IIIB join; a later join with no more queries allocates nothing.
// Frees the per-index IIIB buffers (all of them: a partial set is never kept).
static void free_iiib_buffers(Index* ix) {
  void** bufs[] = {(void**)&ix->iiib_fwd,    (void**)&ix->iiib_cut,    (void**)&ix->iiib_fwd_w,
                   (void**)&ix->iiib_post,   (void**)&ix->iiib_post_s, (void**)&ix->iiib_post_w,
                   (void**)&ix->iiib_freq,   (void**)&ix->iiib_maxw,   (void**)&ix->iiib_big,
                   (void**)&ix->iiib_small,  (void**)&ix->iiib_out_tmp};
  for (void** b : bufs) {
    (void)hipFree(*b);
    *b = nullptr;
  }
}

// Whether every per-index IIIB buffer of this value type is allocated.
static bool iiib_allocated(const Index* ix) {
  const bool common = ix->iiib_fwd && ix->iiib_cut && ix->iiib_freq && ix->iiib_maxw && ix->iiib_big &&
                      ix->iiib_small && ix->iiib_out_tmp;
  return common && (ix->dtype == KNNJ_U8 ? ix->iiib_post != nullptr
                                         : (ix->iiib_post_s && ix->iiib_post_w && ix->iiib_fwd_w));
}

// Allocates the per-index IIIB buffers once, all or nothing: after a failed
// allocation every buffer is released again, so a later call retries instead of
// running on a partial set.
static knnj_status ensure_iiib(Index* ix, int64_t n_r) {
  const int64_t n_keys = int64_t(ix->n_tiles) * ix->n_dims;
  const size_t nnz1 = size_t(ix->nnz > 0 ? ix->nnz : 1);
  if (!iiib_allocated(ix)) {
    free_iiib_buffers(ix);
    if (hipMalloc(&ix->iiib_fwd, sizeof(uint32_t) * nnz1) != hipSuccess ||
        hipMalloc(&ix->iiib_cut, sizeof(uint32_t) * size_t(n_keys) * kLevels) != hipSuccess ||
        (ix->dtype == KNNJ_F32 && hipMalloc(&ix->iiib_fwd_w, sizeof(float) * nnz1) != hipSuccess) ||
        (ix->dtype == KNNJ_U8 && hipMalloc(&ix->iiib_post, sizeof(uint32_t) * (nnz1 + kPostPad)) != hipSuccess) ||
        (ix->dtype == KNNJ_F32 && (hipMalloc(&ix->iiib_post_s, sizeof(uint16_t) * (nnz1 + kPostPad)) != hipSuccess ||
                                   hipMalloc(&ix->iiib_post_w, sizeof(float) * (nnz1 + kPostPad)) != hipSuccess)) ||
        hipMalloc(&ix->iiib_freq, sizeof(uint32_t) * ix->n_dims) != hipSuccess ||
        hipMalloc(&ix->iiib_maxw, sizeof(uint32_t) * ix->n_dims) != hipSuccess ||
        hipMalloc(&ix->iiib_big, sizeof(int64_t) * (n_keys > 0 ? n_keys : 1)) != hipSuccess ||
        hipMalloc(&ix->iiib_small, sizeof(uint32_t) * 8) != hipSuccess ||
        hipMalloc(&ix->iiib_out_tmp, sizeof(uint64_t) * nnz1) != hipSuccess) {
      free_iiib_buffers(ix);
      return fail(KNNJ_ENOMEM, "device allocation for the IIIB index failed");
    }
  }
  if (n_r > ix->iiib_qcap) {
    (void)hipDeviceSynchronize();
    (void)hipFree(ix->iiib_qlist);
    (void)hipFree(ix->iiib_seed2);
    ix->iiib_qlist = nullptr;
    ix->iiib_seed2 = nullptr;
    ix->iiib_qcap = 0;
    if (hipMalloc(&ix->iiib_qlist, sizeof(int32_t) * n_r) != hipSuccess ||
        hipMalloc(&ix->iiib_seed2, sizeof(float) * n_r) != hipSuccess)
      return fail(KNNJ_ENOMEM, "device allocation for the IIIB fallback queue failed");
    ix->iiib_qcap = n_r;
  }
  return KNNJ_OK;
}

// A dense copy of r is used when it takes at most 32 KB; otherwise a hash table
// with 2^lg >= 2 * (longest row of R) slots.
static int32_t r_hash_log2(const Index* ix, int32_t max_r) {
  const size_t wb = ix->dtype == KNNJ_U8 ? 1 : 4;
  if (size_t(ix->n_dims) * wb <= 32768) return 0;
  int32_t lg = 4;
  while ((1 << lg) < 2 * (max_r > 0 ? max_r : 1)) ++lg;
  return lg;
}

static size_t iiib_smem(const Index* ix, int k, int32_t hash_lg) {
  return tile_smem_bytes(ix->tile, k, acc_bytes(ix->dtype)) +
         r_region_bytes(ix->n_dims, ix->dtype == KNNJ_U8 ? 1 : 4, hash_lg);
}

// Builds the IIIB index of R rows [r0, r1) into ix->iiib_*.  Enqueues kernels only.
template <typename V>
static knnj_status build_block(Index* ix, const knnj_csr* R, int64_t r0, int64_t r1, hipStream_t st) {
  const int64_t n_keys = int64_t(ix->n_tiles) * ix->n_dims;
  uint32_t* n_big = ix->iiib_small;
  knnj_status rc;
  if ((rc = launch_fill_u32(ix->iiib_freq, ix->n_dims, 0u, st)) != KNNJ_OK ||
      (rc = launch_fill_u32(ix->iiib_maxw, ix->n_dims, 0u, st)) != KNNJ_OK ||
      (rc = launch_fill_u32(ix->iiib_cut, n_keys * kLevels, 0u, st)) != KNNJ_OK ||
      (rc = launch_fill_u32(n_big, 1, 0u, st)) != KNNJ_OK)
    return rc;
  k_block_stats<V><<<2048, kBlock, 0, st>>>(r0, r1, R->indptr, R->indices, (const V*)R->values, ix->iiib_freq,
                                            ix->iiib_maxw);
  if (ix->n_rows > 0) {
    int p = 1;
    while (p < ix->max_row_nnz) p <<= 1;
    k_split_rows<V><<<unsigned(ix->n_rows), kWave, size_t(p) * 8, st>>>(
        ix->n_rows, ix->n_dims, ix->log2_tile, p, ix->s_indptr, ix->s_indices, (const V*)ix->s_values, ix->iiib_freq,
        ix->iiib_maxw, ix->iiib_fwd, ix->iiib_fwd_w, ix->iiib_cut);
    k_bucket_starts<<<unsigned((n_keys + kBlock - 1) / kBlock), kBlock, 0, st>>>(n_keys, ix->iiib_cut);
    k_split_scatter<V><<<unsigned(ix->n_rows), kWave, 0, st>>>(ix->n_rows, ix->n_dims, ix->log2_tile, ix->s_indptr,
                                                               ix->iiib_fwd, ix->iiib_fwd_w, ix->offsets,
                                                               ix->iiib_cut, ix->rec_tmp);
    k_sort_small<<<unsigned((n_keys + kBlock - 1) / kBlock), kBlock, 0, st>>>(ix->offsets, n_keys, ix->rec_tmp,
                                                                             ix->iiib_big, n_big);
    k_sort_mid<<<kSortGrid, kBlock, 0, st>>>(ix->offsets, ix->iiib_big, n_big, ix->rec_tmp);
    k_sort_buckets<<<kSortGrid, kBlock, kBucketSlots * sizeof(uint32_t), st>>>(
        ix->offsets, ix->iiib_big, n_big, ix->iiib_cut, ix->rec_tmp, ix->iiib_out_tmp, ix->tile);
    if (ix->nnz > 0) {
      const int64_t nbf = (ix->nnz + kBlock - 1) / kBlock;
      const unsigned gf = unsigned(nbf < (int64_t(1) << 20) ? nbf : (int64_t(1) << 20));
      if (ix->dtype == KNNJ_U8) k_finalize_iiib_u8<<<gf, kBlock, 0, st>>>(ix->rec_tmp, ix->nnz, ix->iiib_post);
      else k_finalize_iiib_f32<<<gf, kBlock, 0, st>>>(ix->rec_tmp, ix->nnz, ix->iiib_post_s, ix->iiib_post_w);
    }
  }
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

template <typename V>
static knnj_status join_block(Index* ix, const knnj_csr* R, int64_t r0, int64_t r1, int32_t k,
                              const knnj_join_opts* opt, const int32_t* order, int32_t hash_lg, int32_t* ids,
                              void* scv, int32_t* cnt, uint64_t* slots, hipStream_t st) {
  using S = typename ScoreOf<V>::T;
  S* scores = (S*)scv;
  const size_t smem = iiib_smem(ix, k, hash_lg);
  Postings<V> P;
  if constexpr (sizeof(V) == 1) P = Postings<V>{reinterpret_cast<const uint4*>(ix->iiib_post)};
  else P = Postings<V>{reinterpret_cast<const uint2*>(ix->iiib_post_s), reinterpret_cast<const float4*>(ix->iiib_post_w)};
  const int32_t drop = opt->level_drop;
  const int32_t filt = (opt->flags & KNNJ_FLAG_IIIB_BOUND) ? 1 : 0;
  const int64_t n = r1 - r0;
  uint32_t* qcount = ix->iiib_small + 1;
  for (int pass = 0; pass < (opt->theta_seed ? 2 : 1); ++pass) {
    const bool fallback = pass == 1;
    if (fallback) {
      knnj_status rc = launch_fill_u32(qcount, 1, 0u, st);
      if (rc != KNNJ_OK) return rc;
      k_survivors<S><<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
          r0, n, k, opt->theta_seed, ix->iiib_seed2, ids, scores, cnt, ix->iiib_qlist, qcount, opt->fallback_out,
          slots);
    }
    for (int32_t t = 0; t < ix->n_tiles; ++t) {
      k_iiib_tile<V><<<unsigned(n), kBlock, smem, st>>>(
          t, ix->log2_tile, ix->n_dims, k, r0, fallback ? nullptr : order, fallback ? ix->iiib_qlist : nullptr,
          fallback ? qcount : nullptr, R->indptr, R->indices, (const V*)R->values, ix->offsets, ix->iiib_cut, P,
          ix->s_indptr, ix->iiib_fwd, ix->iiib_fwd_w, fallback ? ix->iiib_seed2 : opt->theta_seed, drop, filt,
          hash_lg, ids, scores, cnt, slots);
    }
  }
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

knnj_status launch_iiib(Index* ix, const knnj_csr* R, int32_t k, const knnj_join_opts* opt, const int32_t* order,
                        int32_t max_r, int32_t* ids, void* scv, int32_t* cnt, uint64_t* slots, hipStream_t st) {
  knnj_status rc = upload_tau();
  if (rc != KNNJ_OK) return rc;
  if (ix->dtype == KNNJ_U8 && ix->n_dims > kFwdMaxDimsU8)
    return fail(KNNJ_EUNSUPPORTED, "IIIB supports at most 2^18 dimensions for uint8 data");
  int max_smem = 0;
  KNNJ_HIP(hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device));
  const int32_t hash_lg = r_hash_log2(ix, max_r);
  if (iiib_smem(ix, k, hash_lg) > size_t(max_smem))
    return fail(KNNJ_EUNSUPPORTED, "IIIB: tile accumulators plus the copy of r exceed workgroup local memory");
  if (opt->level_drop < 0 || opt->level_drop >= kLevels) return fail(KNNJ_EINVAL, "level_drop must be in [0, 63]");
  const int64_t n_r = R->n_rows;
  const int64_t blk = opt->r_block_rows > 0 && opt->r_block_rows < n_r ? opt->r_block_rows : n_r;
  if ((rc = ensure_iiib(ix, n_r)) != KNNJ_OK) return rc;
  for (int64_t r0 = 0; rc == KNNJ_OK && r0 < n_r; r0 += blk) {
    const int64_t r1 = r0 + blk < n_r ? r0 + blk : n_r;
    // the longest-first order covers all of R: used when R is one block
    const int32_t* ord = (r0 == 0 && r1 == n_r) ? order : nullptr;
    if (ix->dtype == KNNJ_U8) {
      rc = build_block<uint8_t>(ix, R, r0, r1, st);
      if (rc == KNNJ_OK) rc = join_block<uint8_t>(ix, R, r0, r1, k, opt, ord, hash_lg, ids, scv, cnt, slots, st);
    } else {
      rc = build_block<float>(ix, R, r0, r1, st);
      if (rc == KNNJ_OK) rc = join_block<float>(ix, R, r0, r1, k, opt, ord, hash_lg, ids, scv, cnt, slots, st);
    }
  }
  return rc;
}

}  // namespace knnj
