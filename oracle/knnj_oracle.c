/*
 * CPU oracle for the exact KNN join of sparse vectors.  TEST INFRASTRUCTURE
 * ONLY: called from the test-suite, the smoke check and the benchmark's CPU
 * baseline; never from the library's product path.  Shares no code with the
 * GPU library.
 *
 * What it computes is the plain definition of the join (Problem definition,
 * Sec. 3, Eq. 1), evaluated by brute force (Sec. 4.2, Algorithm 2):
 *   for every r in R and every s_j in S (ascending j):
 *     v = dot(r, s_j) by the two-pointer merge over ascending dimension ids
 *         (the dot() routine of Algorithm 2);
 *   keep the pairs with v > 0 (Algorithms 1 and 2 start the pruning score at 0
 *   and admit only scores above it, so a zero score is never a neighbour);
 *   order them by (v descending, j ascending) and return the first min(k, #);
 *   unused output slots are id -1, score 0.
 *
 * Precision: u8 values are multiplied and summed in int64 (exact); float
 * values are widened to double, multiplied (exact in double) and summed in
 * ascending dimension order in double.
 *
 * Single-threaded by design.  Build: gcc -O2 -shared -fPIC knnj_oracle.c
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct { double v; int64_t j; } pair_t;

/* (v desc, j asc) */
static int cmp_pair(const void* a, const void* b) {
  const pair_t* x = (const pair_t*)a;
  const pair_t* y = (const pair_t*)b;
  if (x->v > y->v) return -1;
  if (x->v < y->v) return 1;
  return (x->j > y->j) - (x->j < y->j);
}

/* dot(r, s): merge of two ascending feature lists (Algorithm 2, dot()). */
static int64_t dot_u8(const int32_t* ri, const uint8_t* rv, int64_t nr, const int32_t* si, const uint8_t* sv,
                      int64_t ns) {
  int64_t ret = 0, a = 0, b = 0;
  while (a < nr && b < ns) {
    if (ri[a] == si[b]) {
      ret += (int64_t)rv[a] * (int64_t)sv[b];
      ++a;
      ++b;
    } else if (ri[a] > si[b]) {
      ++b;
    } else {
      ++a;
    }
  }
  return ret;
}

static double dot_f32(const int32_t* ri, const float* rv, int64_t nr, const int32_t* si, const float* sv,
                      int64_t ns) {
  double ret = 0.0;
  int64_t a = 0, b = 0;
  while (a < nr && b < ns) {
    if (ri[a] == si[b]) {
      ret += (double)rv[a] * (double)sv[b];
      ++a;
      ++b;
    } else if (ri[a] > si[b]) {
      ++b;
    } else {
      ++a;
    }
  }
  return ret;
}

/*
 * Brute-force top-k for queries [q_begin, q_end) of R against all of S.
 *   dtype 0: u8 values, out_scores is int64[(q_end-q_begin)*k]
 *   dtype 1: f32 values, out_scores is double[(q_end-q_begin)*k]
 * out_ids int32[(q_end-q_begin)*k], out_count int32[q_end-q_begin].
 * Returns 0, -1 on bad arguments, -2 on allocation failure.
 */
int oracle_bf_topk(int64_t q_begin, int64_t q_end, const int64_t* r_ptr, const int32_t* r_idx, const void* r_val,
                   int64_t n_s, const int64_t* s_ptr, const int32_t* s_idx, const void* s_val, int dtype, int32_t k,
                   int32_t* out_ids, void* out_scores, int32_t* out_count) {
  if (k < 1 || q_end < q_begin || n_s < 0 || (dtype != 0 && dtype != 1)) return -1;
  pair_t* buf = (pair_t*)malloc(sizeof(pair_t) * (size_t)(n_s > 0 ? n_s : 1));
  if (!buf) return -2;
  for (int64_t q = q_begin; q < q_end; ++q) {
    const int64_t rb = r_ptr[q], re = r_ptr[q + 1];
    int64_t n = 0;
    for (int64_t j = 0; j < n_s; ++j) {
      const int64_t sb = s_ptr[j], se = s_ptr[j + 1];
      double v;
      if (dtype == 0) {
        v = (double)dot_u8(r_idx + rb, (const uint8_t*)r_val + rb, re - rb, s_idx + sb,
                           (const uint8_t*)s_val + sb, se - sb);
      } else {
        v = dot_f32(r_idx + rb, (const float*)r_val + rb, re - rb, s_idx + sb, (const float*)s_val + sb,
                    se - sb);
      }
      if (v > 0.0) {
        buf[n].v = v;
        buf[n].j = j;
        ++n;
      }
    }
    qsort(buf, (size_t)n, sizeof(pair_t), cmp_pair);
    const int64_t o = (q - q_begin) * (int64_t)k;
    const int64_t m = n < k ? n : k;
    for (int64_t t = 0; t < k; ++t) {
      out_ids[o + t] = t < m ? (int32_t)buf[t].j : -1;
      if (dtype == 0) ((int64_t*)out_scores)[o + t] = t < m ? (int64_t)buf[t].v : 0;
      else ((double*)out_scores)[o + t] = t < m ? buf[t].v : 0.0;
    }
    out_count[q - q_begin] = (int32_t)m;
  }
  free(buf);
  return 0;
}

/* All scores dot(r_q, s_j) for one query q (used to inspect ties and to check
 * sampled outputs one by one).  dtype 0: out is int64[n_s]; dtype 1: double[n_s]. */
int oracle_scores_one(int64_t q, const int64_t* r_ptr, const int32_t* r_idx, const void* r_val, int64_t n_s,
                      const int64_t* s_ptr, const int32_t* s_idx, const void* s_val, int dtype, void* out) {
  if (dtype != 0 && dtype != 1) return -1;
  const int64_t rb = r_ptr[q], re = r_ptr[q + 1];
  for (int64_t j = 0; j < n_s; ++j) {
    const int64_t sb = s_ptr[j], se = s_ptr[j + 1];
    if (dtype == 0)
      ((int64_t*)out)[j] = dot_u8(r_idx + rb, (const uint8_t*)r_val + rb, re - rb, s_idx + sb,
                                  (const uint8_t*)s_val + sb, se - sb);
    else
      ((double*)out)[j] = dot_f32(r_idx + rb, (const float*)r_val + rb, re - rb, s_idx + sb,
                                  (const float*)s_val + sb, se - sb);
  }
  return 0;
}
