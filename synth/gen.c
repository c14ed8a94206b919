/*
 * Seeded synthetic sparse-vector generator (CSR), shared by the oracle side
 * and the GPU side of every test and benchmark.  It holds none of the join's
 * arithmetic: it only draws vectors.
 *
 * Data model (Problem definition, Sec. 3): a sparse vector is a list of
 * features (d, w) in ascending d with w > 0.  Dimension ids here are 0-based.
 *
 * Randomness: a counter-based generator.  Every (seed, stream, row) triple
 * gets its own splitmix64 sequence, so rows can be drawn in parallel and the
 * output does not depend on the thread count.
 *
 *   splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 *   generators", OOPSLA 2014):  state += 0x9e3779b97f4a7c15;
 *   z = state; z = (z ^ z>>30) * 0xbf58476d1ce4e5b9;
 *   z = (z ^ z>>27) * 0x94d049bb133111eb; return z ^ z>>31.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC gen.c -o libsynth.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } rng_t;

static inline uint64_t sm_next(rng_t* r) {
  uint64_t z = (r->s += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* Seed one row's stream: mix (seed, stream tag, row) through splitmix64. */
static inline rng_t row_rng(uint64_t seed, uint64_t tag, uint64_t row) {
  rng_t a = {seed * 0xd1b54a32d192ed03ULL + tag * 0x8cb92ba72f3d8dd7ULL};
  uint64_t x = sm_next(&a) ^ (row * 0x9e3779b97f4a7c15ULL + 0x632be59bd9b4e019ULL);
  rng_t b = {x};
  (void)sm_next(&b);
  return b;
}

/* uniform double in [0,1) with 53 random bits */
static inline double u01(rng_t* r) { return (double)(sm_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0, n) by Lemire's multiply-shift on 32 random bits */
static inline uint32_t below(rng_t* r, uint32_t n) {
  return (uint32_t)(((sm_next(r) >> 32) * (uint64_t)n) >> 32);
}

/* standard normal by Box-Muller (one of the pair) */
static inline double gauss(rng_t* r) {
  double u1 = u01(r), u2 = u01(r);
  if (u1 < 0x1.0p-60) u1 = 0x1.0p-60;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

enum { NNZ_UNIFORM = 0, NNZ_LOGNORMAL = 1 };
enum { FEAT_UNIFORM = 0, FEAT_ZIPF = 1 };
enum { VAL_U8 = 0, VAL_F32_LOGNORMAL_L2 = 1 };

#define TAG_NNZ 0x6e6e7aULL
#define TAG_FEAT 0x66656174ULL
#define TAG_PERM 0x7065726dULL

/* Number of features of each row.
 * NNZ_UNIFORM: uniform integer in [lo, hi].
 * NNZ_LOGNORMAL: round(exp(N(mu, sigma))) clipped to [lo, hi]. */
void synth_row_nnz(uint64_t seed, int64_t n_rows, int kind, int64_t lo, int64_t hi,
                   double mu, double sigma, int64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_rows; ++i) {
    rng_t r = row_rng(seed, TAG_NNZ, (uint64_t)i);
    int64_t v;
    if (kind == NNZ_UNIFORM) {
      v = lo + (int64_t)below(&r, (uint32_t)(hi - lo + 1));
    } else {
      double x = exp(mu + sigma * gauss(&r));
      v = (int64_t)llround(x);
      if (v < lo) v = lo;
      if (v > hi) v = hi;
    }
    out[i] = v;
  }
}

/* A seeded random permutation of [0, n) (Fisher-Yates). */
void synth_permutation(uint64_t seed, int32_t n, int32_t* out) {
  rng_t r = row_rng(seed, TAG_PERM, 0);
  for (int32_t i = 0; i < n; ++i) out[i] = i;
  for (int32_t i = n - 1; i > 0; --i) {
    int32_t j = (int32_t)below(&r, (uint32_t)(i + 1));
    int32_t t = out[i]; out[i] = out[j]; out[j] = t;
  }
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Fill the rows of a CSR matrix whose indptr is already known.
 *   feat_kind FEAT_UNIFORM: ids uniform on [0, n_dims) without replacement.
 *   feat_kind FEAT_ZIPF: rank rho in 1..n_dims with P(rho) proportional to
 *     rho^-zipf_s, mapped to a dimension through perm[rho-1]; distinct ids are
 *     obtained by redrawing duplicates (equal in law to successive sampling
 *     without replacement).
 *   val_kind VAL_U8: uniform integer in [1, 255] into values_u8.
 *   val_kind VAL_F32_LOGNORMAL_L2: exp(N(0,1)) per feature, then the row is
 *     divided by its L2 norm in double precision and stored as float.
 * Each row's ids are sorted ascending.  Returns 0, or -1 on bad arguments. */
int synth_fill_rows(uint64_t seed, int64_t n_rows, int32_t n_dims, const int64_t* indptr,
                    int feat_kind, double zipf_s, const int32_t* perm, int val_kind,
                    int32_t* indices, uint8_t* values_u8, float* values_f32) {
  if (n_dims <= 0 || n_rows < 0) return -1;
  double* cdf = NULL;
  if (feat_kind == FEAT_ZIPF) {
    cdf = (double*)malloc(sizeof(double) * (size_t)n_dims);
    if (!cdf) return -1;
    double acc = 0.0;
    for (int32_t i = 0; i < n_dims; ++i) {
      acc += pow((double)(i + 1), -zipf_s);
      cdf[i] = acc;
    }
    for (int32_t i = 0; i < n_dims; ++i) cdf[i] /= acc;
    cdf[n_dims - 1] = 1.0;
  }
  int bad = 0;
#pragma omp parallel
  {
    int32_t* stamp = (int32_t*)calloc((size_t)n_dims, sizeof(int32_t));
    double* tmp = (double*)malloc(sizeof(double) * 4096);
    if (!stamp || !tmp) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(dynamic, 256)
      for (int64_t i = 0; i < n_rows; ++i) {
        rng_t r = row_rng(seed, TAG_FEAT, (uint64_t)i);
        int64_t b = indptr[i], e = indptr[i + 1];
        int64_t m = e - b;
        if (m > n_dims || m > 4096) {
#pragma omp atomic write
          bad = 1;
          continue;
        }
        int32_t mark = (int32_t)((i % 2147483646) + 1);
        int64_t got = 0;
        while (got < m) {
          int32_t d;
          if (feat_kind == FEAT_UNIFORM) {
            d = (int32_t)below(&r, (uint32_t)n_dims);
          } else {
            double u = u01(&r);
            int32_t lo = 0, hi = n_dims - 1;
            while (lo < hi) {
              int32_t mid = lo + (hi - lo) / 2;
              if (cdf[mid] > u) hi = mid; else lo = mid + 1;
            }
            d = perm ? perm[lo] : lo;
          }
          if (stamp[d] == mark) continue;
          stamp[d] = mark;
          indices[b + got] = d;
          ++got;
        }
        /* a stamp can be reused by row i + 2147483646: clear this row's marks */
        for (int64_t j = b; j < e; ++j) stamp[indices[j]] = 0;
        qsort(indices + b, (size_t)m, sizeof(int32_t), cmp_i32);
        if (val_kind == VAL_U8) {
          for (int64_t j = b; j < e; ++j) values_u8[j] = (uint8_t)(1 + below(&r, 255));
        } else {
          double ss = 0.0;
          for (int64_t j = 0; j < m; ++j) {
            double v = exp(gauss(&r));
            tmp[j] = v;
            ss += v * v;
          }
          double inv = 1.0 / sqrt(ss);
          for (int64_t j = 0; j < m; ++j) values_f32[b + j] = (float)(tmp[j] * inv);
        }
      }
    }
    free(stamp);
    free(tmp);
  }
  free(cdf);
  return bad ? -1 : 0;
}
