// Learned threshold seed: per-query features and a 64-128-128-1 MLP (ReLU,
// bfloat16 weights, float32 accumulation) that predicts a query's k-th score.
// Its prediction seeds IIIB's threshold before any posting is read; the join's
// survivor check keeps results exact whatever the network predicts.
//
// Features of a query r (64 floats):
//   [0]      log(1 + |r|)
//   [1..16]  share of r's features with weight bin b: u8 w >> 4; f32 min(15, floor(16 w))
//   [17..63] share of r's features whose posting list length L = |I_d| falls in
//            bin min(46, floor(2 log2(1 + L)))
// The network sees (x - mean) / std with mean and std taken over the training set,
// and predicts the k-th score divided by the mean training label.
//
// Parameters (flat float vector): W1[128][64] b1[128] W2[128][128] b2[128] w3[128] b3.
// Training: pinball (quantile) loss at tau, minibatch Adam on float32 master
// weights, bfloat16 working weights used by the forward and backward passes.
#include <hip/hip_bf16.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <random>
#include <vector>

#include "common.hpp"

namespace knnj {

constexpr int kIn = 64, kHid = 128;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
              kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid, kParams = kOffB3 + 1;
static_assert(kParams == 24961, "parameter count");
constexpr int kSB = 32;  // samples per workgroup in the per-sample kernels

struct Mlp {
  float* master = nullptr;   // float32 master weights (device)
  float* work = nullptr;     // bfloat16-rounded working weights, stored as float (device)
  float* m1 = nullptr;       // Adam moments
  float* m2 = nullptr;
  float* norm = nullptr;     // mean[64], std[64], label scale (device)
  float h_norm[2 * kIn + 1];
  int64_t step = 0;
};

static float bf16_round_host(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  float r;
  memcpy(&r, &u, 4);
  return r;
}

__device__ __forceinline__ float bf16_round(float x) { return __bfloat162float(__float2bfloat16(x)); }

// ---------------------------------------------------------------- features
template <typename V>
__global__ void k_features(int64_t n, const int64_t* __restrict__ r_ptr, const int32_t* __restrict__ r_idx,
                           const V* __restrict__ r_val, const uint32_t* __restrict__ list_len,
                           float* __restrict__ out) {
  __shared__ uint32_t hist[kBlock / kWave][64];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int64_t q = int64_t(blockIdx.x) * (kBlock / kWave) + wid;
  hist[wid][lane] = 0;
  __syncthreads();
  if (q < n) {
    const int64_t b = r_ptr[q], e = r_ptr[q + 1];
    for (int64_t j = b + lane; j < e; j += kWave) {
      uint32_t bw;
      if constexpr (sizeof(V) == 1) {
        bw = uint32_t(r_val[j]) >> 4;
      } else {
        const float f = floorf(16.0f * r_val[j]);
        bw = f >= 15.0f ? 15u : uint32_t(f);
      }
      const uint64_t x = uint64_t(list_len[r_idx[j]]) + 1u;  // >= 1
      const uint32_t m = 63u - uint32_t(__clzll(x));          // floor(log2 x)
      // floor(2 log2 x) = 2m + [x^2 >= 2^(2m+1)]
      const uint32_t half = (x * x >= (1ull << (2 * m + 1))) ? 1u : 0u;
      uint32_t bl = 2 * m + half;
      if (bl > 46u) bl = 46u;
      atomicAdd(&hist[wid][1 + bw], 1u);
      atomicAdd(&hist[wid][17 + bl], 1u);
    }
  }
  __syncthreads();
  if (q < n) {
    const float nnz = float(r_ptr[q + 1] - r_ptr[q]);
    float v;
    if (lane == 0) v = log1pf(nnz);
    else v = nnz > 0.0f ? float(hist[wid][lane]) / nnz : 0.0f;
    out[q * kIn + lane] = v;
  }
}

// ---------------------------------------------------------------- forward
// One workgroup per kSB samples.  Working weights are staged transposed in local
// memory so lanes (consecutive outputs) read consecutive words.
// x_std, h1, h2 (kSB x 128) are written when save != 0 (training).
__global__ __launch_bounds__(kBlock) void k_mlp_forward(int64_t n, const float* __restrict__ X,
                                                        const int64_t* __restrict__ rows,
                                                        const float* __restrict__ W, const float* __restrict__ norm,
                                                        float* __restrict__ y, float* __restrict__ xs_out,
                                                        float* __restrict__ h1_out, float* __restrict__ h2_out) {
  extern __shared__ float sm[];
  float* w1t = sm;                     // [64][128]
  float* w2t = w1t + kIn * kHid;       // [128][128]
  float* xs = w2t + kHid * kHid;       // [kSB][64]
  float* h1 = xs + kSB * kIn;          // [kSB][128]
  float* h2 = h1 + kSB * kHid;         // [kSB][128]
  for (int i = threadIdx.x; i < kHid * kIn; i += kBlock) {
    const int o = i / kIn, c = i % kIn;
    w1t[c * kHid + o] = W[kOffW1 + i];
  }
  for (int i = threadIdx.x; i < kHid * kHid; i += kBlock) {
    const int o = i / kHid, c = i % kHid;
    w2t[c * kHid + o] = W[kOffW2 + i];
  }
  const int64_t s0 = int64_t(blockIdx.x) * kSB;
  for (int i = threadIdx.x; i < kSB * kIn; i += kBlock) {
    const int s = i / kIn, c = i % kIn;
    float v = 0.0f;
    if (s0 + s < n) {
      const int64_t r = rows ? rows[s0 + s] : s0 + s;
      v = (X[r * kIn + c] - norm[c]) / norm[kIn + c];
    }
    xs[i] = v;
  }
  __syncthreads();
  const int o = threadIdx.x % kHid;
  const int sg = threadIdx.x / kHid;  // 0 or 1: samples sg, sg + 2, ...
  for (int s = sg; s < kSB; s += kBlock / kHid) {
    float a = W[kOffB1 + o];
    for (int c = 0; c < kIn; ++c) a += w1t[c * kHid + o] * xs[s * kIn + c];
    h1[s * kHid + o] = a > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  for (int s = sg; s < kSB; s += kBlock / kHid) {
    float a = W[kOffB2 + o];
    for (int c = 0; c < kHid; ++c) a += w2t[c * kHid + o] * h1[s * kHid + c];
    h2[s * kHid + o] = a > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  // output: one wave per sample group
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  for (int s = wid; s < kSB; s += kBlock / kWave) {
    float a = W[kOffW3 + lane] * h2[s * kHid + lane] + W[kOffW3 + lane + kWave] * h2[s * kHid + lane + kWave];
    for (int off = kWave / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
    if (lane == 0 && s0 + s < n) y[s0 + s] = a + W[kOffB3];
  }
  if (xs_out) {
    for (int i = threadIdx.x; i < kSB * kIn; i += kBlock)
      if (s0 + i / kIn < n) xs_out[s0 * kIn + i] = xs[i];
    for (int i = threadIdx.x; i < kSB * kHid; i += kBlock)
      if (s0 + i / kHid < n) {
        h1_out[s0 * kHid + i] = h1[i];
        h2_out[s0 * kHid + i] = h2[i];
      }
  }
}

// Pinball loss at quantile tau, averaged over the batch: returns dL/dyhat per
// sample into g and adds the batch loss into *loss.
__global__ void k_pinball(int64_t n, const float* __restrict__ yhat, const float* __restrict__ y,
                          const int64_t* __restrict__ rows, const float* __restrict__ norm, float tau,
                          float* __restrict__ g, float* __restrict__ loss) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (i < n) {
    const int64_t r = rows ? rows[i] : i;
    const float t = y[r] / norm[2 * kIn];
    const float d = t - yhat[i];
    l = d >= 0.0f ? tau * d : (tau - 1.0f) * d;
    g[i] = (d > 0.0f ? -tau : (d < 0.0f ? 1.0f - tau : 0.0f)) / float(n);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) l += __shfl_xor(l, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(loss, l / float(n));
}

// Backward through the activations: g2 = g * w3 * [h2 > 0], g1 = (g2 W2) * [h1 > 0].
__global__ __launch_bounds__(kBlock) void k_mlp_backact(int64_t n, const float* __restrict__ W,
                                                        const float* __restrict__ g, const float* __restrict__ h1,
                                                        const float* __restrict__ h2, float* __restrict__ g1,
                                                        float* __restrict__ g2) {
  extern __shared__ float sm[];
  float* w2 = sm;                 // [128 out][128 in] as stored
  float* g2s = w2 + kHid * kHid;  // [kSB][128]
  for (int i = threadIdx.x; i < kHid * kHid; i += kBlock) w2[i] = W[kOffW2 + i];
  const int64_t s0 = int64_t(blockIdx.x) * kSB;
  for (int i = threadIdx.x; i < kSB * kHid; i += kBlock) {
    const int s = i / kHid, o = i % kHid;
    float v = 0.0f;
    if (s0 + s < n) v = h2[s0 * kHid + i] > 0.0f ? g[s0 + s] * W[kOffW3 + o] : 0.0f;
    g2s[i] = v;
    if (s0 + s < n) g2[s0 * kHid + i] = v;
  }
  __syncthreads();
  const int c = threadIdx.x % kHid;   // input unit of W2
  const int sg = threadIdx.x / kHid;
  for (int s = sg; s < kSB; s += kBlock / kHid) {
    if (s0 + s >= n) break;
    float a = 0.0f;
    for (int o = 0; o < kHid; ++o) a += g2s[s * kHid + o] * w2[o * kHid + c];
    g1[(s0 + s) * kHid + c] = h1[(s0 + s) * kHid + c] > 0.0f ? a : 0.0f;
  }
}

// Weight gradients: one thread per parameter, summing over the batch.
__global__ void k_mlp_wgrad(int64_t n, const float* __restrict__ xs, const float* __restrict__ h1,
                            const float* __restrict__ h2, const float* __restrict__ g, const float* __restrict__ g1,
                            const float* __restrict__ g2, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  float a = 0.0f;
  if (p < kOffB1) {
    const int o = p / kIn, c = p % kIn;
    for (int64_t s = 0; s < n; ++s) a += g1[s * kHid + o] * xs[s * kIn + c];
  } else if (p < kOffW2) {
    const int o = p - kOffB1;
    for (int64_t s = 0; s < n; ++s) a += g1[s * kHid + o];
  } else if (p < kOffB2) {
    const int o = (p - kOffW2) / kHid, c = (p - kOffW2) % kHid;
    for (int64_t s = 0; s < n; ++s) a += g2[s * kHid + o] * h1[s * kHid + c];
  } else if (p < kOffW3) {
    const int o = p - kOffB2;
    for (int64_t s = 0; s < n; ++s) a += g2[s * kHid + o];
  } else if (p < kOffB3) {
    const int c = p - kOffW3;
    for (int64_t s = 0; s < n; ++s) a += g[s] * h2[s * kHid + c];
  } else {
    for (int64_t s = 0; s < n; ++s) a += g[s];
  }
  grad[p] = a;
}

// Adam on the master weights, then refresh the bfloat16 working copy.
__global__ void k_adam(const float* __restrict__ grad, float* __restrict__ master, float* __restrict__ work,
                       float* __restrict__ m1, float* __restrict__ m2, float lr, float b1c, float b2c) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float gr = grad[p];
  const float a = 0.9f * m1[p] + 0.1f * gr;
  const float b = 0.999f * m2[p] + 0.001f * gr * gr;
  m1[p] = a;
  m2[p] = b;
  const float w = master[p] - lr * (a / b1c) / (sqrtf(b / b2c) + 1e-8f);
  master[p] = w;
  work[p] = bf16_round(w);
}

// mean and std of each feature over n samples (one workgroup per feature),
// floored at 1e-3 so constant features do not blow up
__global__ void k_feat_stats(int64_t n, const float* __restrict__ X, float* __restrict__ norm) {
  __shared__ double s1[kBlock], s2[kBlock];
  const int c = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) {
    const double v = X[i * kIn + c];
    a += v;
    b += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = s1[0] / double(n);
    double var = s2[0] / double(n) - mean * mean;
    if (var < 0.0) var = 0.0;
    double sd = sqrt(var);
    if (sd < 1e-3) sd = 1e-3;
    norm[c] = float(mean);
    norm[kIn + c] = float(sd);
  }
}

__global__ void k_label_mean(int64_t n, const float* __restrict__ y, float* __restrict__ norm) {
  __shared__ double s1[kBlock];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) a += y[i];
  s1[threadIdx.x] = a;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s1[threadIdx.x] += s1[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double m = s1[0] / double(n);
    norm[2 * kIn] = m > 0.0 ? float(m) : 1.0f;
  }
}

__global__ void k_scale(int64_t n, float* __restrict__ y, const float* __restrict__ norm) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] *= norm[2 * kIn];
}

const uint32_t* index_list_len(const knnj_index* ix);
int index_device(const knnj_index* ix);
knnj_status check_device(int owner, const char* what);

static constexpr size_t kFwdSmem = sizeof(float) * (kIn * kHid + kHid * kHid + kSB * kIn + 2 * kSB * kHid);
static constexpr size_t kBackSmem = sizeof(float) * (kHid * kHid + kSB * kHid);

}  // namespace knnj

using namespace knnj;

struct knnj_mlp {
  Mlp m;
  int device;  // the device its buffers live on
};

extern "C" {

knnj_status knnj_mlp_create(uint64_t seed, knnj_mlp** out) {
  if (!out) return fail(KNNJ_EINVAL, "out is NULL");
  *out = nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(KNNJ_EDEVICE, "hipGetDevice failed");
  knnj_mlp* h = new knnj_mlp();
  h->device = dev;
  Mlp& m = h->m;
  if (hipMalloc(&m.master, sizeof(float) * kParams) != hipSuccess ||
      hipMalloc(&m.work, sizeof(float) * kParams) != hipSuccess ||
      hipMalloc(&m.m1, sizeof(float) * kParams) != hipSuccess ||
      hipMalloc(&m.m2, sizeof(float) * kParams) != hipSuccess ||
      hipMalloc(&m.norm, sizeof(float) * (2 * kIn + 1)) != hipSuccess) {
    knnj_mlp_free(h);
    return fail(KNNJ_ENOMEM, "device allocation for the MLP failed");
  }
  // He-uniform initialisation of the weights, zero biases
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  std::vector<float> p(kParams, 0.0f), w(kParams), z(kParams, 0.0f);
  const double a1 = sqrt(6.0 / kIn), a2 = sqrt(6.0 / kHid), a3 = sqrt(3.0 / kHid);
  for (int i = 0; i < kHid * kIn; ++i) p[kOffW1 + i] = float(a1 * u(rng));
  for (int i = 0; i < kHid * kHid; ++i) p[kOffW2 + i] = float(a2 * u(rng));
  for (int i = 0; i < kHid; ++i) p[kOffW3 + i] = float(a3 * u(rng));
  for (int i = 0; i < kParams; ++i) w[i] = bf16_round_host(p[i]);
  for (int c = 0; c < kIn; ++c) {
    m.h_norm[c] = 0.0f;
    m.h_norm[kIn + c] = 1.0f;
  }
  m.h_norm[2 * kIn] = 1.0f;
  if (hipMemcpy(m.master, p.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m.work, w.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m.m1, z.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m.m2, z.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m.norm, m.h_norm, sizeof(m.h_norm), hipMemcpyHostToDevice) != hipSuccess) {
    knnj_mlp_free(h);
    return fail(KNNJ_EDEVICE, "MLP upload failed");
  }
  *out = h;
  return KNNJ_OK;
}

void knnj_mlp_free(knnj_mlp* h) {
  if (!h) return;
  // wait for and free on the MLP's own device, whichever device is current
  int cur = -1;
  const bool other =
      hipGetDevice(&cur) == hipSuccess && cur != h->device && hipSetDevice(h->device) == hipSuccess;
  (void)hipDeviceSynchronize();
  (void)hipFree(h->m.master);
  (void)hipFree(h->m.work);
  (void)hipFree(h->m.m1);
  (void)hipFree(h->m.m2);
  (void)hipFree(h->m.norm);
  delete h;
  if (other) (void)hipSetDevice(cur);
}

knnj_status knnj_mlp_features(const knnj_index* ix, const knnj_csr* R, float* out, void* stream) {
  if (!ix || !R || (!out && R->n_rows > 0)) return fail(KNNJ_EINVAL, "NULL argument");
  if (const knnj_status rc = check_device(index_device(ix), "the index"); rc != KNNJ_OK) return rc;
  const uint32_t* ll = index_list_len(ix);
  knnj_index_info info;
  knnj_status rc = knnj_index_info_get(ix, &info);
  if (rc != KNNJ_OK) return rc;
  if (R->n_dims != info.n_dims || R->dtype != info.dtype) return fail(KNNJ_EINVAL, "R does not match the index");
  if (R->n_rows == 0) return KNNJ_OK;
  hipStream_t st = (hipStream_t)stream;
  const unsigned g = unsigned((R->n_rows + kBlock / kWave - 1) / (kBlock / kWave));
  if (R->dtype == KNNJ_U8)
    k_features<uint8_t><<<g, kBlock, 0, st>>>(R->n_rows, R->indptr, R->indices, (const uint8_t*)R->values, ll, out);
  else
    k_features<float><<<g, kBlock, 0, st>>>(R->n_rows, R->indptr, R->indices, (const float*)R->values, ll, out);
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

// Scratch for one batch of up to b samples.
struct Batch {
  float *xs = nullptr, *h1 = nullptr, *h2 = nullptr, *yh = nullptr, *g = nullptr, *g1 = nullptr, *g2 = nullptr,
        *grad = nullptr, *loss = nullptr;
  int64_t* rows = nullptr;
  knnj_status alloc(int64_t b) {
    if (hipMalloc(&xs, sizeof(float) * b * kIn) != hipSuccess || hipMalloc(&h1, sizeof(float) * b * kHid) != hipSuccess ||
        hipMalloc(&h2, sizeof(float) * b * kHid) != hipSuccess || hipMalloc(&yh, sizeof(float) * b) != hipSuccess ||
        hipMalloc(&g, sizeof(float) * b) != hipSuccess || hipMalloc(&g1, sizeof(float) * b * kHid) != hipSuccess ||
        hipMalloc(&g2, sizeof(float) * b * kHid) != hipSuccess ||
        hipMalloc(&grad, sizeof(float) * kParams) != hipSuccess || hipMalloc(&loss, sizeof(float)) != hipSuccess ||
        hipMalloc(&rows, sizeof(int64_t) * b) != hipSuccess)
      return fail(KNNJ_ENOMEM, "MLP batch allocation failed");
    return KNNJ_OK;
  }
  ~Batch() {
    (void)hipFree(xs);
    (void)hipFree(h1);
    (void)hipFree(h2);
    (void)hipFree(yh);
    (void)hipFree(g);
    (void)hipFree(g1);
    (void)hipFree(g2);
    (void)hipFree(grad);
    (void)hipFree(loss);
    (void)hipFree(rows);
  }
};

// gradient of the mean pinball loss over the rows (rows == NULL: 0..n-1) into b.grad
static knnj_status batch_grad(const Mlp& m, const float* X, const float* y, const int64_t* rows, int64_t n, float tau,
                              Batch& b, hipStream_t st) {
  const unsigned gs = unsigned((n + kSB - 1) / kSB);
  k_mlp_forward<<<gs, kBlock, kFwdSmem, st>>>(n, X, rows, m.work, m.norm, b.yh, b.xs, b.h1, b.h2);
  k_pinball<<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, b.yh, y, rows, m.norm, tau, b.g, b.loss);
  k_mlp_backact<<<gs, kBlock, kBackSmem, st>>>(n, m.work, b.g, b.h1, b.h2, b.g1, b.g2);
  k_mlp_wgrad<<<unsigned((kParams + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, b.xs, b.h1, b.h2, b.g, b.g1, b.g2,
                                                                           b.grad);
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

knnj_status knnj_mlp_grad(knnj_mlp* h, const float* X, const float* y, int64_t n, float tau, float* grad_out,
                          float* loss_out, void* stream) {
  if (!h || !X || !y || !grad_out || !loss_out || n < 1) return fail(KNNJ_EINVAL, "bad argument");
  if (const knnj_status rc = check_device(h->device, "the MLP"); rc != KNNJ_OK) return rc;
  if (!(tau > 0.0f && tau < 1.0f)) return fail(KNNJ_EINVAL, "tau must be in (0, 1)");
  hipStream_t st = (hipStream_t)stream;
  Batch b;
  knnj_status rc = b.alloc(n);
  if (rc != KNNJ_OK) return rc;
  KNNJ_HIP(hipMemsetAsync(b.loss, 0, sizeof(float), st));
  if ((rc = batch_grad(h->m, X, y, nullptr, n, tau, b, st)) != KNNJ_OK) return rc;
  KNNJ_HIP(hipMemcpyAsync(grad_out, b.grad, sizeof(float) * kParams, hipMemcpyDeviceToDevice, st));
  KNNJ_HIP(hipMemcpyAsync(loss_out, b.loss, sizeof(float), hipMemcpyDeviceToDevice, st));
  KNNJ_HIP(hipStreamSynchronize(st));
  return KNNJ_OK;
}

knnj_status knnj_mlp_train(knnj_mlp* h, const float* X, const float* y, int64_t n, const knnj_train_opts* opt,
                           float* epoch_loss, void* stream) {
  if (!h || !X || !y || n < 1 || !opt) return fail(KNNJ_EINVAL, "bad argument");
  if (const knnj_status rc = check_device(h->device, "the MLP"); rc != KNNJ_OK) return rc;
  if (opt->epochs < 1 || opt->batch < 1 || opt->batch > 65536 || !(opt->lr > 0.0f) || !(opt->tau > 0.0f) ||
      !(opt->tau < 1.0f))
    return fail(KNNJ_EINVAL, "bad training options");
  Mlp& m = h->m;
  hipStream_t st = (hipStream_t)stream;
  // normalisation from the training set
  k_feat_stats<<<kIn, kBlock, 0, st>>>(n, X, m.norm);
  k_label_mean<<<1, kBlock, 0, st>>>(n, y, m.norm);
  KNNJ_HIP(hipGetLastError());
  KNNJ_HIP(hipMemcpyAsync(m.h_norm, m.norm, sizeof(m.h_norm), hipMemcpyDeviceToHost, st));
  Batch b;
  knnj_status rc = b.alloc(opt->batch);
  if (rc != KNNJ_OK) return rc;
  std::mt19937_64 rng(opt->seed);
  std::vector<int64_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  int64_t* dperm = nullptr;
  if (hipMalloc(&dperm, sizeof(int64_t) * n) != hipSuccess) return fail(KNNJ_ENOMEM, "permutation allocation");
  for (int ep = 0; ep < opt->epochs; ++ep) {
    for (int64_t i = n - 1; i > 0; --i) {
      std::uniform_int_distribution<int64_t> pick(0, i);
      std::swap(perm[i], perm[pick(rng)]);
    }
    if (hipMemcpyAsync(dperm, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemsetAsync(b.loss, 0, sizeof(float), st) != hipSuccess) {
      (void)hipFree(dperm);
      return fail(KNNJ_EDEVICE, "training upload failed");
    }
    int64_t nb = 0;
    for (int64_t s0 = 0; s0 < n; s0 += opt->batch, ++nb) {
      const int64_t bn = n - s0 < opt->batch ? n - s0 : opt->batch;
      if ((rc = batch_grad(m, X, y, dperm + s0, bn, opt->tau, b, st)) != KNNJ_OK) break;
      ++m.step;
      const float b1c = float(1.0 - pow(0.9, double(m.step)));
      const float b2c = float(1.0 - pow(0.999, double(m.step)));
      k_adam<<<unsigned((kParams + kBlock - 1) / kBlock), kBlock, 0, st>>>(b.grad, m.master, m.work, m.m1, m.m2,
                                                                          opt->lr, b1c, b2c);
    }
    if (rc != KNNJ_OK) break;
    float l = 0.0f;
    if (hipMemcpyAsync(&l, b.loss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(KNNJ_EDEVICE, "training kernels failed");
      break;
    }
    if (epoch_loss) epoch_loss[ep] = l / float(nb);
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(dperm);
  return rc;
}

knnj_status knnj_mlp_predict(const knnj_mlp* h, const float* X, int64_t n, float* theta_out, void* stream) {
  if (!h || (n > 0 && (!X || !theta_out)) || n < 0) return fail(KNNJ_EINVAL, "bad argument");
  if (const knnj_status rc = check_device(h->device, "the MLP"); rc != KNNJ_OK) return rc;
  if (n == 0) return KNNJ_OK;
  hipStream_t st = (hipStream_t)stream;
  k_mlp_forward<<<unsigned((n + kSB - 1) / kSB), kBlock, kFwdSmem, st>>>(n, X, nullptr, h->m.work, h->m.norm,
                                                                        theta_out, nullptr, nullptr, nullptr);
  k_scale<<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, theta_out, h->m.norm);
  KNNJ_HIP(hipGetLastError());
  return KNNJ_OK;
}

knnj_status knnj_mlp_get_state(const knnj_mlp* h, float* params, float* norm) {
  if (!h || !params || !norm) return fail(KNNJ_EINVAL, "NULL argument");
  if (const knnj_status rc = check_device(h->device, "the MLP"); rc != KNNJ_OK) return rc;
  KNNJ_HIP(hipDeviceSynchronize());
  KNNJ_HIP(hipMemcpy(params, h->m.work, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  KNNJ_HIP(hipMemcpy(norm, h->m.norm, sizeof(float) * (2 * kIn + 1), hipMemcpyDeviceToHost));
  return KNNJ_OK;
}

knnj_status knnj_mlp_set_state(knnj_mlp* h, const float* params, const float* norm) {
  if (!h || !params || !norm) return fail(KNNJ_EINVAL, "NULL argument");
  if (const knnj_status rc = check_device(h->device, "the MLP"); rc != KNNJ_OK) return rc;
  std::vector<float> w(kParams);
  for (int i = 0; i < kParams; ++i) w[i] = bf16_round_host(params[i]);
  for (int c = 0; c < kIn; ++c)
    if (!(norm[kIn + c] > 0.0f)) return fail(KNNJ_EINVAL, "std entries must be > 0");
  if (!(norm[2 * kIn] > 0.0f)) return fail(KNNJ_EINVAL, "label scale must be > 0");
  KNNJ_HIP(hipDeviceSynchronize());
  KNNJ_HIP(hipMemcpy(h->m.master, params, sizeof(float) * kParams, hipMemcpyHostToDevice));
  KNNJ_HIP(hipMemcpy(h->m.work, w.data(), sizeof(float) * kParams, hipMemcpyHostToDevice));
  KNNJ_HIP(hipMemcpy(h->m.norm, norm, sizeof(float) * (2 * kIn + 1), hipMemcpyHostToDevice));
  memcpy(h->m.h_norm, norm, sizeof(h->m.h_norm));
  return KNNJ_OK;
}

}  // extern "C"
