// Warm-start network: forward, loss gradient and Adam on gfx950.
//
// Three dense layers over the spots of one patient (rows of X, B x F):
//   h1 = relu(X W1^T + b1), h2 = relu(h1 W2^T + b2), y = softplus(h2 . w3 + b3)
// and a penalty head lr = mean_b(h2) . wr + br.  Loss
//   L = mean_b (y_b - t_b)^2 + lam (lr - lr_t)^2.
// Flat parameter order W1, b1, W2, b2, w3, b3, wr, br (float32).  Every sum
// over rows is a fixed-order loop in one thread, so gradients are
// deterministic.  The sizes are small (H = 128): these kernels are latency
// bound and use plain fp32 FMA; inference can keep the hidden activations in
// bf16.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/admmbb.h"

namespace {

constexpr int kRows = 16;  // rows per block of the dense kernels

struct HipErr {
  hipError_t e;
};
inline void ck(hipError_t e) {
  if (e != hipSuccess) throw HipErr{e};
}

__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// out[b][k] = sum_i act(in[b][i]) W[k][i] + bias[k]; act = relu when relu_in,
// inputs rounded to bf16 when bf16_in.  Block: H threads (one output column
// each), kRows rows staged in LDS.
__global__ void k_dense(const float* __restrict__ in, int nin, const float* __restrict__ W,
                        const float* __restrict__ bias, float* __restrict__ out, int B, int H, int relu_in,
                        int bf16_in) {
  extern __shared__ float xs[];  // kRows x nin
  const int b0 = blockIdx.x * kRows;
  for (int idx = threadIdx.x; idx < kRows * nin; idx += blockDim.x) {
    const int r = idx / nin, i = idx % nin;
    float v = (b0 + r < B) ? in[static_cast<int64_t>(b0 + r) * nin + i] : 0.0f;
    if (relu_in) v = fmaxf(v, 0.0f);
    if (bf16_in) v = bf16_round(v);
    xs[idx] = v;
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (k >= H) return;
  float acc[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) acc[r] = 0.0f;
  const float* wk = W + static_cast<int64_t>(k) * nin;
  for (int i = 0; i < nin; ++i) {
    const float w = wk[i];
#pragma unroll
    for (int r = 0; r < kRows; ++r) acc[r] = fmaf(xs[r * nin + i], w, acc[r]);
  }
  const float bk = bias[k];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
    if (b0 + r < B) out[static_cast<int64_t>(b0 + r) * H + k] = acc[r] + bk;
}

// bf16 inference with the hidden activations stored as bf16:
// out[b][k] = bf16(relu(sum_i in[b][i] W[k][i] + bias[k])), in given as fp32
// (the network input) or as bf16 bits (a stored hidden layer).
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }
__device__ __forceinline__ uint16_t bf16_bits(float x) { return static_cast<uint16_t>(__float_as_uint(bf16_round(x)) >> 16); }

template <class TIN>
__global__ void k_dense_bf16(const TIN* __restrict__ in, int nin, const float* __restrict__ W,
                             const float* __restrict__ bias, uint16_t* __restrict__ out, int B, int H) {
  extern __shared__ float xs[];  // kRows x nin
  const int b0 = blockIdx.x * kRows;
  for (int idx = threadIdx.x; idx < kRows * nin; idx += blockDim.x) {
    const int r = idx / nin, i = idx % nin;
    float v = 0.0f;
    if (b0 + r < B) {
      if constexpr (std::is_same<TIN, uint16_t>::value)
        v = bf16_value(in[static_cast<int64_t>(b0 + r) * nin + i]);
      else
        v = in[static_cast<int64_t>(b0 + r) * nin + i];
    }
    xs[idx] = v;
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (k >= H) return;
  float acc[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) acc[r] = 0.0f;
  const float* wk = W + static_cast<int64_t>(k) * nin;
  for (int i = 0; i < nin; ++i) {
    const float w = wk[i];
#pragma unroll
    for (int r = 0; r < kRows; ++r) acc[r] = fmaf(xs[r * nin + i], w, acc[r]);
  }
  const float bk = bias[k];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
    if (b0 + r < B) out[static_cast<int64_t>(b0 + r) * H + k] = bf16_bits(fmaxf(acc[r] + bk, 0.0f));
}

// y_b = softplus(sum_k h2[b][k] w3[k] + b3) from the stored bf16 activations
__global__ void k_head_bf16(const uint16_t* __restrict__ h2, const float* __restrict__ w3,
                            const float* __restrict__ b3, float* __restrict__ z3, float* __restrict__ y, int B, int H) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float acc = 0.0f;
  const uint16_t* hr = h2 + static_cast<int64_t>(b) * H;
  for (int k = 0; k < H; ++k) acc = fmaf(bf16_value(hr[k]), w3[k], acc);
  const float z = acc + b3[0];
  z3[b] = z;
  y[b] = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
}

// pooled[k] = mean_b h2[b][k] over the stored bf16 activations (fixed order)
__global__ void k_pool_bf16(const uint16_t* __restrict__ h2, float* __restrict__ pooled, int B, int H) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= H) return;
  double s = 0.0;
  for (int b = 0; b < B; ++b) s += bf16_value(h2[static_cast<int64_t>(b) * H + k]);
  pooled[k] = static_cast<float>(s / B);
}

// y_b = softplus(sum_k relu(z2[b][k]) w3[k] + b3); z3 stored for the backward pass
__global__ void k_head(const float* __restrict__ z2, const float* __restrict__ w3, const float* __restrict__ b3,
                       float* __restrict__ z3, float* __restrict__ y, int B, int H, int bf16_in) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float acc = 0.0f;
  const float* zr = z2 + static_cast<int64_t>(b) * H;
  for (int k = 0; k < H; ++k) {
    float h = fmaxf(zr[k], 0.0f);
    if (bf16_in) h = bf16_round(h);
    acc = fmaf(h, w3[k], acc);
  }
  const float z = acc + b3[0];
  z3[b] = z;
  y[b] = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
}

// pooled[k] = mean_b relu(z2[b][k])  (fixed order)
__global__ void k_pool(const float* __restrict__ z2, float* __restrict__ pooled, int B, int H) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= H) return;
  double s = 0.0;
  for (int b = 0; b < B; ++b) s += fmaxf(z2[static_cast<int64_t>(b) * H + k], 0.0f);
  pooled[k] = static_cast<float>(s / B);
}

// penalty head and loss scalars (one thread): lr, L, dlr
__global__ void k_scalars(const float* __restrict__ pooled, const float* __restrict__ wr,
                          const float* __restrict__ br, const float* __restrict__ y, const float* __restrict__ t,
                          int B, int H, float lr_t, float lam, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lr = br[0];
  for (int k = 0; k < H; ++k) lr += static_cast<double>(pooled[k]) * wr[k];
  double se = 0.0;
  if (t != nullptr)
    for (int b = 0; b < B; ++b) {
      const double d = static_cast<double>(y[b]) - t[b];
      se += d * d;
    }
  out[0] = lr;
  out[1] = se / B + lam * (lr - lr_t) * (lr - lr_t);
  out[2] = 2.0 * lam * (lr - lr_t);  // dL/dlr
}

// dz3_b = 2 (y_b - t_b) / B * sigmoid(z3_b)
__global__ void k_dz3(const float* __restrict__ y, const float* __restrict__ t, const float* __restrict__ z3,
                      float* __restrict__ dz3, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float s = 1.0f / (1.0f + expf(-z3[b]));
  dz3[b] = 2.0f * (y[b] - t[b]) / B * s;
}

// head gradients: g_w3[k] = sum_b dz3_b relu(z2[b][k]); g_b3 = sum_b dz3_b;
// g_wr[k] = dlr * pooled[k]; g_br = dlr
__global__ void k_head_grad(const float* __restrict__ z2, const float* __restrict__ dz3,
                            const float* __restrict__ pooled, const double* __restrict__ sc, float* __restrict__ gw3,
                            float* __restrict__ gb3, float* __restrict__ gwr, float* __restrict__ gbr, int B, int H) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const float dlr = static_cast<float>(sc[2]);
  if (k < H) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += static_cast<double>(dz3[b]) * fmaxf(z2[static_cast<int64_t>(b) * H + k], 0.0f);
    gw3[k] = static_cast<float>(s);
    gwr[k] = dlr * pooled[k];
  }
  if (k == 0) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += dz3[b];
    gb3[0] = static_cast<float>(s);
    gbr[0] = dlr;
  }
}

// dz2[b][k] = (dz3_b w3[k] + dlr wr[k] / B) [z2[b][k] > 0]
__global__ void k_dz2(const float* __restrict__ z2, const float* __restrict__ dz3, const float* __restrict__ w3,
                      const float* __restrict__ wr, const double* __restrict__ sc, float* __restrict__ dz2, int B,
                      int H) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(B) * H) return;
  const int b = static_cast<int>(idx / H), k = static_cast<int>(idx % H);
  const float g = dz3[b] * w3[k] + static_cast<float>(sc[2]) * wr[k] / B;
  dz2[idx] = z2[idx] > 0.0f ? g : 0.0f;
}

// dz1[b][i] = (sum_k dz2[b][k] W2[k][i]) [z1[b][i] > 0]; block: nin threads, kRows rows
__global__ void k_back_data(const float* __restrict__ dz, const float* __restrict__ W, const float* __restrict__ z,
                            float* __restrict__ dzin, int B, int H, int nin) {
  extern __shared__ float ds[];  // kRows x H
  const int b0 = blockIdx.x * kRows;
  for (int idx = threadIdx.x; idx < kRows * H; idx += blockDim.x) {
    const int r = idx / H, k = idx % H;
    ds[idx] = (b0 + r < B) ? dz[static_cast<int64_t>(b0 + r) * H + k] : 0.0f;
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i >= nin) return;
  float acc[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) acc[r] = 0.0f;
  for (int k = 0; k < H; ++k) {
    const float w = W[static_cast<int64_t>(k) * nin + i];
#pragma unroll
    for (int r = 0; r < kRows; ++r) acc[r] = fmaf(ds[r * H + k], w, acc[r]);
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r)
    if (b0 + r < B) {
      const int64_t o = static_cast<int64_t>(b0 + r) * nin + i;
      dzin[o] = z[o] > 0.0f ? acc[r] : 0.0f;
    }
}

// weight gradient gW[k][i] = sum_b dz[b][k] act(in[b][i]); gb[k] = sum_b dz[b][k]
__global__ void k_weight_grad(const float* __restrict__ dz, const float* __restrict__ in, int relu_in,
                              float* __restrict__ gW, float* __restrict__ gb, int B, int H, int nin) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i < nin) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) {
      float x = in[static_cast<int64_t>(b) * nin + i];
      if (relu_in) x = fmaxf(x, 0.0f);
      s += static_cast<double>(dz[static_cast<int64_t>(b) * H + k]) * x;
    }
    gW[static_cast<int64_t>(k) * nin + i] = static_cast<float>(s);
  }
  if (i == 0) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += dz[static_cast<int64_t>(b) * H + k];
    gb[k] = static_cast<float>(s);
  }
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float gj = g[j];
  const float mj = b1 * m[j] + (1.0f - b1) * gj;
  const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  th[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

thread_local std::string g_mlp_error;

}  // namespace

struct admm_mlp {
  int F = 0, H = 0;
  int64_t np = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  float *th = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  int cap = 0;  // rows the activation buffers hold
  float *X = nullptr, *t = nullptr, *z1 = nullptr, *z2 = nullptr, *z3 = nullptr, *y = nullptr, *dz3 = nullptr;
  float *dz2 = nullptr, *dz1 = nullptr, *pooled = nullptr;
  uint16_t *h1b = nullptr, *h2b = nullptr;  // bf16 inference: hidden activations as bf16
  double* sc = nullptr;
  double* h_sc = nullptr;
  int64_t step = 0;
  // parameter offsets
  int64_t oW1, ob1, oW2, ob2, ow3, ob3, owr, obr;

  ~admm_mlp() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : {static_cast<void*>(th), static_cast<void*>(g), static_cast<void*>(m), static_cast<void*>(v)})
      if (p) (void)hipFree(p);
    free_rows();
    if (sc) (void)hipFree(sc);
    if (h_sc) (void)hipHostFree(h_sc);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
  void free_rows() {
    for (float* p : {X, t, z1, z2, z3, y, dz3, dz2, dz1, pooled})
      if (p) (void)hipFree(p);
    for (uint16_t* p : {h1b, h2b})
      if (p) (void)hipFree(p);
    X = t = z1 = z2 = z3 = y = dz3 = dz2 = dz1 = pooled = nullptr;
    h1b = h2b = nullptr;
    cap = 0;
  }
  void ensure(int B) {
    if (B <= cap) return;
    free_rows();
    const int c = std::max(B, 1024);
    auto a = [&](float** p, int64_t n) { ck(hipMalloc(reinterpret_cast<void**>(p), sizeof(float) * n)); };
    a(&X, static_cast<int64_t>(c) * F);
    a(&t, c);
    a(&z1, static_cast<int64_t>(c) * H);
    a(&z2, static_cast<int64_t>(c) * H);
    a(&z3, c);
    a(&y, c);
    a(&dz3, c);
    a(&dz2, static_cast<int64_t>(c) * H);
    a(&dz1, static_cast<int64_t>(c) * H);
    a(&pooled, H);
    ck(hipMalloc(reinterpret_cast<void**>(&h1b), sizeof(uint16_t) * static_cast<int64_t>(c) * H));
    ck(hipMalloc(reinterpret_cast<void**>(&h2b), sizeof(uint16_t) * static_cast<int64_t>(c) * H));
    cap = c;
  }
  void forward(int B, int bf16) {
    const int nb = (B + kRows - 1) / kRows;
    if (bf16) {
      // inference only: the hidden layers are stored as bf16 (fp32 weights and accumulation)
      hipLaunchKernelGGL(k_dense_bf16<float>, dim3(nb), dim3(H), sizeof(float) * kRows * F, stream, X, F, th + oW1,
                         th + ob1, h1b, B, H);
      hipLaunchKernelGGL(k_dense_bf16<uint16_t>, dim3(nb), dim3(H), sizeof(float) * kRows * H, stream, h1b, H,
                         th + oW2, th + ob2, h2b, B, H);
      hipLaunchKernelGGL(k_head_bf16, dim3((B + 255) / 256), dim3(256), 0, stream, h2b, th + ow3, th + ob3, z3, y, B,
                         H);
      hipLaunchKernelGGL(k_pool_bf16, dim3((H + 127) / 128), dim3(128), 0, stream, h2b, pooled, B, H);
      return;
    }
    hipLaunchKernelGGL(k_dense, dim3(nb), dim3(H), sizeof(float) * kRows * F, stream, X, F, th + oW1, th + ob1, z1, B,
                       H, 0, 0);
    hipLaunchKernelGGL(k_dense, dim3(nb), dim3(H), sizeof(float) * kRows * H, stream, z1, H, th + oW2, th + ob2, z2, B,
                       H, 1, bf16);
    hipLaunchKernelGGL(k_head, dim3((B + 255) / 256), dim3(256), 0, stream, z2, th + ow3, th + ob3, z3, y, B, H, bf16);
    hipLaunchKernelGGL(k_pool, dim3((H + 127) / 128), dim3(128), 0, stream, z2, pooled, B, H);
  }
};

namespace {
admm_status mlp_fail(admm_mlp* n, const char* what, hipError_t e) {
  (void)n;
  g_mlp_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? ADMM_E_OOM : ADMM_E_HIP;
}
}  // namespace

extern "C" {

const char* mlp_last_error(void) { return g_mlp_error.c_str(); }

admm_status mlp_create(int32_t nin, int32_t hidden, uint64_t seed, void* stream, admm_mlp** out) {
  if (!out) return ADMM_E_ARG;
  *out = nullptr;
  if (nin < 1 || nin > 1024 || hidden < 1 || hidden > 1024) {
    g_mlp_error = "nin and hidden must be in 1..1024";
    return ADMM_E_ARG;
  }
  admm_mlp* n = new (std::nothrow) admm_mlp();
  if (!n) return ADMM_E_OOM;
  try {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
      delete n;
      g_mlp_error = "no HIP device available";
      return ADMM_E_HIP;
    }
    n->F = nin;
    n->H = hidden;
    const int F = nin, H = hidden;
    n->oW1 = 0;
    n->ob1 = n->oW1 + static_cast<int64_t>(H) * F;
    n->oW2 = n->ob1 + H;
    n->ob2 = n->oW2 + static_cast<int64_t>(H) * H;
    n->ow3 = n->ob2 + H;
    n->ob3 = n->ow3 + H;
    n->owr = n->ob3 + 1;
    n->obr = n->owr + H;
    n->np = n->obr + 1;
    if (stream) {
      n->stream = static_cast<hipStream_t>(stream);
    } else {
      ck(hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking));
      n->own_stream = true;
    }
    for (float** p : {&n->th, &n->g, &n->m, &n->v}) ck(hipMalloc(reinterpret_cast<void**>(p), sizeof(float) * n->np));
    ck(hipMalloc(reinterpret_cast<void**>(&n->sc), sizeof(double) * 4));
    ck(hipHostMalloc(reinterpret_cast<void**>(&n->h_sc), sizeof(double) * 4, hipHostMallocDefault));
    // He-uniform weights from a splitmix64 stream, zero biases
    std::vector<float> th(static_cast<size_t>(n->np), 0.0f);
    uint64_t s = seed;
    auto uni = [&](double lim) {
      const double u = (splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
      return static_cast<float>((2.0 * u - 1.0) * lim);
    };
    for (int64_t j = 0; j < static_cast<int64_t>(H) * F; ++j) th[n->oW1 + j] = uni(std::sqrt(6.0 / F));
    for (int64_t j = 0; j < static_cast<int64_t>(H) * H; ++j) th[n->oW2 + j] = uni(std::sqrt(6.0 / H));
    for (int j = 0; j < H; ++j) th[n->ow3 + j] = uni(std::sqrt(3.0 / H));
    for (int j = 0; j < H; ++j) th[n->owr + j] = uni(std::sqrt(3.0 / H)) * 0.1f;
    ck(hipMemcpy(n->th, th.data(), sizeof(float) * n->np, hipMemcpyHostToDevice));
    ck(hipMemset(n->m, 0, sizeof(float) * n->np));
    ck(hipMemset(n->v, 0, sizeof(float) * n->np));
    ck(hipMemset(n->g, 0, sizeof(float) * n->np));
  } catch (const HipErr& e) {
    delete n;
    return mlp_fail(nullptr, "mlp_create", e.e);
  } catch (const std::exception&) {
    delete n;
    return mlp_fail(nullptr, "mlp_create", hipErrorOutOfMemory);
  }
  *out = n;
  return ADMM_OK;
}

void mlp_destroy(admm_mlp* n) { delete n; }

int64_t mlp_num_params(const admm_mlp* n) { return n ? n->np : 0; }

admm_status mlp_get_params(admm_mlp* n, float* out) {
  if (!n || !out) return ADMM_E_ARG;
  try {
    ck(hipStreamSynchronize(n->stream));
    ck(hipMemcpy(out, n->th, sizeof(float) * n->np, hipMemcpyDeviceToHost));
  } catch (const HipErr& e) {
    return mlp_fail(n, "mlp_get_params", e.e);
  } catch (const std::exception&) {  // host allocation: nothing crosses the C boundary
    return mlp_fail(n, "mlp_get_params", hipErrorOutOfMemory);
  }
  return ADMM_OK;
}

admm_status mlp_set_params(admm_mlp* n, const float* in) {
  if (!n || !in) return ADMM_E_ARG;
  for (int64_t j = 0; j < n->np; ++j)
    if (!std::isfinite(in[j])) {
      g_mlp_error = "parameters not finite";
      return ADMM_E_NONFINITE;
    }
  try {
    ck(hipStreamSynchronize(n->stream));
    ck(hipMemcpy(n->th, in, sizeof(float) * n->np, hipMemcpyHostToDevice));
    ck(hipMemset(n->m, 0, sizeof(float) * n->np));
    ck(hipMemset(n->v, 0, sizeof(float) * n->np));
    n->step = 0;
  } catch (const HipErr& e) {
    return mlp_fail(n, "mlp_set_params", e.e);
  } catch (const std::exception&) {  // host allocation: nothing crosses the C boundary
    return mlp_fail(n, "mlp_set_params", hipErrorOutOfMemory);
  }
  return ADMM_OK;
}

admm_status mlp_forward(admm_mlp* n, const float* X, int32_t rows, int32_t precision, float* y_out,
                        float* log_rho_out) {
  (void)hipGetLastError();  // report only this call's errors
  if (!n || !X || rows < 1 || (precision != ADMM_PREC_FP32 && precision != ADMM_PREC_BF16)) return ADMM_E_ARG;
  try {
    n->ensure(rows);
    ck(hipMemcpyAsync(n->X, X, sizeof(float) * rows * n->F, hipMemcpyHostToDevice, n->stream));
    n->forward(rows, precision == ADMM_PREC_BF16 ? 1 : 0);
    hipLaunchKernelGGL(k_scalars, dim3(1), dim3(1), 0, n->stream, n->pooled, n->th + n->owr, n->th + n->obr, n->y,
                       static_cast<const float*>(nullptr), rows, n->H, 0.0f, 0.0f, n->sc);
    if (y_out) ck(hipMemcpyAsync(y_out, n->y, sizeof(float) * rows, hipMemcpyDeviceToHost, n->stream));
    ck(hipMemcpyAsync(n->h_sc, n->sc, sizeof(double) * 3, hipMemcpyDeviceToHost, n->stream));
    ck(hipStreamSynchronize(n->stream));
    if (log_rho_out) *log_rho_out = static_cast<float>(n->h_sc[0]);
  } catch (const HipErr& e) {
    return mlp_fail(n, "mlp_forward", e.e);
  } catch (const std::exception&) {  // host allocation: nothing crosses the C boundary
    return mlp_fail(n, "mlp_forward", hipErrorOutOfMemory);
  }
  return ADMM_OK;
}

admm_status mlp_loss_grad(admm_mlp* n, const float* X, const float* target, int32_t rows, float target_log_rho,
                          float lam, double* loss_out, float* grad_out) {
  (void)hipGetLastError();  // report only this call's errors
  if (!n || !X || !target || rows < 1 || !std::isfinite(target_log_rho) || !(lam >= 0)) return ADMM_E_ARG;
  try {
    const int B = rows, H = n->H, F = n->F;
    n->ensure(B);
    ck(hipMemcpyAsync(n->X, X, sizeof(float) * B * F, hipMemcpyHostToDevice, n->stream));
    ck(hipMemcpyAsync(n->t, target, sizeof(float) * B, hipMemcpyHostToDevice, n->stream));
    n->forward(B, 0);
    hipLaunchKernelGGL(k_scalars, dim3(1), dim3(1), 0, n->stream, n->pooled, n->th + n->owr, n->th + n->obr, n->y,
                       n->t, B, H, target_log_rho, lam, n->sc);
    hipLaunchKernelGGL(k_dz3, dim3((B + 255) / 256), dim3(256), 0, n->stream, n->y, n->t, n->z3, n->dz3, B);
    hipLaunchKernelGGL(k_head_grad, dim3((H + 127) / 128), dim3(128), 0, n->stream, n->z2, n->dz3, n->pooled, n->sc,
                       n->g + n->ow3, n->g + n->ob3, n->g + n->owr, n->g + n->obr, B, H);
    const int64_t BH = static_cast<int64_t>(B) * H;
    hipLaunchKernelGGL(k_dz2, dim3(static_cast<unsigned>((BH + 255) / 256)), dim3(256), 0, n->stream, n->z2, n->dz3,
                       n->th + n->ow3, n->th + n->owr, n->sc, n->dz2, B, H);
    hipLaunchKernelGGL(k_weight_grad, dim3((H + 127) / 128, H), dim3(128), 0, n->stream, n->dz2, n->z1, 1,
                       n->g + n->oW2, n->g + n->ob2, B, H, H);
    const int nb = (B + kRows - 1) / kRows;
    hipLaunchKernelGGL(k_back_data, dim3(nb), dim3(H), sizeof(float) * kRows * H, n->stream, n->dz2, n->th + n->oW2,
                       n->z1, n->dz1, B, H, H);
    hipLaunchKernelGGL(k_weight_grad, dim3((F + 127) / 128, H), dim3(128), 0, n->stream, n->dz1, n->X, 0,
                       n->g + n->oW1, n->g + n->ob1, B, H, F);
    ck(hipGetLastError());
    ck(hipMemcpyAsync(n->h_sc, n->sc, sizeof(double) * 3, hipMemcpyDeviceToHost, n->stream));
    if (grad_out) ck(hipMemcpyAsync(grad_out, n->g, sizeof(float) * n->np, hipMemcpyDeviceToHost, n->stream));
    ck(hipStreamSynchronize(n->stream));
    if (loss_out) *loss_out = n->h_sc[1];
  } catch (const HipErr& e) {
    return mlp_fail(n, "mlp_loss_grad", e.e);
  } catch (const std::exception&) {  // host allocation: nothing crosses the C boundary
    return mlp_fail(n, "mlp_loss_grad", hipErrorOutOfMemory);
  }
  return ADMM_OK;
}

admm_status mlp_adam_step(admm_mlp* n, float lr, float beta1, float beta2, float eps) {
  (void)hipGetLastError();  // report only this call's errors
  if (!n || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0)) return ADMM_E_ARG;
  try {
    n->step += 1;
    const float c1 = 1.0f - std::pow(beta1, static_cast<float>(n->step));
    const float c2 = 1.0f - std::pow(beta2, static_cast<float>(n->step));
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((n->np + 255) / 256)), dim3(256), 0, n->stream, n->th, n->g,
                       n->m, n->v, n->np, lr, beta1, beta2, eps, c1, c2);
    ck(hipGetLastError());
    ck(hipStreamSynchronize(n->stream));
  } catch (const HipErr& e) {
    return mlp_fail(n, "mlp_adam_step", e.e);
  } catch (const std::exception&) {  // host allocation: nothing crosses the C boundary
    return mlp_fail(n, "mlp_adam_step", hipErrorOutOfMemory);
  }
  return ADMM_OK;
}

}  // extern "C"
