// Per-group dose statistics of a plan: histogram, sum and maximum of the
// voxel doses d = A_s x of one scenario, for the dose-volume evaluation of
// Sec. 3 (dose-volume histograms and D98 / Dmax / D3 / Dmean metrics).
//
// One launch per scenario over the m voxel doses (original voxel order).
// Each block keeps the histogram of every group in LDS (32-bit counters),
// plus per-group double sums and order-preserving 32-bit max keys, and merges
// them into the global arrays with one atomic per nonzero entry.  Counts and
// maxima are exact and order-independent; the sums are double atomics
// (order-dependent only in the last bits).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "internal.h"

namespace admmbb {

namespace {

// order-preserving map from float to uint32 (negative values below positive)
__device__ __forceinline__ uint32_t float_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(kThreads) void k_dose_hist(const float* __restrict__ dose,
                                                        const uint8_t* __restrict__ grp, int m, int G, int nbins,
                                                        float inv_w, uint32_t* __restrict__ counts,
                                                        double* __restrict__ sums, uint32_t* __restrict__ maxkey) {
  extern __shared__ __align__(8) unsigned char smem[];
  double* ssum = reinterpret_cast<double*>(smem);             // G
  uint32_t* smax = reinterpret_cast<uint32_t*>(ssum + G);     // G
  uint32_t* hist = smax + G;                                  // G * nbins
  for (int k = threadIdx.x; k < G * nbins; k += blockDim.x) hist[k] = 0u;
  for (int k = threadIdx.x; k < G; k += blockDim.x) {
    ssum[k] = 0.0;
    smax[k] = 0u;
  }
  __syncthreads();
  // consecutive voxels mostly share a group: accumulate sum and max in
  // registers and flush to LDS when the group changes
  int cur = -1;
  double acc = 0.0;
  uint32_t mk = 0u;
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const int g = grp[i];
    const float d = dose[i];
    int b = static_cast<int>(d * inv_w);
    b = b < 0 ? 0 : (b >= nbins ? nbins - 1 : b);
    if (!(d >= 0.0f)) b = 0;  // negative doses (and NaN) fall in the first bin
    atomicAdd(&hist[g * nbins + b], 1u);
    if (g != cur) {
      if (cur >= 0) {
        atomicAdd(&ssum[cur], acc);
        atomicMax(&smax[cur], mk);
      }
      cur = g;
      acc = 0.0;
      mk = 0u;
    }
    acc += static_cast<double>(d);
    const uint32_t key = float_key(d);
    mk = key > mk ? key : mk;
  }
  if (cur >= 0) {
    atomicAdd(&ssum[cur], acc);
    atomicMax(&smax[cur], mk);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < G * nbins; k += blockDim.x)
    if (hist[k] != 0u) atomicAdd(&counts[k], hist[k]);
  for (int k = threadIdx.x; k < G; k += blockDim.x)
    if (smax[k] != 0u) {
      atomicAdd(&sums[k], ssum[k]);
      atomicMax(&maxkey[k], smax[k]);
    }
}

__global__ __launch_bounds__(kThreads) void k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out,
                                                          int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = static_cast<float>(in[i]);
}

}  // namespace

// Scratch of the allocation-free dose statistics: a fixed array in device
// memory, one copy per GPU, alive until the process ends.  Host code never
// passes the array's own name to a kernel (on the host that name is only a
// stand-in, not a device address); it uses the address hipGetSymbolAddress
// returns for the current device.
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

int dose_hist_smem_bytes(int G, int nbins) { return G * 12 + G * nbins * 4; }

hipError_t noalloc_scratch(void** ptr) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static void* addr[kMaxDev] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

void launch_f64_to_f32(const double* in, float* out, int n, hipStream_t st) {
  int nb = (n + kThreads - 1) / kThreads;
  nb = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
  hipLaunchKernelGGL(k_f64_to_f32, dim3(nb), dim3(kThreads), 0, st, in, out, n);
}

void launch_dose_hist(const float* dose, const uint8_t* grp, int m, int G, int nbins, float inv_w, uint32_t* counts,
                      double* sums, uint32_t* maxkey, hipStream_t st) {
  int nb = (m + kThreads * 8 - 1) / (kThreads * 8);
  nb = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
  hipLaunchKernelGGL(k_dose_hist, dim3(nb), dim3(kThreads), dose_hist_smem_bytes(G, nbins), st, dose, grp, m, G,
                     nbins, inv_w, counts, sums, maxkey);
}

}  // namespace admmbb
