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

}  // namespace

int dose_hist_smem_bytes(int G, int nbins) { return G * 12 + G * nbins * 4; }

void launch_dose_hist(const float* dose, const uint8_t* grp, int m, int G, int nbins, float inv_w, uint32_t* counts,
                      double* sums, uint32_t* maxkey, hipStream_t st) {
  int nb = (m + kThreads * 8 - 1) / (kThreads * 8);
  nb = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
  hipLaunchKernelGGL(k_dose_hist, dim3(nb), dim3(kThreads), dose_hist_smem_bytes(G, nbins), st, dose, grp, m, G,
                     nbins, inv_w, counts, sums, maxkey);
}

}  // namespace admmbb
