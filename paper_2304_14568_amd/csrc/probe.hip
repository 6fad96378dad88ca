// Streaming-read reference: the rate at which this device reads a buffer of a
// given size in one pass (16 KiB per workgroup, every load instruction of a
// wave 1 KiB contiguous, four loads in flight per lane: the fastest shape
// measured at sizes beyond the last-level cache), used to put the measured
// kernel rates next to what the memory system delivers at that size.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/admmbb.h"

namespace {

__global__ __launch_bounds__(256) void k_stream(const float4* __restrict__ a, float* __restrict__ sink, int64_t n4) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * 1024 + threadIdx.x;
  // all four loads in flight before any use
  float4 v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = base + 256 * u;
    v[u] = i < n4 ? a[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  float s = 0.0f;
#pragma unroll
  for (int u = 0; u < 4; ++u) s += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  // a data-dependent store that never happens for the fill used below keeps
  // the loads from being removed
  if (s == -1.0f) sink[blockIdx.x & 1023] = s;
}

__global__ void k_fill4(float4* a, int64_t n4) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n4) a[i] = make_float4(1.0f, 2.0f, 3.0f, 4.0f);
}

}  // namespace

extern "C" admm_status admm_stream_probe(int64_t bytes, int32_t reps, double* gbs_out) {
  if (gbs_out == nullptr || reps < 1 || bytes < (int64_t{1} << 20) || bytes > (int64_t{16} << 30))
    return ADMM_E_ARG;
  (void)hipGetLastError();
  const int64_t n4 = bytes / 16;
  float4* a = nullptr;
  float* sink = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  admm_status rc = ADMM_OK;
  if (hipMalloc(&a, n4 * 16) != hipSuccess || hipMalloc(&sink, 1024 * sizeof(float)) != hipSuccess) {
    rc = ADMM_E_OOM;
  } else if (hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
             hipEventCreate(&e1) != hipSuccess) {
    rc = ADMM_E_HIP;
  } else {
    const unsigned grid = static_cast<unsigned>((n4 + 1023) / 1024);
    hipLaunchKernelGGL(k_fill4, dim3(static_cast<unsigned>((n4 + 255) / 256)), dim3(256), 0, st, a, n4);
    hipLaunchKernelGGL(k_stream, dim3(grid), dim3(256), 0, st, a, sink, n4);  // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_stream, dim3(grid), dim3(256), 0, st, a, sink, n4);
    (void)hipEventRecord(e1, st);
    float ms = 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        hipGetLastError() != hipSuccess || !(ms > 0.0f))
      rc = ADMM_E_HIP;
    else
      *gbs_out = static_cast<double>(n4) * 16.0 * reps / (ms * 1e-3) / 1e9;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  if (a) (void)hipFree(a);
  if (sink) (void)hipFree(sink);
  return rc;
}
