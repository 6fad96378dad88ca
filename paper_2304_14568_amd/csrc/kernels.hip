// gfx950 kernels for ADMM-BB robust planning.
//
// The hot kernel is k_pass: one streaming pass over the length-sorted CSR of
// every (patient, scenario) dose-influence matrix A_s.  For each row i it forms
// the row dot a_i . v, turns it into t_i (c_s w_i a_i.v for a CG product,
// c_s w_i (a_i.v - p_i) for the gradient / objective), and immediately scatters
// t_i a_i into column accumulators held in LDS.  The row's values and column
// indices stay in registers between the two uses, so each nonzero is read from
// HBM once per operator application A_s^T diag(c_s w) A_s v (the x-update
// system of Appendix A without its rho/2 shift).  Each workgroup writes its
// column partial sums; a column-blocked reduction kernel adds them in a fixed
// order.  All scalar reductions are float64 and deterministic (fixed trees).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"
#include "scalars.h"

namespace admmbb {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

template <int VK>
struct ValT;
template <>
struct ValT<VAL_F32> {
  using T = float;
  static __device__ __forceinline__ float f(T v) { return v; }
};
template <>
struct ValT<VAL_BF16> {
  using T = uint16_t;
  static __device__ __forceinline__ float f(T v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }
};
template <>
struct ValT<VAL_F16> {
  using T = _Float16;
  static __device__ __forceinline__ float f(T v) { return static_cast<float>(v); }
};

// ---------------------------------------------------------------------------
// the fused pass
// ---------------------------------------------------------------------------

// Round a scaled contribution d (|d| < 2^50) to the nearest integer, as a
// two's-complement 64-bit value: adding 1.5 * 2^52 moves the rounded integer
// into the low mantissa bits (exact for |d| < 2^51); subtracting the bit
// pattern of 1.5 * 2^52, whose low word is zero, leaves the integer.
__device__ __forceinline__ unsigned long long to_fixed(double d) {
  const double r = d + 0x1.8p52;
  return static_cast<unsigned long long>(__double_as_longlong(r)) - 0x4338000000000000ull;
}

// 4-element chunk types: values (fp32: one 16-byte load; bf16 / fp16: 8 bytes)
// and column indices (uint16: 8 bytes; int32: 16 bytes).
template <int VK>
struct VChunk;
template <>
struct VChunk<VAL_F32> {
  using T = float4;
  static __device__ __forceinline__ void unpack(const T& c, float (&o)[4]) {
    o[0] = c.x;
    o[1] = c.y;
    o[2] = c.z;
    o[3] = c.w;
  }
};
template <>
struct VChunk<VAL_BF16> {
  using T = uint2;
  static __device__ __forceinline__ void unpack(const T& c, float (&o)[4]) {
    o[0] = __uint_as_float(c.x << 16);
    o[1] = __uint_as_float(c.x & 0xffff0000u);
    o[2] = __uint_as_float(c.y << 16);
    o[3] = __uint_as_float(c.y & 0xffff0000u);
  }
};
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
template <>
struct VChunk<VAL_F16> {
  using T = uint2;
  static __device__ __forceinline__ void unpack(const T& c, float (&o)[4]) {
    const half2v a = __builtin_bit_cast(half2v, c.x);
    const half2v b = __builtin_bit_cast(half2v, c.y);
    o[0] = static_cast<float>(a[0]);
    o[1] = static_cast<float>(a[1]);
    o[2] = static_cast<float>(b[0]);
    o[3] = static_cast<float>(b[1]);
  }
};
template <bool C16>
struct CChunk;
template <>
struct CChunk<true> {
  using T = uint2;
  static __device__ __forceinline__ int get(const T& c, int e) {
    const uint32_t w = (e < 2) ? c.x : c.y;
    return static_cast<int>((e & 1) ? (w >> 16) : (w & 0xffffu));
  }
};
template <>
struct CChunk<false> {
  using T = int4;
  static __device__ __forceinline__ int get(const T& c, int e) {
    return e == 0 ? c.x : (e == 1 ? c.y : (e == 2 ? c.z : c.w));
  }
};

// Rows of one tile with L lanes per row.  Rows are stored padded to whole
// 4-element chunks (zero values); lane l of a row loads chunks l, l+L, ... with
// one wide load per chunk and keeps up to kRegChunks of them in registers
// between the row dot product and the scatter.  Rows longer than that (only in
// the 64-lane bin) stream their tail twice.  The next row's offsets are loaded
// while the current row computes.
//
// MODE  PASS_GRAD     t_i = c_s w_i (a_i.v - p_i) (fp64 dot), objective partial, scatter
//       PASS_OBJ      objective partial only
//       PASS_MATVEC   (a_i.v) written to tout[row] (fp64 dot)
//       PASS_CG       t_i = c_s w_i a_i.v (fp32 dot), scatter
//       PASS_RMATVEC  t_i = tin[row], scatter
// ACC   LDS column accumulators (AccKind)
template <int VK, bool C16, int L, int MODE, int ACC, int NT, bool PIPE>
__device__ __forceinline__ void pass_rows(const PassArgs& a, const Tile& t, const Scen& sc, const float* vsh,
                                          void* qacc, double fscale, double& objacc) {
  using VC = typename VChunk<VK>::T;
  using CCk = typename CChunk<C16>::T;
  using VT = typename ValT<VK>::T;
  using CT = std::conditional_t<C16, uint16_t, int32_t>;
  constexpr bool kDot = MODE != PASS_RMATVEC;
  constexpr bool kScatter = MODE == PASS_GRAD || MODE == PASS_CG || MODE == PASS_RMATVEC;
  constexpr bool kDot64 = MODE == PASS_GRAD || MODE == PASS_OBJ || MODE == PASS_MATVEC;
  using DACC = std::conditional_t<kDot64, double, float>;
  constexpr int K = kRegChunks;
  constexpr int G = NT / L;
  const int grp = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  const uint32_t* __restrict__ rp = a.mat.rp + sc.rp_base;
  const VC* __restrict__ valc = reinterpret_cast<const VC*>(static_cast<const VT*>(a.mat.val) + sc.nnz_base);
  const CCk* __restrict__ colc = reinterpret_cast<const CCk*>(static_cast<const CT*>(a.mat.col) + sc.nnz_base);
  // bf16 / fp16 values with 16-bit columns: one 16-byte record per chunk (four
  // values, then their four columns), one load instruction per chunk
  constexpr bool kRec = VK != VAL_F32 && C16;
  const uint4* __restrict__ recc = reinterpret_cast<const uint4*>(a.mat.val) + sc.nnz_base / 4;
  auto ld = [&](uint32_t c, float (&v4)[4], CCk& c4) {
    if constexpr (kRec) {
      const uint4 q = recc[c];
      VChunk<VK>::unpack(VC{q.x, q.y}, v4);
      c4 = CCk{q.z, q.w};
    } else {
      VChunk<VK>::unpack(valc[c], v4);
      c4 = colc[c];
    }
  };
  const int64_t rb = sc.row_base;
  const int rend = t.row_end;
  float* __restrict__ qf = static_cast<float*>(qacc);
  double* __restrict__ qd = static_cast<double*>(qacc);
  unsigned long long* __restrict__ qi = static_cast<unsigned long long*>(qacc);

  auto scatter4 = [&](const CCk& c4, const float (&v4)[4], float tv, double td) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = CChunk<C16>::get(c4, q);
      if constexpr (ACC == ACC_FIX64)
        atomicAdd(&qi[j], to_fixed(td * static_cast<double>(v4[q])));
      else if constexpr (ACC == ACC_F64)
        atomicAdd(&qd[j], static_cast<double>(tv * v4[q]));
      else
        atomicAdd(&qf[j], tv * v4[q]);
    }
  };
  auto dot4 = [&](const CCk& c4, const float (&v4)[4], DACC& dot) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float xv = vsh[CChunk<C16>::get(c4, q)];
      if constexpr (kDot64)
        dot += static_cast<double>(v4[q]) * static_cast<double>(xv);
      else
        dot = fmaf(v4[q], xv, dot);
    }
  };

  // chunks of the row a lane handles next are loaded while the current row computes
  auto load_row = [&](uint32_t s0, uint32_t e0, float (&vv)[K][4], CCk (&cc)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t c = s0 + lane + k * L;
      if (c < e0) {
        ld(c, vv[k], cc[k]);
      } else {
        vv[k][0] = vv[k][1] = vv[k][2] = vv[k][3] = 0.0f;
        cc[k] = CCk{};
      }
    }
  };

  int r = t.row_begin + grp;
  uint32_t s = r < rend ? rp[r] : 0u;
  uint32_t e = r < rend ? rp[r + 1] : 0u;
  float vv[K][4];
  CCk cc[K];
  if constexpr (PIPE) load_row(s, e, vv, cc);
  for (; r < rend; r += G) {
    if constexpr (!PIPE) load_row(s, e, vv, cc);
    float rw;
    float aux = 0.0f;
    if constexpr (MODE == PASS_RMATVEC) {
      rw = a.tin[a.mat.rorig[rb + r]];
    } else if constexpr (MODE == PASS_MATVEC) {
      rw = 0.0f;
    } else {
      rw = a.mat.rw[rb + r];
      if constexpr (kDot64)
        aux = a.mat.rpres[rb + r];
      else if (a.mat.rscale != nullptr)
        aux = a.mat.rscale[rb + r];
      else
        aux = 1.0f;
    }
    // next row: offsets and (when pipelined) its register chunks, in flight while this row computes
    const int rn = r + G;
    const uint32_t sn = rn < rend ? rp[rn] : 0u;
    const uint32_t en = rn < rend ? rp[rn + 1] : 0u;
    float vn[K][4];
    CCk cn[K];
    if constexpr (PIPE) load_row(sn, en, vn, cn);

    float tv = rw;
    if constexpr (kDot) {
      DACC dot = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) dot4(cc[k], vv[k], dot);
      for (uint32_t c = s + lane + K * L; c < e; c += L) {
        float v4[4];
        CCk c4;
        ld(c, v4, c4);
        dot4(c4, v4, dot);
      }
#pragma unroll
      for (int off = L / 2; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
      if constexpr (MODE == PASS_MATVEC) {
        if (lane == 0) a.tout[a.mat.rorig[rb + r]] = static_cast<float>(dot);
      } else if constexpr (kDot64) {
        const double res = dot - static_cast<double>(aux);
        const double wgt = static_cast<double>(rw);
        if (lane == 0) objacc += wgt * res * res;
        tv = static_cast<float>(wgt * res);
      } else {
        tv = rw * dot * aux * aux;
      }
    }
    if constexpr (kScatter) {
      const double td = static_cast<double>(tv) * fscale;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (s + lane + k * L < e) scatter4(cc[k], vv[k], tv, td);
      }
      for (uint32_t c = s + lane + K * L; c < e; c += L) {
        float v4[4];
        CCk c4;
        ld(c, v4, c4);
        scatter4(c4, v4, tv, td);
      }
    }
    s = sn;
    e = en;
    if constexpr (PIPE) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        cc[k] = cn[k];
#pragma unroll
        for (int q = 0; q < 4; ++q) vv[k][q] = vn[k][q];
      }
    }
  }
}

// The same work over the sliced layout (FMT_SELL): wave w of the workgroup
// takes slices w, w + NW, ... of the tile; in a slice, lanes g L .. g L + L - 1
// hold row g (G = 64 / L rows), and the wave's k-th load instruction reads the
// slice's 64 consecutive chunk slots of step k (1 KiB of fp32 values).  The
// number of steps is the slice's, uniform across the wave, so the loads are
// not predicated; padding slots hold zeros and add nothing.
template <int VK, bool C16, int L, int MODE, int ACC, int NT>
__device__ __forceinline__ void pass_slices(const PassArgs& a, const Tile& t, const Scen& sc, const float* vsh,
                                            void* qacc, double fscale, double& objacc) {
  using VC = typename VChunk<VK>::T;
  using CCk = typename CChunk<C16>::T;
  using VT = typename ValT<VK>::T;
  using CT = std::conditional_t<C16, uint16_t, int32_t>;
  constexpr bool kDot = MODE != PASS_RMATVEC;
  constexpr bool kScatter = MODE == PASS_GRAD || MODE == PASS_CG || MODE == PASS_RMATVEC;
  constexpr bool kDot64 = MODE == PASS_GRAD || MODE == PASS_OBJ || MODE == PASS_MATVEC;
  using DACC = std::conditional_t<kDot64, double, float>;
  constexpr int K = kRegChunks;
  constexpr int G = 64 / L;
  constexpr int NW = NT / 64;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int g = lane / L;
  const VC* __restrict__ valc = reinterpret_cast<const VC*>(static_cast<const VT*>(a.mat.val) + sc.sell_base * 4);
  const CCk* __restrict__ colc = reinterpret_cast<const CCk*>(static_cast<const CT*>(a.mat.col) + sc.sell_base * 4);
  constexpr bool kRec = VK != VAL_F32 && C16;
  const uint4* __restrict__ recc = reinterpret_cast<const uint4*>(a.mat.val) + sc.sell_base;
  auto ld = [&](uint32_t c, float (&v4)[4], CCk& c4) {
    if constexpr (kRec) {
      const uint4 q = recc[c];
      VChunk<VK>::unpack(VC{q.x, q.y}, v4);
      c4 = CCk{q.z, q.w};
    } else {
      VChunk<VK>::unpack(valc[c], v4);
      c4 = colc[c];
    }
  };
  const uint32_t* __restrict__ soff = a.mat.soff + t.slice_begin;
  const int64_t rb = sc.row_base;
  const int nsl = (t.row_end - t.row_begin + G - 1) / G;
  float* __restrict__ qf = static_cast<float*>(qacc);
  double* __restrict__ qd = static_cast<double*>(qacc);
  unsigned long long* __restrict__ qi = static_cast<unsigned long long*>(qacc);

  auto scatter4 = [&](const CCk& c4, const float (&v4)[4], float tv, double td) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jc = CChunk<C16>::get(c4, q);
      if constexpr (ACC == ACC_FIX64)
        atomicAdd(&qi[jc], to_fixed(td * static_cast<double>(v4[q])));
      else if constexpr (ACC == ACC_F64)
        atomicAdd(&qd[jc], static_cast<double>(tv * v4[q]));
      else
        atomicAdd(&qf[jc], tv * v4[q]);
    }
  };
  auto dot4 = [&](const CCk& c4, const float (&v4)[4], DACC& dot) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float xv = vsh[CChunk<C16>::get(c4, q)];
      if constexpr (kDot64)
        dot += static_cast<double>(v4[q]) * static_cast<double>(xv);
      else
        dot = fmaf(v4[q], xv, dot);
    }
  };

  for (int j = wave; j < nsl; j += NW) {
    const uint32_t s0 = soff[j];
    const int nk = static_cast<int>((soff[j + 1] - s0) >> 6);
    const int r = t.row_begin + j * G + g;
    const bool real = r < t.row_end;
    float vv[K][4];
    CCk cc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k < nk) {
        const uint32_t c = s0 + static_cast<uint32_t>(k * 64 + lane);
        ld(c, vv[k], cc[k]);
      } else {
        vv[k][0] = vv[k][1] = vv[k][2] = vv[k][3] = 0.0f;
        cc[k] = CCk{};
      }
    }
    float rw = 0.0f, aux = 0.0f;
    if (real) {
      if constexpr (MODE == PASS_RMATVEC) {
        rw = a.tin[a.mat.rorig[rb + r]];
      } else if constexpr (MODE != PASS_MATVEC) {
        rw = a.mat.rw[rb + r];
        if constexpr (kDot64)
          aux = a.mat.rpres[rb + r];
        else if (a.mat.rscale != nullptr)
          aux = a.mat.rscale[rb + r];
        else
          aux = 1.0f;
      }
    }
    float tv = rw;
    if constexpr (kDot) {
      DACC dot = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) dot4(cc[k], vv[k], dot);
      for (int k = K; k < nk; ++k) {
        const uint32_t c = s0 + static_cast<uint32_t>(k * 64 + lane);
        float v4[4];
        CCk c4;
        ld(c, v4, c4);
        dot4(c4, v4, dot);
      }
#pragma unroll
      for (int off = L / 2; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
      if constexpr (MODE == PASS_MATVEC) {
        if (real && (lane % L) == 0) a.tout[a.mat.rorig[rb + r]] = static_cast<float>(dot);
      } else if constexpr (kDot64) {
        const double res = real ? dot - static_cast<double>(aux) : 0.0;
        const double wgt = static_cast<double>(rw);
        if ((lane % L) == 0) objacc += wgt * res * res;
        tv = static_cast<float>(wgt * res);
      } else {
        tv = rw * dot * aux * aux;
      }
    }
    if constexpr (kScatter) {
      const double td = static_cast<double>(tv) * fscale;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < nk) scatter4(cc[k], vv[k], tv, td);
      for (int k = K; k < nk; ++k) {
        const uint32_t c = s0 + static_cast<uint32_t>(k * 64 + lane);
        float v4[4];
        CCk c4;
        ld(c, v4, c4);
        scatter4(c4, v4, tv, td);
      }
    }
  }
}

template <int VK, bool C16, int MODE, int ACC, int NT, bool PIPE, int FMT>
__global__ __launch_bounds__(NT) void k_pass(PassArgs a, int tile_begin) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float vmax_sh[NT / 64];
  constexpr bool kScatter = MODE == PASS_GRAD || MODE == PASS_CG || MODE == PASS_RMATVEC;
  const int ti = tile_begin + static_cast<int>(blockIdx.x);
  const Tile t = a.tiles[ti];
  const Scen sc = a.scen[t.scen];
  if (a.act != nullptr && !a.act[t.scen * kRing + a.step]) return;
  if (a.ps != nullptr && a.ps[sc.patient].stopped) return;
  const int n = sc.n;
  float* vsh = reinterpret_cast<float*>(smem);
  const size_t qoff = (static_cast<size_t>(a.nmax) * 4 + 15) & ~static_cast<size_t>(15);
  void* qacc = static_cast<void*>(smem + qoff);

  float vmax = 0.0f;
  if constexpr (MODE != PASS_RMATVEC) {
    const float* src = a.src + (a.src_per_scen ? sc.vec_base : a.pat[sc.patient].zvec_base);
    for (int j = threadIdx.x; j < n; j += NT) {
      const float x = src[j];
      vsh[j] = x;
      vmax = fmaxf(vmax, fabsf(x));
    }
  }
  if constexpr (kScatter) {
    if constexpr (ACC == ACC_F32)
      for (int j = threadIdx.x; j < n; j += NT) static_cast<float*>(qacc)[j] = 0.0f;
    else
      for (int j = threadIdx.x; j < n; j += NT) static_cast<unsigned long long*>(qacc)[j] = 0ull;
  }
  if constexpr (MODE == PASS_RMATVEC && ACC == ACC_FIX64) {
    // the given t bounds the contributions: max |t_i| over the tile's rows
    const int rb0 = static_cast<int>(sc.row_base);
    for (int r = t.row_begin + static_cast<int>(threadIdx.x); r < t.row_end; r += NT)
      vmax = fmaxf(vmax, fabsf(a.tin[a.mat.rorig[rb0 + r]]));
  }
  // fixed-point scale: every partial column sum of this tile, and every single
  // contribution, is below cmax * (wmax * max|v| + pmax) < 2^50 / 2^F (for the
  // transpose product: cmax * max|t_i|)
  double fscale = 1.0, funscale = 1.0;
  if constexpr (kScatter && ACC == ACC_FIX64) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, off, 64));
    if ((threadIdx.x & 63) == 0) vmax_sh[threadIdx.x >> 6] = vmax;
    __syncthreads();
    float vm = 0.0f;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) vm = fmaxf(vm, vmax_sh[w]);
    const double tb = MODE == PASS_RMATVEC
                          ? static_cast<double>(vm)
                          : static_cast<double>(t.wmax) * vm + (MODE == PASS_GRAD ? static_cast<double>(t.pmax) : 0.0);
    const double bound = 1.0625 * tb * static_cast<double>(t.cmax);
    if (bound > 0.0 && isfinite(bound)) {
      const int F = 49 - ilogb(bound);
      fscale = ldexp(1.0, F);
      funscale = ldexp(1.0, -F);
    }
  }
  __syncthreads();

  double objacc = 0.0;
  if constexpr (FMT == FMT_SELL) {
    switch (t.lanes) {
      case 1: pass_slices<VK, C16, 1, MODE, ACC, NT>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 2: pass_slices<VK, C16, 2, MODE, ACC, NT>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 4: pass_slices<VK, C16, 4, MODE, ACC, NT>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 8: pass_slices<VK, C16, 8, MODE, ACC, NT>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 16: pass_slices<VK, C16, 16, MODE, ACC, NT>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 32: pass_slices<VK, C16, 32, MODE, ACC, NT>(a, t, sc, vsh, qacc, fscale, objacc); break;
      default: pass_slices<VK, C16, 64, MODE, ACC, NT>(a, t, sc, vsh, qacc, fscale, objacc); break;
    }
  } else {
    switch (t.lanes) {
      case 1: pass_rows<VK, C16, 1, MODE, ACC, NT, PIPE>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 2: pass_rows<VK, C16, 2, MODE, ACC, NT, PIPE>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 4: pass_rows<VK, C16, 4, MODE, ACC, NT, PIPE>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 8: pass_rows<VK, C16, 8, MODE, ACC, NT, PIPE>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 16: pass_rows<VK, C16, 16, MODE, ACC, NT, PIPE>(a, t, sc, vsh, qacc, fscale, objacc); break;
      case 32: pass_rows<VK, C16, 32, MODE, ACC, NT, PIPE>(a, t, sc, vsh, qacc, fscale, objacc); break;
      default: pass_rows<VK, C16, 64, MODE, ACC, NT, PIPE>(a, t, sc, vsh, qacc, fscale, objacc); break;
    }
  }

  if constexpr (MODE == PASS_GRAD || MODE == PASS_OBJ) {
    __shared__ double sh[NT / 64];
    double v[1] = {objacc};
    block_sum<1, NT>(v, sh);
    if (threadIdx.x == 0 && a.objpart != nullptr) a.objpart[ti] = v[0];
  } else {
    __syncthreads();
  }
  if constexpr (kScatter) {
    float* out = a.part + t.part_off;
    if constexpr (ACC == ACC_FIX64) {
      const long long* qi = static_cast<const long long*>(qacc);
      for (int j = threadIdx.x; j < n; j += NT) out[j] = static_cast<float>(static_cast<double>(qi[j]) * funscale);
    } else if constexpr (ACC == ACC_F64) {
      const double* qd = static_cast<const double*>(qacc);
      for (int j = threadIdx.x; j < n; j += NT) out[j] = static_cast<float>(qd[j]);
    } else {
      const float* qf = static_cast<const float*>(qacc);
      for (int j = threadIdx.x; j < n; j += NT) out[j] = qf[j];
    }
  }
}

int pass_smem_bytes(int nmax, int acc) {
  const int qoff = (nmax * 4 + 15) & ~15;
  return qoff + nmax * (acc == ACC_F32 ? 4 : 8);
}

template <int VK, bool C16, int MODE, int ACC, int NT, bool PIPE, int FMT>
static void launch_k(const PassArgs& a, int tile_begin, int tile_count, hipStream_t st, hipEvent_t e0,
                     hipEvent_t e1) {
  const int smem = pass_smem_bytes(a.nmax, ACC);
  auto kern = k_pass<VK, C16, MODE, ACC, NT, PIPE, FMT>;
  static bool attr_done = false;
  if (!attr_done && smem > 65536) {
    // a refusal here leaves the launch to report whether the size fits; do not
    // leave the refusal behind as the thread's last error
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            163840) != hipSuccess)
      (void)hipGetLastError();
    attr_done = true;
  }
  if (e0 != nullptr || e1 != nullptr)
    // events stamped by the dispatch itself: kernel start and / or end
    hipExtLaunchKernelGGL(kern, dim3(tile_count), dim3(NT), smem, st, e0, e1, 0, a, tile_begin);
  else
    hipLaunchKernelGGL(kern, dim3(tile_count), dim3(NT), smem, st, a, tile_begin);
}

template <int VK, bool C16, int MODE, int ACC>
static void launch_nt(const PassArgs& a, int tb, int tc, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (C16) {
    // the sliced layout exists for 16-bit column indices (set-up keeps the
    // chunk-row layout for patients with more than 65 535 spots)
    if (a.mat.fmt == FMT_SELL) {
      if (a.threads == 256)
        launch_k<VK, C16, MODE, ACC, 256, false, FMT_SELL>(a, tb, tc, st, e0, e1);
      else
        launch_k<VK, C16, MODE, ACC, 512, false, FMT_SELL>(a, tb, tc, st, e0, e1);
      return;
    }
  }
  const bool pipe = a.unroll == 2;
  if (a.threads == 256) {
    if (pipe)
      launch_k<VK, C16, MODE, ACC, 256, true, FMT_CSR>(a, tb, tc, st, e0, e1);
    else
      launch_k<VK, C16, MODE, ACC, 256, false, FMT_CSR>(a, tb, tc, st, e0, e1);
  } else {
    if (pipe)
      launch_k<VK, C16, MODE, ACC, 512, true, FMT_CSR>(a, tb, tc, st, e0, e1);
    else
      launch_k<VK, C16, MODE, ACC, 512, false, FMT_CSR>(a, tb, tc, st, e0, e1);
  }
}

template <int VK, bool C16, int MODE>
static void launch_acc(const PassArgs& a, int tb, int tc, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (MODE == PASS_OBJ || MODE == PASS_MATVEC) {
    launch_nt<VK, C16, MODE, ACC_F64>(a, tb, tc, st, e0, e1);  // no column accumulators
  } else if constexpr (MODE == PASS_RMATVEC) {
    if (a.acc == ACC_FIX64)
      launch_nt<VK, C16, MODE, ACC_FIX64>(a, tb, tc, st, e0, e1);  // scale from max |t_i| of the tile
    else
      launch_nt<VK, C16, MODE, ACC_F64>(a, tb, tc, st, e0, e1);
  } else {
    if (a.acc == ACC_FIX64)
      launch_nt<VK, C16, MODE, ACC_FIX64>(a, tb, tc, st, e0, e1);
    else if (a.acc == ACC_F32 && MODE == PASS_CG)
      launch_nt<VK, C16, MODE, ACC_F32>(a, tb, tc, st, e0, e1);
    else
      launch_nt<VK, C16, MODE, ACC_F64>(a, tb, tc, st, e0, e1);
  }
}

template <bool C16>
static void launch_mode(int mode, const PassArgs& a, int tb, int tc, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  switch (mode) {
    case PASS_GRAD: launch_acc<VAL_F32, C16, PASS_GRAD>(a, tb, tc, st, e0, e1); break;
    case PASS_OBJ: launch_acc<VAL_F32, C16, PASS_OBJ>(a, tb, tc, st, e0, e1); break;
    case PASS_MATVEC: launch_acc<VAL_F32, C16, PASS_MATVEC>(a, tb, tc, st, e0, e1); break;
    case PASS_RMATVEC: launch_acc<VAL_F32, C16, PASS_RMATVEC>(a, tb, tc, st, e0, e1); break;
    default:
      if (a.mat.vkind == VAL_BF16)
        launch_acc<VAL_BF16, C16, PASS_CG>(a, tb, tc, st, e0, e1);
      else if (a.mat.vkind == VAL_F16)
        launch_acc<VAL_F16, C16, PASS_CG>(a, tb, tc, st, e0, e1);
      else
        launch_acc<VAL_F32, C16, PASS_CG>(a, tb, tc, st, e0, e1);
  }
}

void launch_pass(int mode, const PassArgs& a, int tile_begin, int tile_count, hipStream_t st, hipEvent_t e0,
                 hipEvent_t e1) {
  if (tile_count <= 0) return;
  if (a.mat.col16)
    launch_mode<true>(mode, a, tile_begin, tile_count, st, e0, e1);
  else
    launch_mode<false>(mode, a, tile_begin, tile_count, st, e0, e1);
}

// ---------------------------------------------------------------------------
// column reduction of the tile partials, fused with the vector work that
// needs the completed column sums
// ---------------------------------------------------------------------------

// Sum of the partial column sums of tiles [0, ntiles) (tile t's partials at
// part[t * n + j]) for column j: the four waves of the block take every fourth
// tile, four loads in flight each, then wave 0 adds the four results in a
// fixed order.  Returns the total in wave 0 (lane = column offset).
__device__ __forceinline__ double tile_column_sum(const float* __restrict__ part, int ntiles, int n, int j,
                                                  double (*red)[64]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (j < n) {
    int t = w;
    for (; t + 12 < ntiles; t += 16) {
      s0 += static_cast<double>(part[static_cast<int64_t>(t) * n + j]);
      s1 += static_cast<double>(part[static_cast<int64_t>(t + 4) * n + j]);
      s2 += static_cast<double>(part[static_cast<int64_t>(t + 8) * n + j]);
      s3 += static_cast<double>(part[static_cast<int64_t>(t + 12) * n + j]);
    }
    for (; t < ntiles; t += 4) s0 += static_cast<double>(part[static_cast<int64_t>(t) * n + j]);
  }
  red[w][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  return (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

__global__ __launch_bounds__(kThreads) void k_reduce(VecArgs a, int blk_begin, int mode) {
  __shared__ double red[4][64];
  const int bi = blk_begin + static_cast<int>(blockIdx.x);
  const Blk bk = a.blk[bi];
  const int g = bk.owner;
  const Scen sc = a.scen[g];
  const Pat pt = a.pat[sc.patient];
  PatState* ps = a.ps + sc.patient;
  if (mode == RED_HEAD || mode == RED_CG) {
    if (ps->stopped) return;
    if (mode == RED_CG && !a.act[g * kRing + a.step]) return;
  }
  const int j = bk.col0 + static_cast<int>(threadIdx.x & 63);
  const float* part = a.part + a.tiles[sc.tile_begin].part_off;
  const double s = tile_column_sum(part, sc.tile_end - sc.tile_begin, sc.n, j, red);
  if (threadIdx.x >= 64) return;
  double loc[3] = {0.0, 0.0, 0.0};
  if (j < sc.n) {
    const int64_t vi = sc.vec_base + j;
    if (mode == RED_HEAD) {
      const double rho = ps->rho;
      float yv = a.y[vi];
      if (ps->pending) {
        yv = static_cast<float>(static_cast<double>(yv) + ps->tau * a.dprev[vi]);
        a.y[vi] = yv;
      }
      const float zj = a.z[pt.zvec_base + j];
      // residual of B_s x = c_s at x = z:  c_s - B_s z = -A_s^T c_s W (A_s z - p) - y_s / 2
      const float rf = static_cast<float>(-s - 0.5 * static_cast<double>(yv));
      a.r[vi] = rf;
      a.x[vi] = zj;
      float zpv = rf;
      if (a.dinv != nullptr) {
        zpv = rf * a.dinv[vi];
        a.zp[vi] = zpv;
      }
      a.v[vi] = zpv;
      const double c = static_cast<double>(a.b[vi]) + 0.5 * rho * zj - 0.5 * static_cast<double>(yv);
      loc[0] = static_cast<double>(rf) * zpv;
      loc[1] = c * c;
      loc[2] = static_cast<double>(yv) * yv;
    } else if (mode == RED_CG) {
      const float vj = a.v[vi];
      const float qj = static_cast<float>(s + 0.5 * ps->rho * vj);
      a.q[vi] = qj;
      loc[0] = static_cast<double>(vj) * qj;
    } else if (mode == RED_NORMAL) {
      a.out[j] = static_cast<float>(s + 0.5 * a.rho_out * a.v[vi]);
    } else if (mode == RED_DUALINIT) {
      // s = A_s^T c_s W (A_s z - p) = grad f_s(z) / 2
      a.y[vi] = static_cast<float>(-2.0 * s);
    } else {
      a.out[j] = static_cast<float>(s);
    }
  }
  if (mode == RED_HEAD || mode == RED_CG) {
#pragma unroll
    for (int k = 0; k < 3; ++k) loc[k] = wave_sum(loc[k]);
    if (threadIdx.x == 0) {
      double* bp = a.bpart + static_cast<int64_t>(bi) * 8;
      bp[0] = loc[0];
      bp[1] = loc[1];
      bp[2] = loc[2];
    }
  }
}

void launch_reduce(int mode, const VecArgs& a, int blk_begin, int nblk, hipStream_t st) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(k_reduce, dim3(nblk), dim3(kThreads), 0, st, a, blk_begin, mode);
}

// ---------------------------------------------------------------------------
// head scalars: objective at z, completion of the previous iteration
// (dual-update norm, trace record, stopping test) and CG set-up
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_head_scalars(VecArgs a, int nscen, int cg_setup) {
  head_scalars_run<false>(a, nscen, cg_setup);
}

void launch_head_scalars(const VecArgs& a, int nscen, int cg_setup, hipStream_t st) {
  hipLaunchKernelGGL(k_head_scalars, dim3(1), dim3(kThreads), 0, st, a, nscen, cg_setup);
}

// ---------------------------------------------------------------------------
// CG vector steps
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kColBlock) void k_cg_update(VecArgs a) {
  const int bi = static_cast<int>(blockIdx.x);
  const Blk bk = a.blk[bi];
  const int g = bk.owner;
  const Scen sc = a.scen[g];
  if (!a.act[g * kRing + a.step]) return;
  const double vq = wave_strided_sum(a.bpart + static_cast<int64_t>(sc.blk_begin) * 8 + 0, sc.nblk);
  const double rz = a.rz[g * kRing + a.step];
  const float alpha = (vq > 0.0) ? static_cast<float>(rz / vq) : 0.0f;
  const int j = bk.col0 + static_cast<int>(threadIdx.x);
  double loc[1] = {0.0};
  if (j < sc.n) {
    const int64_t vi = sc.vec_base + j;
    const float vj = a.v[vi];
    a.x[vi] = fmaf(alpha, vj, a.x[vi]);
    const float rj = fmaf(-alpha, a.q[vi], a.r[vi]);
    a.r[vi] = rj;
    float zpv = rj;
    if (a.dinv != nullptr) {
      zpv = rj * a.dinv[vi];
      a.zp[vi] = zpv;
    }
    loc[0] = static_cast<double>(rj) * zpv;
  }
  loc[0] = wave_sum(loc[0]);
  if (threadIdx.x == 0) a.bpart[(int64_t)bi * 8 + 3] = loc[0];
}

__global__ __launch_bounds__(kColBlock) void k_cg_dir(VecArgs a) {
  const int bi = static_cast<int>(blockIdx.x);
  const Blk bk = a.blk[bi];
  const int g = bk.owner;
  const Scen sc = a.scen[g];
  const int k = a.step;
  if (!a.act[g * kRing + k]) {
    if (threadIdx.x == 0) a.act[g * kRing + k + 1] = 0;
    return;
  }
  const double rz1 = wave_strided_sum(a.bpart + static_cast<int64_t>(sc.blk_begin) * 8 + 3, sc.nblk);
  const double rz0 = a.rz[g * kRing + k];
  const float beta = (rz0 > 0.0) ? static_cast<float>(rz1 / rz0) : 0.0f;
  const int j = bk.col0 + static_cast<int>(threadIdx.x);
  if (j < sc.n) {
    const int64_t vi = sc.vec_base + j;
    const float zpv = (a.dinv != nullptr) ? a.zp[vi] : a.r[vi];
    a.v[vi] = fmaf(beta, a.v[vi], zpv);
  }
  if (threadIdx.x == 0) {
    // every block of the scenario writes the same values
    a.rz[g * kRing + k + 1] = rz1;
    a.act[g * kRing + k + 1] = (rz1 > a.tol2[g] && rz1 > 0.0) ? 1 : 0;
    if (bk.col0 == 0) {
      a.cgcount[g] += 1;
      a.cgtotal[g] += 1;
    }
  }
}

void launch_cg_update(const VecArgs& a, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_update, dim3(nblk), dim3(kColBlock), 0, st, a);
}
void launch_cg_dir(const VecArgs& a, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_dir, dim3(nblk), dim3(kColBlock), 0, st, a);
}

// ---------------------------------------------------------------------------
// z-update and residual / BB partial sums, one patient column block per
// workgroup (every quantity is columnwise until the final sums)
// ---------------------------------------------------------------------------

// One workgroup per 16 columns of a patient block: thread (g, c) = (tid / 16,
// tid % 16) takes column c and the scenarios s = g, g + 16, ... (one each for
// N <= 16), so every load of x, y and d_prev is independent of the others.
// Partial sums over scenarios and columns are combined in a fixed order, so
// the result does not depend on timing.  Partials: bpartp[(4 * pblk + sub) * 8 + k].
constexpr int kZCols = 16;
__global__ __launch_bounds__(kThreads) void k_zres(VecArgs a) {
  __shared__ double sacc[kThreads / kZCols][kZCols];
  __shared__ float zsh[kZCols];
  __shared__ double sred[4][8];
  const int bi4 = static_cast<int>(blockIdx.x);
  const Blk bk = a.pblk[bi4 >> 2];
  const int p = bk.owner;
  const Pat pt = a.pat[p];
  const PatState* ps = a.ps + p;
  const int stopped = ps->stopped;  // read beside the loads below; checked before any write
  const double rho = ps->rho;
  const int tid = threadIdx.x;
  const int col = tid % kZCols, grp = tid / kZCols;
  constexpr int kGroups = kThreads / kZCols;
  const int j = bk.col0 + (bi4 & 3) * kZCols + col;
  const bool valid = j < pt.n && (bi4 & 3) * kZCols + col < kColBlock;
  double acc = 0.0;
  if (valid)
    for (int s = grp; s < pt.num_scen; s += kGroups) {
      const int64_t vi = pt.vec_base + static_cast<int64_t>(s) * pt.n + j;
      acc += static_cast<double>(a.x[vi]);
      if (a.prm.z_mode == 0) acc += static_cast<double>(a.y[vi]) / rho;
    }
  if (stopped) return;  // the whole workgroup: one patient
  sacc[grp][col] = acc;
  __syncthreads();
  // ||dz||^2, ||z||^2, ||d||^2, <dd,d_prev>, ||dd||^2, ||x||^2, <y,d>, ||y||^2
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (grp == 0) {
    float znf = 0.0f;
    if (valid) {
      double sum = 0.0;
      for (int g = 0; g < kGroups; ++g) sum += sacc[g][col];
      const int64_t zi = pt.zvec_base + j;
      double zn = sum / pt.num_scen;
      zn = fmin(fmax(zn, static_cast<double>(a.lb[zi])), static_cast<double>(a.ub[zi]));
      znf = static_cast<float>(zn);
      const double dz = static_cast<double>(znf) - static_cast<double>(a.z[zi]);
      a.z[zi] = znf;
      v[0] = dz * dz;
      v[1] = static_cast<double>(znf) * znf;
    }
    zsh[col] = znf;
  }
  __syncthreads();
  if (valid) {
    const double znd = static_cast<double>(zsh[col]);
    for (int s = grp; s < pt.num_scen; s += kGroups) {
      const int64_t vi = pt.vec_base + static_cast<int64_t>(s) * pt.n + j;
      const double xv = static_cast<double>(a.x[vi]);
      const double yv = static_cast<double>(a.y[vi]);
      const double d = xv - znd;
      const double dp = a.dprev[vi];
      const double dd = d - dp;
      v[2] += d * d;
      v[3] += dd * dp;
      v[4] += dd * dd;
      v[5] += xv * xv;
      v[6] += yv * d;
      v[7] += yv * yv;
      a.dprev[vi] = d;
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = wave_sum(v[k]);
  if ((tid & 63) == 0)
    for (int k = 0; k < 8; ++k) sred[tid >> 6][k] = v[k];
  __syncthreads();
  if (tid == 0) {
    double* bp = a.bpartp + static_cast<int64_t>(bi4) * 8;
    for (int k = 0; k < 8; ++k) bp[k] = (sred[0][k] + sred[1][k]) + (sred[2][k] + sred[3][k]);
  }
}

void launch_zres(const VecArgs& a, int npblk, hipStream_t st) {
  hipLaunchKernelGGL(k_zres, dim3(4 * npblk), dim3(kThreads), 0, st, a);
}

// Residual norms, tolerances and the Barzilai-Borwein dual step per patient.
__global__ __launch_bounds__(kThreads) void k_body_scalars(VecArgs a) { body_scalars_run<false>(a); }

void launch_body_scalars(const VecArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_body_scalars, dim3(1), dim3(kThreads), 0, st, a);
}

// ---------------------------------------------------------------------------
// small helpers: cross-scenario gradient sum, objective sum, PGD trial step
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_gsum(const Scen* scen, const Pat* pat, const Blk* pblk,
                                                   const Tile* tiles, const float* part, int blk_begin,
                                                   float scale, float* out) {
  __shared__ double red[4][64];
  const Blk bk = pblk[blk_begin + blockIdx.x];
  const Pat pt = pat[bk.owner];
  const int j = bk.col0 + static_cast<int>(threadIdx.x & 63);
  const double s = tile_column_sum(part + tiles[pt.tile_begin].part_off, pt.tile_end - pt.tile_begin, pt.n, j, red);
  if (threadIdx.x < 64 && j < pt.n) out[j] = static_cast<float>(scale * s);
}

void launch_gsum(const Scen* scen, const Pat* pat, const Blk* pblk, const Tile* tiles, const float* part,
                 int patient_blk_begin, int nblk, float scale, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gsum, dim3(nblk), dim3(kThreads), 0, st, scen, pat, pblk, tiles, part, patient_blk_begin,
                     scale, out);
}

__global__ __launch_bounds__(kThreads) void k_objsum(const double* objpart, int tile_begin, int count, double* out) {
  __shared__ double sh[4];
  const double f = block_list_sum(count, [&](int i) { return objpart[tile_begin + i]; }, sh);
  if (threadIdx.x == 0) *out = f;
}

void launch_objsum(const Tile*, const double* objpart, int tile_begin, int tile_count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_objsum, dim3(1), dim3(kThreads), 0, st, objpart, tile_begin, tile_count, out);
}

__global__ __launch_bounds__(kThreads) void k_pgd_trial(const float* x, const float* g, const float* lb,
                                                        const float* ub, float t, float* xt, int n,
                                                        double* dotpart) {
  __shared__ double sh[4];
  const int j = blockIdx.x * kThreads + threadIdx.x;
  double loc[1] = {0.0};
  if (j < n) {
    const float v = fminf(fmaxf(x[j] - t * g[j], lb[j]), ub[j]);
    xt[j] = v;
    loc[0] = static_cast<double>(g[j]) * (static_cast<double>(v) - static_cast<double>(x[j]));
  }
  block_sum<1>(loc, sh);
  if (threadIdx.x == 0) dotpart[blockIdx.x] = loc[0];
}

void launch_pgd_trial(const float* x, const float* g, const float* lb, const float* ub, float t, float* xt, int n,
                      double* dotpart, hipStream_t st) {
  const int nb = (n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_pgd_trial, dim3(nb), dim3(kThreads), 0, st, x, g, lb, ub, t, xt, n, dotpart);
}

__global__ __launch_bounds__(kThreads) void k_dot_sum(const double* part, int count, double* out) {
  __shared__ double sh[4];
  const double f = block_list_sum(count, [&](int i) { return part[i]; }, sh);
  if (threadIdx.x == 0) *out = f;
}

void launch_dot_sum(const double* part, int count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_sum, dim3(1), dim3(kThreads), 0, st, part, count, out);
}

template <class T>
__global__ void k_fill(T* p, T v, int64_t count) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

template <class T>
static void fill(T* p, T v, int64_t count, hipStream_t st) {
  if (count <= 0) return;
  int64_t nb = (count + kThreads - 1) / kThreads;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill<T>, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, st, p, v, count);
}

void launch_fill_f32(float* p, float v, int64_t count, hipStream_t st) { fill<float>(p, v, count, st); }
void launch_fill_f64(double* p, double v, int64_t count, hipStream_t st) { fill<double>(p, v, count, st); }
void launch_fill_u8(uint8_t* p, uint8_t v, int64_t count, hipStream_t st) { fill<uint8_t>(p, v, count, st); }

}  // namespace admmbb
