// The fused sparse pass (k_pass) and its launch templates, instantiated by
// the pass_*.hip translation units (one per group of value types and modes, so
// that they compile in parallel).
//
// k_pass is one streaming pass over the length-sorted CSR of every (patient,
// scenario) dose-influence matrix A_s.  For each row i it forms the row dot
// a_i . v, turns it into t_i (c_s w_i a_i.v for a CG product, c_s w_i (a_i.v -
// p_i) for the gradient / objective), and immediately scatters t_i a_i into
// column accumulators held in LDS.  The row's values and column indices stay in
// registers between the two uses, so each nonzero is read from HBM once per
// operator application A_s^T diag(c_s w) A_s v (the x-update system of
// Appendix A without its rho/2 shift).  Each workgroup writes its column
// partial sums; a column-blocked reduction kernel adds them in a fixed order.
#pragma once
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
  // transpose product: the row's t_i, two dependent loads with nothing to
  // hide them before the scatter needs it, is requested one row ahead and
  // its original index two rows ahead
  float tin_cur = 0.0f;
  int32_t ro_next = 0;
  if constexpr (MODE == PASS_RMATVEC) {
    tin_cur = r < rend ? a.tin[a.mat.rorig[rb + r]] : 0.0f;
    ro_next = r + G < rend ? a.mat.rorig[rb + r + G] : 0;
  }
  float vv[K][4];
  CCk cc[K];
  if constexpr (PIPE) load_row(s, e, vv, cc);
  for (; r < rend; r += G) {
    if constexpr (!PIPE) load_row(s, e, vv, cc);
    float rw;
    float aux = 0.0f;
    if constexpr (MODE == PASS_RMATVEC) {
      rw = tin_cur;
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
    if constexpr (MODE == PASS_RMATVEC) {
      tin_cur = rn < rend ? a.tin[ro_next] : 0.0f;
      ro_next = rn + G < rend ? a.mat.rorig[rb + rn + G] : 0;
    }
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
      dot = group_allsum<L>(dot);
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
      dot = group_allsum<L>(dot);
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
  static_assert(NT >= kAbsMaxBlocks, "one thread per partial maximum of |t|");
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
    // the given t bounds the contributions: max |t_i| over the whole vector,
    // formed beforehand, or over the tile's rows
    if (a.tmax != nullptr) {
      if (threadIdx.x < kAbsMaxBlocks) vmax = a.tmax[threadIdx.x];
    } else {
      const int rb0 = static_cast<int>(sc.row_base);
      for (int r = t.row_begin + static_cast<int>(threadIdx.x); r < t.row_end; r += NT)
        vmax = fmaxf(vmax, fabsf(a.tin[a.mat.rorig[rb0 + r]]));
    }
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


template <int VK, bool C16, int MODE, int ACC, int NT, bool PIPE, int FMT>
static void launch_k(const PassArgs& a, int tile_begin, int tile_count, hipStream_t st, hipEvent_t e0,
                     hipEvent_t e1) {
  // passes without a scatter need the multiplied vector only, no column accumulators
  constexpr bool kScatter = MODE == PASS_GRAD || MODE == PASS_CG || MODE == PASS_RMATVEC;
  const int smem = kScatter ? pass_smem_bytes(a.nmax, ACC) : ((a.nmax * 4 + 15) & ~15);
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
  if (a.threads == 1024) {
    // patients whose column accumulators leave room for one workgroup per CU
    if (pipe)
      launch_k<VK, C16, MODE, ACC, 1024, true, FMT_CSR>(a, tb, tc, st, e0, e1);
    else
      launch_k<VK, C16, MODE, ACC, 1024, false, FMT_CSR>(a, tb, tc, st, e0, e1);
  } else if (a.threads == 256) {
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

}  // namespace admmbb
