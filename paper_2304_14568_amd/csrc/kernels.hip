// gfx950 kernels for ADMM-BB robust planning: the launch of the fused sparse
// pass (pass.h, instantiated by the pass_*.hip units), the column reduction of
// its partial sums with the CG vector steps, the z-update with the residual
// and Barzilai-Borwein partial sums, and small helpers.  All scalar reductions
// are float64 and deterministic (fixed trees).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "internal.h"
#include "scalars.h"

namespace admmbb {

void launch_pass_f32_io(int mode, const PassArgs& a, int tile_begin, int tile_count, hipStream_t st, hipEvent_t e0,
                        hipEvent_t e1);
void launch_pass_cg_f32(int mode, const PassArgs& a, int tile_begin, int tile_count, hipStream_t st, hipEvent_t e0,
                        hipEvent_t e1);
void launch_pass_cg_lp(int mode, const PassArgs& a, int tile_begin, int tile_count, hipStream_t st, hipEvent_t e0,
                       hipEvent_t e1);

int pass_smem_bytes(int nmax, int acc) {
  const int qoff = (nmax * 4 + 15) & ~15;
  return qoff + nmax * (acc == ACC_F32 ? 4 : 8);
}

void launch_pass(int mode, const PassArgs& a, int tile_begin, int tile_count, hipStream_t st, hipEvent_t e0,
                 hipEvent_t e1) {
  if (tile_count <= 0) return;
  if (mode != PASS_CG)
    launch_pass_f32_io(mode, a, tile_begin, tile_count, st, e0, e1);
  else if (a.mat.vkind == VAL_BF16 || a.mat.vkind == VAL_F16)
    launch_pass_cg_lp(mode, a, tile_begin, tile_count, st, e0, e1);
  else
    launch_pass_cg_f32(mode, a, tile_begin, tile_count, st, e0, e1);
}

// ---------------------------------------------------------------------------
// column reduction of the tile partials, fused with the vector work that
// needs the completed column sums
// ---------------------------------------------------------------------------

// Sum of the partial column sums of tiles [0, ntiles) (tile t's partials at
// part[t * n + j]) for column j: the NW waves of the block take every NW-th
// tile, four loads in flight each, then wave 0 adds the NW results pairwise
// in a fixed order.  Returns the total in wave 0 (lane = column offset).
template <int NW>
__device__ __forceinline__ double tile_column_sum(const float* __restrict__ part, int ntiles, int n, int j,
                                                  double (*red)[64]) {
  static_assert(NW == 4 || NW == 16, "pairwise tree over 4 or 16 waves");
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (j < n) {
    int t = w;
    for (; t + 3 * NW < ntiles; t += 4 * NW) {
      s0 += static_cast<double>(part[static_cast<int64_t>(t) * n + j]);
      s1 += static_cast<double>(part[static_cast<int64_t>(t + NW) * n + j]);
      s2 += static_cast<double>(part[static_cast<int64_t>(t + 2 * NW) * n + j]);
      s3 += static_cast<double>(part[static_cast<int64_t>(t + 3 * NW) * n + j]);
    }
    for (; t < ntiles; t += NW) s0 += static_cast<double>(part[static_cast<int64_t>(t) * n + j]);
  }
  red[w][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  auto q4 = [&](int b) { return (red[b][lane] + red[b + 1][lane]) + (red[b + 2][lane] + red[b + 3][lane]); };
  if constexpr (NW == 4) return q4(0);
  else return (q4(0) + q4(4)) + (q4(8) + q4(12));
}

constexpr int kRedWaves = 16;  // waves per column block of k_reduce

// One workgroup of kRedWaves waves per scenario column block; every address
// comes from the block's job entry, and the partial sums are requested
// before the skip test (a skipped block's partials are read and discarded).
__global__ __launch_bounds__(64 * kRedWaves) void k_reduce(VecArgs a, int blk_begin, int mode) {
  __shared__ double red[kRedWaves][64];
  const int bi = blk_begin + static_cast<int>(blockIdx.x);
  const ColJob cj = a.cjobs[bi];
  PatState* ps = a.ps + cj.patient;
  bool skip = false;
  if (mode == RED_HEAD || mode == RED_CG) {
    skip = ps->stopped != 0;
    if (mode == RED_CG) skip = skip || !a.act[cj.scen * kRing + a.step];
  }
  const int j = cj.col0 + static_cast<int>(threadIdx.x & 63);
  const double s = tile_column_sum<kRedWaves>(a.part + cj.part_off, cj.ntiles, cj.n, j, red);
  if (skip || threadIdx.x >= 64) return;
  double loc[3] = {0.0, 0.0, 0.0};
  if (j < cj.n) {
    const int64_t vi = cj.vec_base + j;
    if (mode == RED_HEAD) {
      const double rho = ps->rho;
      float yv = a.y[vi];
      if (ps->pending) {
        yv = static_cast<float>(static_cast<double>(yv) + ps->tau * a.dprev[vi]);
        a.y[vi] = yv;
      }
      const float zj = a.z[cj.zvec_base + j];
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
  hipLaunchKernelGGL(k_reduce, dim3(nblk), dim3(64 * kRedWaves), 0, st, a, blk_begin, mode);
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

// One workgroup per 16 columns of a patient block (addresses from the block's
// job entry): thread (g, c) = (tid / 16, tid % 16) takes column c and the
// scenarios s = g, g + 16, ... (one each for N <= 16), so every load of x, y
// and d_prev is independent of the others.
// Partial sums over scenarios and columns are combined in a fixed order, so
// the result does not depend on timing.  Partials: bpartp[(4 * pblk + sub) * 8 + k].
constexpr int kZCols = 16;
__global__ __launch_bounds__(kThreads) void k_zres(VecArgs a) {
  __shared__ double sacc[kThreads / kZCols][kZCols];
  __shared__ float zsh[kZCols];
  __shared__ double sred[4][8];
  const int bi4 = static_cast<int>(blockIdx.x);
  const ZJob pt = a.zjobs[bi4 >> 2];
  const PatState* ps = a.ps + pt.patient;
  const int stopped = ps->stopped;  // read beside the loads below; checked before any write
  const double rho = ps->rho;
  const int tid = threadIdx.x;
  const int col = tid % kZCols, grp = tid / kZCols;
  constexpr int kGroups = kThreads / kZCols;
  const int j = pt.col0 + (bi4 & 3) * kZCols + col;
  const bool valid = j < pt.n && (bi4 & 3) * kZCols + col < kColBlock;
  // every input of the thread's first scenario (s = grp) and of the
  // projection, requested at once
  const bool first = valid && grp < pt.N;
  const int64_t vi0 = pt.vec_base + static_cast<int64_t>(grp) * pt.n + j;
  const int64_t zi = pt.zvec_base + j;
  float x0 = 0.0f, y0 = 0.0f, lbv = 0.0f, ubv = 0.0f, zold = 0.0f;
  double dp0 = 0.0;
  if (first) {
    x0 = a.x[vi0];
    y0 = a.y[vi0];
    dp0 = a.dprev[vi0];
  }
  if (valid && grp == 0) {
    lbv = a.lb[zi];
    ubv = a.ub[zi];
    zold = a.z[zi];
  }
  double acc = 0.0;
  if (valid)
    for (int s = grp; s < pt.N; s += kGroups) {
      const int64_t vi = pt.vec_base + static_cast<int64_t>(s) * pt.n + j;
      acc += static_cast<double>(s == grp ? x0 : a.x[vi]);
      if (a.prm.z_mode == 0) acc += static_cast<double>(s == grp ? y0 : a.y[vi]) / rho;
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
      double zn = sum / pt.N;
      zn = fmin(fmax(zn, static_cast<double>(lbv)), static_cast<double>(ubv));
      znf = static_cast<float>(zn);
      const double dz = static_cast<double>(znf) - static_cast<double>(zold);
      a.z[zi] = znf;
      v[0] = dz * dz;
      v[1] = static_cast<double>(znf) * znf;
    }
    zsh[col] = znf;
  }
  __syncthreads();
  if (valid) {
    const double znd = static_cast<double>(zsh[col]);
    for (int s = grp; s < pt.N; s += kGroups) {
      const int64_t vi = pt.vec_base + static_cast<int64_t>(s) * pt.n + j;
      const double xv = static_cast<double>(s == grp ? x0 : a.x[vi]);
      const double yv = static_cast<double>(s == grp ? y0 : a.y[vi]);
      const double d = xv - znd;
      const double dp = s == grp ? dp0 : a.dprev[vi];
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
  const double s = tile_column_sum<4>(part + tiles[pt.tile_begin].part_off, pt.tile_end - pt.tile_begin, pt.n, j, red);
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

__global__ __launch_bounds__(256) void k_absmax(const float* __restrict__ x, int64_t n, float* __restrict__ out) {
  __shared__ float wm[4];
  // four loads in flight per thread
  constexpr int64_t S = int64_t{kAbsMaxBlocks} * 256;
  float v = 0.0f;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += 4 * S) {
    float q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = i + u * S < n ? x[i + u * S] : 0.0f;
#pragma unroll
    for (int u = 0; u < 4; ++u) v = fmaxf(v, fabsf(q[u]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
}

void launch_absmax(const float* x, int64_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_absmax, dim3(kAbsMaxBlocks), dim3(256), 0, st, x, n, out);
}

void launch_fill_f32(float* p, float v, int64_t count, hipStream_t st) { fill<float>(p, v, count, st); }
void launch_fill_f64(double* p, double v, int64_t count, hipStream_t st) { fill<double>(p, v, count, st); }
void launch_fill_u8(uint8_t* p, uint8_t v, int64_t count, hipStream_t st) { fill<uint8_t>(p, v, count, st); }

}  // namespace admmbb
