// Projected gradient descent with Armijo backtracking (Sec. 2.1) on the cached
// dense Gram sum of the dense x-update, driven on the device.
//
// With S = sum_s G_s (packed upper 64 x 64 tiles, fp64) the objective and its
// gradient are f(x) = x^T S x - g0^T x + const and grad f(x) = 2 S x - g0.
// One round evaluates kPgdK backtracking steps at once:
//   k_pgd_tiles   for every tile T of S and every k: T x_k,J and T^T x_k,I,
//                 one read of S for all kPgdK trial points
//   k_pgd_rows    u_k = S x_k from the tile products, and f(x_k) partial sums
//   k_pgd_step    the first k (largest step) with
//                 f(x_k) <= f(x) + beta g^T (x_k - x) is accepted (stopping
//                 tests), x = x_k with gradient 2 u_k - g0, and the next round's
//                 trial points x_k = P(x - t_k g), t_k = t_base gamma^k
// so an iteration whose step is found within kPgdK trials reads S once.
// A round that accepts nothing retries from the same x with the next kPgdK
// steps.  The host launches rounds in chunks and reads the state in between.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace admmbb {

namespace {

constexpr int kT = 64;  // tile size

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t ptile(int I, int J, int nb) {
  return static_cast<int64_t>(I) * nb - static_cast<int64_t>(I) * (I - 1) / 2 + (J - I);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The step of a round (one thread per spot, every workgroup taking the same
// decision from the same sums in the same order):
//   decision  from f(x_k) (tile sums) and g^T (x_k - x) of this round's trial
//             points: the first k (largest step) with sufficient decrease is
//             accepted, else the next kPgdK steps are tried from the same x;
//             stopping tests; workgroup 0 writes the next state
//   apply     x = x_p, grad f(x) = 2 u_p - g0
//   propose   the next trial points x_k = P(x - t_k g), t_k = t_base gamma^k, and
//             the partial sums of g^T (x_k - x) (next buffer)
// State and partial sums are double-buffered by the round's parity: this
// launch reads slot par and writes slot par ^ 1.  mode 0: a round; 1: the first
// round (every trial point is x: record f(x), take its gradient); 2: prime
// (no decision: propose trial points at t_base from x and g).
__global__ __launch_bounds__(256) void k_pgd_step(PgdArgs a, int mode, int par) {
  __shared__ double red[4][kPgdK];
  __shared__ double fk[kPgdK], gd[kPgdK];
  const PgdDevState cur = a.st[par];
  PgdDevState nxt = cur;
  const int tid = threadIdx.x;
  const int j = static_cast<int>(blockIdx.x) * 256 + tid;
  const bool in = j < a.n;
  const double* gdin = a.gdpart + static_cast<int64_t>(par) * kPgdK * a.nblocks;
  double* gdout = a.gdpart + static_cast<int64_t>(par ^ 1) * kPgdK * a.nblocks;
  // loads that do not depend on the decision go out first
  double xj = in ? a.x[j] : 0.0, gj = in ? a.g[j] : 0.0;
  const double g0j = in ? a.g0[j] : 0.0;
  const double lo = in ? a.lb[j] : 0.0, hi = in ? a.ub[j] : 0.0;
  int p = -1;
  if (!cur.done && mode != 2) {
    // f(x_k) and g^T (x_k - x): wave w sums k = w and w + 4, fixed order
    const int w = tid >> 6, lane = tid & 63;
    for (int k = w; k < kPgdK; k += 4) {
      double fs = 0.0, ds = 0.0;
      for (int b = lane; b < a.nb; b += 64) fs += a.fpart[static_cast<int64_t>(k) * a.nb + b];
      for (int b = lane; b < a.nblocks; b += 64) ds += gdin[static_cast<int64_t>(k) * a.nblocks + b];
      fs = wsum(fs);
      ds = wsum(ds);
      if (lane == 0) {
        fk[k] = a.fconst + fs;
        gd[k] = ds;
      }
    }
    __syncthreads();
    bool stop = false;
    if (mode == 1) {
      p = 0;
      nxt.f = fk[0];
      nxt.t_base = cur.alpha;
      if (a.max_iter <= 0) {
        stop = true;
        nxt.status = 3;
      }
    } else {
      for (int kk = 0; kk < kPgdK; ++kk)
        if (cur.trials + kk < a.max_trials && fk[kk] <= cur.f + a.beta * gd[kk]) {
          p = kk;
          break;
        }
      if (p >= 0) {
        nxt.f = fk[p];
        nxt.iter = cur.iter + 1;
        nxt.trials = 0;
        nxt.t_base = cur.alpha;
        if (fabs(cur.f - fk[p]) <= a.tol * fabs(cur.f)) {
          stop = true;
          nxt.status = 1;
        } else if (nxt.iter >= a.max_iter) {
          stop = true;
          nxt.status = 3;
        }
      } else {
        nxt.trials = cur.trials + kPgdK;
        double t = cur.t_base;
        for (int kk = 0; kk < kPgdK; ++kk) t *= a.gamma;
        nxt.t_base = t;
        if (nxt.trials >= a.max_trials) {
          stop = true;
          nxt.status = 2;
        }
      }
    }
    if (stop) nxt.done = 1;
  }
  nxt.pick = p;
  if (blockIdx.x == 0 && tid == 0) a.st[par ^ 1] = nxt;
  if (in && p >= 0) {
    xj = a.xc[static_cast<int64_t>(p) * a.np + j];
    gj = 2.0 * a.u[static_cast<int64_t>(p) * a.np + j] - g0j;
    a.x[j] = xj;
    a.g[j] = gj;
  }
  if (nxt.done) return;
  double loc[kPgdK];
  if (in) {
    double t = nxt.t_base;
#pragma unroll
    for (int k = 0; k < kPgdK; ++k) {
      const double v = fmin(fmax(xj - t * gj, lo), hi);
      a.xc[static_cast<int64_t>(k) * a.np + j] = v;
      loc[k] = gj * (v - xj);
      t *= a.gamma;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kPgdK; ++k) {
      if (j < a.np) a.xc[static_cast<int64_t>(k) * a.np + j] = 0.0;
      loc[k] = 0.0;
    }
  }
#pragma unroll
  for (int k = 0; k < kPgdK; ++k) {
    const double sum = wsum(loc[k]);
    if ((tid & 63) == 0) red[tid >> 6][k] = sum;
  }
  __syncthreads();
  if (tid < kPgdK)
    gdout[static_cast<int64_t>(tid) * a.nblocks + blockIdx.x] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// One tile T = S_IJ (I <= J) per workgroup, staged once through LDS (32 KB,
// five workgroups per CU) with coalesced 16-byte loads; element (r, c) sits at
// r * 64 + (c ^ sw(r)), an even swizzle that keeps column pairs together and
// spreads both read patterns below over distinct banks.
// Wave w takes rows 16w..16w+15 of T for T v_k,J and columns 16w..16w+15 for
// T^T v_k,I, both as products (16 x 64 trial-point rows, zero beyond KC) x
// (64 x 16 slice of T) on the fp64 16x16x4 MFMA: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16] of each step and receives D[l / 16 + 4 r][l % 16] in
// item r.  The k index of the 16 steps is a free permutation of the 64 tile
// columns (rows), chosen so that every lane reads contiguous doubles of the
// trial points.  v_k = v + k * vstride, vstride and the vectors padded with
// zeros to whole 64-blocks.
// part[(t * KC + k) * 128 + i]      = (T v_k,J)_i
// part[(t * KC + k) * 128 + 64 + i] = (T^T v_k,I)_i   (off-diagonal tiles)
__device__ __forceinline__ int sw(int r) { return ((2 * r) & 30) ^ (r & 16); }

template <int KC>
__global__ __launch_bounds__(256) void k_pgd_tiles(PgdArgs a, const double* __restrict__ v, int64_t vstride,
                                                   int par) {
  __shared__ double tl[kT * kT];
  const int64_t t = blockIdx.x;  // jobs are the tiles in packed order
  const int tid = threadIdx.x;
  {
    // the tile's loads go out first (in bounds whatever the state), so their
    // latency overlaps that of the state and job reads
    const double2* T = reinterpret_cast<const double2*>(a.Gp + t * kT * kT);
    double2 g[8];
#pragma unroll
    for (int it = 0; it < 8; ++it) g[it] = T[it * 256 + tid];
    if (a.st[par].done) return;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int e = 2 * (it * 256 + tid), r = e / kT, c = e % kT;
      *reinterpret_cast<double2*>(&tl[r * kT + (c ^ sw(r))]) = g[it];
    }
  }
  const XJob job = a.jobs[blockIdx.x];
  const int I = job.ij >> 16, J = job.ij & 0xffff;
  const int lane = tid & 63, w = tid >> 6;
  const int m = lane & 15, kk = lane >> 4;
  const bool live = m < KC;
  double* out = a.part + t * (KC * 2 * kT);
  // trial-point operands (global, cached): columns of block J, rows of block I
  double2 vaJ[8], vaI[8];
  {
    const double2* vJ = reinterpret_cast<const double2*>(v + m * vstride + J * kT + 2 * kk);
    const double2* vI = reinterpret_cast<const double2*>(v + m * vstride + I * kT + 16 * kk);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      vaJ[s] = live ? vJ[4 * s] : make_double2(0.0, 0.0);
      vaI[s] = live ? vI[s] : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  // T v_J: step (s, h) uses tile column 8 s + 2 kk + h
  {
    const int r = 16 * w + m;
    const double* Tr = &tl[r * kT];
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const double2 b = *reinterpret_cast<const double2*>(Tr + ((8 * s + 2 * kk) ^ sw(r)));
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vaJ[s].x, b.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vaJ[s].y, b.y, acc, 0, 0, 0);
    }
    // item r: trial point kk + 4 r, tile row 16 w + m
#pragma unroll
    for (int r = 0; r < 2; ++r)
      if (kk + 4 * r < KC) out[(kk + 4 * r) * 2 * kT + 16 * w + m] = acc[r];
  }
  if (I == J) return;
  // T^T v_I: step s uses tile row 16 kk + s
  {
    const int c = 16 * w + m;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int r0 = 16 * kk + 2 * s, r1 = r0 + 1;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vaI[s].x, tl[r0 * kT + (c ^ sw(r0))], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vaI[s].y, tl[r1 * kT + (c ^ sw(r1))], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
      if (kk + 4 * r < KC) out[(kk + 4 * r) * 2 * kT + kT + 16 * w + m] = acc[r];
  }
}

// Block row I of u_k = S v_k (workgroup (I, k)) from the tile products, and
// fpart[k * nb + I] = sum over the block's rows of v_k (u_k - g0).
// Four waves take every fourth tile of the block row; fixed summation order.
template <int KC>
__global__ __launch_bounds__(256) void k_pgd_rows(PgdArgs a, const double* __restrict__ v, int64_t vstride,
                                                  int par) {
  __shared__ double red[4][kT];
  const int I = static_cast<int>(blockIdx.x), k = static_cast<int>(blockIdx.y);
  const int i = threadIdx.x & 63, w = threadIdx.x >> 6;
  // four independent loads in flight per lane, then a fixed-order sum
  double s = 0.0;
  for (int J0 = w; J0 < a.nb; J0 += 16) {
    double e[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int J = J0 + 4 * q;
      const int64_t t = J < I ? ptile(J, I, a.nb) : ptile(I, J, a.nb);
      e[q] = J < a.nb ? a.part[(t * KC + k) * (2 * kT) + (J < I ? kT : 0) + i] : 0.0;
    }
    s += (e[0] + e[1]) + (e[2] + e[3]);
  }
  if (a.st[par].done) return;  // checked after the (in-bounds) loads are under way
  red[w][i] = s;
  __syncthreads();
  if (w != 0) return;
  s = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
  const int row = I * kT + i;
  double d = 0.0;
  if (row < a.n) {
    a.u[static_cast<int64_t>(k) * a.np + row] = s;
    d = v[k * vstride + row] * (s - a.g0[row]);
  }
  d = wsum(d);
  if (i == 0) a.fpart[static_cast<int64_t>(k) * a.nb + I] = d;
}

// Power iteration step: v = u / ||u|| with u = 2 S v_old (rows of u[0]),
// alpha = 10 / ||u|| (1 when u = 0).
__global__ __launch_bounds__(1024) void k_pgd_normalize(PgdArgs a, double* __restrict__ v) {
  __shared__ double red[16];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int j = tid; j < a.n; j += 1024) {
    const double e = 2.0 * a.u[j];
    s = fma(e, e, s);
  }
  s = wsum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double tot = 0.0;
#pragma unroll
  for (int w = 0; w < 16; ++w) tot += red[w];
  const double nrm = sqrt(tot);
  if (!(nrm > 0)) {
    if (tid == 0) a.st[0].alpha = 1.0;
    return;
  }
  for (int j = tid; j < a.n; j += 1024) v[j] = 2.0 * a.u[j] / nrm;
  if (tid == 0) a.st[0].alpha = 10.0 / nrm;
}

}  // namespace

// One power-iteration step on H = 2 S; v is replaced by the next unit vector.
// Slot 0 of the state must have done = 0.
void launch_pgd_power(const PgdArgs& a, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_pgd_tiles<1>, dim3(a.njobs), dim3(256), 0, st, a, static_cast<const double*>(v),
                     int64_t{0}, 0);
  hipLaunchKernelGGL(k_pgd_rows<1>, dim3(a.nb, 1), dim3(256), 0, st, a, static_cast<const double*>(v), int64_t{0},
                     0);
  hipLaunchKernelGGL(k_pgd_normalize, dim3(1), dim3(1024), 0, st, a, v);
}

void launch_pgd_prime(const PgdArgs& a, int par, hipStream_t st) {
  hipLaunchKernelGGL(k_pgd_step, dim3(a.nblocks), dim3(256), 0, st, a, 2, par);
}

void launch_pgd_round(const PgdArgs& a, int first, int par, hipStream_t st) {
  const double* xc = a.xc;
  const int64_t n = a.np;
  hipLaunchKernelGGL(k_pgd_tiles<kPgdK>, dim3(a.njobs), dim3(256), 0, st, a, xc, n, par);
  hipLaunchKernelGGL(k_pgd_rows<kPgdK>, dim3(a.nb, kPgdK), dim3(256), 0, st, a, xc, n, par);
  hipLaunchKernelGGL(k_pgd_step, dim3(a.nblocks), dim3(256), 0, st, a, first ? 1 : 0, par);
}

}  // namespace admmbb
