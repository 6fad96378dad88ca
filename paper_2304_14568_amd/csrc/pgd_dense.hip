// Projected gradient descent with Armijo backtracking (Sec. 2.1) on the cached
// dense Gram sum of the dense x-update, driven on the device.
//
// With S = sum_s G_s (packed upper 64 x 64 tiles, fp64) the objective and its
// gradient are f(x) = x^T S x - g0^T x + const and grad f(x) = 2 S x - g0.
// One round evaluates kPgdK backtracking steps at once:
//   k_pgd_cand    trial points x_k = P(x - t_k g), t_k = t_base gamma^k, and the
//                 partial sums of g^T (x_k - x)
//   k_pgd_tiles   for every tile T of S and every k: T x_k,J and T^T x_k,I,
//                 one read of S for all kPgdK trial points
//   k_pgd_rows    u_k = S x_k from the tile products, and f(x_k) partial sums
//   k_pgd_select  the first k (largest step) with
//                 f(x_k) <= f(x) + beta g^T (x_k - x) becomes x, with gradient
//                 2 u_k - g0; stopping tests
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

// K trial points and g^T (x_k - x) partial sums, gdpart[k * nblocks + block]
__global__ __launch_bounds__(256) void k_pgd_cand(PgdArgs a) {
  if (a.st->done) return;
  __shared__ double red[4][kPgdK];
  const int j = static_cast<int>(blockIdx.x) * 256 + threadIdx.x;
  double loc[kPgdK];
  if (j >= a.n) {
    // zero padding up to whole 64-blocks (read by the tile products)
    if (j < a.np)
#pragma unroll
      for (int k = 0; k < kPgdK; ++k) a.xc[static_cast<int64_t>(k) * a.np + j] = 0.0;
  }
  if (j < a.n) {
    const double xj = a.x[j], gj = a.g[j];
    const double lo = a.lb[j], hi = a.ub[j];
    double t = a.st->t_base;
#pragma unroll
    for (int k = 0; k < kPgdK; ++k) {
      const double v = fmin(fmax(xj - t * gj, lo), hi);
      a.xc[static_cast<int64_t>(k) * a.np + j] = v;
      loc[k] = gj * (v - xj);
      t *= a.gamma;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kPgdK; ++k) loc[k] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < kPgdK; ++k) {
    const double s = wsum(loc[k]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < kPgdK) {
    const int k = threadIdx.x;
    a.gdpart[static_cast<int64_t>(k) * a.nblocks + blockIdx.x] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
  }
}

// One tile T = S_IJ (I <= J) per workgroup; wave w takes rows 16w..16w+15 of
// T for T v_k,J and columns 16w..16w+15 for T^T v_k,I, both as products
// (16 x 64 trial-point rows, zero beyond KC) x (64 x 16 slice of T) on the
// fp64 16x16x4 MFMA: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] of
// each step and receives D[l / 16 + 4 r][l % 16] in item r.  The k index of
// the 16 steps is a free permutation of the 64 tile columns (rows), chosen so
// that every lane loads contiguous doubles.  v_k = v + k * vstride, vstride and
// the vectors padded with zeros to whole 64-blocks.
// part[(t * KC + k) * 128 + i]      = (T v_k,J)_i
// part[(t * KC + k) * 128 + 64 + i] = (T^T v_k,I)_i   (off-diagonal tiles)
template <int KC>
__global__ __launch_bounds__(256) void k_pgd_tiles(PgdArgs a, const double* __restrict__ v, int64_t vstride) {
  if (a.st->done) return;
  const XJob job = a.jobs[blockIdx.x];
  const int I = job.ij >> 16, J = job.ij & 0xffff;
  const int64_t t = blockIdx.x;  // jobs are the tiles in packed order
  const double* T = a.Gp + t * kT * kT;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 15, kk = lane >> 4;
  const bool live = m < KC;
  double* out = a.part + t * (KC * 2 * kT);
  // T v_J: step (s, h) uses tile column 8 s + 2 kk + h
  {
    const double2* Tr = reinterpret_cast<const double2*>(T + (16 * w + m) * kT + 2 * kk);
    const double2* vr = reinterpret_cast<const double2*>(v + m * vstride + J * kT + 2 * kk);
    double2 tb[8], va[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      tb[s] = Tr[4 * s];
      va[s] = live ? vr[4 * s] : make_double2(0.0, 0.0);
    }
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[s].x, tb[s].x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[s].y, tb[s].y, acc, 0, 0, 0);
    }
    // item r: trial point kk + 4 r, tile row 16 w + m
#pragma unroll
    for (int r = 0; r < 2; ++r)
      if (kk + 4 * r < KC) out[(kk + 4 * r) * 2 * kT + 16 * w + m] = acc[r];
  }
  if (I == J) return;
  // T^T v_I: step s uses tile row 16 kk + s
  {
    const double* Tc = T + (16 * kk) * kT + 16 * w + m;
    const double2* vr = reinterpret_cast<const double2*>(v + m * vstride + I * kT + 16 * kk);
    double tb[16];
    double2 va[8];
#pragma unroll
    for (int s = 0; s < 16; ++s) tb[s] = Tc[s * kT];
#pragma unroll
    for (int s = 0; s < 8; ++s) va[s] = live ? vr[s] : make_double2(0.0, 0.0);
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[s].x, tb[2 * s], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[s].y, tb[2 * s + 1], acc, 0, 0, 0);
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
__global__ __launch_bounds__(256) void k_pgd_rows(PgdArgs a, const double* __restrict__ v, int64_t vstride) {
  if (a.st->done) return;
  __shared__ double red[4][kT];
  const int I = static_cast<int>(blockIdx.x), k = static_cast<int>(blockIdx.y);
  const int i = threadIdx.x & 63, w = threadIdx.x >> 6;
  double s = 0.0;
  for (int J = w; J < a.nb; J += 4) {
    const int64_t t = J < I ? ptile(J, I, a.nb) : ptile(I, J, a.nb);
    s += a.part[(t * KC + k) * (2 * kT) + (J < I ? kT : 0) + i];
  }
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

// Acceptance, step update and stopping tests, then x and grad f(x) = 2 S x - g0
// of the accepted point; 2 waves per trial point for the sums.
__global__ __launch_bounds__(128 * kPgdK) void k_pgd_select(PgdArgs a, int first) {
  PgdDevState* st = a.st;
  if (st->done) return;
  __shared__ double rf[2 * kPgdK], rd[2 * kPgdK];
  __shared__ double fk[kPgdK], gd[kPgdK];
  __shared__ int pick;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int k = w >> 1, h = w & 1;
  double f = 0.0, d = 0.0;
  for (int b = h * 64 + lane; b < a.nb; b += 128) f += a.fpart[static_cast<int64_t>(k) * a.nb + b];
  for (int b = h * 64 + lane; b < a.nblocks; b += 128) d += a.gdpart[static_cast<int64_t>(k) * a.nblocks + b];
  f = wsum(f);
  d = wsum(d);
  if (lane == 0) {
    rf[w] = f;
    rd[w] = d;
  }
  __syncthreads();
  if (tid < kPgdK) {
    fk[tid] = a.fconst + (rf[2 * tid] + rf[2 * tid + 1]);
    gd[tid] = rd[2 * tid] + rd[2 * tid + 1];
  }
  __syncthreads();
  if (tid == 0) {
    int p = -1;
    bool stop = false;
    if (first) {
      // every trial point is x itself (t_base = 0): record f(x), take its gradient
      p = 0;
      st->f = fk[0];
      st->t_base = st->alpha;
      if (a.max_iter <= 0) {
        stop = true;
        st->status = 3;
      }
    } else {
      for (int kk = 0; kk < kPgdK; ++kk)
        if (st->trials + kk < a.max_trials && fk[kk] <= st->f + a.beta * gd[kk]) {
          p = kk;
          break;
        }
      if (p >= 0) {
        const double f_old = st->f, f_new = fk[p];
        st->f = f_new;
        st->iter += 1;
        st->trials = 0;
        st->t_base = st->alpha;
        if (fabs(f_old - f_new) <= a.tol * fabs(f_old)) {
          stop = true;
          st->status = 1;
        } else if (st->iter >= a.max_iter) {
          stop = true;
          st->status = 3;
        }
      } else {
        st->trials += kPgdK;
        double t = st->t_base;
        for (int kk = 0; kk < kPgdK; ++kk) t *= a.gamma;
        st->t_base = t;
        if (st->trials >= a.max_trials) {
          stop = true;
          st->status = 2;
        }
      }
    }
    if (stop) st->done = 1;
    st->pick = p;
    pick = p;
  }
  __syncthreads();
  const int p = pick;
  if (p < 0) return;
  const double* xp = a.xc + static_cast<int64_t>(p) * a.np;
  const double* up = a.u + static_cast<int64_t>(p) * a.np;
  for (int j = tid; j < a.n; j += blockDim.x) {
    a.x[j] = xp[j];
    a.g[j] = 2.0 * up[j] - a.g0[j];
  }
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
    if (tid == 0) a.st->alpha = 1.0;
    return;
  }
  for (int j = tid; j < a.n; j += 1024) v[j] = 2.0 * a.u[j] / nrm;
  if (tid == 0) a.st->alpha = 10.0 / nrm;
}

}  // namespace

// One power-iteration step on H = 2 S; v is replaced by the next unit vector.
// The state must have done = 0.
void launch_pgd_power(const PgdArgs& a, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_pgd_tiles<1>, dim3(a.njobs), dim3(256), 0, st, a, static_cast<const double*>(v),
                     int64_t{0});
  hipLaunchKernelGGL(k_pgd_rows<1>, dim3(a.nb, 1), dim3(256), 0, st, a, static_cast<const double*>(v), int64_t{0});
  hipLaunchKernelGGL(k_pgd_normalize, dim3(1), dim3(1024), 0, st, a, v);
}

void launch_pgd_round(const PgdArgs& a, int first, hipStream_t st) {
  const double* xc = a.xc;
  const int64_t n = a.np;
  hipLaunchKernelGGL(k_pgd_cand, dim3(a.nblocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_pgd_tiles<kPgdK>, dim3(a.njobs), dim3(256), 0, st, a, xc, n);
  hipLaunchKernelGGL(k_pgd_rows<kPgdK>, dim3(a.nb, kPgdK), dim3(256), 0, st, a, xc, n);
  hipLaunchKernelGGL(k_pgd_select, dim3(1), dim3(128 * kPgdK), 0, st, a, first);
}

}  // namespace admmbb
