// Dense x-update: the exact solve of every scenario subproblem through a
// cached inverse of its system matrix (Appendix A factors B_s = A_s^T W~_s A_s
// + rho/2 I once and reuses the factor in every iteration; here the factor is
// the inverse itself, so that each x-update is one bandwidth-bound GEMV).
//
//  1. G_s = A_s^T diag(c_s w) A_s, upper 64 x 64 tiles: lists of the rows
//     that reach each tile (k_gram_rows, k_gram_scan), then one workgroup per
//     tile adds its rows' products in LDS (k_gram_tiles).  k_gram (one fp64
//     atomic per product, one wave per stored row) is the fallback when the
//     lists do not fit in device memory.
//  2. k_gram_finish: the upper tiles of the sweep work matrix
//     A = G_s + rho/2 I (identity on the padding to npad) and sum_s G_s.
//     Steps 1-3 run on chunks of scenarios, so that only a chunk's fp64
//     set-up matrices occupy device memory at a time.
//  3. block sweep (Gauss-Jordan on 64-blocks, no pivoting: the pivot blocks
//     are Schur complements of an SPD matrix): for each block K,
//        P = A_KK^-1, U = A_:K P, R = A_K: (old),
//        A_ij -= U_i R_j off the block row and column,
//        A_:K = U, A_K: = U^T, A_KK = -P;
//     after the last block A = -B_s^-1.  The sweep matrix stays symmetric, so
//     only its upper 64 x 64 tiles are updated (half the work).  k_sweep_store writes M_s = B_s^-1 in fp32.
//  4. k_gq_pack: sum_s G_s rounded to 48 bits for the objective tiles.
//  5. every iteration, three launches: k_dense_x (x_s = M_s c_s tile by tile,
//     the previous iteration's stopping test in workgroup 0), k_xzres (the
//     partial sums of x_s with the z-update), k_dense_tail_dual (residual
//     norms and dual step, the dual
//     update with the next right-hand sides c_s, the objective at the new z
//     from the quadratic form).  k_fheadobj forms the right-hand sides and the
//     objective of the state a run starts from.
// The symmetric matrices used in every iteration (M_s and sum_s G_s) are stored
// as their upper 64 x 64 tiles only, which halves the bytes each iteration reads.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.h"
#include "scalars.h"

namespace admmbb {

namespace {

constexpr int kFb = 64;  // sweep block size and packed tile size

__host__ __device__ __forceinline__ int64_t tile_index(int I, int J, int nb) {
  return static_cast<int64_t>(I) * nb - static_cast<int64_t>(I) * (I - 1) / 2 + (J - I);
}

__device__ __forceinline__ double wave_sum_d(double v) { return group_allsum<64>(v); }

// ---------------------------------------------------------------------------
// Gram matrix
// ---------------------------------------------------------------------------

template <bool C16>
__global__ __launch_bounds__(256) void k_gram(MatDev mat, const double* __restrict__ rw64, Scen sc,
                                              double* __restrict__ G, int ld) {
  const int row = static_cast<int>(blockIdx.x) * 4 + static_cast<int>(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= sc.rows) return;
  const uint32_t c0 = mat.rp[sc.rp_base + row], c1 = mat.rp[sc.rp_base + row + 1];
  const int64_t e0 = sc.nnz_base + 4 * static_cast<int64_t>(c0);
  const int k = 4 * static_cast<int>(c1 - c0);
  const double rw = rw64[sc.row_base + row];
  const float* val = static_cast<const float*>(mat.val);
  auto colat = [&](int64_t e) -> int {
    if constexpr (C16)
      return static_cast<const uint16_t*>(mat.col)[e];
    else
      return static_cast<const int32_t*>(mat.col)[e];
  };
  for (int base = 0; base < k; base += 64) {
    const int kk = base + lane;
    const bool valid = kk < k;
    const int ck = valid ? colat(e0 + kk) : 0;
    const double vk = valid ? rw * static_cast<double>(val[e0 + kk]) : 0.0;
    const int jend = base + 64 < k ? base + 64 : k;
    for (int jj = 0; jj < jend; ++jj) {
      const float vj = val[e0 + jj];
      if (vj == 0.0f) continue;  // chunk padding
      const int cj = colat(e0 + jj);
      // columns increase along a stored row, so jj <= kk gives cj <= ck
      if (valid && jj <= kk && vk != 0.0)
        unsafeAtomicAdd(&G[static_cast<int64_t>(cj) * ld + ck], vk * static_cast<double>(vj));
    }
  }
}

// Gram matrix by output tiles.  Every stored row adds w_i a_i a_i^T to the
// 64 x 64 tiles (I, J), I <= J, of the blocks its nonzeros fall in.  Lists of
// the rows that reach each tile are built first (count, scan, fill); one
// workgroup per tile then adds its rows' products in LDS and writes the tile
// once, instead of one global fp64 atomic per product.

template <bool C16>
__device__ __forceinline__ int col_at(const MatDev& mat, int64_t e) {
  if constexpr (C16)
    return static_cast<const uint16_t*>(mat.col)[e];
  else
    return static_cast<const int32_t*>(mat.col)[e];
}

// LDS written by some lanes of a wave and then read by others of the same wave
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kMaxBlocks = 128;  // 64-column blocks of a patient (n <= 8192)

// FILL = false: count[t] += 1 for every tile t = (b_p, b_q), p <= q, of the
// distinct blocks b_1 < ... < b_r of each row; FILL = true: the row and its
// extent at off[t] + (a slot taken from cur[t]).  One wave per stored row.
template <bool C16, bool FILL>
__global__ __launch_bounds__(256) void k_gram_rows(MatDev mat, Scen sc, int nb, int32_t* __restrict__ cnt,
                                                   const int64_t* __restrict__ off, GramEntry* __restrict__ list) {
  __shared__ int bl[4][kMaxBlocks];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = static_cast<int>(blockIdx.x) * 4 + w;
  if (row >= sc.rows) return;  // no workgroup barrier below
  const uint32_t c0 = mat.rp[sc.rp_base + row], c1 = mat.rp[sc.rp_base + row + 1];
  const int64_t e0 = sc.nnz_base + 4 * static_cast<int64_t>(c0);
  const int k = 4 * static_cast<int>(c1 - c0);
  int r = 0;
  for (int base = 0; base < k; base += 64) {
    const int kk = base + lane;
    int b = -1, bp = -1;
    if (kk < k) {
      b = col_at<C16>(mat, e0 + kk) >> 6;
      if (kk > 0) bp = col_at<C16>(mat, e0 + kk - 1) >> 6;
    }
    const bool start = kk < k && b != bp;  // columns are non-decreasing along a row
    const uint64_t m = __ballot(start);
    const int at = r + __popcll(m & ((uint64_t{1} << lane) - 1));
    if (start && at < kMaxBlocks) bl[w][at] = b;
    r += __popcll(m);
  }
  if (r > kMaxBlocks) r = kMaxBlocks;  // cannot happen for n <= 8192
  wave_lds_sync();
  for (int t = lane; t < r * r; t += 64) {
    const int p = t / r, q = t - p * r;
    if (p > q) continue;
    const int64_t ti = tile_index(bl[w][p], bl[w][q], nb);
    if constexpr (FILL)
      list[off[ti] + atomicAdd(&cnt[ti], 1)] = GramEntry{row, c0, c1, 0};
    else
      atomicAdd(&cnt[ti], 1);
  }
}

// off[i] = cnt[0] + ... + cnt[i - 1] for i <= nt (one workgroup)
__global__ __launch_bounds__(1024) void k_gram_scan(const int32_t* __restrict__ cnt, int64_t nt,
                                                    int64_t* __restrict__ off) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (nt + 1023) / 1024;
  const int64_t b = t * per < nt ? t * per : nt, e = b + per < nt ? b + per : nt;
  int64_t sum = 0;
  for (int64_t i = b; i < e; ++i) sum += cnt[i];
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int i = 0; i < 1024; ++i) {
      const int64_t v = part[i];
      part[i] = run;
      run += v;
    }
    off[nt] = run;
  }
  __syncthreads();
  int64_t run = part[t];
  for (int64_t i = b; i < e; ++i) {
    off[i] = run;
    run += cnt[i];
  }
}

// One workgroup per tile (I, J) of scenario g0 + blockIdx.y: the rows of its
// list add c_s w_i a_ij a_ik for j in block I, k in block J (j <= k inside a
// diagonal tile) to an fp64 LDS tile, which is then written to G (upper part).
// The tile is accumulated in 64-bit fixed point (gscale[s], a power of two,
// keeps every partial sum below 2^61: all products are nonnegative, so no
// partial sum exceeds its entry G_jk <= sqrt(G_jj G_kk) <= max_j G_jj), which
// makes it exact and independent of the order of the atomics.
// A row's nonzeros in one block are contiguous (at most 64, plus padding of
// value 0).  Each wave takes one listed row at a time: its columns and values
// are read once (with the next list entry already in flight) and staged in the
// wave's LDS area, from which the products are formed; rows longer than the
// staging area are read from memory instead.
constexpr int kGramWaves = 8;
constexpr int kGramStage = 320;

template <bool C16>
__global__ __launch_bounds__(64 * kGramWaves) void k_gram_tiles(MatDev mat, const double* __restrict__ rw64,
                                                                const Scen* __restrict__ scen, int g0, int nb,
                                                                const int64_t* __restrict__ off,
                                                                const GramEntry* __restrict__ list,
                                                                const double* __restrict__ gscale,
                                                                double* __restrict__ G, int ld) {
  // row stride kFb + 1: the lanes of one atomic instruction mostly share a
  // column and differ in the row, so rows must fall in different banks
  __shared__ unsigned long long acc[kFb * (kFb + 1)];
  __shared__ float sval[kGramWaves][kGramStage];
  __shared__ uint8_t scol[kGramWaves][kGramStage];
  const int64_t ntiles = static_cast<int64_t>(nb) * (nb + 1) / 2;
  const int64_t t = blockIdx.x;
  const int s = static_cast<int>(blockIdx.y);
  int I = 0;
  int64_t rem = t;
  while (rem >= nb - I) {
    rem -= nb - I;
    ++I;
  }
  const int J = I + static_cast<int>(rem);
  for (int e = threadIdx.x; e < kFb * (kFb + 1); e += 64 * kGramWaves) acc[e] = 0ull;
  __syncthreads();
  const Scen sc = scen[g0 + s];
  const double scale = gscale[s];
  const float* val = static_cast<const float*>(mat.val);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* sv = sval[w];
  uint8_t* scl = scol[w];
  const int64_t le = off[s * ntiles + t + 1];
  int64_t li = off[s * ntiles + t] + w;
  GramEntry cur{};
  if (li < le) cur = list[li];
  for (; li < le; li += kGramWaves) {
    GramEntry nxt{};
    if (li + kGramWaves < le) nxt = list[li + kGramWaves];
    const int64_t e0 = sc.nnz_base + 4 * static_cast<int64_t>(cur.c0);
    const int k = 4 * static_cast<int>(cur.c1 - cur.c0);
    const bool staged = k <= kGramStage;
    const double rw = rw64[sc.row_base + cur.row];
    int fI = 0, nI = 0, fJ = 0, nJ = 0;
    for (int base = 0; base < k; base += 64) {
      const int kk = base + lane;
      int b = -1;
      if (kk < k) {
        const int c = col_at<C16>(mat, e0 + kk);
        b = c >> 6;
        if (staged) {
          sv[kk] = val[e0 + kk];
          scl[kk] = static_cast<uint8_t>(c & (kFb - 1));
        }
      }
      const uint64_t mI = __ballot(b == I), mJ = __ballot(b == J);
      if (nI == 0 && mI) fI = base + __ffsll(static_cast<unsigned long long>(mI)) - 1;
      if (nJ == 0 && mJ) fJ = base + __ffsll(static_cast<unsigned long long>(mJ)) - 1;
      nI += __popcll(mI);
      nJ += __popcll(mJ);
    }
    wave_lds_sync();
    // a = p / nJ as (p * mJ) >> 19: exact for p < 67 * 67 and nJ <= 67, the
    // largest segments (64 columns of a block plus 3 entries of padding)
    const int np = nI * nJ;
    const uint32_t mJ = nJ > 0 ? (uint32_t{1} << 19) / static_cast<uint32_t>(nJ) + 1 : 0;
    for (int p = lane; p < np; p += 64) {
      const int a = static_cast<int>((static_cast<uint32_t>(p) * mJ) >> 19), q = p - a * nJ;
      if (I == J && a > q) continue;
      const int pa = fI + a, pb = fJ + q;
      double va, vb;
      int ca, cb;
      if (staged) {
        va = sv[pa];
        vb = sv[pb];
        ca = scl[pa];
        cb = scl[pb];
      } else {
        va = val[e0 + pa];
        vb = val[e0 + pb];
        ca = col_at<C16>(mat, e0 + pa) & (kFb - 1);
        cb = col_at<C16>(mat, e0 + pb) & (kFb - 1);
      }
      const double prod = (rw * va) * vb;
      if (prod != 0.0) atomicAdd(&acc[ca * (kFb + 1) + cb], __double2ull_rn(prod * scale));
    }
    wave_lds_sync();  // the next row overwrites the staging area
    cur = nxt;
  }
  __syncthreads();
  double* Gs = G + static_cast<int64_t>(s) * ld * ld;
  const double unscale = 1.0 / scale;  // exact: a power of two
  for (int e = threadIdx.x; e < kFb * kFb; e += 64 * kGramWaves) {
    const int r = e / kFb, c = e % kFb;
    if (I != J || r <= c) Gs[static_cast<int64_t>(I * kFb + r) * ld + J * kFb + c] = static_cast<double>(acc[r * (kFb + 1) + c]) * unscale;
  }
}

// For the chunk of scenarios [scen_begin, scen_begin + nscen) of one patient
// (chunk buffers, npad x npad per scenario, upper triangle of G accumulated):
// the upper tiles of A = G + rho/2 I (identity on the padding; inside a
// diagonal tile both triangles, the lower one read from the upper), and, when
// accumulate_gsum, their sum over the chunk added to the packed sum_s G_s.
__global__ __launch_bounds__(256) void k_gram_finish(FactorArgs f, int patient, int scen_begin, int nscen,
                                                     int npad, int n, double rho, int accumulate_gsum) {
  const Pat pt = f.pat[patient];
  const int64_t nn = static_cast<int64_t>(npad) * npad;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  (void)scen_begin;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < nn; idx += stride) {
    const int i = static_cast<int>(idx / npad), j = static_cast<int>(idx % npad);
    const int I = i / kFb, J = j / kFb;
    if (I > J) continue;  // only the upper tiles are used from here on
    const int64_t src = (i <= j) ? idx : static_cast<int64_t>(j) * npad + i;
    double sum = 0.0;
    for (int s = 0; s < nscen; ++s) {
      const double gv = f.G[s * nn + src];
      sum += gv;
      double a = gv;
      if (i == j) a += (i < n) ? 0.5 * rho : 1.0;
      f.A[s * nn + idx] = a;
    }
    if (accumulate_gsum)
      f.Gp[pt.gpack_off + tile_index(I, J, pt.nbk) * kFb * kFb + (i % kFb) * kFb + (j % kFb)] += sum;
  }
}

// ---------------------------------------------------------------------------
// block sweep
// ---------------------------------------------------------------------------

// P = A_KK^-1 by the scalar sweep (one workgroup per scenario)
__global__ __launch_bounds__(256) void k_sweep_pivot(FactorArgs f, int scen_begin, int npad, int k0) {
  // thread (i0, j) keeps rows i0, i0 + 4, ..., i0 + 60 of column j in
  // registers; each step publishes only the pivot row and column (their values
  // before the step) through LDS
  __shared__ double prow[kFb], pcol[kFb];
  const int g = scen_begin + static_cast<int>(blockIdx.x);
  const double* A = f.A + static_cast<int64_t>(blockIdx.x) * npad * npad;  // chunk buffer
  const int j = threadIdx.x & (kFb - 1), i0 = threadIdx.x >> 6;
  double r[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) r[q] = A[static_cast<int64_t>(k0 + i0 + 4 * q) * npad + k0 + j];
#pragma unroll
  for (int t = 0; t < kFb; ++t) {
    if (i0 == (t & 3)) prow[j] = r[t >> 2];
    if (j == t) {
#pragma unroll
      for (int q = 0; q < 16; ++q) pcol[i0 + 4 * q] = r[q];
    }
    __syncthreads();
    const double inv = 1.0 / prow[t];
    const double atj = prow[j];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = i0 + 4 * q;
      const double ait = pcol[i];
      double v;
      if (i == t && j == t)
        v = -inv;
      else if (i == t)
        v = atj * inv;
      else if (j == t)
        v = ait * inv;
      else
        v = r[q] - ait * atj * inv;
      r[q] = v;
    }
    __syncthreads();  // the next step overwrites the pivot row and column
  }
  // the swept block is -A_KK^-1
  double* P = f.P + static_cast<int64_t>(g) * kFb * kFb;
#pragma unroll
  for (int q = 0; q < 16; ++q) P[(i0 + 4 * q) * kFb + j] = -r[q];
}

// U_I = A_IK P (64 x 64 per workgroup) and R tile = A_K,I (old row panel copy).
// Only the upper tiles (I <= J) of the sweep matrix are kept up to date (it
// stays symmetric), so blocks on the other side of the pivot are read from the
// mirrored tile, transposed.
__global__ __launch_bounds__(256) void k_sweep_panel(FactorArgs f, int scen_begin, int npad, int k0) {
  __shared__ double at[kFb][kFb];  // A_IK
  __shared__ double p[kFb][kFb];   // P
  const int g = scen_begin + static_cast<int>(blockIdx.y);
  const double* A = f.A + static_cast<int64_t>(blockIdx.y) * npad * npad;  // chunk buffer
  const int i0 = static_cast<int>(blockIdx.x) * kFb;
  const double* Pg = f.P + static_cast<int64_t>(g) * kFb * kFb;
  double* Ut = f.U + static_cast<int64_t>(g) * f.npmax * kFb;
  double* R = f.R + static_cast<int64_t>(g) * f.npmax * kFb;
  for (int e = threadIdx.x; e < kFb * kFb; e += 256) {
    const int r = e / kFb, c = e % kFb;
    p[r][c] = Pg[e];
    if (i0 <= k0) {
      at[r][c] = A[static_cast<int64_t>(i0 + r) * npad + k0 + c];  // tile (I, K), stored
    } else {
      at[c][r] = A[static_cast<int64_t>(k0 + r) * npad + i0 + c];  // tile (K, I), transposed
    }
    // row panel R[t][i0 + j] = A[k0 + t][i0 + j]
    if (i0 >= k0)
      R[static_cast<int64_t>(r) * npad + i0 + c] = A[static_cast<int64_t>(k0 + r) * npad + i0 + c];
    else
      R[static_cast<int64_t>(c) * npad + i0 + r] = A[static_cast<int64_t>(i0 + r) * npad + k0 + c];
  }
  __syncthreads();
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;  // 4 x 4 outputs each
  double acc[4][4] = {};
  for (int t = 0; t < kFb; ++t) {
    double av[4], pv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      av[q] = at[4 * ti + q][t];
      pv[q] = p[t][4 * tj + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[q][r] = fma(av[q], pv[r], acc[q][r]);
  }
  // stored transposed: Ut[c][i] = U[i][c]
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) Ut[static_cast<int64_t>(4 * tj + r) * npad + i0 + 4 * ti + q] = acc[q][r];
}

// rank-64 update of every upper tile off the pivot row and column; panel tiles replaced
__global__ __launch_bounds__(256) void k_sweep_update(FactorArgs f, int scen_begin, int npad, int k0) {
  __shared__ double ut[kFb][kFb];  // ut[t][i] = U[i0 + i][t]
  __shared__ double rs[kFb][kFb];  // rs[t][j] = R[t][j0 + j]
  const int nbk = npad / kFb;
  // upper tile number -> (bi, bj), bi <= bj
  int t0 = static_cast<int>(blockIdx.x), bi = 0;
  while (t0 >= nbk - bi) {
    t0 -= nbk - bi;
    ++bi;
  }
  const int bj = bi + t0;
  const int g = scen_begin + static_cast<int>(blockIdx.y);
  double* A = f.A + static_cast<int64_t>(blockIdx.y) * npad * npad;  // chunk buffer
  const int i0 = bi * kFb, j0 = bj * kFb, kb = k0 / kFb;
  const double* Ut = f.U + static_cast<int64_t>(g) * f.npmax * kFb;
  const double* R = f.R + static_cast<int64_t>(g) * f.npmax * kFb;
  if (bi == kb || bj == kb) {
    const double* Pg = f.P + static_cast<int64_t>(g) * kFb * kFb;
    for (int e = threadIdx.x; e < kFb * kFb; e += 256) {
      const int i = e / kFb, j = e % kFb;
      double v;
      if (bi == kb && bj == kb)
        v = -Pg[e];
      else if (bj == kb)
        v = Ut[static_cast<int64_t>(j) * npad + i0 + i];  // U[i0 + i][j]
      else
        v = Ut[static_cast<int64_t>(i) * npad + j0 + j];  // U[j0 + j][i]
      A[static_cast<int64_t>(i0 + i) * npad + j0 + j] = v;
    }
    return;
  }
  // thread (ti, tj) updates rows 4 ti .. 4 ti + 3 and columns tj, tj + 16,
  // tj + 32, tj + 48 of the tile; its old values and both panels are all
  // requested before the first use
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  double a_old[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) a_old[q][r] = A[static_cast<int64_t>(i0 + 4 * ti + q) * npad + j0 + tj + 16 * r];
  double us[16], rr[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = threadIdx.x + 256 * k;
    const int t = e / kFb, c = e % kFb;
    us[k] = Ut[static_cast<int64_t>(t) * npad + i0 + c];
    rr[k] = R[static_cast<int64_t>(t) * npad + j0 + c];
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = threadIdx.x + 256 * k;
    ut[e / kFb][e % kFb] = us[k];
    rs[e / kFb][e % kFb] = rr[k];
  }
  __syncthreads();
  double acc[4][4] = {};
  for (int t = 0; t < kFb; ++t) {
    double uv[4], rv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uv[q] = ut[t][4 * ti + q];
      rv[q] = rs[t][tj + 16 * q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[q][r] = fma(uv[q], rv[r], acc[q][r]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      A[static_cast<int64_t>(i0 + 4 * ti + q) * npad + j0 + tj + 16 * r] = a_old[q][r] - acc[q][r];
}

// Position of entry (r, c) inside a stored 64 x 64 tile of M_s.  Thread t of
// the x-update holds the 4 x 4 block of rows 4 (t / 16) .. + 3 and columns
// 4 (t % 16) .. + 3 as four float4 (row k = 0..3 of the block); float4 k of
// thread t is stored at k * 256 + t, so that every wave load instruction of
// the x-update reads 1 KiB contiguous.
__host__ __device__ __forceinline__ int xtile_pos(int r, int c) {
  return 4 * ((r & 3) * 256 + (r >> 2) * 16 + (c >> 2)) + (c & 3);
}

// packed M = -A (upper tiles) in fp32, for the chunk of scenarios starting at scen_begin
__global__ __launch_bounds__(256) void k_sweep_store(FactorArgs f, int patient, int scen_begin, int npad) {
  const Pat pt = f.pat[patient];
  const Scen sc = f.scen[scen_begin + static_cast<int>(blockIdx.y)];
  const int64_t nn = static_cast<int64_t>(npad) * npad;
  const double* A = f.A + static_cast<int64_t>(blockIdx.y) * nn;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < nn; idx += stride) {
    const int i = static_cast<int>(idx / npad), j = static_cast<int>(idx % npad);
    const int I = i / kFb, J = j / kFb;
    if (I <= J)
      f.Mp[sc.mpack_off + tile_index(I, J, pt.nbk) * kFb * kFb + xtile_pos(i % kFb, j % kFb)] =
          static_cast<float>(-A[idx]);
  }
}

// ---------------------------------------------------------------------------
// per-iteration kernels
// ---------------------------------------------------------------------------

// Row rotations by DPP for the x-update's row sums (the pair and quad
// exchanges are those of scalars.h).
constexpr int kDppRor4 = 0x124;
constexpr int kDppRor8 = 0x128;

// One packed tile T = M_s[I, J] (I <= J) per workgroup: a = T c_J and, off
// the diagonal, b = T^T c_I (the tile's contribution to the rows of block J).
// Thread t holds the 4 x 4 block at rows 4 rb, columns 4 cb (rb = t / 16,
// cb = t % 16; four float4 loads, each a 1 KiB contiguous read per wave in
// the stored order of xtile_pos), so both products use the registers as
// loaded: the row sums are reduced over the 16 lanes of a DPP row, the column
// sums over the wave's four rows by shuffles and over the four waves in
// shared memory.  The tile table entry carries every address, so the tile
// load depends on one table read only.  The right-hand side and all sums are
// fp64: the inverse has entries of both signs and |M| |c| exceeds |M c| by two
// orders of magnitude, so fp32 sums would put a floor of about 1e-5 relative
// under every x-update; the fp32 storage of M itself contributes about 1e-6.
// kLoadsFirst (a context of one patient): the tile's 16 KB (tile idx of the
// table is stored at Mp + 4096 idx) are requested before the table and
// stop-flag reads, and the empty statement keeps the compiler from moving the
// loads below the early exit (a stopped patient ends the run within an
// iteration).  Otherwise (a batch, whose other patients go on iterating) the
// flag is read first and a stopped patient's tiles are not loaded at all.
template <bool kLoadsFirst>
__device__ __forceinline__ void xsym_tile(const FactorArgs& f, const double* __restrict__ c, int idx) {
  __shared__ double2 cI[kFb / 2], cJ[kFb / 2];
  __shared__ double bpart[4][kFb];  // column sums of each wave
  const int tid = threadIdx.x;
  const int rb = tid >> 4, cb = tid & 15, lane = tid & 63;
  const float4* T = reinterpret_cast<const float4*>(f.Mp) + static_cast<int64_t>(idx) * 1024;
  float4 m[4];
  XTile tj;
  if constexpr (kLoadsFirst) {
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = T[k * 256 + tid];
    tj = f.xtiles[idx];
    const bool stopped = f.ps[tj.patient].stopped != 0;
    asm volatile("" ::: "memory");
    if (stopped) return;
  } else {
    tj = f.xtiles[idx];
    if (f.ps[tj.patient].stopped) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = T[k * 256 + tid];
  }
  if (tid < kFb) {
    const int jc = tj.J * kFb + tid, ic = tj.I * kFb + tid;
    reinterpret_cast<double*>(cJ)[tid] = jc < tj.n ? c[tj.vbase + jc] : 0.0;
    reinterpret_cast<double*>(cI)[tid] = ic < tj.n ? c[tj.vbase + ic] : 0.0;
  }
  __syncthreads();
  // a: row 4 rb + k over this block's four columns
  const double2 j01 = cJ[2 * cb], j23 = cJ[2 * cb + 1];
  double a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double v = static_cast<double>(m[k].x) * j01.x;
    v = fma(static_cast<double>(m[k].y), j01.y, v);
    v = fma(static_cast<double>(m[k].z), j23.x, v);
    a[k] = fma(static_cast<double>(m[k].w), j23.y, v);
  }
  // sum over the 16 column blocks (the lanes of one DPP row), scattered so
  // that lane cb ends with row 4 rb + (cb % 4): lane pairs (xor 1) keep rows of
  // their own parity, quad pairs (xor 2) one row each, then the four lanes of
  // a row add up by rotations of 4 and 8
  const bool b0 = (cb & 1) != 0, b1 = (cb & 2) != 0;
  double k0 = b0 ? a[1] : a[0], k1 = b0 ? a[3] : a[2];
  k0 += dpp_move<kDppXor1>(b0 ? a[0] : a[1]);
  k1 += dpp_move<kDppXor1>(b0 ? a[2] : a[3]);
  double r = (b1 ? k1 : k0) + dpp_move<kDppXor2>(b1 ? k0 : k1);
  r += dpp_move<kDppRor8>(r);
  r += dpp_move<kDppRor4>(r);
  double* out = f.xpart + static_cast<int64_t>(idx) * (2 * kFb);
  if (cb < 4) out[4 * rb + cb] = r;
  if (tj.I == tj.J) return;
  // b: column 4 cb + j over this block's four rows
  const double2 i01 = cI[2 * rb], i23 = cI[2 * rb + 1];
  double bv[4];
  {
    const float* m0 = reinterpret_cast<const float*>(&m[0]);
    const float* m1 = reinterpret_cast<const float*>(&m[1]);
    const float* m2 = reinterpret_cast<const float*>(&m[2]);
    const float* m3 = reinterpret_cast<const float*>(&m[3]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double v = static_cast<double>(m0[j]) * i01.x;
      v = fma(static_cast<double>(m1[j]), i01.y, v);
      v = fma(static_cast<double>(m2[j]), i23.x, v);
      bv[j] = fma(static_cast<double>(m3[j]), i23.y, v);
    }
  }
  // sum over the wave's four row blocks (lane bits 4 and 5), scattered so
  // that the lane ends with column 4 cb + lane / 16
  const bool g0 = (lane & 16) != 0, g1 = (lane & 32) != 0;
  double h0 = g0 ? bv[1] : bv[0], h1 = g0 ? bv[3] : bv[2];
  h0 += __shfl_xor(g0 ? bv[0] : bv[1], 16, 64);
  h1 += __shfl_xor(g0 ? bv[2] : bv[3], 16, 64);
  const double u = (g1 ? h1 : h0) + __shfl_xor(g1 ? h0 : h1, 32, 64);
  bpart[tid >> 6][4 * cb + (lane >> 4)] = u;
  __syncthreads();
  if (tid < kFb) out[kFb + tid] = (bpart[0][tid] + bpart[1][tid]) + (bpart[2][tid] + bpart[3][tid]);
}

// Table index of the tile that workgroup b of an x-update launch takes: the
// order reverses from one iteration to the next (by the parity of the first
// patient's iteration count, which only the previous launches write), so that
// an iteration starts on the tiles the last one read most recently, while
// they may still sit in the memory-side cache.  Every tile is taken once
// either way, and the results do not depend on the order.
__device__ __forceinline__ int xsym_order(const FactorArgs& f, int b) {
  return (f.ps[0].iter & 1) ? f.nxtiles - 1 - b : b;
}

template <bool kLoadsFirst>
__global__ __launch_bounds__(256) void k_xsym(FactorArgs f, const double* __restrict__ c) {
  xsym_tile<kLoadsFirst>(f, c, xsym_order(f, static_cast<int>(blockIdx.x)));
}

// The reduction of the x-update partials fused with the z-update (the dense
// x-update's iteration, both launch orders): one workgroup per 16 spots of a
// patient (a quarter of a column block, the z-update's job), one wave per
// scenario (waves w, w + 16, ... for more than 16).  For the wave's scenario
// its four 16-lane groups g add the partials of the tiles J = g, g + 4, ...
// of the spots' row block I (T_IJ c_J for J >= I, T_JI^T c_J below), each
// lane one spot, then across the groups by lane swaps: x_s of the 16 spots,
// rounded to fp32 as stored.  Then the z-update of k_zres on the same spots:
// z = P(mean_s(x_s + y_s / rho)) in a fixed order over the waves, d = x_s - z
// and the eight fp64 partial sums of the residuals and the dual step.
constexpr int kXzWaves = 16;
constexpr int kXzCols = 16;
__global__ __launch_bounds__(64 * kXzWaves) void k_xzres(FactorArgs f, VecArgs a) {
  __shared__ double sacc[kXzWaves][kXzCols];
  __shared__ float zsh[kXzCols];
  __shared__ double sred[kXzWaves][8];
  const int bi4 = static_cast<int>(blockIdx.x);
  const ZJob pt = a.zjobs[bi4 >> 2];
  const PatState* ps = a.ps + pt.patient;
  const int stopped = ps->stopped;  // read beside the loads below; checked before any write
  const double rho = ps->rho;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const int r = (bi4 & 3) * kXzCols + c;  // row within the block of 64 spots
  const int j = pt.col0 + r;
  const bool valid = j < pt.n;
  const int I = pt.col0 / kFb, nb = (pt.n + kFb - 1) / kFb;
  const int64_t ntile = static_cast<int64_t>(nb) * (nb + 1) / 2;
  const int64_t zi = pt.zvec_base + j;
  // the first scenario's vectors and the projection's inputs, requested first
  float y0 = 0.0f, lbv = 0.0f, ubv = 0.0f, zold = 0.0f;
  double dp0 = 0.0;
  if (valid && g == 0 && w < pt.N) {
    const int64_t vi = pt.vec_base + static_cast<int64_t>(w) * pt.n + j;
    y0 = a.y[vi];
    dp0 = a.dprev[vi];
  }
  if (valid && tid < kXzCols) {
    lbv = a.lb[zi];
    ubv = a.ub[zi];
    zold = a.z[zi];
  }
  // x_s of the wave's scenarios and their sum with y_s / rho
  float x0 = 0.0f;
  double zacc = 0.0;
  const int wu = __builtin_amdgcn_readfirstlane(w);  // the wave's index, as a scalar
  for (int s = wu; s < pt.N; s += kXzWaves) {
    // the scenario's partials (a scalar base) and 32-bit offsets per lane
    const double* xp = f.xpart + (pt.xtile0 + static_cast<int64_t>(s) * ntile) * (2 * kFb);
    // the group's tiles J = g + 4k, twelve loads in flight per lane, added in
    // the order of k
    double acc = 0.0;
    if (valid) {
      for (int J0 = g; J0 < nb; J0 += 48) {
        double q[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          const int J = J0 + 4 * k;
          const int off = J < I ? static_cast<int>(tile_index(J, I, nb)) * (2 * kFb) + kFb + r
                                : static_cast<int>(tile_index(I, J, nb)) * (2 * kFb) + r;
          q[k] = J >= nb ? 0.0 : xp[off];
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) acc += q[k];
      }
    }
    const double xs = swap_sum<32>(swap_sum<16>(acc));
    const float xf = static_cast<float>(xs);
    const int64_t vi = pt.vec_base + static_cast<int64_t>(s) * pt.n + j;
    if (g == 0 && valid) {
      const float yv = s == wu ? y0 : a.y[vi];
      if (!stopped) a.x[vi] = xf;
      zacc += static_cast<double>(xf);
      if (a.prm.z_mode == 0) zacc += static_cast<double>(yv) / rho;
    }
    if (s == wu) x0 = xf;
  }
  if (stopped) return;  // the whole workgroup: one patient
  if (g == 0) sacc[w][c] = zacc;
  __syncthreads();
  // ||dz||^2, ||z||^2, ||d||^2, <dd,d_prev>, ||dd||^2, ||x||^2, <y,d>, ||y||^2
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (tid < kXzCols) {
    float znf = 0.0f;
    if (valid) {
      double sum = 0.0;
      for (int q = 0; q < kXzWaves; ++q) sum += sacc[q][c];
      double zn = sum / pt.N;
      zn = fmin(fmax(zn, static_cast<double>(lbv)), static_cast<double>(ubv));
      znf = static_cast<float>(zn);
      const double dz = static_cast<double>(znf) - static_cast<double>(zold);
      a.z[zi] = znf;
      v[0] = dz * dz;
      v[1] = static_cast<double>(znf) * znf;
    }
    zsh[c] = znf;
  }
  __syncthreads();
  if (valid && g == 0) {
    const double znd = static_cast<double>(zsh[c]);
    for (int s = w; s < pt.N; s += kXzWaves) {
      const int64_t vi = pt.vec_base + static_cast<int64_t>(s) * pt.n + j;
      const double xv = static_cast<double>(s == w ? x0 : a.x[vi]);
      const double yv = static_cast<double>(s == w ? y0 : a.y[vi]);
      const double d = xv - znd;
      const double dp = s == w ? dp0 : a.dprev[vi];
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
  for (int k = 0; k < 8; ++k) v[k] = group_allsum<64>(v[k]);
  if (lane == 0)
    for (int k = 0; k < 8; ++k) sred[w][k] = v[k];
  __syncthreads();
  if (tid < 8) {
    auto q4 = [&](int b) { return (sred[b][tid] + sred[b + 1][tid]) + (sred[b + 2][tid] + sred[b + 3][tid]); };
    a.bpartp[static_cast<int64_t>(bi4) * 8 + tid] = (q4(0) + q4(4)) + (q4(8) + q4(12));
  }
}

// The dual update y_s += tau d_s at one spot (when `update`) and the
// right-hand side c_s = b_s + rho/2 z - y_s/2 of the next x-update there, with
// the roundings written out, so that every launch order that applies them
// gives the same bits.  Returns y_s at the spot.
__device__ __forceinline__ float dual_rhs_at(const VecArgs& a, int64_t vi, bool update, float yv, double dp,
                                             double bv, float zj, double tau, double rho) {
  if (update) {
    yv = static_cast<float>(fma(tau, dp, static_cast<double>(yv)));
    a.y[vi] = yv;
  }
  a.c64[vi] = fma(-0.5, static_cast<double>(yv), fma(0.5 * rho, static_cast<double>(zj), bv));
  return yv;
}

// completion of the pending dual update and the right-hand side
// c_s = b_s + rho/2 z - y_s/2 (one scenario column block of 64 per workgroup)
// one wave: column block bi of one scenario, lane = column within the block
__device__ __forceinline__ void fhead_block(const VecArgs& a, int bi, int lane) {
  const Blk bk = a.blk[bi];
  const Scen sc = a.scen[bk.owner];
  const int j = bk.col0 + lane;
  const bool in = j < sc.n;
  const int64_t vi = sc.vec_base + j;
  // the scenario's vectors are requested beside the patient's entries
  float yv = 0.0f;
  double dp = 0.0, bv = 0.0;
  if (in) {
    yv = a.y[vi];
    dp = a.dprev[vi];
    bv = a.b64[vi];
  }
  const Pat pt = a.pat[sc.patient];
  const PatState* ps = a.ps + sc.patient;
  const float zj = in ? a.z[pt.zvec_base + j] : 0.0f;
  if (ps->stopped) return;
  double yy = 0.0;
  if (in) {
    yv = dual_rhs_at(a, vi, ps->pending != 0, yv, dp, bv, zj, ps->tau, ps->rho);
    yy = static_cast<double>(yv) * yv;
  }
  yy = wave_sum_d(yy);
  if (lane == 0) {
    double* bp = a.bpart + static_cast<int64_t>(bi) * 8;
    bp[0] = 0.0;
    bp[1] = 0.0;
    bp[2] = yy;
  }
}

// The objective tiles read sum_s G_s rounded to 48 bits (sign, exponent and
// the leading 36 of the 52 fraction bits, to nearest): 24 KB a tile instead of
// 32 KB, relative error at most 2^-37 per entry.  Thread t of fobj_tile takes
// the 16 entries e = 0..15 at (row 8 (e / 2) + t / 32, column 2 (t % 32) +
// e % 2) of the tile; their upper 32 bits are four 16-byte words at
// 256 k + t (k = 0..3, entries 4k .. 4k + 3) of the tile's first 16 KB, their
// next 16 bits two 16-byte words at 256 k + t (k = 0..1, entries 8k .. 8k + 7)
// of its last 8 KB, so every wave load reads 1 KiB contiguous.
constexpr int kGqWords = 6144;  // 32-bit words of one tile
__global__ __launch_bounds__(256) void k_gq_pack(const double* __restrict__ Gp, uint32_t* __restrict__ Gq,
                                                 int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < n; idx += stride) {
    const int64_t tile = idx >> 12;
    const int L = static_cast<int>(idx & 4095);  // row-major within the tile: 512 (e / 2) + 2 t + e % 2
    const int t = (L & 511) >> 1, e = 2 * (L >> 9) + (L & 1);
    const unsigned long long r = static_cast<unsigned long long>(__double_as_longlong(Gp[idx])) + 0x8000ull;
    uint32_t* q = Gq + tile * kGqWords;
    q[((e >> 2) * 256 + t) * 4 + (e & 3)] = static_cast<uint32_t>(r >> 32);
    reinterpret_cast<uint16_t*>(q + 4096)[((e >> 3) * 256 + t) * 8 + (e & 7)] =
        static_cast<uint16_t>((r >> 16) & 0xffffu);
  }
}

__device__ __forceinline__ uint32_t word_of(const uint4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// objective partial of one packed tile T of sum_s G_s: z_I^T T z_J, doubled off
// the diagonal; a diagonal tile also carries -g0_I^T z_I.  fp64 arithmetic on
// the 48-bit entries above.  The tile's 24 KB are requested first, from its
// list index alone.
__device__ __forceinline__ void fobj_tile(const FactorArgs& f, const float* __restrict__ z, int jb) {
  __shared__ double zI[kFb], zJ[kFb], red[4];
  const int tid = threadIdx.x;
  const uint4* Q = reinterpret_cast<const uint4*>(f.Gq + static_cast<int64_t>(jb) * kGqWords);
  uint4 hi[4], lo[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) hi[k] = Q[k * 256 + tid];
#pragma unroll
  for (int k = 0; k < 2; ++k) lo[k] = Q[1024 + k * 256 + tid];
  const XJob job = f.fjobs[jb];
  if (f.ps[job.g].stopped) return;
  const Pat pt = f.pat[job.g];
  const int I = job.ij >> 16, J = job.ij & 0xffff;
  if (tid < kFb) {
    const int jc = J * kFb + tid, ic = I * kFb + tid;
    zJ[tid] = jc < pt.n ? static_cast<double>(z[pt.zvec_base + jc]) : 0.0;
    zI[tid] = ic < pt.n ? static_cast<double>(z[pt.zvec_base + ic]) : 0.0;
  }
  __syncthreads();
  auto entry = [&](int e) {
    const uint32_t h = word_of(hi[e >> 2], e & 3);
    const uint32_t l2 = word_of(lo[e >> 3], (e & 7) >> 1);
    const uint32_t l = (e & 1) ? (l2 >> 16) : (l2 & 0xffffu);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h) << 32) |
                                                       (static_cast<unsigned long long>(l) << 16)));
  };
  const int c = 2 * (tid & 31), r0 = tid >> 5;
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) a = fma(zI[8 * k + r0], fma(entry(2 * k), zJ[c], entry(2 * k + 1) * zJ[c + 1]), a);
  double v = (I == J ? 1.0 : 2.0) * a;
  if (I == J && tid < kFb) {
    const int row = I * kFb + tid;
    if (row < pt.n) v -= f.g0[pt.zvec_base + row] * zI[tid];
  }
  v = wave_sum_d(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) f.fpart[jb] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The four-launch dense iteration ends with two launches that each pair one
// scalar workgroup with independent wide work:
//   tail: workgroup 0 the residual norms, tolerances and BB step of every
//         patient (body_scalars_run), the others the objective tiles at the
//         new z;
//   head: workgroup 0 the objective sums and stopping tests
//         (head_scalars_run), the others the dual update y_s += tau d_s and
//         the right-hand sides c_s of the next x-update, gated by dual_go,
//         which the tail set (the stopping test of the same launch does not
//         gate them: as in the six-launch order, the dual update of an
//         iteration precedes its stopping test).
__device__ __forceinline__ void dense_head_block(const VecArgs& a, int bi, int lane) {
  const Blk bk = a.blk[bi];
  const Scen sc = a.scen[bk.owner];
  const int j = bk.col0 + lane;
  const bool in = j < sc.n;
  const int64_t vi = sc.vec_base + j;
  float yv = 0.0f;
  double dp = 0.0, bv = 0.0;
  if (in) {
    yv = a.y[vi];
    dp = a.dprev[vi];
    bv = a.b64[vi];
  }
  const Pat pt = a.pat[sc.patient];
  const PatState* ps = a.ps + sc.patient;
  const float zj = in ? a.z[pt.zvec_base + j] : 0.0f;
  if (!ps->dual_go) return;
  if (in) (void)dual_rhs_at(a, vi, true, yv, dp, bv, zj, ps->tau, ps->rho);
}

// The same update in the launch that forms tau: every wave forms its
// patient's tau itself, from the z-update's partial sums in the order of
// wave_strided_sums and the inputs the last head recorded, which gives the
// bits the scalar workgroup of that launch (body_scalars_run) stores.
__device__ __forceinline__ void dense_dual_block(const VecArgs& a, int bi, int lane) {
  const Blk bk = a.blk[bi];
  const Scen sc = a.scen[bk.owner];
  const int j = bk.col0 + lane;
  const bool in = j < sc.n;
  const int64_t vi = sc.vec_base + j;
  float yv = 0.0f;
  double dp = 0.0, bv = 0.0;
  if (in) {
    yv = a.y[vi];
    dp = a.dprev[vi];
    bv = a.b64[vi];
  }
  const Pat pt = a.pat[sc.patient];
  const PatState* ps = a.ps + sc.patient;
  const float zj = in ? a.z[pt.zvec_base + j] : 0.0f;
  const int stopped = ps->stopped;
  const double rho = ps->rho, tau0 = ps->bb_tau0;
  const int it0 = ps->bb_iter0;
  double v[2];
  wave_strided_sums<2>(a.bpartp + static_cast<int64_t>(4 * pt.blk_begin) * 8, 4 * pt.nblk, 3, v);
  if (stopped) return;
  const double tau = bb_dual_step(a.prm, rho, tau0, it0, v[0], v[1]);
  if (in) (void)dual_rhs_at(a, vi, true, yv, dp, bv, zj, tau, rho);
}

__global__ __launch_bounds__(256) void k_dense_tail(FactorArgs f, VecArgs a, int nfobj) {
  const int b = static_cast<int>(blockIdx.x);
  if (b == 0) {
    body_scalars_run<true>(a);
    return;
  }
  if (b - 1 < nfobj) fobj_tile(f, a.z, b - 1);
}

__global__ __launch_bounds__(256) void k_dense_head(VecArgs a, int nblk) {
  const int b = static_cast<int>(blockIdx.x);
  if (b == 0) {
    head_scalars_run<true>(a, 0, 0);
    return;
  }
  const int bi = 4 * (b - 1) + static_cast<int>(threadIdx.x >> 6);
  if (bi < nblk) dense_head_block(a, bi, threadIdx.x & 63);
}

// The three-launch dense iteration (the reduction and the z-update between them):
//   x:    workgroup 0 the objective sums and stopping test of the previous
//         iteration (head_scalars_run), the others the x-update tiles.  The
//         tiles read the stop flag that workgroup 0 may be setting: a tile of
//         a patient that stops there writes partial sums that nothing reads
//         (the reduction and the z-update read the flag after the launch),
//         and none writes the iteration count that orders the tiles;
//   tail: workgroup 0 the residual norms, tolerances and dual step
//         (body_scalars_run), then the dual update with the next right-hand
//         sides (each wave forms tau itself, dense_dual_block), then the
//         objective tiles at the new z.
// Every value equals the four-launch order's; the stopping test of the last
// iteration of a run follows in a launch of its own.
template <bool kLoadsFirst>
__global__ __launch_bounds__(256) void k_dense_x(FactorArgs f, VecArgs a, const double* __restrict__ c) {
  if (blockIdx.x == 0) {
    head_scalars_run<true>(a, 0, 0);
    return;
  }
  xsym_tile<kLoadsFirst>(f, c, xsym_order(f, static_cast<int>(blockIdx.x) - 1));
}

__global__ __launch_bounds__(256) void k_dense_tail_dual(FactorArgs f, VecArgs a, int nfobj, int nblk) {
  const int b = static_cast<int>(blockIdx.x);
  if (b == 0) {
    body_scalars_run<true>(a);
    return;
  }
  const int ndual = (nblk + 3) / 4;
  if (b - 1 < ndual) {
    const int bi = 4 * (b - 1) + static_cast<int>(threadIdx.x >> 6);
    if (bi < nblk) dense_dual_block(a, bi, threadIdx.x & 63);
    return;
  }
  if (b - 1 - ndual < nfobj) fobj_tile(f, a.z, b - 1 - ndual);
}

// The head of a dense iteration in one launch: workgroups [0, nfobj) take the
// objective tiles, the rest four column blocks each of the pending dual update
// and right-hand sides (the two parts are independent).
__global__ __launch_bounds__(256) void k_fheadobj(FactorArgs f, VecArgs a, int nfobj, int nblk) {
  const int b = static_cast<int>(blockIdx.x);
  if (b < nfobj) {
    fobj_tile(f, a.z, b);
    return;
  }
  const int bi = 4 * (b - nfobj) + static_cast<int>(threadIdx.x >> 6);
  if (bi < nblk) fhead_block(a, bi, threadIdx.x & 63);
}

}  // namespace

void launch_gram(const MatDev& m, const double* rw64, const Scen& sc, double* G, int ld, hipStream_t st) {
  if (sc.rows <= 0) return;
  const unsigned nb = static_cast<unsigned>((sc.rows + 3) / 4);
  if (m.col16)
    hipLaunchKernelGGL(k_gram<true>, dim3(nb), dim3(256), 0, st, m, rw64, sc, G, ld);
  else
    hipLaunchKernelGGL(k_gram<false>, dim3(nb), dim3(256), 0, st, m, rw64, sc, G, ld);
}

void launch_gram_rows(const MatDev& m, const Scen& sc, int nb, int32_t* cnt, const int64_t* off, GramEntry* list,
                      hipStream_t st) {
  if (sc.rows <= 0) return;
  const unsigned g = static_cast<unsigned>((sc.rows + 3) / 4);
  if (m.col16) {
    if (list)
      hipLaunchKernelGGL((k_gram_rows<true, true>), dim3(g), dim3(256), 0, st, m, sc, nb, cnt, off, list);
    else
      hipLaunchKernelGGL((k_gram_rows<true, false>), dim3(g), dim3(256), 0, st, m, sc, nb, cnt, off, list);
  } else {
    if (list)
      hipLaunchKernelGGL((k_gram_rows<false, true>), dim3(g), dim3(256), 0, st, m, sc, nb, cnt, off, list);
    else
      hipLaunchKernelGGL((k_gram_rows<false, false>), dim3(g), dim3(256), 0, st, m, sc, nb, cnt, off, list);
  }
}

void launch_gram_scan(const int32_t* cnt, int64_t nt, int64_t* off, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_scan, dim3(1), dim3(1024), 0, st, cnt, nt, off);
}

void launch_gram_tiles(const MatDev& m, const double* rw64, const Scen* scen, int g0, int nscen, int nb,
                       const int64_t* off, const GramEntry* list, const double* gscale, double* G, int ld,
                       hipStream_t st) {
  const unsigned nt = static_cast<unsigned>(static_cast<int64_t>(nb) * (nb + 1) / 2);
  const dim3 grid(nt, static_cast<unsigned>(nscen)), block(64 * kGramWaves);
  if (m.col16)
    hipLaunchKernelGGL(k_gram_tiles<true>, grid, block, 0, st, m, rw64, scen, g0, nb, off, list, gscale, G, ld);
  else
    hipLaunchKernelGGL(k_gram_tiles<false>, grid, block, 0, st, m, rw64, scen, g0, nb, off, list, gscale, G, ld);
}

void launch_gram_finish(FactorArgs f, int patient, int scen_begin, int nscen, int npad, int n, double rho,
                        int accumulate_gsum, hipStream_t st) {
  int64_t nb = (static_cast<int64_t>(npad) * npad + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_gram_finish, dim3(static_cast<unsigned>(nb)), dim3(256), 0, st, f, patient, scen_begin,
                     nscen, npad, n, rho, accumulate_gsum);
}

void launch_sweep_step(FactorArgs f, int scen_begin, int nscen, int npad, int k0, hipStream_t st) {
  const int nbk = npad / kFb;
  hipLaunchKernelGGL(k_sweep_pivot, dim3(nscen), dim3(256), 0, st, f, scen_begin, npad, k0);
  hipLaunchKernelGGL(k_sweep_panel, dim3(nbk, nscen), dim3(256), 0, st, f, scen_begin, npad, k0);
  hipLaunchKernelGGL(k_sweep_update, dim3(nbk * (nbk + 1) / 2, nscen), dim3(256), 0, st, f, scen_begin, npad, k0);
}

void launch_gq_pack(const double* Gp, uint32_t* Gq, int64_t ntiles, hipStream_t st) {
  if (ntiles <= 0) return;
  const int64_t n = ntiles * 4096;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(k_gq_pack, dim3(grid), dim3(256), 0, st, Gp, Gq, n);
}

void launch_sweep_store(FactorArgs f, int patient, int scen_begin, int nscen, int npad, hipStream_t st) {
  int64_t nb = (static_cast<int64_t>(npad) * npad + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_sweep_store, dim3(static_cast<unsigned>(nb), nscen), dim3(256), 0, st, f, patient,
                     scen_begin, npad);
}

void launch_xsym(const FactorArgs& f, const double* c, int njobs, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (njobs <= 0) return;
  const int grid = njobs;
  auto kern = f.npat == 1 ? k_xsym<true> : k_xsym<false>;
  if (e0 != nullptr)
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, e0, e1, 0, f, c);
  else
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, f, c);
}

void launch_xzres(const FactorArgs& f, const VecArgs& a, int npblk, hipStream_t st) {
  if (npblk <= 0) return;
  hipLaunchKernelGGL(k_xzres, dim3(static_cast<unsigned>(4 * npblk)), dim3(64 * kXzWaves), 0, st, f, a);
}

void launch_dense_tail(const FactorArgs& f, const VecArgs& a, int nfobj, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_tail, dim3(1 + nfobj), dim3(256), 0, st, f, a, nfobj);
}

void launch_dense_head(const VecArgs& a, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_head, dim3(1 + (nblk + 3) / 4), dim3(256), 0, st, a, nblk);
}

void launch_dense_x(const FactorArgs& f, const VecArgs& a, const double* c, int njobs, hipStream_t st, hipEvent_t e0,
                    hipEvent_t e1) {
  const dim3 grid(static_cast<unsigned>(1 + njobs));
  auto kern = f.npat == 1 ? k_dense_x<true> : k_dense_x<false>;
  if (e0 != nullptr)
    hipExtLaunchKernelGGL(kern, grid, dim3(256), 0, st, e0, e1, 0, f, a, c);
  else
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, f, a, c);
}

void launch_dense_tail_dual(const FactorArgs& f, const VecArgs& a, int nfobj, int nblk, hipStream_t st) {
  const int grid = 1 + (nblk + 3) / 4 + nfobj;
  hipLaunchKernelGGL(k_dense_tail_dual, dim3(static_cast<unsigned>(grid)), dim3(256), 0, st, f, a, nfobj, nblk);
}

void launch_fheadobj(const FactorArgs& f, const VecArgs& a, int nfobj, int nblk, hipStream_t st) {
  const int grid = nfobj + (nblk + 3) / 4;
  if (grid <= 0) return;
  hipLaunchKernelGGL(k_fheadobj, dim3(grid), dim3(256), 0, st, f, a, nfobj, nblk);
}

}  // namespace admmbb
