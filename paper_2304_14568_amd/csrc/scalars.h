// Device-side reductions and the per-patient scalar steps of an ADMM-BB
// iteration (objective sum and stopping test; residual norms, tolerances and
// the Barzilai-Borwein dual step), shared by the launch sequences of the CG
// and the dense x-updates.  Every sum is in a fixed order.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace admmbb {

// Lane exchanges inside a row of 16 lanes by DPP moves (vector ALU, no LDS):
// pairs (kDppXor1), pairs of pairs (kDppXor2), lane 7 - i of each half-row
// (kDppHalfMirror) and lane 15 - i of the row (kDppMirror).
constexpr int kDppXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
template <int kCtrl>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), kCtrl, 0xF, 0xF, false));
}
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(v), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(v >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// x[l] + x[l ^ 16] (k = 16) or x[l] + x[l ^ 32] (k = 32) in every lane, by the
// gfx950 lane swaps: v_permlane16_swap of (x, x) leaves rows 0 and 2 of x in
// the first result and rows 1 and 3 in the second, each beside its partner
// row, and v_permlane32_swap the lower and the upper half likewise; both
// partners add the same two operands in the same order.
template <int k>
__device__ __forceinline__ void lane_swap(uint32_t u, uint32_t& first, uint32_t& second) {
  static_assert(k == 16 || k == 32, "rows or half-waves");
  if constexpr (k == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    first = r[0];
    second = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    first = r[0];
    second = r[1];
  }
}
template <int k>
__device__ __forceinline__ float swap_sum(float x) {
  uint32_t a = 0, b = 0;
  lane_swap<k>(__float_as_uint(x), a, b);
  return __uint_as_float(a) + __uint_as_float(b);
}
template <int k>
__device__ __forceinline__ double swap_sum(double x) {
  const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(x));
  uint32_t la = 0, lb = 0, ha = 0, hb = 0;
  lane_swap<k>(static_cast<uint32_t>(u), la, lb);
  lane_swap<k>(static_cast<uint32_t>(u >> 32), ha, hb);
  const double a = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(ha) << 32) | la));
  const double b = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hb) << 32) | lb));
  return a + b;
}

// Sum over aligned groups of L lanes (L a power of two, at most 64; every lane
// of a group active), every lane of a group getting the same bits: at each
// step the two partners add the same two values.  Pairs and quads exchange by
// DPP; after that every lane of a quad holds the quad's sum, so the mirror of
// a half-row pairs whole quads and the mirror of a row whole half-rows; rows
// and half-waves by the lane swaps above.  All on the vector ALU, in a fixed
// order: the same inputs give the same bits.
template <int L, class T>
__device__ __forceinline__ T group_allsum(T x) {
  static_assert(L >= 1 && L <= 64 && (L & (L - 1)) == 0, "L a power of two up to 64");
  if constexpr (L >= 2) x += dpp_move<kDppXor1>(x);
  if constexpr (L >= 4) x += dpp_move<kDppXor2>(x);
  if constexpr (L >= 8) x += dpp_move<kDppHalfMirror>(x);
  if constexpr (L >= 16) x += dpp_move<kDppMirror>(x);
  if constexpr (L >= 32) x = swap_sum<16>(x);
  if constexpr (L >= 64) x = swap_sum<32>(x);
  return x;
}

// Sum over the wave; every lane returns it.
__device__ __forceinline__ double wave_sum(double x) { return group_allsum<64>(x); }

// Sum of p[b * 8] for b < count by one wave: lane l adds entries l, l+64, ...
// then group_allsum; every lane returns the same total.
__device__ __forceinline__ double wave_strided_sum(const double* p, int count) {
  double s = 0.0;
  for (int b = threadIdx.x & 63; b < count; b += 64) s += p[static_cast<int64_t>(b) * 8];
  return group_allsum<64>(s);
}

// NV interleaved sums by one wave: v[k] = sum over b < count of p[b * 8 + k0 + k],
// lane l adding entries l, l + 64, ... in order, then group_allsum; every
// lane returns the totals.  Any subset of k gives the same bits for its sums.
template <int NV>
__device__ __forceinline__ void wave_strided_sums(const double* p, int count, int k0, double (&v)[NV]) {
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (int b = threadIdx.x & 63; b < count; b += 64) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += p[static_cast<int64_t>(b) * 8 + k0 + k];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = group_allsum<64>(v[k]);
}

// Dual step of Sec. 2.2: the Barzilai-Borwein value beta = -<dd, dy> / ||dd||^2
// when it is positive and finite (after the first iteration), else rho, then
// the optional clamp.  dy = y^k - y^{k-1} = tau_{k-1} d^k, so <dd, dy> =
// tau_{k-1} <dd, d^k> with <dd, d^k> = dd_dp and ||dd||^2 = dd2.
__device__ __forceinline__ double bb_dual_step(const AlgoParams& P, double rho, double tau0, int iter0, double dd_dp,
                                               double dd2) {
  double tau = rho;
  if (P.bb && iter0 >= 1 && dd2 > 0.0) {
    const double beta = -tau0 * dd_dp / dd2;
    if (isfinite(beta) && beta > 0.0) tau = beta;
  }
  if (P.bb_clamp > 0.0) tau = fmin(fmax(tau, rho / P.bb_clamp), rho * P.bb_clamp);
  return tau;
}

// Deterministic block sum of NV doubles over NT threads; result valid in thread 0.
template <int NV, int NT = kThreads>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh) {
  constexpr int NW = NT / 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wave * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double acc = 0.0;
      for (int w = 0; w < NW; ++w) acc += sh[w * NV + k];
      v[k] = acc;
    }
  }
  __syncthreads();
}

// Block sum of a strided list: thread i adds items i, i+256, ... in order,
// then a fixed tree.  Deterministic for a given count.
template <class F>
__device__ __forceinline__ double block_list_sum(int count, F item, double* sh) {
  double v[1] = {0.0};
  // four independent loads in flight, added in the same order as one at a time
  int i = threadIdx.x;
  for (; i + 3 * kThreads < count; i += 4 * kThreads) {
    const double e0 = item(i), e1 = item(i + kThreads), e2 = item(i + 2 * kThreads), e3 = item(i + 3 * kThreads);
    v[0] += e0;
    v[0] += e1;
    v[0] += e2;
    v[0] += e3;
  }
  for (; i < count; i += kThreads) v[0] += item(i);
  block_sum<1>(v, sh);
  return v[0];
}

// Two strided lists at once, so that their loads overlap; each is added in
// the order block_list_sum uses, and block_sum reduces the two independently,
// so either result equals its own block_list_sum.  Valid in thread 0.
template <class F1, class F2>
__device__ __forceinline__ void block_list_sum2(int n1, F1 item1, int n2, F2 item2, double* sh, double& s1,
                                                double& s2) {
  double v[2] = {0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 3 * kThreads < n1; i += 4 * kThreads) {
    const double e0 = item1(i), e1 = item1(i + kThreads), e2 = item1(i + 2 * kThreads), e3 = item1(i + 3 * kThreads);
    v[0] += e0;
    v[0] += e1;
    v[0] += e2;
    v[0] += e3;
  }
  for (; i < n1; i += kThreads) v[0] += item1(i);
  i = threadIdx.x;
  for (; i + 3 * kThreads < n2; i += 4 * kThreads) {
    const double e0 = item2(i), e1 = item2(i + kThreads), e2 = item2(i + 2 * kThreads), e3 = item2(i + 3 * kThreads);
    v[1] += e0;
    v[1] += e1;
    v[1] += e2;
    v[1] += e3;
  }
  for (; i < n2; i += kThreads) v[1] += item2(i);
  block_sum<2>(v, sh);
  s1 = v[0];
  s2 = v[1];
}

// Objective at z, completion of the previous iteration (dual tolerance, trace
// record, stopping test) and, with cg_setup, the CG set-up; one workgroup of
// kThreads threads.  DENSE: the dual tolerance was already formed by
// body_scalars_run from the updated duals' norm, and no CG set-up follows.
template <bool DENSE>
__device__ __forceinline__ void head_scalars_run(const VecArgs& a, int nscen, int cg_setup) {
  __shared__ double sh[4 * 2];
  const AlgoParams& P = a.prm;
  for (int p = 0; p < P.num_pat; ++p) {
    const Pat pt = a.pat[p];
    PatState* ps = a.ps + p;
    const int stopped = ps->stopped;  // read beside the partial sums
    // objective partials and the blocks' sums of squares of y, loaded together
    const int sb0 = pt.sblk_begin;
    auto yitem = [&](int i) { return a.bpart[(int64_t)(sb0 + i) * 8 + 2]; };
    double fs = 0.0, yy = 0.0;
    if (a.fpart != nullptr)
      block_list_sum2(pt.fobj_end - pt.fobj_begin, [&](int i) { return a.fpart[pt.fobj_begin + i]; },
                      DENSE ? 0 : pt.sblk_end - sb0, yitem, sh, fs, yy);
    else
      block_list_sum2(pt.tile_end - pt.tile_begin, [&](int i) { return a.objpart[pt.tile_begin + i]; },
                      pt.sblk_end - sb0, yitem, sh, fs, yy);
    if (stopped) continue;  // uniform
    const double f = (a.fpart != nullptr ? pt.fconst : pt.fzero) + fs;
    if (threadIdx.x == 0) {
      ps->f_cur = f;
      if (ps->pending) {
        const int N = pt.num_scen;
        if constexpr (!DENSE) {
          const double base = P.eps_abs * sqrt(static_cast<double>(N) * pt.n);
          ps->eps_dual = base + P.eps_rel * sqrt(yy);
        }
        const int k = ps->iter;  // iterations completed, >= 1
        if (a.trace != nullptr && k - 1 < P.trace_cap) {
          IterRecord rec;
          rec.iter = k;
          rec.cg_steps = ps->cg_steps;
          rec.obj = f;
          rec.r_prim = ps->r_prim;
          rec.r_dual = ps->r_dual;
          rec.eps_prim = ps->eps_prim;
          rec.eps_dual = ps->eps_dual;
          rec.tau = ps->tau;
          a.trace[static_cast<int64_t>(p) * P.trace_cap + (k - 1)] = rec;
        }
        if (!isfinite(f) || !isfinite(ps->r_prim)) {
          ps->stopped = 1;
          ps->status = 2;
        } else if (P.stop_enabled) {
          bool obj_ok = true;
          if (P.obj_rel_tol > 0.0) obj_ok = (k >= 2) && fabs(f - ps->f_prev) <= P.obj_rel_tol * fabs(ps->f_prev);
          if (ps->r_prim <= ps->eps_prim && ps->r_dual <= ps->eps_dual && obj_ok) {
            ps->stopped = 1;
            ps->status = 1;
          }
        }
        ps->pending = 0;
      }
      ps->f_prev = f;
      // inputs of the next dual step, stable while the launch that forms it
      // runs (the dense x-update forms it in several workgroups at once)
      ps->bb_tau0 = ps->tau;
      ps->bb_iter0 = ps->iter;
    }
    __syncthreads();
  }
  if (DENSE || !cg_setup) return;
  // per-scenario CG set-up: one thread per scenario, fixed-order sums over its blocks
  for (int g = threadIdx.x; g < nscen; g += kThreads) {
    const Scen sc = a.scen[g];
    const PatState* ps = a.ps + sc.patient;
    double rz0 = 0.0, cc = 0.0;
    for (int b = 0; b < sc.nblk; ++b) {
      rz0 += a.bpart[(int64_t)(sc.blk_begin + b) * 8 + 0];
      cc += a.bpart[(int64_t)(sc.blk_begin + b) * 8 + 1];
    }
    double eta = P.eta_factor;
    if (ps->iter > 0) {
      const double rel = ps->r_prim / fmax(ps->xnorm, 1e-30);
      eta = fmax(P.eta_floor, P.eta_factor * fmin(1.0, rel));
    }
    const double tol2 = eta * eta * cc;
    a.tol2[g] = tol2;
    a.rz[g * kRing + 0] = rz0;
    a.act[g * kRing + 0] = (!ps->stopped && rz0 > tol2 && rz0 > 0.0) ? 1 : 0;
    a.cgcount[g] = 0;
  }
}

// Residual norms, tolerances and the Barzilai-Borwein dual step per patient,
// from the z-update's partial sums; one workgroup of kThreads threads.
// DENSE: the partial sums are added by wave 0 in the order of
// wave_strided_sums, and the step from the inputs the last head recorded
// (bb_tau0, bb_iter0), so that a workgroup that forms the same step in the
// same launch gets the same bits; also the dual tolerance, from the norm of
// the duals after the update y + tau d (||y||^2 + 2 tau <y, d> + tau^2 ||d||^2
// from the same partial sums), and the flag dual_go for a launch that applies
// that update after this one (0 for a patient that has stopped).
template <bool DENSE>
__device__ __forceinline__ void body_scalars_run(const VecArgs& a) {
  __shared__ double sh[4 * 8];
  const AlgoParams& P = a.prm;
  for (int p = 0; p < P.num_pat; ++p) {
    const Pat pt = a.pat[p];
    PatState* ps = a.ps + p;
    const int stopped = ps->stopped;  // read beside the partial sums
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if constexpr (DENSE) {
      if (threadIdx.x < 64) wave_strided_sums<8>(a.bpartp + (int64_t)(4 * pt.blk_begin) * 8, 4 * pt.nblk, 0, v);
    } else {
      for (int b = threadIdx.x; b < 4 * pt.nblk; b += kThreads)
        for (int k = 0; k < 6; ++k) v[k] += a.bpartp[(int64_t)(4 * pt.blk_begin + b) * 8 + k];
    }
    // thread 0's inputs from the patient's state, requested before the reduction
    int cg = 0, iter0 = 0, cgt0 = 0, itb = 0;
    double rho = 0.0, tau0 = 0.0;
    if (threadIdx.x == 0) {
      for (int s = 0; s < pt.num_scen; ++s) cg += a.cgcount[pt.scen_begin + s];
      rho = ps->rho;
      tau0 = DENSE ? ps->bb_tau0 : ps->tau;
      itb = DENSE ? ps->bb_iter0 : ps->iter;
      iter0 = ps->iter;
      cgt0 = ps->cg_total;
    }
    if (stopped) {  // uniform
      if (DENSE && threadIdx.x == 0) ps->dual_go = 0;
      continue;
    }
    if constexpr (!DENSE) block_sum<8>(v, sh);
    if (threadIdx.x == 0) {
      const int N = pt.num_scen;
      const double rp = sqrt(v[2]);
      const double rd = sqrt(static_cast<double>(N)) * rho * sqrt(v[0]);
      const double tau = bb_dual_step(P, rho, tau0, itb, v[3], v[4]);
      const double base = P.eps_abs * sqrt(static_cast<double>(N) * pt.n);
      ps->xnorm = sqrt(v[5]);
      ps->znorm = sqrt(v[1]);
      ps->eps_prim = base + P.eps_rel * fmax(ps->xnorm, sqrt(static_cast<double>(N)) * ps->znorm);
      ps->r_prim = rp;
      ps->r_dual = rd;
      ps->tau = tau;
      ps->cg_steps = cg;
      ps->cg_total = cgt0 + cg;
      ps->iter = iter0 + 1;
      ps->pending = 1;
      if constexpr (DENSE) {
        const double yy = fmax(0.0, v[7] + 2.0 * tau * v[6] + tau * tau * v[2]);
        ps->eps_dual = base + P.eps_rel * sqrt(yy);
        ps->dual_go = 1;
      }
    }
    __syncthreads();
  }
}

}  // namespace admmbb
