// Host-side validation of admm_problem (no device calls; usable without a GPU).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/admmbb.h"
#include "host.h"

namespace admmbb {

static admm_status fail(std::string* msg, admm_status st, const char* fmt, long long a = 0, long long b = 0,
                        long long c = 0) {
  if (msg) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), fmt, a, b, c);
    *msg = buf;
  }
  return st;
}

admm_status validate_problem(const admm_problem* p, std::string* msg) {
  if (!p) return fail(msg, ADMM_E_ARG, "problem is NULL");
  if (p->mem_kind != ADMM_MEM_HOST && p->mem_kind != ADMM_MEM_DEVICE)
    return fail(msg, ADMM_E_ARG, "mem_kind=%lld is neither ADMM_MEM_HOST nor ADMM_MEM_DEVICE", p->mem_kind);
  if (p->mem_kind == ADMM_MEM_DEVICE)
    return fail(msg, ADMM_E_ARG, "device-resident CSR arrays are staged to the host by admm_setup first");
  if (p->m <= 0 || p->n <= 0 || p->num_scen <= 0)
    return fail(msg, ADMM_E_ARG, "sizes must be positive (m=%lld n=%lld num_scen=%lld)", p->m, p->n, p->num_scen);
  if (p->n > 1 << 24) return fail(msg, ADMM_E_ARG, "n=%lld exceeds the supported 2^24 spots", p->n);
  if (!p->A || !p->struct_id || !p->struct_weight || !p->presc)
    return fail(msg, ADMM_E_ARG, "NULL array in problem (A, struct_id, struct_weight or presc)");
  if (p->num_struct <= 0 || p->num_struct > 256) return fail(msg, ADMM_E_ARG, "num_struct=%lld not in 1..256", p->num_struct);
  for (int k = 0; k < p->num_struct; ++k) {
    const double w = p->struct_weight[k];
    if (!std::isfinite(w)) return fail(msg, ADMM_E_NONFINITE, "struct_weight[%lld] is not finite", k);
    if (w < 0) return fail(msg, ADMM_E_NEGATIVE, "struct_weight[%lld] < 0", k);
  }
  for (int i = 0; i < p->m; ++i) {
    if (p->struct_id[i] >= p->num_struct)
      return fail(msg, ADMM_E_ARG, "struct_id[%lld]=%lld >= num_struct", i, p->struct_id[i]);
    const double v = p->presc[i];
    if (!std::isfinite(v)) return fail(msg, ADMM_E_NONFINITE, "presc[%lld] is not finite", i);
    if (v < 0) return fail(msg, ADMM_E_NEGATIVE, "presc[%lld] < 0", i);
  }
  for (int j = 0; j < p->n; ++j) {
    const double lo = p->lb ? p->lb[j] : 0.0;
    const double hi = p->ub ? p->ub[j] : INFINITY;
    if (std::isnan(lo) || std::isnan(hi) || std::isinf(lo))
      return fail(msg, ADMM_E_NONFINITE, "bound of spot %lld is NaN or lb is infinite", j);
    if (lo > hi) return fail(msg, ADMM_E_ARG, "lb > ub at spot %lld", j);
  }
  // scenarios are checked by parallel host threads; the first failing
  // scenario in index order decides the status and message
  const int N = p->num_scen;
  std::vector<admm_status> st(N, ADMM_OK);
  std::vector<std::string> ms(N);
  auto check_scen = [&](int s) -> admm_status {
    std::string* msg1 = &ms[s];
    const admm_csr& A = p->A[s];
    if (!A.row_ptr || (A.nnz > 0 && (!A.col || !A.val)))
      return fail(msg1, ADMM_E_ARG, "scenario %lld: NULL CSR array", s);
    if (A.nnz < 0 || A.nnz > (int64_t)0xFFFFFFFFLL)
      return fail(msg1, ADMM_E_CSR, "scenario %lld: nnz=%lld outside 0..2^32-1", s, A.nnz);
    if (!std::isfinite(A.prob)) return fail(msg1, ADMM_E_NONFINITE, "scenario %lld: probability not finite", s);
    if (A.prob < 0) return fail(msg1, ADMM_E_NEGATIVE, "scenario %lld: probability < 0", s);
    if (A.row_ptr[0] != 0) return fail(msg1, ADMM_E_CSR, "scenario %lld: row_ptr[0] != 0", s);
    if (A.row_ptr[p->m] != A.nnz)
      return fail(msg1, ADMM_E_CSR, "scenario %lld: row_ptr[m]=%lld != nnz=%lld", s, A.row_ptr[p->m], A.nnz);
    for (int i = 0; i < p->m; ++i) {
      const int64_t b = A.row_ptr[i], e = A.row_ptr[i + 1];
      if (e < b) return fail(msg1, ADMM_E_CSR, "scenario %lld: row_ptr decreases at row %lld", s, i);
      if (e - b > p->n) return fail(msg1, ADMM_E_CSR, "scenario %lld: row %lld has more than n entries", s, i);
      int32_t prev = -1;
      for (int64_t k = b; k < e; ++k) {
        const int32_t c = A.col[k];
        if (c < 0 || c >= p->n)
          return fail(msg1, ADMM_E_CSR, "scenario %lld: column %lld out of range at row %lld", s, c, i);
        if (c <= prev) return fail(msg1, ADMM_E_CSR, "scenario %lld: columns not increasing in row %lld", s, i);
        prev = c;
        const float v = A.val[k];
        if (!std::isfinite(v)) return fail(msg1, ADMM_E_NONFINITE, "scenario %lld: non-finite value at row %lld", s, i);
        if (v < 0) return fail(msg1, ADMM_E_NEGATIVE, "scenario %lld: negative value at row %lld", s, i);
      }
    }
    return ADMM_OK;
  };
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nt = static_cast<int>(std::min<unsigned>(hw, static_cast<unsigned>(N)));
  std::atomic<int> next{0};
  auto worker = [&]() {
    for (int s = next++; s < N; s = next++) {
      try {
        st[s] = check_scen(s);
      } catch (...) {  // nothing may leave a worker thread
        st[s] = ADMM_E_OOM;
        ms[s] = "host allocation failed while validating";
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) {
    try {
      th.emplace_back(worker);
    } catch (const std::system_error&) {
      break;  // fewer threads: the calling thread checks the remaining scenarios
    }
  }
  worker();
  for (auto& t : th) t.join();
  for (int s = 0; s < N; ++s)
    if (st[s] != ADMM_OK) {
      if (msg) *msg = ms[s];
      return st[s];
    }
  return ADMM_OK;
}

admm_status validate_options(const admm_options* o, std::string* msg) {
  if (!o) return ADMM_OK;
  if (!(o->eps_abs >= 0) || !(o->eps_rel >= 0) || !(o->obj_rel_tol >= 0) || !(o->bb_clamp >= 0) ||
      !std::isfinite(o->rho))
    return fail(msg, ADMM_E_ARG, "tolerances, bb_clamp must be >= 0 and rho finite");
  if (o->max_iter < 0) return fail(msg, ADMM_E_ARG, "max_iter < 0");
  if (o->cg_max < 1 || o->cg_max > kMaxCg) return fail(msg, ADMM_E_ARG, "cg_max=%lld not in 1..64", o->cg_max);
  if (!(o->cg_eta >= 0) || !(o->cg_eta_floor >= 0)) return fail(msg, ADMM_E_ARG, "cg_eta must be >= 0");
  if (o->precision < ADMM_PREC_FP32 || o->precision > ADMM_PREC_FP16)
    return fail(msg, ADMM_E_ARG, "unknown precision %lld", o->precision);
  if (o->z_mode < 0 || o->z_mode > 1) return fail(msg, ADMM_E_ARG, "z_mode must be 0 or 1");
  if (o->check_every < 1) return fail(msg, ADMM_E_ARG, "check_every must be >= 1");
  if (o->lds_acc < -1 || o->lds_acc > 2) return fail(msg, ADMM_E_ARG, "lds_acc must be -1, 0, 1 or 2");
  if (o->tile_nnz < 0) return fail(msg, ADMM_E_ARG, "tile_nnz < 0");
  if (o->pass_threads != 0 && o->pass_threads != 256 && o->pass_threads != 512 && o->pass_threads != 1024)
    return fail(msg, ADMM_E_ARG, "pass_threads must be 0, 256, 512 or 1024");
  if (o->pass_threads == 1024 && o->format == 1)
    return fail(msg, ADMM_E_ARG, "the sliced layout has no 1024-thread pass (pass_threads 0, 256 or 512)");
  if (o->pass_unroll != 0 && o->pass_unroll != 1 && o->pass_unroll != 2)
    return fail(msg, ADMM_E_ARG, "pass_unroll must be 0, 1 or 2");
  if (o->format < -1 || o->format > 1) return fail(msg, ADMM_E_ARG, "format must be -1, 0 or 1");
  if (o->deterministic != 0 && o->deterministic != 1) return fail(msg, ADMM_E_ARG, "deterministic must be 0 or 1");
  if (o->deterministic && o->lds_acc >= 0 && o->lds_acc != 2)
    return fail(msg, ADMM_E_ARG, "deterministic needs lds_acc -1 or 2 (64-bit fixed-point column sums)");
  if (o->xupdate < -1 || o->xupdate > 1) return fail(msg, ADMM_E_ARG, "xupdate must be -1, 0 or 1");
  if (o->dense_launches != 3 && o->dense_launches != 4) return fail(msg, ADMM_E_ARG, "dense_launches must be 3 or 4");
  return ADMM_OK;
}

}  // namespace admmbb
