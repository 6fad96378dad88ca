// Host packing: validated CSR inputs -> length-sorted CSR tiles for the fused
// pass, plus the per-scenario constants the iteration needs.
//
// Rows of each A_s are reordered by decreasing length (zero rows dropped).
// The fused pass never has to write a voxel-indexed vector, so the order of
// rows is free; sorting lets each workgroup tile use one lanes-per-row width
// that keeps a row's nonzeros in registers (at most kRegChunks per lane),
// and makes neighbouring rows of a tile equally long.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"

namespace admmbb {

uint16_t to_bf16_bits(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>(u >> 16);  // inf / nan
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<uint16_t>(u >> 16);
}

uint16_t to_f16_bits(float v) {
  _Float16 h = static_cast<_Float16>(v);
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

// lanes per row for a row of `chunks` 4-element chunks: each lane holds up to
// kRegChunks chunks in registers
static int lanes_for(int64_t chunks) {
  int L = 1;
  while (L < 64 && static_cast<int64_t>(L) * kRegChunks < chunks) L <<= 1;
  return L;
}

admm_status pack_problems(const admm_problem* probs, int num_patients, const admm_options& o, Packed* out,
                          std::string* msg) {
  Packed& P = *out;
  int64_t nnz_all = 0;
  for (int p = 0; p < num_patients; ++p)
    for (int s = 0; s < probs[p].num_scen; ++s) nnz_all += probs[p].A[s].nnz;
  int64_t tile_nnz = o.tile_nnz > 0 ? o.tile_nnz : nnz_all / (256 * 8);
  tile_nnz = std::max<int64_t>(8192, std::min<int64_t>(tile_nnz, 1 << 22));
  const int64_t tile_chunks = std::max<int64_t>(1, tile_nnz / 4);

  P.col16_used = true;
  for (int p = 0; p < num_patients; ++p) {
    P.nmax = std::max(P.nmax, probs[p].n);
    P.mmax = std::max(P.mmax, probs[p].m);
    if (probs[p].n > 65535) P.col16_used = false;
  }
  const bool lp = o.precision != ADMM_PREC_FP32;
  try {
    const size_t cap = static_cast<size_t>(nnz_all + nnz_all / 16 + 1024);
    P.val.reserve(cap);
    if (P.col16_used)
      P.col16.reserve(cap);
    else
      P.col32.reserve(cap);
    if (lp) P.val_lp.reserve(cap);
  } catch (const std::bad_alloc&) {
    if (msg) *msg = "host allocation failed while packing";
    return ADMM_E_OOM;
  }

  int64_t nnz_base = 0, row_base = 0, rp_base = 0;
  int blk_s = 0, blk_p = 0;
  P.g0.resize(num_patients);
  P.gdiag_mean.resize(num_patients);
  try {
    for (int p = 0; p < num_patients; ++p) {
      const admm_problem& pr = probs[p];
      const int n = pr.n, m = pr.m, N = pr.num_scen;
      Pat pt{};
      pt.n = n;
      pt.m = m;
      pt.num_scen = N;
      pt.scen_begin = static_cast<int32_t>(P.scen.size());
      pt.zvec_base = P.zvec_total;
      pt.tile_begin = static_cast<int32_t>(P.tiles.size());
      pt.blk_begin = blk_p;
      pt.nblk = (n + kColBlock - 1) / kColBlock;
      for (int b = 0; b < pt.nblk; ++b) P.pblk.push_back(Blk{p, b * kColBlock});
      blk_p += pt.nblk;

      std::vector<double> w(m);
      for (int i = 0; i < m; ++i) w[i] = pr.struct_weight[pr.struct_id[i]];
      std::vector<double> g0(n, 0.0);
      std::vector<std::vector<double>> gdiag(N, std::vector<double>(n, 0.0));
      double gsum = 0.0;
      std::vector<int64_t> cnt;
      std::vector<int32_t> order;
      for (int s = 0; s < N; ++s) {
        const admm_csr& A = pr.A[s];
        const double c = A.prob == 0.0 ? 1.0 : A.prob;
        Scen sc{};
        sc.patient = p;
        sc.n = n;
        sc.m = m;
        sc.cw = static_cast<float>(c);
        sc.row_base = row_base;
        sc.rp_base = rp_base;
        sc.nnz_base = nnz_base;
        sc.vec_base = P.vec_total;
        sc.blk_begin = blk_s;
        sc.nblk = (n + kColBlock - 1) / kColBlock;
        const int g = static_cast<int>(P.scen.size());
        for (int b = 0; b < sc.nblk; ++b) P.blk.push_back(Blk{g, b * kColBlock});
        blk_s += sc.nblk;

        // counting sort of the nonzero rows by decreasing length (stable)
        int64_t maxlen = 0;
        for (int i = 0; i < m; ++i) maxlen = std::max<int64_t>(maxlen, A.row_ptr[i + 1] - A.row_ptr[i]);
        cnt.assign(static_cast<size_t>(maxlen) + 2, 0);
        int64_t rows = 0;
        for (int i = 0; i < m; ++i) {
          const int64_t len = A.row_ptr[i + 1] - A.row_ptr[i];
          if (len > 0) {
            cnt[static_cast<size_t>(maxlen - len)]++;
            rows++;
          }
        }
        int64_t acc = 0;
        for (auto& c2 : cnt) {
          const int64_t t = c2;
          c2 = acc;
          acc += t;
        }
        order.assign(static_cast<size_t>(rows), 0);
        for (int i = 0; i < m; ++i) {
          const int64_t len = A.row_ptr[i + 1] - A.row_ptr[i];
          if (len > 0) order[static_cast<size_t>(cnt[static_cast<size_t>(maxlen - len)]++)] = i;
        }
        sc.rows = static_cast<int32_t>(rows);
        for (int i = 0; i < m; ++i) {
          const double wp2 = c * w[i] * pr.presc[i] * pr.presc[i];
          pt.fconst += wp2;
          if (A.row_ptr[i + 1] == A.row_ptr[i]) pt.fzero += wp2;
        }

        // rows, values, per-row constants
        uint32_t off = 0;
        P.rp.push_back(0);
        std::vector<double> bs(n, 0.0);
        std::vector<double> row_w(static_cast<size_t>(rows)), row_p(static_cast<size_t>(rows));
        for (int64_t r = 0; r < rows; ++r) {
          const int i = order[static_cast<size_t>(r)];
          const int64_t b = A.row_ptr[i], e = A.row_ptr[i + 1];
          const double cwi = c * w[i];
          float rmax = 0.0f;
          double rsum = 0.0;
          for (int64_t k = b; k < e; ++k) rsum += A.val[k];
          row_w[static_cast<size_t>(r)] = cwi * rsum;
          row_p[static_cast<size_t>(r)] = cwi * pr.presc[i];
          for (int64_t k = b; k < e; ++k) {
            const int32_t j = A.col[k];
            const float v = A.val[k];
            if (P.col16_used)
              P.col16.push_back(static_cast<uint16_t>(j));
            else
              P.col32.push_back(j);
            P.val.push_back(v);
            rmax = std::max(rmax, v);
            bs[j] += cwi * pr.presc[i] * static_cast<double>(v);
            gdiag[s][j] += cwi * static_cast<double>(v) * static_cast<double>(v);
          }
          if (lp) {
            const float scl = rmax > 0.0f ? rmax : 1.0f;
            P.rscale.push_back(scl);
            for (int64_t k = b; k < e; ++k) {
              const float q = A.val[k] / scl;
              P.val_lp.push_back(o.precision == ADMM_PREC_BF16 ? to_bf16_bits(q) : to_f16_bits(q));
            }
          }
          // pad the row to whole 4-element chunks: value 0, column = the row's last column
          const int64_t len = e - b, len4 = (len + 3) & ~int64_t(3);
          for (int64_t k = len; k < len4; ++k) {
            const int32_t j = A.col[e - 1];
            if (P.col16_used)
              P.col16.push_back(static_cast<uint16_t>(j));
            else
              P.col32.push_back(j);
            P.val.push_back(0.0f);
            if (lp) P.val_lp.push_back(0);
          }
          P.rw.push_back(static_cast<float>(cwi));
          P.rw64.push_back(cwi);
          P.rpres.push_back(static_cast<float>(pr.presc[i]));
          P.rorig.push_back(i);
          off += static_cast<uint32_t>(len4 / 4);
          P.rp.push_back(off);
        }
        for (int j = 0; j < n; ++j) {
          P.gdiag.push_back(static_cast<float>(gdiag[s][j]));
          P.b.push_back(static_cast<float>(bs[j]));
          g0[j] += 2.0 * bs[j];
          gsum += gdiag[s][j];
        }

        // tiles: consecutive rows with one lanes-per-row width, ~tile_nnz nonzeros each
        sc.tile_begin = static_cast<int32_t>(P.tiles.size());
        int64_t r = 0;
        const uint32_t* rpp = P.rp.data() + rp_base;
        std::vector<double> colsum(n, 0.0);
        std::vector<int32_t> touched;
        auto round_up = [](double x) { return static_cast<float>(x * (1.0 + 1e-6)) ; };
        while (r < rows) {
          const int L = lanes_for(rpp[r + 1] - rpp[r]);
          int64_t r1 = r;
          int64_t nz = 0;
          while (r1 < rows && lanes_for(rpp[r1 + 1] - rpp[r1]) == L && (nz < tile_chunks || r1 == r)) {
            nz += rpp[r1 + 1] - rpp[r1];
            ++r1;
          }
          Tile t{};
          t.scen = g;
          t.row_begin = static_cast<int32_t>(r);
          t.row_end = static_cast<int32_t>(r1);
          t.lanes = L;
          double wm = 0.0, pm = 0.0, cm = 0.0;
          for (int64_t rr = r; rr < r1; ++rr) {
            wm = std::max(wm, row_w[static_cast<size_t>(rr)]);
            pm = std::max(pm, row_p[static_cast<size_t>(rr)]);
            for (int64_t k = nnz_base + 4 * static_cast<int64_t>(rpp[rr]); k < nnz_base + 4 * static_cast<int64_t>(rpp[rr + 1]); ++k) {
              const int32_t j = P.col16_used ? P.col16[static_cast<size_t>(k)] : P.col32[static_cast<size_t>(k)];
              if (colsum[j] == 0.0) touched.push_back(j);
              colsum[j] += P.val[static_cast<size_t>(k)];
            }
          }
          for (int32_t j : touched) {
            cm = std::max(cm, colsum[j]);
            colsum[j] = 0.0;
          }
          touched.clear();
          t.wmax = round_up(wm);
          t.pmax = round_up(pm);
          t.cmax = round_up(cm);
          t.part_off = P.part_total;
          P.part_total += n;
          P.tiles.push_back(t);
          r = r1;
        }
        sc.tile_end = static_cast<int32_t>(P.tiles.size());
        P.scen.push_back(sc);
        P.scen_nnz.push_back(A.nnz);
        nnz_base += static_cast<int64_t>(off) * 4;
        row_base += rows;
        rp_base += rows + 1;
        P.vec_total += n;
      }
      const double mean_diag = gsum / (static_cast<double>(N) * n);
      P.gdiag_mean[p] = mean_diag;
      const double rho = o.rho > 0 ? o.rho : 2.0 * mean_diag;
      if (o.precond) {
        for (int s = 0; s < N; ++s)
          for (int j = 0; j < n; ++j) {
            const double d = gdiag[s][j] + 0.5 * rho;
            P.dinv.push_back(d > 0 ? static_cast<float>(1.0 / d) : 1.0f);
          }
      }
      P.g0[p] = std::move(g0);
      for (int j = 0; j < n; ++j) {
        P.lb.push_back(static_cast<float>(pr.lb ? pr.lb[j] : 0.0));
        P.ub.push_back(pr.ub ? static_cast<float>(pr.ub[j]) : INFINITY);
      }
      pt.tile_end = static_cast<int32_t>(P.tiles.size());
      P.pat.push_back(pt);
      P.zvec_total += n;
    }
  } catch (const std::bad_alloc&) {
    if (msg) *msg = "host allocation failed while packing";
    return ADMM_E_OOM;
  }
  // trailing zero chunks so that no chunk load can leave the arrays
  for (int k = 0; k < 256; ++k) {
    P.val.push_back(0.0f);
    if (P.col16_used)
      P.col16.push_back(0);
    else
      P.col32.push_back(0);
    if (lp) P.val_lp.push_back(0);
  }
  // the column reductions address tile t's partials as first_tile_offset + (t - first) * n
  for (const Pat& pt : P.pat)
    for (int t = pt.tile_begin; t < pt.tile_end; ++t)
      if (P.tiles[t].part_off != P.tiles[pt.tile_begin].part_off + static_cast<int64_t>(t - pt.tile_begin) * pt.n) {
        if (msg) *msg = "internal: tile partials are not contiguous";
        return ADMM_E_STATE;
      }
  P.nnz_total = nnz_base;
  P.rows_total = row_base;
  return ADMM_OK;
}

}  // namespace admmbb
