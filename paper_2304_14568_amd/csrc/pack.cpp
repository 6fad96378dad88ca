// Host packing: validated CSR inputs -> length-sorted CSR tiles for the fused
// pass, plus the per-scenario constants the iteration needs.
//
// Rows of each A_s are reordered by decreasing length (zero rows dropped).
// The fused pass never has to write a voxel-indexed vector, so the order of
// rows is free; sorting lets each workgroup tile use one lanes-per-row width
// that keeps a row's nonzeros in registers (at most kRegChunks per lane),
// and makes neighbouring rows of a tile equally long.
//
// Every (patient, scenario) pair is packed by its own host thread into
// preallocated ranges of the shared arrays; the per-patient sums are then
// formed in scenario order, so the result does not depend on the threads.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <stdexcept>
#include <system_error>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_set>

#include "host.h"

namespace admmbb {

namespace {
std::atomic<int64_t> g_pin_budget{0};  // bytes the packing may still place in pinned memory
std::mutex g_pin_mu;
std::unordered_set<void*> g_pinned;  // blocks from hipHostMalloc
constexpr size_t kPinMin = size_t{1} << 20;
}  // namespace

void* host_alloc(size_t bytes) {
  if (bytes >= kPinMin) {
    int64_t left = g_pin_budget.load();
    while (left >= static_cast<int64_t>(bytes) &&
           !g_pin_budget.compare_exchange_weak(left, left - static_cast<int64_t>(bytes))) {
    }
    if (left >= static_cast<int64_t>(bytes)) {
      void* p = nullptr;
      if (hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess && p != nullptr) {
        std::lock_guard<std::mutex> lk(g_pin_mu);
        g_pinned.insert(p);
        return p;
      }
      (void)hipGetLastError();  // no device or no pinned memory: the heap serves
      g_pin_budget.fetch_add(static_cast<int64_t>(bytes));
    }
  }
  return ::operator new(bytes);
}

void host_free(void* p) noexcept {
  if (p == nullptr) return;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto it = g_pinned.find(p);
    if (it != g_pinned.end()) {
      g_pinned.erase(it);
      (void)hipHostFree(p);
      return;
    }
  }
  ::operator delete(p);
}

PinnedBudget::PinnedBudget(size_t bytes) : saved(static_cast<size_t>(g_pin_budget.exchange(static_cast<int64_t>(bytes)))) {}
PinnedBudget::~PinnedBudget() { g_pin_budget.store(static_cast<int64_t>(saved)); }

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

// Rows of equal length sit in voxel order after the sort, so the rows that
// one wave instruction handles are neighbouring voxels reached by nearly the
// same spots: their scatters hit the same LDS column accumulators at once.
// Within every class of equal length the rows are visited with a stride near
// 0.618 of the class size (coprime to it), which spreads neighbours apart.

static void scramble_length_classes(const admm_csr& A, std::vector<int32_t>& order) {
  std::vector<int32_t> tmp;
  const size_t R = order.size();
  size_t a = 0;
  while (a < R) {
    const int64_t len = A.row_ptr[order[a] + 1] - A.row_ptr[order[a]];
    size_t b = a + 1;
    while (b < R && A.row_ptr[order[b] + 1] - A.row_ptr[order[b]] == len) ++b;
    const size_t c = b - a;
    if (c > 2) {
      size_t step = std::max<size_t>(1, static_cast<size_t>(0.6180339887498949 * static_cast<double>(c)));
      while (std::gcd(step, c) != 1) ++step;
      tmp.assign(order.begin() + static_cast<std::ptrdiff_t>(a), order.begin() + static_cast<std::ptrdiff_t>(b));
      size_t q = 0;
      for (size_t p = 0; p < c; ++p) {
        order[a + p] = tmp[q];
        q += step;
        if (q >= c) q -= c;
      }
    }
    a = b;
  }
}

namespace {

// What one thread produces for one (patient, scenario) pair besides the shared arrays.
struct ScenOut {
  int64_t rows = 0, chunks = 0;        // nonempty rows, 4-element chunks after padding
  int64_t nnz_base = 0, row_base = 0, rp_base = 0;
  std::vector<Tile> tiles;             // part_off filled at the merge; slice_begin local
  std::vector<double> b, gdiag;        // n each
  double fzero = 0.0, fconst = 0.0;
  std::vector<uint32_t> soff;          // sliced layout: slot offset of every slice, then a terminal entry
};

// The sliced copy of one scenario's rows (MatDev FMT_SELL), read from its
// chunk-row copy: tile by tile, slices of G = 64 / L consecutive rows, each
// row's chunk c at slot 64 (c / L) + g L + (c % L) of its slice, every slice
// padded to the most chunk slots per lane any of its rows needs.
template <class CT>
void build_sliced(ScenOut& r, const uint32_t* rpp, const float* val, const CT* col, const uint16_t* lp,
                  RawVec<float>& sval, RawVec<CT>& scol, RawVec<uint16_t>* slp) {
  r.soff.clear();
  uint64_t slots = 0;
  for (Tile& t : r.tiles) {
    const int L = t.lanes, G = 64 / L;
    t.slice_begin = static_cast<int32_t>(r.soff.size());
    for (int32_t rb = t.row_begin; rb < t.row_end; rb += G) {
      const int32_t re = std::min(rb + G, t.row_end);
      uint32_t K = 0;
      for (int32_t q = rb; q < re; ++q) K = std::max<uint32_t>(K, (rpp[q + 1] - rpp[q] + L - 1) / L);
      r.soff.push_back(static_cast<uint32_t>(slots));
      slots += 64ull * K;
    }
  }
  if (slots >= (1ull << 32)) throw std::length_error("sliced layout of one scenario exceeds 2^32 slots");
  r.soff.push_back(static_cast<uint32_t>(slots));
  sval.resize(static_cast<size_t>(slots) * 4);
  scol.resize(static_cast<size_t>(slots) * 4);
  if (slp) slp->resize(static_cast<size_t>(slots) * 8);  // records: four values, four columns
  size_t sl = 0;
  for (const Tile& t : r.tiles) {
    const int L = t.lanes, G = 64 / L;
    for (int32_t rb = t.row_begin; rb < t.row_end; rb += G, ++sl) {
      const uint32_t s0 = r.soff[sl], K = (r.soff[sl + 1] - s0) / 64;
      for (int g = 0; g < G; ++g) {
        const int32_t q = rb + g;
        const bool real = q < t.row_end;
        const uint32_t ch = real ? rpp[q + 1] - rpp[q] : 0;
        const size_t src = real ? static_cast<size_t>(rpp[q]) * 4 : 0;
        const CT pad_col = real ? col[src + 4 * static_cast<size_t>(ch) - 1] : CT{0};
        for (uint32_t c = 0; c < K * static_cast<uint32_t>(L); ++c) {
          const size_t dst = (static_cast<size_t>(s0) + 64ull * (c / L) + static_cast<size_t>(g) * L + c % L) * 4;
          if (c < ch) {
            for (int e = 0; e < 4; ++e) {
              sval[dst + e] = val[src + 4 * c + e];
              scol[dst + e] = col[src + 4 * c + e];
            }
            if (slp)
              for (int e = 0; e < 8; ++e) (*slp)[2 * dst + e] = lp[2 * (src + 4 * c) + e];
          } else {
            for (int e = 0; e < 4; ++e) {
              sval[dst + e] = 0.0f;
              scol[dst + e] = pad_col;
              if (slp) {
                (*slp)[2 * dst + e] = 0;
                (*slp)[2 * dst + 4 + e] = static_cast<uint16_t>(pad_col);
              }
            }
          }
        }
      }
    }
  }
}

template <class F>
void parallel_for(int count, F&& fn) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nt = static_cast<int>(std::min<unsigned>(hw, static_cast<unsigned>(std::max(1, count))));
  std::atomic<int> next{0};
  std::atomic<bool> oom{false}, failed{false};
  auto worker = [&]() {
    for (int k = next++; k < count; k = next++) {
      try {
        fn(k);
      } catch (const std::bad_alloc&) {
        oom = true;
      } catch (const std::exception&) {
        failed = true;
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) {
    try {
      th.emplace_back(worker);
    } catch (const std::system_error&) {
      break;  // fewer threads: the calling thread takes the remaining jobs
    }
  }
  worker();
  for (auto& t : th) t.join();
  if (oom) throw std::bad_alloc();
  if (failed) throw std::length_error("a scenario exceeds the packed layout's 32-bit chunk offsets");
}

}  // namespace

admm_status pack_problems(const admm_problem* probs, int num_patients, const admm_options& o, Packed* out,
                          std::string* msg) {
  Packed& P = *out;
  // the packed arrays go to the device next: up to 4 GiB of them in pinned
  // memory, which the upload reads at the link's DMA rate
  PinnedBudget pin(size_t{4} << 30);
  int64_t nnz_all = 0;
  for (int p = 0; p < num_patients; ++p)
    for (int s = 0; s < probs[p].num_scen; ++s) nnz_all += probs[p].A[s].nnz;
  // about 2048 tiles (8 workgroups per CU) for every patient: the passes are
  // launched per patient, so each patient's tiles are sized for its own
  // nonzeros (a small patient in a batch must not get a few huge tiles, nor a
  // large one thousands of tiny ones)
  (void)nnz_all;
  std::vector<int64_t> tile_chunks_of(num_patients);
  for (int p = 0; p < num_patients; ++p) {
    int64_t np = 0;
    for (int s = 0; s < probs[p].num_scen; ++s) np += probs[p].A[s].nnz;
    int64_t tile_nnz = o.tile_nnz > 0 ? o.tile_nnz : np / (256 * 8);
    tile_nnz = std::max<int64_t>(8192, std::min<int64_t>(tile_nnz, 1 << 22));
    tile_chunks_of[p] = std::max<int64_t>(1, tile_nnz / 4);
  }

  P.col16_used = true;
  for (int p = 0; p < num_patients; ++p) {
    P.nmax = std::max(P.nmax, probs[p].n);
    P.mmax = std::max(P.mmax, probs[p].m);
    if (probs[p].n > 65535) P.col16_used = false;
  }
  const bool lp = o.precision != ADMM_PREC_FP32;

  // jobs in (patient, scenario) order
  std::vector<int> job_p, job_s;
  for (int p = 0; p < num_patients; ++p)
    for (int s = 0; s < probs[p].num_scen; ++s) {
      job_p.push_back(p);
      job_s.push_back(s);
    }
  const int J = static_cast<int>(job_p.size());
  try {
    std::vector<ScenOut> so(J);
    // sizes: nonempty rows and padded chunks of every scenario
    parallel_for(J, [&](int k) {
      const admm_csr& A = probs[job_p[k]].A[job_s[k]];
      const int m = probs[job_p[k]].m;
      int64_t rows = 0, chunks = 0;
      for (int i = 0; i < m; ++i) {
        const int64_t len = A.row_ptr[i + 1] - A.row_ptr[i];
        if (len > 0) {
          rows++;
          chunks += (len + 3) / 4;
        }
      }
      so[k].rows = rows;
      so[k].chunks = chunks;
    });
    int64_t nnz_base = 0, row_base = 0, rp_base = 0;
    for (int k = 0; k < J; ++k) {
      so[k].nnz_base = nnz_base;
      so[k].row_base = row_base;
      so[k].rp_base = rp_base;
      nnz_base += 4 * so[k].chunks;
      row_base += so[k].rows;
      rp_base += so[k].rows + 1;
    }
    // the scenarios' ranges tile [0, nnz_base) and are written in full below;
    // only the trailing zero chunks are cleared here
    const size_t ntot = static_cast<size_t>(nnz_base + 4 * 256);
    const size_t tail = static_cast<size_t>(nnz_base);
    P.val.resize(ntot);
    std::fill(P.val.begin() + tail, P.val.end(), 0.0f);
    if (P.col16_used) {
      P.col16.resize(ntot);
      std::fill(P.col16.begin() + tail, P.col16.end(), uint16_t{0});
    } else {
      P.col32.resize(ntot);
      std::fill(P.col32.begin() + tail, P.col32.end(), 0);
    }
    // low-precision values with 16-bit columns: one 8 x 16-bit record per
    // chunk (its four values, then its four columns)
    const size_t lpw = P.col16_used ? 2 : 1;
    if (lp) {
      P.val_lp.resize(lpw * ntot);
      std::fill(P.val_lp.begin() + lpw * tail, P.val_lp.end(), uint16_t{0});
      P.rscale.resize(static_cast<size_t>(row_base));
    }
    P.rw.resize(static_cast<size_t>(row_base));
    P.rw64.resize(static_cast<size_t>(row_base));
    P.rpres.resize(static_cast<size_t>(row_base));
    P.rorig.resize(static_cast<size_t>(row_base));
    P.rp.resize(static_cast<size_t>(rp_base));
    // the sliced layout is built for 16-bit columns unless the chunk-row layout is asked for
    const bool sell = P.col16_used && o.format != ADMM_FORMAT_CSR;
    if (sell) {
      P.sell_val.resize(static_cast<size_t>(J));
      P.sell_col16.resize(static_cast<size_t>(J));
      if (lp) P.sell_val_lp.resize(static_cast<size_t>(J));
    }

    // fill every scenario's ranges
    parallel_for(J, [&](int k) {
      const admm_problem& pr = probs[job_p[k]];
      const admm_csr& A = pr.A[job_s[k]];
      const int n = pr.n, m = pr.m;
      const int64_t tile_chunks = tile_chunks_of[job_p[k]];
      ScenOut& r = so[k];
      const double c = A.prob == 0.0 ? 1.0 : A.prob;
      // counting sort of the nonzero rows by decreasing length (stable)
      int64_t maxlen = 0;
      for (int i = 0; i < m; ++i) maxlen = std::max<int64_t>(maxlen, A.row_ptr[i + 1] - A.row_ptr[i]);
      std::vector<int64_t> cnt(static_cast<size_t>(maxlen) + 2, 0);
      for (int i = 0; i < m; ++i) {
        const int64_t len = A.row_ptr[i + 1] - A.row_ptr[i];
        if (len > 0) cnt[static_cast<size_t>(maxlen - len)]++;
      }
      int64_t acc = 0;
      for (auto& c2 : cnt) {
        const int64_t t = c2;
        c2 = acc;
        acc += t;
      }
      std::vector<int32_t> order(static_cast<size_t>(r.rows));
      for (int i = 0; i < m; ++i) {
        const int64_t len = A.row_ptr[i + 1] - A.row_ptr[i];
        if (len > 0) order[static_cast<size_t>(cnt[static_cast<size_t>(maxlen - len)]++)] = i;
      }
      scramble_length_classes(A, order);
      for (int i = 0; i < m; ++i) {
        const double wp2 = c * pr.struct_weight[pr.struct_id[i]] * pr.presc[i] * pr.presc[i];
        r.fconst += wp2;
        if (A.row_ptr[i + 1] == A.row_ptr[i]) r.fzero += wp2;
      }
      r.b.assign(n, 0.0);
      r.gdiag.assign(n, 0.0);
      uint32_t* rpp = P.rp.data() + r.rp_base;
      rpp[0] = 0;
      uint32_t off = 0;
      // tiles: consecutive rows of one lanes-per-row width, ~tile_chunks chunks
      // each (a row whose width differs, or a full tile, starts the next one);
      // their accumulator bounds are gathered in the same pass
      std::vector<double> colsum(n, 0.0);
      std::vector<int32_t> touched;
      auto round_up = [](double x) { return static_cast<float>(x * (1.0 + 1e-6)); };
      int64_t t_begin = 0, t_chunks = 0;
      int t_lanes = -1;
      double wm = 0.0, pm = 0.0;
      auto close_tile = [&](int64_t t_end) {
        double cm = 0.0;
        for (int32_t j : touched) {
          cm = std::max(cm, colsum[j]);
          colsum[j] = 0.0;
        }
        touched.clear();
        Tile t{};
        t.scen = k;  // global scenario index = job index
        t.row_begin = static_cast<int32_t>(t_begin);
        t.row_end = static_cast<int32_t>(t_end);
        t.lanes = t_lanes;
        t.wmax = round_up(wm);
        t.pmax = round_up(pm);
        t.cmax = round_up(cm);
        r.tiles.push_back(t);
      };
      // rows are visited in the sorted order, so their source entries are
      // scattered: the entries of the row kPrefetch places ahead are requested
      // early, and the row pointers of the one twice as far
      constexpr int64_t kPrefetch = 8;
      for (int64_t q = 0; q < r.rows; ++q) {
        if (q + 2 * kPrefetch < r.rows) __builtin_prefetch(A.row_ptr + order[static_cast<size_t>(q + 2 * kPrefetch)]);
        if (q + kPrefetch < r.rows) {
          const int ia = order[static_cast<size_t>(q + kPrefetch)];
          const int64_t ba = A.row_ptr[ia], ea = A.row_ptr[ia + 1];
          for (int64_t t = ba; t < ea; t += 16) __builtin_prefetch(A.col + t);
          for (int64_t t = ba; t < ea; t += 16) __builtin_prefetch(A.val + t);
          __builtin_prefetch(pr.presc + ia);
          __builtin_prefetch(pr.struct_id + ia);
        }
        const int i = order[static_cast<size_t>(q)];
        const int64_t b = A.row_ptr[i], e = A.row_ptr[i + 1];
        const int64_t len = e - b, len4 = (len + 3) & ~int64_t(3);
        const int lanes = lanes_for(len4 / 4);
        if (q > 0 && (lanes != t_lanes || t_chunks >= tile_chunks)) {
          close_tile(q);
          t_begin = q;
          t_chunks = 0;
          wm = pm = 0.0;
        }
        t_lanes = lanes;
        const double wi = pr.struct_weight[pr.struct_id[i]];
        const double cwi = c * wi;
        float rmax = 0.0f;
        double rsum = 0.0;
        for (int64_t t = b; t < e; ++t) {
          rsum += A.val[t];
          rmax = std::max(rmax, A.val[t]);
        }
        wm = std::max(wm, cwi * rsum);
        pm = std::max(pm, cwi * pr.presc[i]);
        const int64_t dst = r.nnz_base + 4 * static_cast<int64_t>(off);
        const float scl = rmax > 0.0f ? rmax : 1.0f;
        const int32_t* colp = A.col + b;
        const float* valp = A.val + b;
        // the row, padded to whole 4-element chunks (value 0, column = the
        // row's last column)
        if (P.col16_used) {
          uint16_t* cd = P.col16.data() + dst;
          for (int64_t t = 0; t < len; ++t) cd[t] = static_cast<uint16_t>(colp[t]);
          for (int64_t t = len; t < len4; ++t) cd[t] = static_cast<uint16_t>(colp[len - 1]);
        } else {
          int32_t* cd = P.col32.data() + dst;
          for (int64_t t = 0; t < len; ++t) cd[t] = colp[t];
          for (int64_t t = len; t < len4; ++t) cd[t] = colp[len - 1];
        }
        float* vd = P.val.data() + dst;
        for (int64_t t = 0; t < len; ++t) vd[t] = valp[t];
        for (int64_t t = len; t < len4; ++t) vd[t] = 0.0f;
        if (lp) {
          const bool bf = o.precision == ADMM_PREC_BF16;
          if (lpw == 2) {
            uint16_t* ld = P.val_lp.data() + 2 * dst;
            const uint16_t* cd = P.col16.data() + dst;
            for (int64_t t = 0; t < len4; ++t) {
              const float qv = t < len ? valp[t] / scl : 0.0f;
              const int64_t rec = 8 * (t / 4), e = t % 4;
              ld[rec + e] = t < len ? (bf ? to_bf16_bits(qv) : to_f16_bits(qv)) : uint16_t{0};
              ld[rec + 4 + e] = cd[t];
            }
          } else {
            uint16_t* ld = P.val_lp.data() + dst;
            for (int64_t t = 0; t < len; ++t) {
              const float qv = valp[t] / scl;
              ld[t] = bf ? to_bf16_bits(qv) : to_f16_bits(qv);
            }
            for (int64_t t = len; t < len4; ++t) ld[t] = 0;
          }
        }
        for (int64_t t = 0; t < len; ++t) {
          const int32_t j = colp[t];
          const float v = valp[t];
          r.b[j] += cwi * pr.presc[i] * static_cast<double>(v);
          r.gdiag[j] += cwi * static_cast<double>(v) * static_cast<double>(v);
          if (colsum[j] == 0.0) touched.push_back(j);
          colsum[j] += v;
        }
        const int64_t ro = r.row_base + q;
        if (lp) P.rscale[static_cast<size_t>(ro)] = scl;
        P.rw[static_cast<size_t>(ro)] = static_cast<float>(cwi);
        P.rw64[static_cast<size_t>(ro)] = cwi;
        P.rpres[static_cast<size_t>(ro)] = static_cast<float>(pr.presc[i]);
        P.rorig[static_cast<size_t>(ro)] = i;
        off += static_cast<uint32_t>(len4 / 4);
        rpp[q + 1] = off;
        t_chunks += len4 / 4;
      }
      if (r.rows > 0) close_tile(r.rows);
      // the sliced copy of the same rows
      if (sell) {
        const float* v0 = P.val.data() + r.nnz_base;
        const uint16_t* lp0 = lp ? P.val_lp.data() + 2 * r.nnz_base : nullptr;
        RawVec<uint16_t>* slp = lp ? &P.sell_val_lp[static_cast<size_t>(k)] : nullptr;
        build_sliced<uint16_t>(r, rpp, v0, P.col16.data() + r.nnz_base, lp0, P.sell_val[static_cast<size_t>(k)],
                               P.sell_col16[static_cast<size_t>(k)], slp);
      }
    });

    // merge in (patient, scenario) order
    P.g0.resize(num_patients);
    P.gdiag_mean.resize(num_patients);
    int blk_s = 0, blk_p = 0;
    int k = 0;
    for (int p = 0; p < num_patients; ++p) {
      const admm_problem& pr = probs[p];
      const int n = pr.n, m = pr.m, N = pr.num_scen;
      Pat pt{};
      pt.n = n;
      pt.m = m;
      pt.num_scen = N;
      pt.scen_begin = static_cast<int32_t>(P.scen.size());
      pt.zvec_base = P.zvec_total;
      pt.vec_base = P.vec_total;
      pt.tile_begin = static_cast<int32_t>(P.tiles.size());
      pt.blk_begin = blk_p;
      pt.nblk = (n + kColBlock - 1) / kColBlock;
      for (int b = 0; b < pt.nblk; ++b) P.pblk.push_back(Blk{p, b * kColBlock});
      blk_p += pt.nblk;
      std::vector<double> g0(n, 0.0);
      double gsum = 0.0;
      const int k0 = k;
      pt.sblk_begin = blk_s;
      for (int s = 0; s < N; ++s, ++k) {
        ScenOut& r = so[k];
        const admm_csr& A = pr.A[s];
        Scen sc{};
        sc.patient = p;
        sc.n = n;
        sc.m = m;
        sc.cw = static_cast<float>(A.prob == 0.0 ? 1.0 : A.prob);
        sc.rows = static_cast<int32_t>(r.rows);
        sc.row_base = r.row_base;
        sc.rp_base = r.rp_base;
        sc.nnz_base = r.nnz_base;
        sc.vec_base = P.vec_total;
        sc.blk_begin = blk_s;
        sc.nblk = (n + kColBlock - 1) / kColBlock;
        for (int b = 0; b < sc.nblk; ++b) P.blk.push_back(Blk{k, b * kColBlock});
        blk_s += sc.nblk;
        sc.tile_begin = static_cast<int32_t>(P.tiles.size());
        const int32_t slice_base = static_cast<int32_t>(P.soff.size());
        for (Tile t : r.tiles) {
          t.part_off = P.part_total;
          t.slice_begin += slice_base;
          P.part_total += n;
          P.tiles.push_back(t);
        }
        P.soff.insert(P.soff.end(), r.soff.begin(), r.soff.end());
        sc.sell_base = P.sell_total;
        P.sell_total += r.soff.empty() ? 0 : static_cast<int64_t>(r.soff.back());
        sc.tile_end = static_cast<int32_t>(P.tiles.size());
        P.scen.push_back(sc);
        P.scen_nnz.push_back(A.nnz);
        pt.fzero += r.fzero;
        pt.fconst += r.fconst;
        double gdmax = 0.0;
        for (int j = 0; j < n; ++j) {
          P.gdiag.push_back(static_cast<float>(r.gdiag[j]));
          gdmax = std::max(gdmax, r.gdiag[j]);
          P.b.push_back(static_cast<float>(r.b[j]));
          P.b64.push_back(r.b[j]);
          g0[j] += 2.0 * r.b[j];
          gsum += r.gdiag[j];
        }
        P.gdiag_max.push_back(gdmax);
        P.vec_total += n;
      }
      pt.sblk_end = blk_s;
      const double mean_diag = gsum / (static_cast<double>(N) * n);
      P.gdiag_mean[p] = mean_diag;
      const double rho = o.rho > 0 ? o.rho : 2.0 * mean_diag;
      if (o.precond) {
        for (int s = 0; s < N; ++s)
          for (int j = 0; j < n; ++j) {
            const double d = so[k0 + s].gdiag[j] + 0.5 * rho;
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
    P.nnz_total = nnz_base;
    P.rows_total = row_base;
  } catch (const std::bad_alloc&) {
    if (msg) *msg = "host allocation failed while packing";
    return ADMM_E_OOM;
  }
  // the column reductions address tile t's partials as first_tile_offset + (t - first) * n
  for (const Pat& pt : P.pat)
    for (int t = pt.tile_begin; t < pt.tile_end; ++t)
      if (P.tiles[t].part_off != P.tiles[pt.tile_begin].part_off + static_cast<int64_t>(t - pt.tile_begin) * pt.n) {
        if (msg) *msg = "internal: tile partials are not contiguous";
        return ADMM_E_STATE;
      }
  return ADMM_OK;
}

}  // namespace admmbb
