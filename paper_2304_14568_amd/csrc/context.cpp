// Host runtime: device state of a context, the launch sequence of one ADMM-BB
// iteration (captured once into a HIP graph and replayed), the PGD loop and the
// extern "C" entry points of include/admmbb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <system_error>
#include <thread>
#include <utility>
#include <vector>

#include "host.h"

using namespace admmbb;

namespace {

thread_local std::string g_setup_error;

struct HipError {
  hipError_t code;
  const char* what;
};

inline void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError{e, what};
}

// Waits for a stream when it goes out of scope: declared after the host
// buffers that queued copies read or write, it keeps them alive until the
// copies are done, also when a failed call leaves the scope by an exception.
struct StreamDrain {
  hipStream_t s;
  explicit StreamDrain(hipStream_t st) : s(st) {}
  StreamDrain(const StreamDrain&) = delete;
  StreamDrain& operator=(const StreamDrain&) = delete;
  ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

}  // namespace

struct admm_ctx {
  std::string err;
  admm_options opts{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Packed H;  // host image (kept for sizes, g0, bounds)
  int P = 0, G = 0, T = 0, NB = 0, NPB = 0;
  std::vector<double> rho;  // per patient
  std::vector<void*> allocs;
  // device tables
  Scen* d_scen = nullptr;
  Pat* d_pat = nullptr;
  Tile* d_tiles = nullptr;
  Blk* d_blk = nullptr;
  ColJob* d_cjobs = nullptr;
  ZJob* d_zjobs = nullptr;
  Blk* d_pblk = nullptr;
  // the sparse passes read mat32 / matlp (the layout in use); the Gram
  // kernels of the dense set-up read the chunk-row layout csr32
  MatDev mat32{}, matlp{};
  MatDev csr32{}, csrlp{}, sell32{}, selllp{};
  bool has_sell = false;
  int fmt = FMT_CSR;
  void use_format(int f) {
    fmt = (f == FMT_SELL && has_sell) ? FMT_SELL : FMT_CSR;
    mat32 = fmt == FMT_SELL ? sell32 : csr32;
    matlp = fmt == FMT_SELL ? selllp : csrlp;
  }
  // device vectors
  float *d_x = nullptr, *d_r = nullptr, *d_v = nullptr, *d_q = nullptr, *d_zp = nullptr, *d_y = nullptr;
  float *d_b = nullptr, *d_dinv = nullptr, *d_z = nullptr, *d_lb = nullptr, *d_ub = nullptr;
  float *d_pvec = nullptr, *d_pvec2 = nullptr, *d_pvec3 = nullptr, *d_mvec = nullptr;
  float* d_tmax = nullptr;  // kAbsMaxBlocks partial maxima of the transpose product's input
  double* d_dprev = nullptr;
  float* d_part = nullptr;
  double* d_objpart = nullptr;
  double *d_bpart = nullptr, *d_bpartp = nullptr, *d_scratch = nullptr;
  uint8_t* d_act = nullptr;
  double *d_rz = nullptr, *d_tol2 = nullptr;
  int32_t* d_cgcount = nullptr;
  int64_t* d_cgtotal = nullptr;
  PatState* d_ps = nullptr;
  IterRecord* d_trace = nullptr;
  int trace_cap = 0;
  PatState* h_ps = nullptr;  // pinned
  double* h_scr = nullptr;   // pinned scratch
  hipGraphExec_t g_solve = nullptr, g_iter = nullptr;
  hipGraph_t gr_solve = nullptr, gr_iter = nullptr;
  int acc = ACC_F64;
  int pass_threads = 512, pass_unroll = 1;
  double tuned_ms = 0.0;
  // configuration of the sparse passes per patient (workgroup size, row
  // pipelining, LDS accumulator, layout): the passes are launched once per
  // patient, each with its own; the members above hold the common default
  struct PassCfg {
    int threads, unroll, acc, fmt;
    double ms;  // tuned pass time (0 where the tuner did not run)
    // the products other than the CG operator and the gradient pass (forward
    // product and objective, transpose product): workgroup size, row
    // pipelining and the tuned forward-product time
    int fthreads, funroll;
    double fms;
  };
  std::vector<PassCfg> pcfg;
  void set_all_cfg() {
    pcfg.assign(static_cast<size_t>(P),
                PassCfg{pass_threads, pass_unroll, acc, fmt, 0.0, pass_threads, pass_unroll, 0.0});
  }
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;  // pairs around the CG passes inside the captured iteration
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  double total_ms = 0.0, pass_ms_sum = 0.0;
  int64_t pass_count = 0;
  // dense x-update (cached inverses)
  bool dense = false;
  double *d_G = nullptr, *d_Aw = nullptr, *d_Gp = nullptr, *d_g0 = nullptr;
  double *d_Pb = nullptr, *d_U = nullptr, *d_R = nullptr, *d_fpart = nullptr;
  float* d_Mp = nullptr;
  double *d_xpart = nullptr, *d_c64 = nullptr, *d_b64 = nullptr;
  double* d_rw64 = nullptr;
  XJob* d_fjobs = nullptr;
  uint32_t* d_Gq = nullptr;
  XTile* d_xtiles = nullptr;
  int n_xjobs = 0, n_fjobs = 0, ld_max = 0;
  int64_t gp_elems = 0;
  std::vector<double> factored_rho;  // per patient: penalty of the cached inverse
  std::vector<int> chunk_scen;       // per patient: scenarios per set-up chunk
  double factor_ms = 0.0;            // time of the last set-up of the cached inverses
  // dense PGD work buffers, sized for the largest patient on first use
  double* d_pgd = nullptr;
  PgdDevState* d_pgdst = nullptr;

  template <class T>
  T* alloc(size_t count) {
    if (count == 0) count = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) throw HipError{e, "hipMalloc"};
    allocs.push_back(p);
    return static_cast<T*>(p);
  }
  // Copies of more than 64 MiB are split over host threads: a copy from
  // pageable memory is staged through pinned buffers by the calling thread, so
  // several threads keep more of the link busy.
  template <class T, class Alloc>
  T* upload(const std::vector<T, Alloc>& v) {
    T* p = alloc<T>(v.size());
    const size_t bytes = v.size() * sizeof(T);
    if (bytes == 0) return p;
    constexpr size_t kSplit = size_t{64} << 20;
    if (bytes <= kSplit) {
      check(hipMemcpy(p, v.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy H2D");
      return p;
    }
    int dev = 0;
    check(hipGetDevice(&dev), "hipGetDevice");
    const int parts = 8;
    const size_t per = (v.size() + parts - 1) / parts;
    std::vector<hipError_t> rc(parts, hipSuccess);
    std::vector<std::thread> th;
    auto copy_part = [&](int k, size_t b, size_t e) {
      rc[k] = hipSetDevice(dev);
      if (rc[k] == hipSuccess) rc[k] = hipMemcpy(p + b, v.data() + b, (e - b) * sizeof(T), hipMemcpyHostToDevice);
    };
    for (int k = 0; k < parts; ++k) {
      const size_t b = std::min(v.size(), k * per), e = std::min(v.size(), b + per);
      if (e <= b) break;
      try {
        th.emplace_back(copy_part, k, b, e);
      } catch (const std::system_error&) {
        copy_part(k, b, e);  // no thread: copy this part here
      }
    }
    for (auto& t : th) t.join();
    for (hipError_t e : rc) check(e, "hipMemcpy H2D");
    return p;
  }
  // One device array holding per-scenario host parts one after the other
  // (the sliced layout, 4 elements per chunk slot).
  template <class T>
  T* upload_parts(const std::vector<RawVec<T>>& parts, int64_t total_elems) {
    T* p = alloc<T>(static_cast<size_t>(std::max<int64_t>(total_elems, 1)));
    int64_t o = 0;
    for (const auto& v : parts) {
      if (!v.empty())
        check(hipMemcpy(p + o, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy H2D");
      o += static_cast<int64_t>(v.size());
    }
    return p;
  }
  ~admm_ctx() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (g_solve) (void)hipGraphExecDestroy(g_solve);
    if (g_iter) (void)hipGraphExecDestroy(g_iter);
    if (gr_solve) (void)hipGraphDestroy(gr_solve);
    if (gr_iter) (void)hipGraphDestroy(gr_iter);
    for (auto e : ev) (void)hipEventDestroy(e);
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
    for (void* p : allocs) (void)hipFree(p);
    if (h_ps) (void)hipHostFree(h_ps);
    if (h_scr) (void)hipHostFree(h_scr);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  // A sparse pass over the tiles [tile_begin, tile_begin + tile_count), one
  // launch per patient they cover, each sized for that patient's spot count
  // (the LDS of a workgroup holds n floats of v and n accumulators, so sizing
  // every launch for the largest patient of a batch would cost occupancy).
  // e0 / e1 stamp the start of the first and the end of the last launch.
  void pass_launch(int mode, PassArgs pa, int tile_begin, int tile_count, hipEvent_t e0 = nullptr,
                   hipEvent_t e1 = nullptr) const {
    const int tile_end = tile_begin + tile_count;
    int first = -1, last = -1;
    for (int p = 0; p < P; ++p)
      if (H.pat[p].tile_end > tile_begin && H.pat[p].tile_begin < tile_end) {
        if (first < 0) first = p;
        last = p;
      }
    for (int p = first; p >= 0 && p <= last; ++p) {
      const Pat& pt = H.pat[p];
      const int b = std::max(tile_begin, pt.tile_begin), e = std::min(tile_end, pt.tile_end);
      if (e <= b) continue;
      pa.nmax = pt.n;
      if (static_cast<size_t>(p) < pcfg.size()) {
        const PassCfg& c = pcfg[static_cast<size_t>(p)];
        const bool fwd = mode == PASS_OBJ || mode == PASS_MATVEC || mode == PASS_RMATVEC;
        pa.threads = fwd ? c.fthreads : c.threads;
        pa.unroll = fwd ? c.funroll : c.unroll;
        pa.acc = c.acc;
        const bool sl = c.fmt == FMT_SELL && has_sell;
        pa.mat = pa.mat.vkind == VAL_F32 ? (sl ? sell32 : csr32) : (sl ? selllp : csrlp);
      }
      launch_pass(mode, pa, b, e - b, stream, p == first ? e0 : nullptr, p == last ? e1 : nullptr);
    }
  }

  // Transpose product A_s^T t over tiles [tile_begin, tile_begin + tile_count)
  // of one patient (t: its m-vector): max |t_i| first, which bounds the
  // fixed-point column sums of every tile.
  void rmatvec_launch(PassArgs pa, const float* t, int64_t m, int tile_begin, int tile_count) {
    launch_absmax(t, m, d_tmax, stream);
    pa.tin = t;
    pa.tmax = d_tmax;
    pass_launch(PASS_RMATVEC, pa, tile_begin, tile_count);
  }

  PassArgs pass_args(const MatDev& m) const {
    PassArgs a{};
    a.tiles = d_tiles;
    a.scen = d_scen;
    a.pat = d_pat;
    a.mat = m;
    a.part = d_part;
    a.objpart = d_objpart;
    a.nmax = H.nmax;
    a.acc = acc;
    a.threads = pass_threads;
    a.unroll = pass_unroll;
    return a;
  }

  VecArgs vec_args(int stop_enabled) const {
    VecArgs a{};
    a.scen = d_scen;
    a.pat = d_pat;
    a.blk = d_blk;
    a.pblk = d_pblk;
    a.cjobs = d_cjobs;
    a.zjobs = d_zjobs;
    a.tiles = d_tiles;
    a.part = d_part;
    a.objpart = d_objpart;
    a.ps = d_ps;
    a.act = d_act;
    a.rz = d_rz;
    a.tol2 = d_tol2;
    a.cgcount = d_cgcount;
    a.cgtotal = d_cgtotal;
    a.x = d_x;
    a.r = d_r;
    a.v = d_v;
    a.q = d_q;
    a.zp = d_zp;
    a.y = d_y;
    a.b = d_b;
    a.dinv = d_dinv;
    a.z = d_z;
    a.lb = d_lb;
    a.ub = d_ub;
    a.dprev = d_dprev;
    a.bpart = d_bpart;
    a.bpartp = d_bpartp;
    a.trace = d_trace;
    a.prm.eps_abs = opts.eps_abs;
    a.prm.eps_rel = opts.eps_rel;
    a.prm.obj_rel_tol = opts.obj_rel_tol;
    a.prm.bb_clamp = opts.bb_clamp;
    a.prm.eta_factor = opts.cg_eta;
    a.prm.eta_floor = opts.cg_eta_floor;
    a.prm.bb = opts.bb;
    a.prm.z_mode = opts.z_mode;
    a.prm.stop_enabled = stop_enabled;
    a.prm.precond = opts.precond;
    a.prm.trace_cap = trace_cap;
    a.prm.num_pat = P;
    a.fpart = dense ? d_fpart : nullptr;
    a.c64 = d_c64;
    a.b64 = d_b64;
    return a;
  }

  FactorArgs fargs() const {
    FactorArgs f{};
    f.scen = d_scen;
    f.pat = d_pat;
    f.ps = d_ps;
    f.G = d_G;
    f.A = d_Aw;
    f.Mp = d_Mp;
    f.Gp = d_Gp;
    f.g0 = d_g0;
    f.P = d_Pb;
    f.U = d_U;
    f.R = d_R;
    f.xpart = d_xpart;
    f.xtiles = d_xtiles;
    f.nxtiles = n_xjobs;
    f.fjobs = d_fjobs;
    f.Gq = d_Gq;
    f.fpart = d_fpart;
    f.npmax = ld_max;
    f.npat = P;
    return f;
  }

  // Gram matrices G_s of the scenarios [g0, g0 + cs) of patient pt into the
  // chunk buffer (the upper tiles are what the next steps read): per-tile row
  // lists and one LDS accumulation per tile; where the lists do not fit in
  // device memory, one fp64 atomic per product (also taken when the
  // environment sets ADMMBB_GRAM_ATOMIC, which tests use to compare the two).
  void gram_chunk(const Pat& pt, int g0, int cs, int64_t nn) {
    struct DevBuf {
      void* p = nullptr;
      ~DevBuf() {
        if (p) (void)hipFree(p);
      }
    } bc, bo, bl, bsc;
    const int nb = pt.nbk;
    const int64_t ntl = static_cast<int64_t>(nb) * (nb + 1) / 2, nt = ntl * cs;
    bool lists = std::getenv("ADMMBB_GRAM_ATOMIC") == nullptr &&
                 hipMalloc(&bc.p, sizeof(int32_t) * 2 * nt) == hipSuccess &&
                 hipMalloc(&bo.p, sizeof(int64_t) * (nt + 1)) == hipSuccess;
    if (lists) {
      int32_t* cnt = static_cast<int32_t*>(bc.p);
      int32_t* cur = cnt + nt;
      int64_t* off = static_cast<int64_t*>(bo.p);
      launch_fill_f32(reinterpret_cast<float*>(cnt), 0.0f, 2 * nt, stream);  // counts and cursors
      for (int s = 0; s < cs; ++s) launch_gram_rows(csr32, H.scen[g0 + s], nb, cnt + s * ntl, nullptr, nullptr, stream);
      launch_gram_scan(cnt, nt, off, stream);
      check(hipMemcpyAsync(h_scr, off + nt, sizeof(int64_t), hipMemcpyDeviceToHost, stream), "D2H");
      check(hipStreamSynchronize(stream), "sync");
      int64_t total = 0;
      std::memcpy(&total, h_scr, sizeof(total));
      lists = total >= 0 && hipMalloc(&bl.p, sizeof(GramEntry) * static_cast<size_t>(std::max<int64_t>(total, 1))) ==
                                hipSuccess;
      // fixed-point scale of each scenario's tiles: a power of two that keeps
      // 2 max_j (G_s)_jj, a bound of every partial sum, below 2^62 (from the
      // fp64 diagonal).  A diagonal beyond fp64 range, or so small that the
      // scale would leave it, takes the fp64 atomic path instead.
      std::vector<double> gs(static_cast<size_t>(cs), 1.0);
      for (int s = 0; s < cs; ++s) {
        const double gmax = H.gdiag_max[static_cast<size_t>(g0 + s)];
        int e = 0;
        if (!(2.0 * gmax <= std::numeric_limits<double>::max())) {
          lists = false;
        } else if (gmax > 0.0) {
          (void)std::frexp(2.0 * gmax, &e);  // 2 gmax = f 2^e, 1/2 <= f < 1
          if (62 - e > 1000) lists = false;
          gs[static_cast<size_t>(s)] = std::ldexp(1.0, std::min(62 - e, 1000));
        }
      }
      lists = lists && hipMalloc(&bsc.p, sizeof(double) * static_cast<size_t>(cs)) == hipSuccess;
      if (lists) {
        check(hipMemcpy(bsc.p, gs.data(), sizeof(double) * static_cast<size_t>(cs), hipMemcpyHostToDevice), "H2D");
        GramEntry* list = static_cast<GramEntry*>(bl.p);
        for (int s = 0; s < cs; ++s)
          launch_gram_rows(csr32, H.scen[g0 + s], nb, cur + s * ntl, off + s * ntl, list, stream);
        launch_gram_tiles(csr32, d_rw64, d_scen, g0, cs, nb, off, list, static_cast<const double*>(bsc.p), d_G,
                          pt.npad, stream);
      }
    }
    if (!lists) {
      (void)hipGetLastError();  // the failed allocation
      launch_fill_f64(d_G, 0.0, nn * cs, stream);
      for (int s = 0; s < cs; ++s) launch_gram(csr32, d_rw64, H.scen[g0 + s], d_G + s * nn, pt.npad, stream);
    }
    check(hipGetLastError(), "Gram launch");
    check(hipStreamSynchronize(stream), "sync");  // before the lists are freed
  }

  // (Re)build the cached inverses of patient p at its current penalty, a
  // chunk of scenarios at a time: Gram matrices, B_s = G_s + rho/2 I swept in
  // place, packed fp32 inverses.  With accumulate_gsum (the first time) the
  // chunks also add up the packed sum_s G_s of the objective.
  void factorize(int p, bool accumulate_gsum) {
    const Pat& pt = H.pat[p];
    const int npad = pt.npad;
    const int64_t nn = static_cast<int64_t>(npad) * npad;
    FactorArgs f = fargs();
    const int chunk = chunk_scen[p];
    for (int c0 = 0; c0 < pt.num_scen; c0 += chunk) {
      const int cs = std::min(chunk, pt.num_scen - c0);
      const int g0 = pt.scen_begin + c0;
      gram_chunk(pt, g0, cs, nn);
      launch_gram_finish(f, p, g0, cs, npad, pt.n, rho[p], accumulate_gsum ? 1 : 0, stream);
      for (int k0 = 0; k0 < npad; k0 += 64) launch_sweep_step(f, g0, cs, npad, k0, stream);
      launch_sweep_store(f, p, g0, cs, npad, stream);
    }
    check(hipGetLastError(), "factor launch");
    factored_rho[p] = rho[p];
  }

  // head: gradient pass at z (objective + residual of the x-update system at x = z),
  // completion of the previous iteration, CG set-up
  void launch_head(int stop_enabled, int cg_setup) {
    if (dense) {
      VecArgs va = vec_args(stop_enabled);
      launch_fheadobj(fargs(), va, n_fjobs, NB, stream);
      launch_head_scalars(va, G, 0, stream);
      return;
    }
    PassArgs pa = pass_args(mat32);
    pa.src = d_z;
    pa.src_per_scen = 0;
    pa.ps = d_ps;
    pass_launch(PASS_GRAD, pa, 0, T);
    VecArgs va = vec_args(stop_enabled);
    launch_reduce(RED_HEAD, va, 0, NB, stream);
    launch_head_scalars(va, G, cg_setup, stream);
  }

  void launch_body(int stop_enabled, bool with_events) {
    const MatDev& m = (opts.precision == ADMM_PREC_FP32) ? mat32 : matlp;
    VecArgs va = vec_args(stop_enabled);
    if (dense) {
      const FactorArgs f = fargs();
      if (opts.dense_launches == 3) {
        // the previous iteration's stopping test beside the x-update tiles;
        // the reduction and z-update; residual norms and dual step beside the
        // dual update, the next right-hand sides and the objective tiles
        if (with_events)
          launch_dense_x(f, va, d_c64, n_xjobs, stream, ev[0], ev[1]);
        else
          launch_dense_x(f, va, d_c64, n_xjobs, stream);
        launch_xzres(f, va, NPB, stream);
        launch_dense_tail_dual(f, va, n_fjobs, NB, stream);
        return;
      }
      if (with_events)
        launch_xsym(f, d_c64, n_xjobs, stream, ev[0], ev[1]);
      else
        launch_xsym(f, d_c64, n_xjobs, stream);
      launch_xzres(f, va, NPB, stream);
      // residual norms and BB step beside the objective tiles at the new z,
      // then the stopping test beside the dual update and the next right-hand
      // sides: the iteration ends complete, with no head of its own next time
      launch_dense_tail(f, va, n_fjobs, stream);
      launch_dense_head(va, NB, stream);
      return;
    }
    for (int k = 0; k < opts.cg_max; ++k) {
      PassArgs pa = pass_args(m);
      pa.src = d_v;
      pa.src_per_scen = 1;
      pa.step = k;
      pa.act = d_act;
      pa.ps = d_ps;
      pa.objpart = nullptr;
      if (with_events)
        pass_launch(PASS_CG, pa, 0, T, ev[2 * k], ev[2 * k + 1]);
      else
        pass_launch(PASS_CG, pa, 0, T);
      va.step = k;
      launch_reduce(RED_CG, va, 0, NB, stream);
      launch_cg_update(va, NB, stream);
      launch_cg_dir(va, NB, stream);
    }
    launch_zres(va, NPB, stream);
    launch_body_scalars(va, stream);
  }

  // One iteration recorded into a graph.  No event is ever recorded inside a
  // capture: timed runs launch directly (one_iteration), and the body is
  // captured without its timing events, so a replayed graph holds kernel nodes
  // only and nothing the host reads back between replays.
  void capture(int stop_enabled, hipGraph_t* gr, hipGraphExec_t* ge) {
    if (timing) throw HipError{hipErrorInvalidValue, "graph capture refused while timing events are enabled"};
    check(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
      if (!dense) launch_head(stop_enabled, 1);
      launch_body(stop_enabled, false);
    } catch (...) {
      hipGraph_t tmp = nullptr;
      (void)hipStreamEndCapture(stream, &tmp);
      if (tmp) (void)hipGraphDestroy(tmp);
      throw;
    }
    check(hipStreamEndCapture(stream, gr), "hipStreamEndCapture");
    check(hipGraphInstantiate(ge, *gr, nullptr, nullptr, 0), "hipGraphInstantiate");
  }

  void one_iteration(int stop_enabled) {
    // timed runs launch directly: events recorded around each pass launch must
    // be readable after every iteration, which graph-captured events are not
    if (opts.use_graph && !timing) {
      hipGraphExec_t& ge = stop_enabled ? g_solve : g_iter;
      hipGraph_t& gr = stop_enabled ? gr_solve : gr_iter;
      if (!ge) capture(stop_enabled, &gr, &ge);
      check(hipGraphLaunch(ge, stream), "hipGraphLaunch");
    } else {
      if (!dense) launch_head(stop_enabled, 1);
      launch_body(stop_enabled, timing);
    }
  }

  void accumulate_pass_times() {
    if (!timing) return;
    const int nev = dense ? 1 : opts.cg_max;
    for (int k = 0; k < nev; ++k) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) == hipSuccess) {
        pass_ms_sum += ms;
        pass_count += 1;
      }
    }
  }

  void read_state() {
    check(hipMemcpyAsync(h_ps, d_ps, sizeof(PatState) * P, hipMemcpyDeviceToHost, stream), "hipMemcpyAsync");
    check(hipStreamSynchronize(stream), "hipStreamSynchronize");
  }

  // Run up to `k` iterations.  With stop_enabled the loop ends early once every
  // patient has stopped.  CG x-update: every iteration starts with its head (the
  // gradient pass at z, completion of the previous iteration, CG set-up) and a
  // final head completes the bookkeeping of the last one.  Dense x-update: one
  // head before the first iteration forms the right-hand sides and the
  // objective of the state the run starts from (completing a pending dual
  // update, as left by a checkpoint); in the four-launch order each iteration
  // then ends complete (stopping test, dual update, next right-hand sides), in
  // the three-launch order the stopping test of each iteration runs in the
  // next one's first launch, and a final one follows the loop.  There the host
  // sees a stop one iteration late; the iteration between is skipped on the
  // device.
  void run(int k, int stop_enabled) {
    if (timing) {
      check(hipEventRecord(ev_a, stream), "hipEventRecord");
      pass_ms_sum = 0.0;
      pass_count = 0;
    }
    if (dense) launch_head(stop_enabled, 0);
    const int every = std::max(1, opts.check_every);
    for (int it = 0; it < k; ++it) {
      one_iteration(stop_enabled);
      const bool last = (it + 1 == k);
      // without the stopping test the device skips stopped patients by itself:
      // the host only waits when it needs the flags or the pass timings
      if (timing || last || (stop_enabled && (it + 1) % every == 0)) {
        read_state();
        accumulate_pass_times();
        bool all = true;
        for (int p = 0; p < P; ++p) all = all && (h_ps[p].stopped != 0);
        if (all) break;
      }
    }
    if (!dense) launch_head(stop_enabled, 0);
    if (dense && opts.dense_launches == 3) launch_dense_head(vec_args(stop_enabled), 0, stream);
    if (timing) {
      check(hipEventRecord(ev_b, stream), "hipEventRecord");
      check(hipEventSynchronize(ev_b), "hipEventSynchronize");
      float ms = 0.0f;
      check(hipEventElapsedTime(&ms, ev_a, ev_b), "hipEventElapsedTime");
      total_ms = ms;
    }
    read_state();
  }

  void fill_info(admm_info* info) {
    if (!info) return;
    for (int p = 0; p < P; ++p) {
      const PatState& s = h_ps[p];
      admm_info& o = info[p];
      std::memset(&o, 0, sizeof(o));
      o.iter = s.iter;
      o.cg_steps = s.cg_total;
      o.status = s.status == 2 ? ADMM_E_DIVERGED : (s.status == 1 ? ADMM_OK : ADMM_MAX_ITER);
      o.obj = s.f_cur;
      o.r_prim = s.r_prim;
      o.r_dual = s.r_dual;
      o.eps_prim = s.eps_prim;
      o.eps_dual = s.eps_dual;
      o.tau = s.tau;
      o.kkt = -1.0;
    }
  }

  // Time each patient's fused CG pass (its own launch) for every candidate
  // configuration and keep that patient's fastest (values of the multiplied
  // vector do not change the work).
  void autotune() {
    std::vector<int> th = {256, 512, 1024}, un = {1, 2}, ac = {ACC_FIX64, ACC_F64}, fm = {FMT_CSR};
    if (opts.pass_threads) th = {opts.pass_threads};
    if (opts.pass_unroll) un = {opts.pass_unroll};
    if (opts.lds_acc >= 0) ac = {opts.lds_acc};
    if (opts.deterministic) ac = {ACC_FIX64};
    if (has_sell) fm = opts.format == FMT_SELL ? std::vector<int>{FMT_SELL} : std::vector<int>{FMT_CSR, FMT_SELL};
    hipEvent_t e0, e1;
    check(hipEventCreate(&e0), "hipEventCreate");
    check(hipEventCreate(&e1), "hipEventCreate");
    std::vector<PassCfg> best = pcfg;
    for (auto& b : best) {
      b.threads = th[0];
      b.unroll = un[0];
      b.acc = ac[0];
      b.fmt = fm[0];
      b.ms = 1e30;
    }
    const int reps = 3;
    for (int f : fm)
      for (int a64 : ac)
        for (int t : th)
          for (int u : un) {
            // the sliced layout has neither a row pipelining nor a 1024-thread variant
            if (f == FMT_SELL && (u != un[0] || t > 512)) continue;
            for (auto& c : pcfg) {
              c.threads = t;
              c.unroll = u;
              c.acc = a64;
              c.fmt = f;
            }
            PassArgs pa = pass_args(opts.precision == ADMM_PREC_FP32 ? csr32 : csrlp);
            pa.src = d_v;
            pa.src_per_scen = 1;
            pa.objpart = nullptr;
            for (int p = 0; p < P; ++p) {
              const Pat& pt = H.pat[p];
              const int tc = pt.tile_end - pt.tile_begin;
              if (tc <= 0) continue;
              pass_launch(PASS_CG, pa, pt.tile_begin, tc);
              check(hipEventRecord(e0, stream), "hipEventRecord");
              for (int r = 0; r < reps; ++r) pass_launch(PASS_CG, pa, pt.tile_begin, tc);
              check(hipEventRecord(e1, stream), "hipEventRecord");
              check(hipEventSynchronize(e1), "hipEventSynchronize");
              float ms = 0.0f;
              check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
              PassCfg& b = best[static_cast<size_t>(p)];
              if (ms / reps < b.ms) {
                b.threads = t;
                b.unroll = u;
                b.acc = a64;
                b.fmt = f;
                b.ms = ms / reps;
              }
            }
          }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    pcfg = best;
    tuned_ms = 0.0;
    for (auto& c : pcfg) {
      if (!(c.ms < 1e30)) c.ms = 0.0;
      tuned_ms += c.ms;
    }
    // the common default (reported by admm_get_tuning): patient 0's
    use_format(pcfg[0].fmt);
    acc = pcfg[0].acc;
    pass_threads = pcfg[0].threads;
    pass_unroll = pcfg[0].unroll;
  }

  // Per patient, the workgroup size and row pipelining of the products other
  // than the CG operator: the fastest forward product (objective pass at z,
  // fp32 values) of 512 or 1024 threads, with or without pipelining, in the
  // patient's layout (the sliced layout has 512 threads at most and no
  // pipelining).  Options that fix either keep it.  Run once, before the
  // context's first such product (the iterations use none).
  bool fwd_tuned = false;
  void ensure_forward_tuned() {
    if (!fwd_tuned) tune_forward();
  }
  void tune_forward() {
    fwd_tuned = true;
    std::vector<int> th = {512, 1024}, un = {1, 2};
    if (opts.pass_threads) th = {opts.pass_threads};
    if (opts.pass_unroll) un = {opts.pass_unroll};
    hipEvent_t e0, e1;
    check(hipEventCreate(&e0), "hipEventCreate");
    check(hipEventCreate(&e1), "hipEventCreate");
    // the candidates differ by a few per cent: each is timed over 4 passes in
    // each of 3 rounds taken in turn, and keeps its best round
    const int reps = 4, rounds = 3;
    try {
      for (int p = 0; p < P; ++p) {
        const Pat& pt = H.pat[p];
        const int tc = pt.tile_end - pt.tile_begin;
        PassCfg& c = pcfg[static_cast<size_t>(p)];
        if (tc <= 0) continue;
        const bool sl = c.fmt == FMT_SELL && has_sell;
        std::vector<std::pair<int, int>> cand;
        for (int t : th)
          for (int u : un)
            if (!(sl && (t > 512 || u != un[0]))) cand.emplace_back(t, u);
        std::vector<double> best(cand.size(), 1e30);
        PassArgs pa = pass_args(mat32);
        pa.src = d_z;
        pa.src_per_scen = 0;
        pa.part = nullptr;
        for (int round = 0; round < rounds; ++round)
          for (size_t k = 0; k < cand.size(); ++k) {
            c.fthreads = cand[k].first;
            c.funroll = cand[k].second;
            pass_launch(PASS_OBJ, pa, pt.tile_begin, tc);
            check(hipEventRecord(e0, stream), "hipEventRecord");
            for (int r = 0; r < reps; ++r) pass_launch(PASS_OBJ, pa, pt.tile_begin, tc);
            check(hipEventRecord(e1, stream), "hipEventRecord");
            check(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.0f;
            check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            best[k] = std::min(best[k], static_cast<double>(ms) / reps);
          }
        size_t kb = 0;
        for (size_t k = 1; k < cand.size(); ++k)
          if (best[k] < best[kb]) kb = k;
        c.fthreads = cand[kb].first;
        c.funroll = cand[kb].second;
        c.fms = best[kb] < 1e30 ? best[kb] : 0.0;
      }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }

  void reset_patient(int p, const double* z0, double new_rho) {
    const Pat& pt = H.pat[p];
    std::vector<float> z(pt.n);
    StreamDrain drain{stream};
    for (int j = 0; j < pt.n; ++j) {
      double v = z0 ? z0[j] : 0.0;
      v = std::min(std::max(v, static_cast<double>(H.lb[pt.zvec_base + j])), static_cast<double>(H.ub[pt.zvec_base + j]));
      z[j] = static_cast<float>(v);
    }
    check(hipMemcpyAsync(d_z + pt.zvec_base, z.data(), sizeof(float) * pt.n, hipMemcpyHostToDevice, stream), "H2D");
    const Scen& s0 = H.scen[pt.scen_begin];
    const int64_t len = static_cast<int64_t>(pt.num_scen) * pt.n;
    launch_fill_f32(d_y + s0.vec_base, 0.0f, len, stream);
    launch_fill_f32(d_x + s0.vec_base, 0.0f, len, stream);
    launch_fill_f64(d_dprev + s0.vec_base, 0.0, len, stream);
    check(hipMemsetAsync(d_cgtotal + pt.scen_begin, 0, sizeof(int64_t) * pt.num_scen, stream), "memset");
    if (new_rho > 0) rho[p] = new_rho;
    if (dense && factored_rho[p] != rho[p]) factorize(p, false);  // Sum_s G_s does not depend on rho
    PatState st{};
    st.rho = rho[p];
    st.tau = rho[p];
    st.bb_tau0 = rho[p];
    std::memcpy(h_ps + p, &st, sizeof(st));
    check(hipMemcpyAsync(d_ps + p, h_ps + p, sizeof(PatState), hipMemcpyHostToDevice, stream), "H2D");
    check(hipStreamSynchronize(stream), "sync");
  }

  void upload_pvec(int p, const double* x, float* dst) {
    const Pat& pt = H.pat[p];
    std::vector<float> v(pt.n);
    StreamDrain drain{stream};
    for (int j = 0; j < pt.n; ++j) v[j] = static_cast<float>(x[j]);
    check(hipMemcpyAsync(dst + pt.zvec_base, v.data(), sizeof(float) * pt.n, hipMemcpyHostToDevice, stream), "H2D");
    check(hipStreamSynchronize(stream), "sync");
  }

  // f(x) and (optionally) grad f(x) for patient p, x already in d_pvec at zvec_base
  double objective_dev(int p, float* grad_dev) {
    if (!grad_dev) ensure_forward_tuned();
    const Pat& pt = H.pat[p];
    PassArgs pa = pass_args(mat32);
    pa.src = d_pvec;
    pa.src_per_scen = 0;
    pass_launch(grad_dev ? PASS_GRAD : PASS_OBJ, pa, pt.tile_begin, pt.tile_end - pt.tile_begin);
    if (grad_dev)
      launch_gsum(d_scen, d_pat, d_pblk, d_tiles, d_part, pt.blk_begin, pt.nblk, 2.0f, grad_dev, stream);
    launch_objsum(d_tiles, d_objpart, pt.tile_begin, pt.tile_end - pt.tile_begin, d_scratch, stream);
    check(hipMemcpyAsync(h_scr, d_scratch, sizeof(double), hipMemcpyDeviceToHost, stream), "D2H");
    check(hipStreamSynchronize(stream), "sync");
    return h_scr[0] + pt.fzero;
  }
};

namespace {

admm_status set_err(admm_ctx* c, admm_status st, const std::string& m) {
  if (c)
    c->err = m;
  else
    g_setup_error = m;
  return st;
}

admm_status from_hip(admm_ctx* c, const HipError& e) {
  std::string m = std::string(e.what) + ": " + hipGetErrorString(e.code);
  return set_err(c, e.code == hipErrorOutOfMemory ? ADMM_E_OOM : ADMM_E_HIP, m);
}

// A failed entry point waits for the work it already queued before it
// returns, so that no copy into a caller's buffer is still pending once the
// caller sees the error.
void drain_after_error(admm_ctx* c) {
  if (c) (void)hipStreamSynchronize(c->stream);
  (void)hipGetLastError();
}

// every entry reports only its own HIP errors: a stale last-error left by an
// earlier call of the thread is cleared first
#define GUARD_BEGIN      \
  (void)hipGetLastError(); \
  try {
#define GUARD_END(ctx)                                              \
  }                                                                 \
  catch (const HipError& e) {                                       \
    const admm_status guard_st = from_hip(ctx, e);                  \
    drain_after_error(ctx);                                         \
    return guard_st;                                                \
  }                                                                 \
  catch (const std::bad_alloc&) {                                   \
    drain_after_error(ctx);                                         \
    return set_err(ctx, ADMM_E_OOM, "host allocation failed");      \
  }                                                                 \
  catch (...) {                                                     \
    drain_after_error(ctx);                                         \
    return set_err(ctx, ADMM_E_HIP, "unexpected exception");        \
  }

admm_status check_patient(const admm_ctx* c, int32_t p) {
  if (!c) return ADMM_E_ARG;
  if (p < 0 || p >= c->P) return set_err(const_cast<admm_ctx*>(c), ADMM_E_ARG, "patient index out of range");
  return ADMM_OK;
}

}  // namespace

extern "C" {

admm_status admm_default_options(admm_options* o) {
  if (!o) return ADMM_E_ARG;
  std::memset(o, 0, sizeof(*o));
  o->rho = 0.0;
  o->eps_abs = 1e-6;
  o->eps_rel = 1e-6;
  o->obj_rel_tol = 1e-5;
  o->max_iter = 1000;
  o->bb = 1;
  o->z_mode = 0;
  o->bb_clamp = 0.0;
  o->cg_max = 8;
  o->cg_eta = 0.01;
  o->cg_eta_floor = 1e-8;
  o->precision = ADMM_PREC_FP32;
  o->precond = 0;
  o->use_graph = 1;
  o->check_every = 1;
  o->lds_acc = -1;
  o->tile_nnz = 0;
  o->pass_threads = 0;
  o->pass_unroll = 0;
  o->format = -1;
  o->deterministic = 0;
  o->dense_launches = 3;
  o->xupdate = ADMM_XUPDATE_AUTO;
  o->stream = nullptr;
  return ADMM_OK;
}

admm_status pgd_default_options(pgd_options* o) {
  if (!o) return ADMM_E_ARG;
  std::memset(o, 0, sizeof(*o));
  o->alpha = 0.0;
  o->beta = 1e-4;
  o->gamma = 0.5;
  o->obj_rel_tol = 1e-5;
  o->max_iter = 10000;
  o->max_trials = 60;
  o->dense = -1;
  o->reserved = 0;
  return ADMM_OK;
}

admm_status admm_validate(const admm_problem* prob) {
  std::string m;
  admm_status st = validate_problem(prob, &m);
  if (st != ADMM_OK) g_setup_error = m;
  return st;
}

const char* admm_last_error(const admm_ctx* ctx) {
  if (!ctx) return g_setup_error.c_str();
  return ctx->err.c_str();
}

namespace {

// Wall-clock phases of admm_setup, printed to stderr when ADMMBB_SETUP_TIMING is set.
struct SetupClock {
  bool on = std::getenv("ADMMBB_SETUP_TIMING") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[admm_setup] %-28s %8.1f ms\n", what,
                 std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

}  // namespace

// Device bytes the dense set-up's fp64 matrices (Gram and sweep, npad^2 each
// per scenario) may take at once: 8 GiB, or ADMMBB_DENSE_CHUNK_MB.
static int64_t dense_chunk_bytes() {
  int64_t b = int64_t(8) << 30;
  if (const char* env = std::getenv("ADMMBB_DENSE_CHUNK_MB")) {
    const long long mb = std::atoll(env);
    if (mb > 0) b = static_cast<int64_t>(mb) << 20;
  }
  return b;
}

admm_status admm_setup_batch(const admm_problem* probs, int32_t num_patients, const admm_options* opts,
                             admm_ctx** out) {
  SetupClock clk;
  if (!out) return set_err(nullptr, ADMM_E_ARG, "out is NULL");
  *out = nullptr;
  if (!probs || num_patients <= 0) return set_err(nullptr, ADMM_E_ARG, "no problems given");
  admm_options o;
  admm_default_options(&o);
  if (opts) o = *opts;
  std::string msg;
  admm_status st = validate_options(&o, &msg);
  if (st != ADMM_OK) return set_err(nullptr, st, msg);
  // device-resident CSR arrays: host staging copies, then the host path
  std::vector<admm_problem> staged;
  std::vector<std::vector<admm_csr>> staged_csr;
  std::vector<std::vector<int64_t>> st_rp;
  std::vector<std::vector<int32_t>> st_col;
  std::vector<std::vector<float>> st_val;
  bool any_device = false;
  for (int p = 0; p < num_patients; ++p) any_device = any_device || probs[p].mem_kind == ADMM_MEM_DEVICE;
  if (any_device) {
    try {
      staged.assign(probs, probs + num_patients);
      staged_csr.resize(num_patients);
      for (int p = 0; p < num_patients; ++p) {
        admm_problem& q = staged[p];
        if (q.mem_kind != ADMM_MEM_DEVICE) continue;
        if (!q.A || q.m <= 0 || q.num_scen <= 0)
          return set_err(nullptr, ADMM_E_ARG, "patient " + std::to_string(p) + ": NULL A or non-positive sizes");
        for (int s = 0; s < q.num_scen; ++s) {
          const admm_csr& a = q.A[s];
          if (a.nnz < 0 || !a.row_ptr || (a.nnz > 0 && (!a.col || !a.val)))
            return set_err(nullptr, ADMM_E_ARG,
                           "patient " + std::to_string(p) + " scenario " + std::to_string(s) + ": bad device CSR");
          st_rp.emplace_back(static_cast<size_t>(q.m) + 1);
          st_col.emplace_back(static_cast<size_t>(a.nnz));
          st_val.emplace_back(static_cast<size_t>(a.nnz));
          hipError_t e = hipMemcpy(st_rp.back().data(), a.row_ptr, sizeof(int64_t) * (q.m + 1), hipMemcpyDeviceToHost);
          if (e == hipSuccess && a.nnz > 0)
            e = hipMemcpy(st_col.back().data(), a.col, sizeof(int32_t) * a.nnz, hipMemcpyDeviceToHost);
          if (e == hipSuccess && a.nnz > 0)
            e = hipMemcpy(st_val.back().data(), a.val, sizeof(float) * a.nnz, hipMemcpyDeviceToHost);
          if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_err(nullptr, ADMM_E_HIP,
                           "patient " + std::to_string(p) + " scenario " + std::to_string(s) +
                               ": copying the device CSR arrays failed: " + hipGetErrorString(e));
          }
          admm_csr h = a;
          h.row_ptr = st_rp.back().data();
          h.col = st_col.back().data();
          h.val = st_val.back().data();
          staged_csr[p].push_back(h);
        }
        q.A = staged_csr[p].data();
        q.mem_kind = ADMM_MEM_HOST;
      }
    } catch (const std::bad_alloc&) {
      return set_err(nullptr, ADMM_E_OOM, "host allocation failed while staging device input");
    }
    probs = staged.data();
  }
  for (int p = 0; p < num_patients; ++p) {
    st = validate_problem(&probs[p], &msg);
    if (st != ADMM_OK) return set_err(nullptr, st, "patient " + std::to_string(p) + ": " + msg);
  }
  // the sparse pass keeps v (n floats) and one 64-bit column accumulator per
  // spot of a patient in the 160 KiB of LDS of a workgroup
  for (int p = 0; p < num_patients; ++p)
    if (pass_smem_bytes(probs[p].n, ACC_FIX64) > 163840)
      return set_err(nullptr, ADMM_E_ARG,
                     "patient " + std::to_string(p) + ": n = " + std::to_string(probs[p].n) +
                         " spots exceeds the 13 600 the sparse pass holds in LDS");
  std::unique_ptr<admm_ctx> c;
  try {
    c.reset(new admm_ctx());
  } catch (const std::bad_alloc&) {
    return set_err(nullptr, ADMM_E_OOM, "host allocation failed");
  }
  c->opts = o;
  clk.mark("validate");
  // the x-update form, decided before packing (it needs only the sizes and the
  // free device memory): the dense form runs no CG pass per iteration, so
  // under the automatic layout choice it gets the chunk-row layout alone
  {
    int ndev = 0;
    (void)hipGetLastError();  // report only this call's errors
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
      return set_err(nullptr, ADMM_E_HIP, "no HIP device available");
    const int64_t kChunkBytes = dense_chunk_bytes();
    int64_t need = 0, chunk_need = 0;
    bool fits_n = true;
    for (int p = 0; p < num_patients; ++p) {
      const int64_t n = probs[p].n, N = probs[p].num_scen;
      const int64_t npad = (n + 63) / 64 * 64, nb = npad / 64, tiles = nb * (nb + 1) / 2;
      fits_n = fits_n && n <= 8128;
      const int64_t per_scen = 16 * npad * npad;
      const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(N, kChunkBytes / per_scen));
      chunk_need = std::max(chunk_need, chunk * per_scen);
      // every iteration: packed fp32 inverses, packed fp64 sum of G, tile partials; U, R panels
      need += tiles * 4096 * (4 * N + 8) + tiles * 1024 * N + 2 * 8 * 64 * npad * N;
    }
    need += chunk_need;
    size_t free_b = 0, total_b = 0;
    const hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return set_err(nullptr, ADMM_E_HIP, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
    if (o.xupdate == ADMM_XUPDATE_DENSE) {
      if (!fits_n) return set_err(nullptr, ADMM_E_ARG, "dense x-update needs n <= 8128 for every patient");
      if (static_cast<size_t>(need) > free_b)
        return set_err(nullptr, ADMM_E_OOM, "dense x-update matrices do not fit in device memory");
      c->dense = true;
    } else if (o.xupdate == ADMM_XUPDATE_AUTO) {
      c->dense = fits_n && static_cast<size_t>(need) <= free_b / 4;
    }
  }
  admm_options po = o;
  if (c->dense && o.format == ADMM_FORMAT_AUTO) po.format = ADMM_FORMAT_CSR;
  try {
    st = pack_problems(probs, num_patients, po, &c->H, &msg);
  } catch (const std::bad_alloc&) {
    return set_err(nullptr, ADMM_E_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_err(nullptr, ADMM_E_HIP, std::string("packing failed: ") + e.what());
  }
  if (st != ADMM_OK) return set_err(nullptr, st, msg);
  clk.mark("pack");
  try {
    Packed& H = c->H;
    c->P = num_patients;
    c->G = static_cast<int>(H.scen.size());
    c->T = static_cast<int>(H.tiles.size());
    c->NB = static_cast<int>(H.blk.size());
    c->NPB = static_cast<int>(H.pblk.size());
    c->acc = (o.lds_acc >= 0 && !o.deterministic) ? o.lds_acc : ACC_FIX64;
    if (o.stream) {
      c->stream = static_cast<hipStream_t>(o.stream);
    } else {
      check(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate");
      c->own_stream = true;
    }
    {
      // device address of the allocation-free entry point's fixed scratch,
      // looked up once per device while it is current
      void* sp = nullptr;
      check(noalloc_scratch(&sp), "hipGetSymbolAddress");
    }
    c->rho.resize(num_patients);
    for (int p = 0; p < num_patients; ++p) c->rho[p] = o.rho > 0 ? o.rho : 2.0 * H.gdiag_mean[p];
    c->trace_cap = std::max(1, o.max_iter + 2);

    // dense x-update: sizes, offsets and work lists (before the tables go to the device)
    std::vector<XJob> fjobs;
    std::vector<XTile> xtiles;
    // dense set-up works on chunks of scenarios: G and the sweep matrix (fp64,
    // npad^2 each) for at most kChunkBytes at a time
    const int64_t kChunkBytes = dense_chunk_bytes();
    if (c->dense) {
      int64_t chunk_elems = 0, moff = 0, goff = 0;
      c->chunk_scen.assign(num_patients, 1);
      for (int p = 0; p < num_patients; ++p) {
        Pat& pt = H.pat[p];
        pt.npad = (pt.n + 63) / 64 * 64;
        pt.nbk = pt.npad / 64;
        c->ld_max = std::max(c->ld_max, pt.npad);
        const int64_t nn = static_cast<int64_t>(pt.npad) * pt.npad;
        const int64_t tiles = static_cast<int64_t>(pt.nbk) * (pt.nbk + 1) / 2;
        const int chunk = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(pt.num_scen, kChunkBytes / (16 * nn))));
        c->chunk_scen[p] = chunk;
        chunk_elems = std::max(chunk_elems, chunk * nn);
        pt.gpack_off = goff;
        goff += tiles * 4096;
        pt.fobj_begin = static_cast<int32_t>(fjobs.size());
        for (int I = 0; I < pt.nbk; ++I)
          for (int J = I; J < pt.nbk; ++J) {
            // the upper tiles in row-major order: the job's rank is the tile's index
            // objective job k is the tile stored at 4096 k of Gp (6144 k words of Gq)
            if (pt.gpack_off + static_cast<int64_t>(fjobs.size() - pt.fobj_begin) * 4096 !=
                static_cast<int64_t>(fjobs.size()) * 4096)
              throw std::logic_error("objective tile list out of storage order");
            fjobs.push_back(XJob{p, I * 65536 + J});
          }
        pt.fobj_end = static_cast<int32_t>(fjobs.size());
        for (int s = 0; s < pt.num_scen; ++s) {
          const int g = pt.scen_begin + s;
          Scen& sc = H.scen[g];
          sc.mpack_off = moff;
          moff += tiles * 4096;
          for (int I = 0; I < pt.nbk; ++I)
            for (int J = I; J < pt.nbk; ++J) {
              XTile xt{};
              const int64_t t = static_cast<int64_t>(I) * pt.nbk - static_cast<int64_t>(I) * (I - 1) / 2 + (J - I);
              if (sc.mpack_off / 4096 + t != static_cast<int64_t>(xtiles.size()))
                throw std::logic_error("dense tile table out of storage order");
              xt.vbase = sc.vec_base;
              xt.n = pt.n;
              xt.patient = p;
              xt.I = I;
              xt.J = J;
              xtiles.push_back(xt);
            }
        }
      }
      c->n_xjobs = static_cast<int>(xtiles.size());
      c->n_fjobs = static_cast<int>(fjobs.size());
      c->d_G = c->alloc<double>(static_cast<size_t>(chunk_elems));
      c->d_Aw = c->alloc<double>(static_cast<size_t>(chunk_elems));
      c->d_Mp = c->alloc<float>(static_cast<size_t>(moff));
      c->d_xpart = c->alloc<double>(static_cast<size_t>(moff / 4096) * 128);
      c->d_c64 = c->alloc<double>(static_cast<size_t>(H.vec_total));
      c->d_b64 = c->upload(H.b64);
      c->d_Gp = c->alloc<double>(static_cast<size_t>(goff));
      c->gp_elems = goff;
      c->d_Pb = c->alloc<double>(static_cast<size_t>(c->G) * 64 * 64);
      c->d_U = c->alloc<double>(static_cast<size_t>(c->G) * 64 * c->ld_max);
      c->d_R = c->alloc<double>(static_cast<size_t>(c->G) * 64 * c->ld_max);
      c->d_fpart = c->alloc<double>(fjobs.size());
      c->d_xtiles = c->upload(xtiles);
      c->d_fjobs = c->upload(fjobs);
      c->d_Gq = c->alloc<uint32_t>(static_cast<size_t>(goff / 4096) * 6144);
      std::vector<double> g0all(static_cast<size_t>(H.zvec_total));
      for (int p = 0; p < num_patients; ++p)
        std::copy(H.g0[p].begin(), H.g0[p].end(), g0all.begin() + H.pat[p].zvec_base);
      c->d_g0 = c->upload(g0all);
      c->d_rw64 = c->upload(H.rw64);
      c->factored_rho.assign(num_patients, 0.0);
    }
    clk.mark("dense buffers and tables");
    c->d_scen = c->upload(H.scen);
    c->d_pat = c->upload(H.pat);
    c->d_tiles = c->upload(H.tiles);
    c->d_blk = c->upload(H.blk);
    {
      std::vector<ColJob> cj(H.blk.size());
      for (size_t b = 0; b < H.blk.size(); ++b) {
        const Scen& sc = H.scen[static_cast<size_t>(H.blk[b].owner)];
        ColJob& j = cj[b];
        j = ColJob{};
        j.ntiles = sc.tile_end - sc.tile_begin;
        j.part_off = j.ntiles > 0 ? H.tiles[static_cast<size_t>(sc.tile_begin)].part_off : 0;
        j.vec_base = sc.vec_base;
        j.zvec_base = H.pat[static_cast<size_t>(sc.patient)].zvec_base;
        j.n = sc.n;
        j.col0 = H.blk[b].col0;
        j.scen = H.blk[b].owner;
        j.patient = sc.patient;
      }
      c->d_cjobs = c->upload(cj);
      std::vector<ZJob> zj(H.pblk.size());
      for (size_t b = 0; b < H.pblk.size(); ++b) {
        const Pat& pt = H.pat[static_cast<size_t>(H.pblk[b].owner)];
        const int64_t xt0 = c->dense ? H.scen[static_cast<size_t>(pt.scen_begin)].mpack_off / 4096 : 0;
        zj[b] = ZJob{pt.vec_base, pt.zvec_base, pt.n, pt.num_scen, H.pblk[b].col0, H.pblk[b].owner, xt0};
      }
      c->d_zjobs = c->upload(zj);
    }
    c->d_pblk = c->upload(H.pblk);
    const uint32_t* d_rp = c->upload(H.rp);
    const void* d_col = H.col16_used ? static_cast<const void*>(c->upload(H.col16))
                                     : static_cast<const void*>(c->upload(H.col32));
    const float* d_rw = c->upload(H.rw);
    const float* d_rpres = c->upload(H.rpres);
    const int32_t* d_rorig = c->upload(H.rorig);
    const int c16 = H.col16_used ? 1 : 0;
    const int vlp = o.precision == ADMM_PREC_BF16 ? VAL_BF16 : VAL_F16;
    c->csr32 = MatDev{d_rp, d_col, c->upload(H.val), nullptr, d_rw, d_rpres, d_rorig, nullptr, c16, VAL_F32,
                      FMT_CSR, 0};
    // the host copies of the largest arrays are not needed after upload
    decltype(H.val)().swap(H.val);
    const float* d_rscale = nullptr;
    if (o.precision != ADMM_PREC_FP32) {
      d_rscale = c->upload(H.rscale);
      c->csrlp = MatDev{d_rp, d_col, c->upload(H.val_lp), d_rscale, d_rw, d_rpres, d_rorig, nullptr, c16, vlp,
                        FMT_CSR, 0};
      decltype(H.val_lp)().swap(H.val_lp);
    }
    c->has_sell = !H.soff.empty() && !H.sell_val.empty();
    if (c->has_sell) {
      const uint32_t* d_soff = c->upload(H.soff);
      const int64_t ne = 4 * H.sell_total;  // elements: four per chunk slot (low-precision records: eight)
      const void* d_scol = c->upload_parts(H.sell_col16, ne);
      c->sell32 = MatDev{d_rp, d_scol, c->upload_parts(H.sell_val, ne), nullptr, d_rw, d_rpres, d_rorig, d_soff,
                         c16, VAL_F32, FMT_SELL, 0};
      if (o.precision != ADMM_PREC_FP32)
        c->selllp = MatDev{d_rp, d_scol, c->upload_parts(H.sell_val_lp, 2 * ne), d_rscale, d_rw, d_rpres, d_rorig,
                           d_soff, c16, vlp, FMT_SELL, 0};
      decltype(H.sell_val)().swap(H.sell_val);
      decltype(H.sell_col16)().swap(H.sell_col16);
      decltype(H.sell_val_lp)().swap(H.sell_val_lp);
    }
    // the layout asked for; under AUTO the chunk-row layout until the set-up
    // autotuner (CG x-update, LDS within 64 KiB) measures both
    c->use_format(o.format == FMT_SELL ? FMT_SELL : FMT_CSR);
    clk.mark("sparse matrix upload");
    decltype(H.col16)().swap(H.col16);
    decltype(H.col32)().swap(H.col32);
    decltype(H.rp)().swap(H.rp);
    decltype(H.rw64)().swap(H.rw64);

    const size_t V = static_cast<size_t>(H.vec_total);
    c->d_x = c->alloc<float>(V);
    c->d_r = c->alloc<float>(V);
    c->d_v = c->alloc<float>(V);
    c->d_q = c->alloc<float>(V);
    c->d_y = c->alloc<float>(V);
    c->d_zp = o.precond ? c->alloc<float>(V) : c->d_r;
    c->d_dinv = o.precond ? c->upload(H.dinv) : nullptr;
    c->d_b = c->upload(H.b);
    c->d_dprev = c->alloc<double>(V);
    c->d_z = c->alloc<float>(H.zvec_total);
    c->d_lb = c->upload(H.lb);
    c->d_ub = c->upload(H.ub);
    c->d_pvec = c->alloc<float>(H.zvec_total);
    c->d_pvec2 = c->alloc<float>(H.zvec_total);
    c->d_pvec3 = c->alloc<float>(H.zvec_total);
    c->d_mvec = c->alloc<float>(H.mmax);
    c->d_tmax = c->alloc<float>(kAbsMaxBlocks);
    c->d_part = c->alloc<float>(static_cast<size_t>(H.part_total));
    c->d_objpart = c->alloc<double>(c->T);
    c->d_bpart = c->alloc<double>(static_cast<size_t>(c->NB) * 8);
    c->d_bpartp = c->alloc<double>(static_cast<size_t>(c->NPB) * 4 * 8);
    c->d_scratch = c->alloc<double>(std::max(64, (H.nmax + kThreads - 1) / kThreads + 8));
    c->d_act = c->alloc<uint8_t>(static_cast<size_t>(c->G) * kRing);
    c->d_rz = c->alloc<double>(static_cast<size_t>(c->G) * kRing);
    c->d_tol2 = c->alloc<double>(c->G);
    c->d_cgcount = c->alloc<int32_t>(c->G);
    c->d_cgtotal = c->alloc<int64_t>(c->G);
    c->d_ps = c->alloc<PatState>(c->P);
    c->d_trace = c->alloc<IterRecord>(static_cast<size_t>(c->P) * c->trace_cap);
    check(hipHostMalloc(reinterpret_cast<void**>(&c->h_ps), sizeof(PatState) * c->P, hipHostMallocDefault),
          "hipHostMalloc");
    check(hipHostMalloc(reinterpret_cast<void**>(&c->h_scr), sizeof(double) * 64, hipHostMallocDefault),
          "hipHostMalloc");
    launch_fill_f32(c->d_v, 0.0f, V, c->stream);
    launch_fill_f32(c->d_q, 0.0f, V, c->stream);
    launch_fill_f32(c->d_r, 0.0f, V, c->stream);
    launch_fill_u8(c->d_act, 0, static_cast<int64_t>(c->G) * kRing, c->stream);
    launch_fill_f64(c->d_rz, 0.0, static_cast<int64_t>(c->G) * kRing, c->stream);
    check(hipMemsetAsync(c->d_cgcount, 0, sizeof(int32_t) * c->G, c->stream), "memset");
    check(hipMemsetAsync(c->d_cgtotal, 0, sizeof(int64_t) * c->G, c->stream), "memset");
    check(hipStreamSynchronize(c->stream), "setup sync");
    clk.mark("other buffers and uploads");
    if (c->dense) {
      hipEvent_t f0, f1;
      check(hipEventCreate(&f0), "hipEventCreate");
      check(hipEventCreate(&f1), "hipEventCreate");
      check(hipEventRecord(f0, c->stream), "hipEventRecord");
      launch_fill_f64(c->d_Gp, 0.0, c->gp_elems, c->stream);
      for (int p = 0; p < num_patients; ++p) c->factorize(p, true);
      launch_gq_pack(c->d_Gp, c->d_Gq, c->gp_elems / 4096, c->stream);
      check(hipEventRecord(f1, c->stream), "hipEventRecord");
      check(hipEventSynchronize(f1), "hipEventSynchronize");
      float ms = 0.0f;
      check(hipEventElapsedTime(&ms, f0, f1), "hipEventElapsedTime");
      c->factor_ms = ms;
      (void)hipEventDestroy(f0);
      (void)hipEventDestroy(f1);
    }
    for (int p = 0; p < num_patients; ++p) c->reset_patient(p, nullptr, 0.0);
    if (o.pass_threads) c->pass_threads = o.pass_threads;
    if (o.pass_unroll) c->pass_unroll = o.pass_unroll;
    c->set_all_cfg();
    clk.mark("cached inverses");
    if (!c->dense) c->autotune();  // the dense x-update does not run the CG pass per iteration
    check(hipEventCreate(&c->ev_a), "hipEventCreate");
    check(hipEventCreate(&c->ev_b), "hipEventCreate");
    check(hipStreamSynchronize(c->stream), "setup sync");
    clk.mark("autotune and state");
  } catch (const HipError& e) {
    std::string m = std::string(e.what) + ": " + hipGetErrorString(e.code);
    return set_err(nullptr, e.code == hipErrorOutOfMemory ? ADMM_E_OOM : ADMM_E_HIP, m);
  } catch (const std::bad_alloc&) {
    return set_err(nullptr, ADMM_E_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_err(nullptr, ADMM_E_HIP, std::string("set-up failed: ") + e.what());
  }
  *out = c.release();
  return ADMM_OK;
}

admm_status admm_setup(const admm_problem* prob, const admm_options* opts, admm_ctx** out) {
  return admm_setup_batch(prob, 1, opts, out);
}

void admm_destroy(admm_ctx* ctx) { delete ctx; }

admm_status admm_enable_timing(admm_ctx* ctx, int32_t on) {
  if (!ctx) return ADMM_E_ARG;
  GUARD_BEGIN
  const bool want = on != 0;
  if (want == ctx->timing) return ADMM_OK;
  ctx->timing = want;
  if (want && ctx->ev.empty()) {
    ctx->ev.resize(2 * static_cast<size_t>(ctx->opts.cg_max));
    for (auto& e : ctx->ev) check(hipEventCreate(&e), "hipEventCreate");
  }
  // graphs captured with the other setting are rebuilt on next use
  if (ctx->g_solve) { (void)hipGraphExecDestroy(ctx->g_solve); ctx->g_solve = nullptr; }
  if (ctx->g_iter) { (void)hipGraphExecDestroy(ctx->g_iter); ctx->g_iter = nullptr; }
  if (ctx->gr_solve) { (void)hipGraphDestroy(ctx->gr_solve); ctx->gr_solve = nullptr; }
  if (ctx->gr_iter) { (void)hipGraphDestroy(ctx->gr_iter); ctx->gr_iter = nullptr; }
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_get_timing(const admm_ctx* ctx, double* total_ms, double* pass_ms, int32_t* pass_launches) {
  if (!ctx) return ADMM_E_ARG;
  if (total_ms) *total_ms = ctx->total_ms;
  if (pass_ms) *pass_ms = ctx->pass_count ? ctx->pass_ms_sum / ctx->pass_count : 0.0;
  if (pass_launches) *pass_launches = static_cast<int32_t>(ctx->pass_count);
  return ADMM_OK;
}

admm_status admm_get_xupdate(const admm_ctx* ctx, int32_t* mode, double* setup_ms) {
  if (!ctx) return ADMM_E_ARG;
  if (mode) *mode = ctx->dense ? ADMM_XUPDATE_DENSE : ADMM_XUPDATE_CG;
  if (setup_ms) *setup_ms = ctx->factor_ms;
  return ADMM_OK;
}

admm_status admm_warm_start(admm_ctx* ctx, int32_t patient, const double* z0, double rho, int32_t dual_init) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!std::isfinite(rho)) return set_err(ctx, ADMM_E_ARG, "rho not finite");
  if (z0)
    for (int j = 0; j < ctx->H.pat[patient].n; ++j)
      if (!std::isfinite(z0[j])) return set_err(ctx, ADMM_E_NONFINITE, "z0 has a non-finite entry");
  if (rho > 0 && ctx->opts.precond)
    return set_err(ctx, ADMM_E_STATE, "changing rho is not supported with the Jacobi preconditioner");
  if (dual_init != 0 && dual_init != 1) return set_err(ctx, ADMM_E_ARG, "dual_init must be 0 or 1");
  GUARD_BEGIN
  ctx->reset_patient(patient, z0, rho);
  if (dual_init) {
    // y_s = -grad f_s(z): one gradient pass at z over this patient's tiles
    const Pat& pt = ctx->H.pat[patient];
    PassArgs pa = ctx->pass_args(ctx->mat32);
    pa.src = ctx->d_z;
    pa.src_per_scen = 0;
    ctx->pass_launch(PASS_GRAD, pa, pt.tile_begin, pt.tile_end - pt.tile_begin);
    VecArgs va = ctx->vec_args(0);
    const Scen& s0 = ctx->H.scen[pt.scen_begin];
    const Scen& s1 = ctx->H.scen[pt.scen_begin + pt.num_scen - 1];
    launch_reduce(RED_DUALINIT, va, s0.blk_begin, s1.blk_begin + s1.nblk - s0.blk_begin, ctx->stream);
    check(hipStreamSynchronize(ctx->stream), "sync");
  }
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_spot_features(admm_ctx* ctx, int32_t patient, const uint8_t* voxel_class, float* feat) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!voxel_class || !feat) return set_err(ctx, ADMM_E_ARG, "NULL argument");
  const Pat& pt = ctx->H.pat[patient];
  for (int i = 0; i < pt.m; ++i)
    if (voxel_class[i] > 2) return set_err(ctx, ADMM_E_ARG, "voxel_class entries must be 0, 1 or 2");
  GUARD_BEGIN
  ctx->ensure_forward_tuned();
  const int n = pt.n, m = pt.m, N = pt.num_scen;
  // indicator vectors of targets, organs at risk and all voxels
  std::vector<float> ind(static_cast<size_t>(3) * m);
  for (int i = 0; i < m; ++i) {
    ind[i] = voxel_class[i] == 1 ? 1.0f : 0.0f;
    ind[static_cast<size_t>(m) + i] = voxel_class[i] == 2 ? 1.0f : 0.0f;
    ind[static_cast<size_t>(2) * m + i] = 1.0f;
  }
  float* d_ind = nullptr;
  check(hipMalloc(reinterpret_cast<void**>(&d_ind), sizeof(float) * ind.size()), "hipMalloc");
  std::vector<float> col(static_cast<size_t>(3) * N * n);
  try {
    check(hipMemcpy(d_ind, ind.data(), sizeof(float) * ind.size(), hipMemcpyHostToDevice), "H2D");
    for (int s = 0; s < N; ++s) {
      const Scen& sc = ctx->H.scen[pt.scen_begin + s];
      for (int c = 0; c < 3; ++c) {
        PassArgs pa = ctx->pass_args(ctx->mat32);
        pa.objpart = nullptr;
        ctx->rmatvec_launch(pa, d_ind + static_cast<size_t>(c) * m, m, sc.tile_begin, sc.tile_end - sc.tile_begin);
        VecArgs va = ctx->vec_args(0);
        va.out = ctx->d_pvec2 + pt.zvec_base;
        launch_reduce(RED_RMAT, va, sc.blk_begin, sc.nblk, ctx->stream);
        check(hipMemcpyAsync(col.data() + (static_cast<size_t>(c) * N + s) * n, va.out, sizeof(float) * n,
                             hipMemcpyDeviceToHost, ctx->stream),
              "D2H");
      }
    }
    check(hipStreamSynchronize(ctx->stream), "sync");
  } catch (...) {
    (void)hipFree(d_ind);
    throw;
  }
  (void)hipFree(d_ind);
  const int64_t vb = ctx->H.scen[pt.scen_begin].vec_base;
  for (int j = 0; j < n; ++j) {
    double ft_sum = 0, ft_min = 1e300, ft_max = -1e300, fo_sum = 0, fo_max = -1e300, mass_sum = 0, bsum = 0, gsum = 0;
    for (int s = 0; s < N; ++s) {
      const double T = col[(static_cast<size_t>(0) * N + s) * n + j];
      const double O = col[(static_cast<size_t>(1) * N + s) * n + j];
      const double M = col[(static_cast<size_t>(2) * N + s) * n + j];
      const double ft = M > 0 ? T / M : 0.0, fo = M > 0 ? O / M : 0.0;
      ft_sum += ft;
      ft_min = std::min(ft_min, ft);
      ft_max = std::max(ft_max, ft);
      fo_sum += fo;
      fo_max = std::max(fo_max, fo);
      mass_sum += M;
      bsum += ctx->H.b[vb + static_cast<int64_t>(s) * n + j];
      gsum += ctx->H.gdiag[vb + static_cast<int64_t>(s) * n + j];
    }
    float* f = feat + static_cast<size_t>(j) * ADMM_NUM_DOSE_FEATURES;
    f[0] = static_cast<float>(ft_sum / N);
    f[1] = static_cast<float>(ft_min);
    f[2] = static_cast<float>(ft_max);
    f[3] = static_cast<float>(fo_sum / N);
    f[4] = static_cast<float>(fo_max);
    f[5] = static_cast<float>(std::log1p(mass_sum / N));
    f[6] = static_cast<float>(gsum > 0 ? bsum / gsum : 0.0);
  }
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_reset(admm_ctx* ctx) {
  if (!ctx) return ADMM_E_ARG;
  GUARD_BEGIN
  for (int p = 0; p < ctx->P; ++p) ctx->reset_patient(p, nullptr, 0.0);
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_iterate(admm_ctx* ctx, int32_t k, admm_info* info) {
  if (!ctx || k < 0) return set_err(ctx, ADMM_E_ARG, "bad argument");
  GUARD_BEGIN
  // iterate ignores earlier stops: clear the stop flags
  ctx->read_state();
  for (int p = 0; p < ctx->P; ++p) ctx->h_ps[p].stopped = ctx->h_ps[p].status == 2 ? 1 : 0;
  check(hipMemcpyAsync(ctx->d_ps, ctx->h_ps, sizeof(PatState) * ctx->P, hipMemcpyHostToDevice, ctx->stream), "H2D");
  ctx->run(k, 0);
  ctx->fill_info(info);
  for (int p = 0; p < ctx->P; ++p)
    if (ctx->h_ps[p].status == 2) return set_err(ctx, ADMM_E_DIVERGED, "iterates became non-finite");
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_solve(admm_ctx* ctx, double* z_out, admm_info* info) {
  if (!ctx) return ADMM_E_ARG;
  GUARD_BEGIN
  ctx->read_state();
  int done = 0;
  for (int p = 0; p < ctx->P; ++p) done = std::max(done, ctx->h_ps[p].iter);
  const int k = std::max(0, ctx->opts.max_iter - done);
  ctx->run(k, 1);
  ctx->fill_info(info);
  std::vector<float> z(static_cast<size_t>(ctx->H.zvec_total));
  if (z_out || info) {
    check(hipStreamSynchronize(ctx->stream), "sync");
    check(hipMemcpy(z.data(), ctx->d_z, sizeof(float) * z.size(), hipMemcpyDeviceToHost), "D2H");
  }
  if (z_out)
    for (size_t i = 0; i < z.size(); ++i) z_out[i] = z[i];
  admm_status worst = ADMM_OK;
  for (int p = 0; p < ctx->P; ++p) {
    if (ctx->h_ps[p].status == 2) return set_err(ctx, ADMM_E_DIVERGED, "iterates became non-finite");
    if (ctx->h_ps[p].status != 1) worst = ADMM_MAX_ITER;
  }
  if (info) {
    // KKT residual of every returned z (one gradient pass per patient)
    for (int p = 0; p < ctx->P; ++p) {
      const Pat& pt = ctx->H.pat[p];
      std::vector<double> zp(z.begin() + pt.zvec_base, z.begin() + pt.zvec_base + pt.n);
      double r = -1.0;
      const admm_status ks = admm_kkt(ctx, p, zp.data(), &r);
      if (ks != ADMM_OK) return ks;
      info[p].kkt = r;
    }
  }
  return worst;
  GUARD_END(ctx)
}

admm_status admm_get_z(admm_ctx* ctx, int32_t patient, double* z) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!z) return set_err(ctx, ADMM_E_ARG, "z is NULL");
  GUARD_BEGIN
  const Pat& pt = ctx->H.pat[patient];
  std::vector<float> v(pt.n);
  check(hipStreamSynchronize(ctx->stream), "sync");
  check(hipMemcpy(v.data(), ctx->d_z + pt.zvec_base, sizeof(float) * pt.n, hipMemcpyDeviceToHost), "D2H");
  for (int j = 0; j < pt.n; ++j) z[j] = v[j];
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_get_rho(const admm_ctx* ctx, int32_t patient, double* rho) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (rho) *rho = ctx->rho[patient];
  return ADMM_OK;
}

admm_status admm_get_sizes(const admm_ctx* ctx, int32_t patient, int32_t* n, int32_t* m, int32_t* num_scen,
                           int64_t* nnz) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  const Pat& pt = ctx->H.pat[patient];
  if (n) *n = pt.n;
  if (m) *m = pt.m;
  if (num_scen) *num_scen = pt.num_scen;
  if (nnz) {
    int64_t t = 0;
    for (int s = 0; s < pt.num_scen; ++s) t += ctx->H.scen_nnz[pt.scen_begin + s];
    *nnz = t;
  }
  return ADMM_OK;
}

admm_status admm_objective(admm_ctx* ctx, int32_t patient, const double* x, double* f_out) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!x || !f_out) return set_err(ctx, ADMM_E_ARG, "NULL argument");
  GUARD_BEGIN
  ctx->upload_pvec(patient, x, ctx->d_pvec);
  *f_out = ctx->objective_dev(patient, nullptr);
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_gradient(admm_ctx* ctx, int32_t patient, const double* x, double* grad_out, double* f_out) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!x || !grad_out) return set_err(ctx, ADMM_E_ARG, "NULL argument");
  GUARD_BEGIN
  const Pat& pt = ctx->H.pat[patient];
  ctx->upload_pvec(patient, x, ctx->d_pvec);
  const double f = ctx->objective_dev(patient, ctx->d_pvec2 + pt.zvec_base);
  std::vector<float> g(pt.n);
  check(hipMemcpy(g.data(), ctx->d_pvec2 + pt.zvec_base, sizeof(float) * pt.n, hipMemcpyDeviceToHost), "D2H");
  for (int j = 0; j < pt.n; ++j) grad_out[j] = g[j];
  if (f_out) *f_out = f;
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_kkt(admm_ctx* ctx, int32_t patient, const double* x, double* r_out) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!x || !r_out) return set_err(ctx, ADMM_E_ARG, "NULL argument");
  const Pat& pt = ctx->H.pat[patient];
  std::vector<double> g(pt.n);
  st = admm_gradient(ctx, patient, x, g.data(), nullptr);
  if (st != ADMM_OK) return st;
  double gi = 0.0, r = 0.0;
  for (int j = 0; j < pt.n; ++j) gi = std::max(gi, std::fabs(ctx->H.g0[patient][j]));
  for (int j = 0; j < pt.n; ++j) {
    const double lo = ctx->H.lb[pt.zvec_base + j], hi = ctx->H.ub[pt.zvec_base + j];
    const double pj = std::min(std::max(x[j] - g[j], lo), hi);
    r = std::max(r, std::fabs(x[j] - pj));
  }
  *r_out = r / std::max(1.0, gi);
  return ADMM_OK;
}

static admm_status scen_index(admm_ctx* ctx, int32_t patient, int32_t scen, int* g) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  const Pat& pt = ctx->H.pat[patient];
  if (scen < 0 || scen >= pt.num_scen) return set_err(ctx, ADMM_E_ARG, "scenario index out of range");
  *g = pt.scen_begin + scen;
  return ADMM_OK;
}

admm_status admm_matvec(admm_ctx* ctx, int32_t patient, int32_t scen, const float* v, float* out) {
  int g = 0;
  admm_status st = scen_index(ctx, patient, scen, &g);
  if (st != ADMM_OK) return st;
  if (!v || !out) return set_err(ctx, ADMM_E_ARG, "NULL argument");
  GUARD_BEGIN
  ctx->ensure_forward_tuned();
  const Pat& pt = ctx->H.pat[patient];
  const Scen& sc = ctx->H.scen[g];
  check(hipMemcpyAsync(ctx->d_pvec + pt.zvec_base, v, sizeof(float) * pt.n, hipMemcpyHostToDevice, ctx->stream), "H2D");
  launch_fill_f32(ctx->d_mvec, 0.0f, pt.m, ctx->stream);
  PassArgs pa = ctx->pass_args(ctx->mat32);
  pa.src = ctx->d_pvec;
  pa.src_per_scen = 0;
  pa.tout = ctx->d_mvec;
  pa.objpart = nullptr;
  ctx->pass_launch(PASS_MATVEC, pa, sc.tile_begin, sc.tile_end - sc.tile_begin);
  check(hipMemcpyAsync(out, ctx->d_mvec, sizeof(float) * pt.m, hipMemcpyDeviceToHost, ctx->stream), "D2H");
  check(hipStreamSynchronize(ctx->stream), "sync");
  return ADMM_OK;
  GUARD_END(ctx)
}

}  // extern "C"

namespace {

admm_status dose_stats_check(admm_ctx* ctx, int32_t patient, const double* x, const uint8_t* voxel_group,
                             int32_t num_groups, int32_t nbins, double dmax, uint32_t* counts, double* sums,
                             float* maxes) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!x || !voxel_group || !counts || !sums || !maxes) return set_err(ctx, ADMM_E_ARG, "NULL argument");
  if (num_groups < 1 || num_groups > 256 || nbins < 1 || !(dmax > 0) || !std::isfinite(dmax) ||
      dose_hist_smem_bytes(num_groups, nbins) > 65536)
    return set_err(ctx, ADMM_E_ARG, "need 1 <= num_groups <= 256, nbins >= 1, 12 G + 4 G nbins <= 65536, dmax > 0");
  const Pat& pt = ctx->H.pat[patient];
  for (int i = 0; i < pt.m; ++i)
    if (voxel_group[i] >= num_groups) return set_err(ctx, ADMM_E_ARG, "voxel_group entry >= num_groups");
  for (int j = 0; j < pt.n; ++j)
    if (!std::isfinite(x[j])) return set_err(ctx, ADMM_E_NONFINITE, "x is not finite");
  return ADMM_OK;
}

// Queue the dose statistics of the plan already in d_pvec (fp32) into the
// device arrays grp / cnt / key / sum (cnt, key, sum cleared here by fill
// kernels), and the doses into dose_out when given; then the copies of the
// counts, sums and max keys (into maxes, as 32-bit keys) back to the host, and
// wait for them.
void dose_stats_queue(admm_ctx* ctx, int32_t patient, const uint8_t* d_grp, uint32_t* d_cnt, uint32_t* d_key,
                      double* d_sum, int G, int nbins, double dmax, uint32_t* counts, double* sums, float* maxes,
                      float* dose_out) {
  const Pat& pt = ctx->H.pat[patient];
  const int N = pt.num_scen, m = pt.m;
  const size_t per = static_cast<size_t>(G) * nbins;
  static_assert(sizeof(float) == sizeof(uint32_t), "fill by bit pattern");
  launch_fill_f32(reinterpret_cast<float*>(d_cnt), 0.0f, static_cast<int64_t>(per * N), ctx->stream);
  launch_fill_f32(reinterpret_cast<float*>(d_key), 0.0f, static_cast<int64_t>(G) * N, ctx->stream);
  launch_fill_f64(d_sum, 0.0, static_cast<int64_t>(G) * N, ctx->stream);
  const float inv_w = static_cast<float>(nbins / dmax);
  for (int s = 0; s < N; ++s) {
    const Scen& sc = ctx->H.scen[pt.scen_begin + s];
    launch_fill_f32(ctx->d_mvec, 0.0f, m, ctx->stream);
    PassArgs pa = ctx->pass_args(ctx->mat32);
    pa.src = ctx->d_pvec;
    pa.src_per_scen = 0;
    pa.tout = ctx->d_mvec;
    pa.objpart = nullptr;
    ctx->pass_launch(PASS_MATVEC, pa, sc.tile_begin, sc.tile_end - sc.tile_begin);
    launch_dose_hist(ctx->d_mvec, d_grp, m, G, nbins, inv_w, d_cnt + per * s, d_sum + static_cast<size_t>(G) * s,
                     d_key + static_cast<size_t>(G) * s, ctx->stream);
    if (dose_out)
      check(hipMemcpyAsync(dose_out + static_cast<size_t>(s) * m, ctx->d_mvec, sizeof(float) * m,
                           hipMemcpyDeviceToHost, ctx->stream),
            "D2H");
  }
  check(hipGetLastError(), "launch");
  check(hipMemcpyAsync(counts, d_cnt, sizeof(uint32_t) * per * N, hipMemcpyDeviceToHost, ctx->stream), "D2H");
  check(hipMemcpyAsync(sums, d_sum, sizeof(double) * G * N, hipMemcpyDeviceToHost, ctx->stream), "D2H");
  check(hipMemcpyAsync(maxes, d_key, sizeof(uint32_t) * G * N, hipMemcpyDeviceToHost, ctx->stream), "D2H");
  check(hipStreamSynchronize(ctx->stream), "sync");
  // order-preserving keys back to floats, in place (0 marks an empty group)
  for (size_t k = 0; k < static_cast<size_t>(G) * N; ++k) {
    uint32_t key;
    std::memcpy(&key, maxes + k, sizeof(key));
    if (key == 0u) {
      maxes[k] = -INFINITY;
      continue;
    }
    const uint32_t u = (key & 0x80000000u) ? (key & 0x7fffffffu) : ~key;
    std::memcpy(maxes + k, &u, sizeof(u));
  }
}

}  // namespace

extern "C" {

admm_status admm_dose_stats(admm_ctx* ctx, int32_t patient, const double* x, const uint8_t* voxel_group,
                            int32_t num_groups, int32_t nbins, double dmax, uint32_t* counts, double* sums,
                            float* maxes, float* dose_out) {
  admm_status st = dose_stats_check(ctx, patient, x, voxel_group, num_groups, nbins, dmax, counts, sums, maxes);
  if (st != ADMM_OK) return st;
  GUARD_BEGIN
  const Pat& pt = ctx->H.pat[patient];
  const int N = pt.num_scen, m = pt.m, G = num_groups;
  const size_t per = static_cast<size_t>(G) * nbins;
  uint8_t* d_grp = nullptr;
  uint32_t* d_cnt = nullptr;
  uint32_t* d_key = nullptr;
  double* d_sum = nullptr;
  auto release = [&]() {
    if (d_grp) (void)hipFree(d_grp);
    if (d_cnt) (void)hipFree(d_cnt);
    if (d_key) (void)hipFree(d_key);
    if (d_sum) (void)hipFree(d_sum);
  };
  try {
    check(hipMalloc(reinterpret_cast<void**>(&d_grp), m), "hipMalloc");
    check(hipMalloc(reinterpret_cast<void**>(&d_cnt), sizeof(uint32_t) * per * N), "hipMalloc");
    check(hipMalloc(reinterpret_cast<void**>(&d_key), sizeof(uint32_t) * G * N), "hipMalloc");
    check(hipMalloc(reinterpret_cast<void**>(&d_sum), sizeof(double) * G * N), "hipMalloc");
    check(hipMemcpyAsync(d_grp, voxel_group, m, hipMemcpyHostToDevice, ctx->stream), "H2D");
    ctx->upload_pvec(patient, x, ctx->d_pvec);
    dose_stats_queue(ctx, patient, d_grp, d_cnt, d_key, d_sum, G, nbins, dmax, counts, sums, maxes, dose_out);
  } catch (...) {
    release();
    throw;
  }
  release();
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_dose_stats_noalloc(admm_ctx* ctx, int32_t patient, const double* x, const uint8_t* voxel_group,
                                    int32_t num_groups, int32_t nbins, double dmax, uint32_t* counts, double* sums,
                                    float* maxes, float* dose_out) {
  admm_status st = dose_stats_check(ctx, patient, x, voxel_group, num_groups, nbins, dmax, counts, sums, maxes);
  if (st != ADMM_OK) return st;
  const Pat& pt = ctx->H.pat[patient];
  const size_t N = static_cast<size_t>(pt.num_scen), G = static_cast<size_t>(num_groups);
  auto up = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
  const size_t o_cnt = up(static_cast<size_t>(pt.m));
  const size_t o_key = o_cnt + up(sizeof(uint32_t) * N * G * static_cast<size_t>(nbins));
  const size_t o_sum = o_key + up(sizeof(uint32_t) * N * G);
  const size_t o_x = o_sum + up(sizeof(double) * N * G);
  const size_t need = o_x + up(sizeof(double) * static_cast<size_t>(pt.n));
  if (need > kNoAllocScratchBytes)
    return set_err(ctx, ADMM_E_ARG,
                   "admm_dose_stats_noalloc needs " + std::to_string(need) + " bytes of scratch (m + 4 N G nbins + "
                   "12 N G + 8 n, each rounded up to 256); the fixed scratch holds " +
                       std::to_string(kNoAllocScratchBytes));
  GUARD_BEGIN
  void* base = nullptr;
  check(noalloc_scratch(&base), "hipGetSymbolAddress");
  unsigned char* sp = static_cast<unsigned char*>(base);
  uint8_t* d_grp = sp;
  uint32_t* d_cnt = reinterpret_cast<uint32_t*>(sp + o_cnt);
  uint32_t* d_key = reinterpret_cast<uint32_t*>(sp + o_key);
  double* d_sum = reinterpret_cast<double*>(sp + o_sum);
  double* d_x = reinterpret_cast<double*>(sp + o_x);
  check(hipMemcpyAsync(d_grp, voxel_group, static_cast<size_t>(pt.m), hipMemcpyHostToDevice, ctx->stream), "H2D");
  check(hipMemcpyAsync(d_x, x, sizeof(double) * static_cast<size_t>(pt.n), hipMemcpyHostToDevice, ctx->stream), "H2D");
  launch_f64_to_f32(d_x, ctx->d_pvec + pt.zvec_base, pt.n, ctx->stream);
  dose_stats_queue(ctx, patient, d_grp, d_cnt, d_key, d_sum, num_groups, nbins, dmax, counts, sums, maxes, dose_out);
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_rmatvec(admm_ctx* ctx, int32_t patient, int32_t scen, const float* t, float* out) {
  int g = 0;
  admm_status st = scen_index(ctx, patient, scen, &g);
  if (st != ADMM_OK) return st;
  if (!t || !out) return set_err(ctx, ADMM_E_ARG, "NULL argument");
  GUARD_BEGIN
  ctx->ensure_forward_tuned();
  const Pat& pt = ctx->H.pat[patient];
  const Scen& sc = ctx->H.scen[g];
  check(hipMemcpyAsync(ctx->d_mvec, t, sizeof(float) * pt.m, hipMemcpyHostToDevice, ctx->stream), "H2D");
  PassArgs pa = ctx->pass_args(ctx->mat32);
  pa.objpart = nullptr;
  ctx->rmatvec_launch(pa, ctx->d_mvec, pt.m, sc.tile_begin, sc.tile_end - sc.tile_begin);
  VecArgs va = ctx->vec_args(0);
  va.out = ctx->d_pvec2 + pt.zvec_base;
  launch_reduce(RED_RMAT, va, sc.blk_begin, sc.nblk, ctx->stream);
  check(hipMemcpyAsync(out, va.out, sizeof(float) * pt.n, hipMemcpyDeviceToHost, ctx->stream), "D2H");
  check(hipStreamSynchronize(ctx->stream), "sync");
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_normal_apply(admm_ctx* ctx, int32_t patient, int32_t scen, int32_t precision, const float* v,
                              float* out) {
  int g = 0;
  admm_status st = scen_index(ctx, patient, scen, &g);
  if (st != ADMM_OK) return st;
  if (!v || !out) return set_err(ctx, ADMM_E_ARG, "NULL argument");
  if (precision != ADMM_PREC_FP32 && precision != ctx->opts.precision)
    return set_err(ctx, ADMM_E_ARG, "that value precision was not set up for this context");
  GUARD_BEGIN
  const Pat& pt = ctx->H.pat[patient];
  const Scen& sc = ctx->H.scen[g];
  // the input goes where the CG direction of this scenario lives (scratch between iterations)
  check(hipMemcpyAsync(ctx->d_v + sc.vec_base, v, sizeof(float) * pt.n, hipMemcpyHostToDevice, ctx->stream), "H2D");
  PassArgs pa = ctx->pass_args(precision == ADMM_PREC_FP32 ? ctx->mat32 : ctx->matlp);
  pa.src = ctx->d_v;
  pa.src_per_scen = 1;
  pa.objpart = nullptr;
  ctx->pass_launch(PASS_CG, pa, sc.tile_begin, sc.tile_end - sc.tile_begin);
  VecArgs va = ctx->vec_args(0);
  va.out = ctx->d_pvec2 + pt.zvec_base;
  va.rho_out = ctx->rho[patient];
  launch_reduce(RED_NORMAL, va, sc.blk_begin, sc.nblk, ctx->stream);
  check(hipMemcpyAsync(out, va.out, sizeof(float) * pt.n, hipMemcpyDeviceToHost, ctx->stream), "D2H");
  check(hipStreamSynchronize(ctx->stream), "sync");
  return ADMM_OK;
  GUARD_END(ctx)
}

namespace {

// PGD on the packed fp64 sum of the Gram matrices, every iteration on the device.
admm_status pgd_dense(admm_ctx* ctx, const pgd_options& o, int32_t patient, const double* x0, double* x_out,
                      admm_info* info) {
  const Pat& pt = ctx->H.pat[patient];
  const int n = pt.n;
  hipStream_t s = ctx->stream;
  if (!ctx->d_pgd) {
    int64_t words = 0;
    for (const Pat& q : ctx->H.pat) {
      const int64_t nj = q.fobj_end - q.fobj_begin, nbl = (q.npad + 255) / 256;
      words = std::max(words, (2 + 2 * kPgdK) * static_cast<int64_t>(q.npad) + nj * kPgdK * 128 + q.nbk * kPgdK +
                                  2 * nbl * kPgdK);
    }
    ctx->d_pgd = ctx->alloc<double>(static_cast<size_t>(words));
    ctx->d_pgdst = ctx->alloc<PgdDevState>(2);
  }
  PgdArgs a{};
  a.Gp = ctx->d_Gp + pt.gpack_off;
  a.g0 = ctx->d_g0 + pt.zvec_base;
  a.lb = ctx->d_lb + pt.zvec_base;
  a.ub = ctx->d_ub + pt.zvec_base;
  a.jobs = ctx->d_fjobs + pt.fobj_begin;
  a.njobs = pt.fobj_end - pt.fobj_begin;
  a.nb = pt.nbk;
  a.n = n;
  a.np = pt.npad;
  a.nblocks = (a.np + 255) / 256;
  a.x = ctx->d_pgd;
  a.g = a.x + a.np;
  a.xc = a.g + a.np;
  a.u = a.xc + static_cast<int64_t>(kPgdK) * a.np;
  a.part = a.u + static_cast<int64_t>(kPgdK) * a.np;
  a.fpart = a.part + static_cast<int64_t>(a.njobs) * kPgdK * 128;
  a.gdpart = a.fpart + static_cast<int64_t>(a.nb) * kPgdK;
  a.st = ctx->d_pgdst;
  a.fconst = pt.fconst;
  a.beta = o.beta;
  a.gamma = o.gamma;
  a.tol = o.obj_rel_tol;
  a.max_iter = o.max_iter;
  a.max_trials = o.max_trials;

  // host sources stay alive and unchanged until the final synchronisation,
  // also when a failed call below leaves the function by an exception
  PgdDevState h0[2] = {}, h{};
  std::vector<double> pv, hv(n);
  StreamDrain drain{s};
  for (PgdDevState& e : h0) {
    e.alpha = o.alpha > 0 ? o.alpha : 1.0;
    e.pick = -1;
  }
  check(hipMemcpyAsync(a.st, h0, sizeof(h0), hipMemcpyHostToDevice, s), "H2D");
  launch_fill_f64(a.x, 0.0, 2 * static_cast<int64_t>(a.np), s);  // x and g, with their zero padding
  if (!(o.alpha > 0)) {
    // alpha = 10 / lambda_max(H), H = 2 sum_s G_s, 30 power iterations
    pv.assign(n, 1.0 / std::sqrt(static_cast<double>(n)));
    check(hipMemcpyAsync(a.x, pv.data(), sizeof(double) * n, hipMemcpyHostToDevice, s), "H2D");
    for (int it = 0; it < 30; ++it) launch_pgd_power(a, a.x, s);
  }
  for (int j = 0; j < n; ++j) {
    const double v = x0 ? x0[j] : 0.0;
    hv[j] = std::min(std::max(v, static_cast<double>(ctx->H.lb[pt.zvec_base + j])),
                     static_cast<double>(ctx->H.ub[pt.zvec_base + j]));
  }
  check(hipMemcpyAsync(a.x, hv.data(), sizeof(double) * n, hipMemcpyHostToDevice, s), "H2D");
  launch_fill_f64(a.g, 0.0, n, s);
  static_assert(kPgdK % 2 == 0, "sub-buffers of the PGD work area stay 16-byte aligned");
  // state slot 0 carries alpha from the power iteration; every launch of the
  // step kernel reads slot par and writes slot par ^ 1
  int par = 0;
  launch_pgd_prime(a, par, s);  // t_base = 0: every trial point is x
  par ^= 1;
  launch_pgd_round(a, 1, par, s);
  par ^= 1;
  // every round either accepts a step or rejects kPgdK trial steps, so the
  // device state reaches done within this many rounds
  const int64_t max_rounds =
      1 + static_cast<int64_t>(o.max_iter) * ((o.max_trials + kPgdK - 1) / kPgdK);
  constexpr int kChunk = 16;
  for (int64_t r = 1; r <= max_rounds; r += kChunk) {
    const int64_t c = std::min<int64_t>(kChunk, max_rounds - r + 1);
    for (int64_t k = 0; k < c; ++k) {
      launch_pgd_round(a, 0, par, s);
      par ^= 1;
    }
    check(hipGetLastError(), "PGD launch");
    check(hipMemcpyAsync(&h, a.st + par, sizeof(h), hipMemcpyDeviceToHost, s), "D2H");
    check(hipStreamSynchronize(s), "sync");
    if (h.done) break;
  }
  check(hipMemcpyAsync(&h, a.st + par, sizeof(h), hipMemcpyDeviceToHost, s), "D2H");
  if (x_out) check(hipMemcpyAsync(x_out, a.x, sizeof(double) * n, hipMemcpyDeviceToHost, s), "D2H");
  check(hipStreamSynchronize(s), "sync");
  const bool converged = h.done && h.status == 1;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->iter = h.iter;
    info->obj = h.f;
    info->tau = h.alpha;
    info->status = converged ? ADMM_OK : ADMM_MAX_ITER;
  }
  return converged ? ADMM_OK : ADMM_MAX_ITER;
}

}  // namespace

namespace {
admm_status pgd_solve_impl(admm_ctx* ctx, const pgd_options* popts, int32_t patient, const double* x0,
                           double* x_out, admm_info* info) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  pgd_options o;
  pgd_default_options(&o);
  if (popts) o = *popts;
  if (!(o.beta > 0 && o.beta < 1) || !(o.gamma > 0 && o.gamma < 1) || o.max_trials < 1 || o.max_iter < 0 ||
      !(o.obj_rel_tol >= 0) || !std::isfinite(o.alpha) || o.dense < -1 || o.dense > 1)
    return set_err(ctx, ADMM_E_ARG, "invalid PGD options");
  if (o.dense == 1 && !ctx->dense)
    return set_err(ctx, ADMM_E_ARG, "dense PGD needs a context set up with the dense x-update");
  if (o.dense != 0 && ctx->dense) {
    GUARD_BEGIN
    return pgd_dense(ctx, o, patient, x0, x_out, info);
    GUARD_END(ctx)
  }
  GUARD_BEGIN
  ctx->ensure_forward_tuned();
  const Pat& pt = ctx->H.pat[patient];
  const int n = pt.n;
  float* x = ctx->d_pvec + pt.zvec_base;
  float* g = ctx->d_pvec2 + pt.zvec_base;
  float* xt = ctx->d_pvec3 + pt.zvec_base;
  const float* lb = ctx->d_lb + pt.zvec_base;
  const float* ub = ctx->d_ub + pt.zvec_base;
  hipStream_t s = ctx->stream;
  double alpha = o.alpha;
  if (!(alpha > 0)) {
    // largest eigenvalue of H = 2 sum_s A_s^T c_s W A_s by power iteration
    std::vector<float> v(n, static_cast<float>(1.0 / std::sqrt(static_cast<double>(n))));
    StreamDrain drain{s};
    double lam = 0.0;
    for (int it = 0; it < 30; ++it) {
      check(hipMemcpyAsync(xt, v.data(), sizeof(float) * n, hipMemcpyHostToDevice, s), "H2D");
      PassArgs pa = ctx->pass_args(ctx->mat32);
      pa.src = ctx->d_pvec3;
      pa.src_per_scen = 0;
      pa.objpart = nullptr;
      ctx->pass_launch(PASS_CG, pa, pt.tile_begin, pt.tile_end - pt.tile_begin);
      launch_gsum(ctx->d_scen, ctx->d_pat, ctx->d_pblk, ctx->d_tiles, ctx->d_part, pt.blk_begin, pt.nblk, 2.0f, g, s);
      check(hipMemcpyAsync(v.data(), g, sizeof(float) * n, hipMemcpyDeviceToHost, s), "D2H");
      check(hipStreamSynchronize(s), "sync");
      double nrm = 0.0;
      for (float e : v) nrm += static_cast<double>(e) * e;
      nrm = std::sqrt(nrm);
      lam = nrm;
      if (!(nrm > 0)) break;
      for (float& e : v) e = static_cast<float>(e / nrm);
    }
    alpha = lam > 0 ? 10.0 / lam : 1.0;
  }
  std::vector<double> x0v(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double v = x0 ? x0[j] : 0.0;
    x0v[j] = std::min(std::max(v, static_cast<double>(ctx->H.lb[pt.zvec_base + j])),
                      static_cast<double>(ctx->H.ub[pt.zvec_base + j]));
  }
  ctx->upload_pvec(patient, x0v.data(), ctx->d_pvec);
  double f = ctx->objective_dev(patient, g);
  const int nb = (n + kThreads - 1) / kThreads;
  int iters = 0;
  bool converged = false, failed = false;
  for (int k = 0; k < o.max_iter; ++k) {
    double t = alpha;
    bool accepted = false;
    double ft = 0.0;
    for (int trial = 0; trial < o.max_trials; ++trial) {
      launch_pgd_trial(x, g, lb, ub, static_cast<float>(t), xt, n, ctx->d_scratch + 8, s);
      launch_dot_sum(ctx->d_scratch + 8, nb, ctx->d_scratch + 1, s);
      PassArgs pa = ctx->pass_args(ctx->mat32);
      pa.src = ctx->d_pvec3;
      pa.src_per_scen = 0;
      pa.part = nullptr;  // objective only
      ctx->pass_launch(PASS_OBJ, pa, pt.tile_begin, pt.tile_end - pt.tile_begin);
      launch_objsum(ctx->d_tiles, ctx->d_objpart, pt.tile_begin, pt.tile_end - pt.tile_begin, ctx->d_scratch, s);
      check(hipMemcpyAsync(ctx->h_scr, ctx->d_scratch, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "D2H");
      check(hipStreamSynchronize(s), "sync");
      ft = ctx->h_scr[0] + pt.fzero;
      const double gd = ctx->h_scr[1];
      if (ft <= f + o.beta * gd) {
        accepted = true;
        break;
      }
      t *= o.gamma;
    }
    iters = k + 1;
    if (!accepted) {
      failed = true;
      break;
    }
    check(hipMemcpyAsync(x, xt, sizeof(float) * n, hipMemcpyDeviceToDevice, s), "D2D");
    const double f_old = f;
    f = ctx->objective_dev(patient, g);
    if (std::fabs(f_old - f) <= o.obj_rel_tol * std::fabs(f_old)) {
      converged = true;
      break;
    }
  }
  if (x_out) {
    std::vector<float> xv(n);
    check(hipMemcpyAsync(xv.data(), x, sizeof(float) * n, hipMemcpyDeviceToHost, s), "D2H");
    check(hipStreamSynchronize(s), "sync");
    for (int j = 0; j < n; ++j) x_out[j] = xv[j];
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->iter = iters;
    info->obj = f;
    info->tau = alpha;
    info->status = converged ? ADMM_OK : ADMM_MAX_ITER;
  }
  (void)failed;
  return converged ? ADMM_OK : ADMM_MAX_ITER;
  GUARD_END(ctx)
}
}  // namespace

admm_status pgd_solve(admm_ctx* ctx, const pgd_options* popts, int32_t patient, const double* x0, double* x_out,
                      admm_info* info) {
  const admm_status st = pgd_solve_impl(ctx, popts, patient, x0, x_out, info);
  if (st < 0 || !info) return st;
  info->kkt = -1.0;
  if (x_out) {
    double r = -1.0;
    const admm_status ks = admm_kkt(ctx, patient, x_out, &r);
    if (ks != ADMM_OK) return ks;
    info->kkt = r;
  }
  return st;
}

admm_status admm_get_state(admm_ctx* ctx, int32_t patient, double* z, double* y, double* d, double* scalars) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  GUARD_BEGIN
  const Pat& pt = ctx->H.pat[patient];
  const int64_t len = static_cast<int64_t>(pt.num_scen) * pt.n;
  const int64_t base = ctx->H.scen[pt.scen_begin].vec_base;
  check(hipStreamSynchronize(ctx->stream), "sync");
  if (z) {
    std::vector<float> v(pt.n);
    check(hipMemcpy(v.data(), ctx->d_z + pt.zvec_base, sizeof(float) * pt.n, hipMemcpyDeviceToHost), "D2H");
    for (int j = 0; j < pt.n; ++j) z[j] = v[j];
  }
  if (y) {
    std::vector<float> v(len);
    check(hipMemcpy(v.data(), ctx->d_y + base, sizeof(float) * len, hipMemcpyDeviceToHost), "D2H");
    for (int64_t j = 0; j < len; ++j) y[j] = v[j];
  }
  if (d) check(hipMemcpy(d, ctx->d_dprev + base, sizeof(double) * len, hipMemcpyDeviceToHost), "D2H");
  if (scalars) {
    ctx->read_state();
    const PatState& s = ctx->h_ps[patient];
    scalars[0] = s.iter;
    scalars[1] = s.tau;
    scalars[2] = s.f_prev;
    scalars[3] = s.pending;
    scalars[4] = s.stopped;
    scalars[5] = s.status;
    scalars[6] = s.rho;
    scalars[7] = s.cg_total;
    scalars[8] = s.f_cur;
    scalars[9] = s.r_prim;
    scalars[10] = s.r_dual;
    scalars[11] = s.eps_prim;
    scalars[12] = s.eps_dual;
    scalars[13] = s.xnorm;
    scalars[14] = s.znorm;
    scalars[15] = s.cg_steps;
  }
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_set_state(admm_ctx* ctx, int32_t patient, const double* z, const double* y, const double* d,
                           const double* scalars) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!z || !y || !d || !scalars) return set_err(ctx, ADMM_E_ARG, "NULL argument");
  const Pat& pt = ctx->H.pat[patient];
  const int64_t len = static_cast<int64_t>(pt.num_scen) * pt.n;
  for (int64_t j = 0; j < len; ++j)
    if (!std::isfinite(y[j]) || !std::isfinite(d[j])) return set_err(ctx, ADMM_E_NONFINITE, "state not finite");
  if (scalars[6] > 0 && scalars[6] != ctx->rho[patient] && ctx->opts.precond)
    return set_err(ctx, ADMM_E_STATE, "rho differs from the preconditioner's");
  GUARD_BEGIN
  const int64_t base = ctx->H.scen[pt.scen_begin].vec_base;
  std::vector<float> zf(pt.n), yf(len);
  for (int j = 0; j < pt.n; ++j) zf[j] = static_cast<float>(z[j]);
  for (int64_t j = 0; j < len; ++j) yf[j] = static_cast<float>(y[j]);
  check(hipStreamSynchronize(ctx->stream), "sync");
  check(hipMemcpy(ctx->d_z + pt.zvec_base, zf.data(), sizeof(float) * pt.n, hipMemcpyHostToDevice), "H2D");
  check(hipMemcpy(ctx->d_y + base, yf.data(), sizeof(float) * len, hipMemcpyHostToDevice), "H2D");
  check(hipMemcpy(ctx->d_dprev + base, d, sizeof(double) * len, hipMemcpyHostToDevice), "H2D");
  if (scalars[6] > 0) ctx->rho[patient] = scalars[6];
  if (ctx->dense && ctx->factored_rho[patient] != ctx->rho[patient]) ctx->factorize(patient, false);
  PatState s{};
  s.iter = static_cast<int32_t>(scalars[0]);
  s.tau = scalars[1];
  s.f_prev = scalars[2];
  s.pending = static_cast<int32_t>(scalars[3]);
  s.stopped = static_cast<int32_t>(scalars[4]);
  s.status = static_cast<int32_t>(scalars[5]);
  s.rho = ctx->rho[patient];
  s.cg_total = static_cast<int32_t>(scalars[7]);
  s.f_cur = scalars[8];
  s.r_prim = scalars[9];
  s.r_dual = scalars[10];
  s.eps_prim = scalars[11];
  s.eps_dual = scalars[12];
  s.xnorm = scalars[13];
  s.znorm = scalars[14];
  s.cg_steps = static_cast<int32_t>(scalars[15]);
  s.bb_tau0 = s.tau;
  s.bb_iter0 = s.iter;
  ctx->h_ps[patient] = s;
  check(hipMemcpy(ctx->d_ps + patient, &s, sizeof(PatState), hipMemcpyHostToDevice), "H2D");
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_time_pass(admm_ctx* ctx, int32_t kind, int32_t reps, double* ms_out) {
  if (!ctx || !ms_out || kind < 0 || kind > 2 || reps < 1) return set_err(ctx, ADMM_E_ARG, "bad argument");
  GUARD_BEGIN
  ctx->ensure_forward_tuned();
  PassArgs pa = ctx->pass_args(ctx->mat32);
  int mode = PASS_CG;
  if (kind == 0) {
    mode = PASS_OBJ;
    pa.src = ctx->d_z;
    pa.src_per_scen = 0;
    pa.part = nullptr;
  } else if (kind == 1) {
    mode = PASS_RMATVEC;
    launch_fill_f32(ctx->d_mvec, 1.0f, ctx->H.mmax, ctx->stream);
    pa.objpart = nullptr;
  } else {
    pa.src = ctx->d_v;
    pa.src_per_scen = 1;
    pa.objpart = nullptr;
  }
  hipEvent_t e0, e1;
  check(hipEventCreate(&e0), "hipEventCreate");
  check(hipEventCreate(&e1), "hipEventCreate");
  float ms = 0.0f;
  // every pass over all tiles; the transpose product with its max |t| launch
  auto one = [&]() {
    if (mode == PASS_RMATVEC)
      ctx->rmatvec_launch(pa, ctx->d_mvec, ctx->H.mmax, 0, ctx->T);
    else
      ctx->pass_launch(mode, pa, 0, ctx->T);
  };
  try {
    one();  // warm
    check(hipEventRecord(e0, ctx->stream), "hipEventRecord");
    for (int r = 0; r < reps; ++r) one();
    check(hipEventRecord(e1, ctx->stream), "hipEventRecord");
    check(hipEventSynchronize(e1), "hipEventSynchronize");
    check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_out = static_cast<double>(ms) / reps;
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_get_format(const admm_ctx* ctx, int32_t* format) {
  if (!ctx || !format) return ADMM_E_ARG;
  *format = ctx->fmt == FMT_SELL ? ADMM_FORMAT_SELL : ADMM_FORMAT_CSR;
  return ADMM_OK;
}

admm_status admm_get_tuning(const admm_ctx* ctx, int32_t* threads, int32_t* unroll, int32_t* lds_acc, double* ms) {
  if (!ctx) return ADMM_E_ARG;
  if (threads) *threads = ctx->pass_threads;
  if (unroll) *unroll = ctx->pass_unroll;
  if (lds_acc) *lds_acc = ctx->acc;
  if (ms) *ms = ctx->tuned_ms;
  return ADMM_OK;
}

admm_status admm_get_pass_config(const admm_ctx* ctx, int32_t patient, int32_t* threads, int32_t* unroll,
                                 int32_t* lds_acc, int32_t* format, double* ms) {
  if (!ctx) return ADMM_E_ARG;
  if (patient < 0 || patient >= ctx->P || static_cast<size_t>(patient) >= ctx->pcfg.size()) return ADMM_E_ARG;
  const auto& c = ctx->pcfg[static_cast<size_t>(patient)];
  if (threads) *threads = c.threads;
  if (unroll) *unroll = c.unroll;
  if (lds_acc) *lds_acc = c.acc;
  if (format) *format = (c.fmt == FMT_SELL && ctx->has_sell) ? ADMM_FORMAT_SELL : ADMM_FORMAT_CSR;
  if (ms) *ms = c.ms;
  return ADMM_OK;
}

admm_status admm_get_forward_config(const admm_ctx* ctx, int32_t patient, int32_t* threads, int32_t* unroll,
                                    double* ms) {
  if (!ctx) return ADMM_E_ARG;
  if (patient < 0 || patient >= ctx->P || static_cast<size_t>(patient) >= ctx->pcfg.size()) return ADMM_E_ARG;
  const auto& c = ctx->pcfg[static_cast<size_t>(patient)];
  if (threads) *threads = c.fthreads;
  if (unroll) *unroll = c.funroll;
  if (ms) *ms = c.fms;
  return ADMM_OK;
}

admm_status admm_get_cg_counts(admm_ctx* ctx, int32_t patient, int64_t* counts) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!counts) return set_err(ctx, ADMM_E_ARG, "counts is NULL");
  GUARD_BEGIN
  const Pat& pt = ctx->H.pat[patient];
  check(hipStreamSynchronize(ctx->stream), "sync");
  check(hipMemcpy(counts, ctx->d_cgtotal + pt.scen_begin, sizeof(int64_t) * pt.num_scen, hipMemcpyDeviceToHost),
        "D2H");
  return ADMM_OK;
  GUARD_END(ctx)
}

admm_status admm_get_trace(admm_ctx* ctx, int32_t patient, admm_info* buf, int32_t cap, int32_t* count) {
  admm_status st = check_patient(ctx, patient);
  if (st != ADMM_OK) return st;
  if (!buf || cap < 0) return set_err(ctx, ADMM_E_ARG, "bad buffer");
  GUARD_BEGIN
  ctx->read_state();
  const int have = std::min(ctx->h_ps[patient].iter, ctx->trace_cap);
  const int k = std::min(have, cap);
  std::vector<IterRecord> rec(static_cast<size_t>(std::max(k, 1)));
  if (k > 0)
    check(hipMemcpy(rec.data(), ctx->d_trace + static_cast<int64_t>(patient) * ctx->trace_cap,
                    sizeof(IterRecord) * k, hipMemcpyDeviceToHost),
          "D2H");
  for (int i = 0; i < k; ++i) {
    std::memset(&buf[i], 0, sizeof(admm_info));
    buf[i].iter = rec[i].iter;
    buf[i].cg_steps = rec[i].cg_steps;
    buf[i].obj = rec[i].obj;
    buf[i].r_prim = rec[i].r_prim;
    buf[i].r_dual = rec[i].r_dual;
    buf[i].eps_prim = rec[i].eps_prim;
    buf[i].eps_dual = rec[i].eps_dual;
    buf[i].tau = rec[i].tau;
  }
  if (count) *count = k;
  return ADMM_OK;
  GUARD_END(ctx)
}

}  // extern "C"
