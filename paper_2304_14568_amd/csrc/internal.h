// Device-side tables and launch interfaces shared by the host runtime and the
// gfx950 kernels.  Plain structs only; no torch or HIP types in here except
// hipStream_t in the launcher declarations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace admmbb {

constexpr int kThreads = 256;       // threads per workgroup, all kernels
constexpr int kColBlock = 64;       // columns handled by one block of a vector kernel (one wave)
constexpr int kMaxCg = 64;          // CG steps per ADMM iteration, upper limit
constexpr int kRing = kMaxCg + 2;   // per-scenario CG scalar slots
constexpr int kRegChunks = 4;       // 4-element chunks of a row kept in registers per lane

enum PassMode { PASS_GRAD = 0, PASS_CG = 1, PASS_OBJ = 2, PASS_MATVEC = 3, PASS_RMATVEC = 4 };
enum ValKind { VAL_F32 = 0, VAL_BF16 = 1, VAL_F16 = 2 };
enum RedMode { RED_HEAD = 0, RED_CG = 1, RED_NORMAL = 2, RED_RMAT = 3, RED_DUALINIT = 4 };
// LDS column accumulators of the fused pass: float atomics, double atomics, or
// 64-bit fixed point (integer atomics, exact and order-independent sums).
enum AccKind { ACC_F32 = 0, ACC_F64 = 1, ACC_FIX64 = 2 };

// One per (patient, scenario).
struct Scen {
  int32_t patient;
  int32_t n;            // spots of the patient
  int32_t m;            // voxels of the patient
  int32_t rows;         // rows holding at least one nonzero (length-sorted)
  int64_t row_base;     // into per-row arrays (rw, rpres, rorig, rscale)
  int64_t rp_base;      // into rp (rows + 1 entries per scenario)
  int64_t nnz_base;     // into col / val arrays
  int64_t vec_base;     // into the stacked per-scenario n-vectors
  int32_t blk_begin;    // first scenario column block
  int32_t nblk;
  int32_t tile_begin, tile_end;
  float cw;             // scenario probability c_s (already folded into rw)
  int32_t pad;
  int64_t mpack_off;    // dense x-update: offset of its packed inverse (upper 64 x 64 tiles, 4096 each)
  int64_t sell_base;    // sliced layout: first 4-element chunk slot of the scenario
};

// One per patient.
struct Pat {
  int32_t n, m;
  int32_t num_scen, scen_begin;
  int32_t blk_begin, nblk;      // patient column blocks (z kernels)
  int32_t tile_begin, tile_end; // tiles of all its scenarios (contiguous)
  int64_t zvec_base;            // into per-patient n-vectors (z, lb, ub, dinv-free)
  double fzero;                 // sum_s c_s sum_{i: row i of A_s empty} w_i p_i^2 (objective of dropped rows)
  double fconst;                // sum_s c_s sum_i w_i p_i^2 (objective at x = 0)
  int32_t npad;                 // dense x-update: n rounded up to whole 64-blocks
  int32_t fobj_begin, fobj_end; // dense x-update: objective workgroups (one per packed tile) of this patient
  int32_t nbk;                  // dense x-update: npad / 64
  int64_t gpack_off;            // dense x-update: offset of sum_s G_s, packed upper tiles, fp64
  int64_t vec_base;             // its first scenario's offset in the stacked n-vectors (the others follow, n apart)
  int32_t sblk_begin, sblk_end; // column blocks of all its scenarios (contiguous)
};

// A contiguous range of length-sorted rows of one scenario, handled by one
// workgroup with `lanes` lanes per row.
struct Tile {
  int32_t scen;
  int32_t row_begin, row_end;
  int32_t lanes;
  int64_t part_off;   // offset of this tile's n-vector of partial column sums
  // bounds for the fixed-point column accumulators (rounded up):
  float wmax;         // max over the tile's rows of c_s w_i sum_j |a_ij|
  float pmax;         // max over the tile's rows of c_s w_i p_i
  float cmax;         // max over columns of sum over the tile's rows of |a_ij|
  int32_t slice_begin; // sliced layout: index of the tile's first slice in MatDev::soff
};

// Column block of a scenario (owner = scenario) or of a patient (owner = patient).
struct Blk {
  int32_t owner;
  int32_t col0;
};

// Per-patient scalars living on the device.
struct PatState {
  double rho;
  double tau;          // dual step used by the pending dual update
  double f_prev;       // objective at the previous z
  double f_cur;
  double r_prim, r_dual, eps_prim, eps_dual;
  double xnorm, znorm;
  int32_t iter;        // completed ADMM iterations
  int32_t pending;     // body done: the next head completes the dual update and the stop test
  int32_t stopped;
  int32_t status;      // 0 running, 1 converged, 2 diverged (non-finite)
  int32_t cg_steps;    // CG steps (summed over scenarios) of the last iteration
  int32_t cg_total;
  int32_t dual_go;     // dense four-launch iteration: the head launch applies the pending dual update
  int32_t bb_iter0;    // iter and tau as the last head left them: the inputs of the next
  double bb_tau0;      // dual step, stable while the dense iteration's tail forms it
};

struct IterRecord {
  int32_t iter;
  int32_t cg_steps;
  double obj, r_prim, r_dual, eps_prim, eps_dual, tau;
};

struct AlgoParams {
  double eps_abs, eps_rel, obj_rel_tol;
  double bb_clamp;
  double eta_factor, eta_floor;
  int32_t bb;
  int32_t z_mode;
  int32_t stop_enabled;
  int32_t precond;
  int32_t trace_cap;
  int32_t num_pat;
};

// Matrix storage of all (patient, scenario) pairs, length-sorted rows, in one
// of two layouts of the same 4-element chunks:
//   FMT_CSR   every row's chunks one after the other (row r at rp[r]);
//   FMT_SELL  sliced: the rows of a tile in slices of G = 64 / L consecutive
//             rows (L = the tile's lanes per row), each slice padded to K
//             chunk slots per lane; slot (k, lane) of a slice at
//             soff[slice] + 64 k + lane, lane = g L + l holding chunk k L + l
//             of the slice's row g, so that one wave load instruction reads 64
//             consecutive chunks.  Padding slots hold value 0 and a valid column.
enum MatFmt { FMT_CSR = 0, FMT_SELL = 1 };
struct MatDev {
  const uint32_t* rp;      // row starts in 4-element chunks relative to nnz_base (rows padded to whole chunks)
  const void* col;         // uint16 (n <= 65535) or int32 column indices (in the layout of fmt)
  const void* val;         // float / bf16 bits / fp16 values (in the layout of fmt)
  const float* rscale;     // per-row scale for low-precision values (nullptr for fp32)
  const float* rw;         // c_s * w_i per sorted row
  const float* rpres;      // p_i per sorted row
  const int32_t* rorig;    // original row index per sorted row
  const uint32_t* soff;    // FMT_SELL: slot offset of every slice relative to the scenario's sell_base
  int32_t col16;           // 1 when col holds uint16
  int32_t vkind;           // ValKind
  int32_t fmt;             // MatFmt
  int32_t pad;
};

struct PassArgs {
  const Tile* tiles;
  const Scen* scen;
  const Pat* pat;
  MatDev mat;
  const float* src;        // multiplied vector: per scenario (src + vec_base) or per patient (src + zvec_base)
  int32_t src_per_scen;
  int32_t step;            // CG step (selects the active flag slot)
  const uint8_t* act;      // [scen * kRing + step], nullptr = all active
  const PatState* ps;      // skip stopped patients when non-null
  float* part;             // tile partial column sums
  double* objpart;         // per-tile objective partial (GRAD / OBJ)
  const float* tin;        // RMATVEC input (m-vector of the scenario)
  const float* tmax;       // RMATVEC: kAbsMaxBlocks partial maxima of |tin| (launch_absmax); nullptr: each
                           // tile takes the maximum over its own rows first
  float* tout;             // MATVEC output (m-vector of the scenario)
  int32_t nmax;
  int32_t acc;             // LDS column accumulators: ACC_F32, ACC_F64 or ACC_FIX64
  int32_t threads;         // workgroup size of the pass: 256 or 512
  int32_t unroll;          // rows per lane group in flight: 1, 2 or 4
};

// Column reduction of the tile partials: one column block of one scenario,
// with every address its loads need
struct ColJob {
  int64_t part_off;   // the scenario's first tile partials
  int64_t vec_base;   // the scenario in the stacked n-vectors
  int64_t zvec_base;  // its patient in the per-patient n-vectors
  int32_t ntiles, n, col0, scen;
  int32_t patient, pad;
};

// z-update: one patient column block, with every address its loads need
struct ZJob {
  int64_t vec_base;   // the patient's first scenario in the stacked n-vectors
  int64_t zvec_base;  // the patient in the per-patient n-vectors
  int32_t n, N, col0, patient;
  int64_t xtile0;     // dense x-update: table index of the first tile of the patient's first scenario
};

struct VecArgs {
  const Scen* scen;
  const Pat* pat;
  const Blk* blk;           // scenario column blocks
  const Blk* pblk;          // patient column blocks
  const ColJob* cjobs;      // one per scenario column block (blk)
  const ZJob* zjobs;        // one per patient column block (pblk)
  const Tile* tiles;
  const float* part;
  const double* objpart;
  PatState* ps;
  int32_t step;
  uint8_t* act;            // [scen * kRing + k]
  double* rz;              // [scen * kRing + k]
  double* tol2;            // [scen]
  int32_t* cgcount;        // [scen], CG steps of the current iteration
  int64_t* cgtotal;        // [scen], CG steps since the last reset
  float* x;
  float* r;
  float* v;
  float* q;
  float* zp;               // preconditioned residual (== r when no preconditioner)
  float* y;
  const float* b;          // A_s^T c_s W p
  const float* dinv;       // Jacobi inverse diagonal (per scenario), may be null
  float* z;                // per patient
  const float* lb;
  const float* ub;
  double* dprev;           // d = x - z of the last iteration (stacked, fp64)
  double* bpart;           // per scenario-block partials [blk * 8 + k]
  double* bpartp;          // per quarter patient-block partials [(4 * pblk + quarter) * 8 + k]
  float* out;              // RMAT / NORMAL output vector (n)
  double rho_out;          // NORMAL: diagonal shift rho/2 * v added when > 0
  const double* fpart;     // dense x-update: objective partials per workgroup (nullptr: tile partials)
  double* c64;             // dense x-update: right-hand sides c_s in fp64 (stacked)
  const double* b64;       // dense x-update: A_s^T c_s W p in fp64 (stacked)
  AlgoParams prm;
  IterRecord* trace;
};

// Dense x-update (cached inverse of every B_s): device arrays and work tables.
// One packed tile of an inverse M_s, with everything its x-update workgroup
// needs to address it (no dependent table lookups before the tile load).
// Tile k of the table is stored at Mp + 4096 k and its partial pair at
// xpart + 128 k (the scenarios' packed inverses follow each other).
struct XTile {
  int64_t vbase;   // vec_base of the scenario
  int32_t n;       // spots of the patient
  int32_t patient;
  int32_t I, J;    // block row and block column
};

struct XJob {
  int32_t g;    // scenario (x-update) or patient (objective)
  int32_t ij;   // tile (I, J) as I * 65536 + J
};

// x-update reduction: block row I of one scenario's x_s, with every address
// it needs, so that its loads depend on this entry only

// Symmetric matrices of the dense x-update are stored as their upper 64 x 64
// tiles (I <= J) in the order t(I, J) = I nb - I (I - 1) / 2 + (J - I), each
// tile row-major.
struct FactorArgs {
  const Scen* scen;
  const Pat* pat;
  const PatState* ps;
  double* G;          // set-up chunk: G_s = A_s^T c_s W A_s per scenario, npad x npad, fp64
  double* A;          // set-up chunk: sweep work matrices, end as -(G_s + rho/2 I)^-1
  float* Mp;          // per scenario: packed (G_s + rho/2 I)^-1, fp32
  double* Gp;         // per patient: packed sum_s G_s, fp64
  const double* g0;   // per patient: 2 sum_s A_s^T c_s W p, fp64 (zvec layout)
  double* P;          // per scenario: 64 x 64 pivot-block inverse
  double* U;          // per scenario: 64 x npmax column panel, transposed
  double* R;          // per scenario: 64 x npmax row panel
  double* xpart;      // per packed tile of every scenario: T c_J (64) and T^T c_I (64), fp64
  const XTile* xtiles; // x-update: one per packed tile of every scenario
  int32_t nxtiles;
  const XJob* fjobs;  // objective: one per packed tile of every patient
  uint32_t* Gq;       // objective: Gp rounded to 48 bits, tile k of fjobs at 6144 k (layout in fobj_tile)
  double* fpart;      // objective partial per objective job
  int32_t npmax;      // largest npad
  int32_t npat;       // patients of the context
};

// ---- launchers (kernels.hip) ----
// e0 / e1 (optional): events stamped at the start and end of the kernel itself
void launch_pass(int mode, const PassArgs& a, int tile_begin, int tile_count, hipStream_t st,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_reduce(int mode, const VecArgs& a, int blk_begin, int nblk, hipStream_t st);
void launch_head_scalars(const VecArgs& a, int nscen, int cg_setup, hipStream_t st);
void launch_cg_update(const VecArgs& a, int nblk, hipStream_t st);
void launch_cg_dir(const VecArgs& a, int nblk, hipStream_t st);
void launch_zres(const VecArgs& a, int npblk, hipStream_t st);
void launch_body_scalars(const VecArgs& a, hipStream_t st);
void launch_gsum(const Scen* scen, const Pat* pat, const Blk* pblk, const Tile* tiles, const float* part,
                 int patient_blk_begin, int nblk, float scale, float* out, hipStream_t st);
void launch_objsum(const Tile* tiles, const double* objpart, int tile_begin, int tile_count, double* out,
                   hipStream_t st);
void launch_pgd_trial(const float* x, const float* g, const float* lb, const float* ub, float t, float* xt,
                      int n, double* dotpart, hipStream_t st);
void launch_dot_sum(const double* part, int count, double* out, hipStream_t st);
void launch_fill_f32(float* p, float v, int64_t count, hipStream_t st);
// max |x_i| over x[0, n) as kAbsMaxBlocks partial maxima (NaN entries ignored)
constexpr int kAbsMaxBlocks = 256;
void launch_absmax(const float* x, int64_t n, float* out, hipStream_t st);
void launch_fill_f64(double* p, double v, int64_t count, hipStream_t st);
void launch_fill_u8(uint8_t* p, uint8_t v, int64_t count, hipStream_t st);
int pass_smem_bytes(int nmax, int acc);
int dose_hist_smem_bytes(int G, int nbins);
void launch_gram(const MatDev& m, const double* rw64, const Scen& sc, double* G, int ld, hipStream_t st);
// Gram matrix by output tiles: per-tile row lists (count with list == nullptr,
// then fill), their offsets, and one workgroup per tile and scenario
struct GramEntry {  // one stored row in a tile's list: its index and its extent in 4-element chunks
  int32_t row;
  uint32_t c0, c1;
  int32_t pad;
};
void launch_gram_rows(const MatDev& m, const Scen& sc, int nb, int32_t* cnt, const int64_t* off, GramEntry* list,
                      hipStream_t st);
void launch_gram_scan(const int32_t* cnt, int64_t nt, int64_t* off, hipStream_t st);
void launch_gram_tiles(const MatDev& m, const double* rw64, const Scen* scen, int g0, int nscen, int nb,
                       const int64_t* off, const GramEntry* list, const double* gscale, double* G, int ld,
                       hipStream_t st);
void launch_gram_finish(FactorArgs f, int patient, int scen_begin, int nscen, int npad, int n, double rho,
                        int accumulate_gsum, hipStream_t st);
void launch_sweep_step(FactorArgs f, int scen_begin, int nscen, int npad, int k0, hipStream_t st);
void launch_sweep_store(FactorArgs f, int patient, int scen_begin, int nscen, int npad, hipStream_t st);
void launch_gq_pack(const double* Gp, uint32_t* Gq, int64_t ntiles, hipStream_t st);
void launch_xsym(const FactorArgs& f, const double* c, int njobs, hipStream_t st, hipEvent_t e0 = nullptr,
                 hipEvent_t e1 = nullptr);
void launch_fheadobj(const FactorArgs& f, const VecArgs& a, int nfobj, int nblk, hipStream_t st);
// dense four-launch iteration: body scalars beside the objective tiles, then
// the stopping test beside the dual update and right-hand sides
void launch_dense_tail(const FactorArgs& f, const VecArgs& a, int nfobj, hipStream_t st);
void launch_dense_head(const VecArgs& a, int nblk, hipStream_t st);
// dense three-launch iteration: the stopping test of the previous iteration
// beside the x-update tiles; the reduction; the z-update; body scalars beside
// the dual update with the next right-hand sides and the objective tiles
void launch_xzres(const FactorArgs& f, const VecArgs& a, int npblk, hipStream_t st);
void launch_dense_x(const FactorArgs& f, const VecArgs& a, const double* c, int njobs, hipStream_t st,
                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_dense_tail_dual(const FactorArgs& f, const VecArgs& a, int nfobj, int nblk, hipStream_t st);
void launch_dose_hist(const float* dose, const uint8_t* grp, int m, int G, int nbins, float inv_w, uint32_t* counts,
                      double* sums, uint32_t* maxkey, hipStream_t st);
// Allocation-free dose statistics: device address of the fixed scratch array
// (dose.hip) on the current device, looked up once per device; and a
// double-to-float copy kernel for the plan it receives.
constexpr size_t kNoAllocScratchBytes = size_t{16} << 20;
hipError_t noalloc_scratch(void** ptr);
void launch_f64_to_f32(const double* in, float* out, int n, hipStream_t st);

// ---- dense PGD (pgd_dense.hip) ----
constexpr int kPgdK = 8;  // backtracking steps evaluated per round

struct PgdDevState {
  double f;       // objective at x
  double t_base;  // step of the first trial point of the next round
  double alpha;   // initial step of every iteration
  int32_t iter;   // accepted steps
  int32_t trials; // rejected trial steps at the current x
  int32_t done;
  int32_t status; // 1 converged, 2 no step accepted within max_trials, 3 iteration limit
  int32_t pick;   // trial point accepted by the last round, -1 none
  int32_t pad;
};

struct PgdArgs {
  const double* Gp;  // sum_s G_s of the patient, packed upper tiles, fp64
  const double* g0;  // 2 sum_s A_s^T c_s W p of the patient, fp64
  const float* lb;
  const float* ub;
  const XJob* jobs;  // the patient's packed tiles in packed order
  int32_t njobs, nb, n, nblocks;  // tiles, block rows, spots, 256-spot blocks of np
  int32_t np, pad;   // n rounded up to whole 64-blocks: length of every vector below
  double* x;         // np, zero beyond n
  double* g;         // np, gradient at x
  double* xc;        // kPgdK x np trial points, zero beyond n
  double* u;         // kPgdK x np: S x_k
  double* part;      // per tile and trial point: 64 row and 64 column products
  double* fpart;     // [k][block row]
  double* gdpart;    // [2][k][block]: double-buffered by round parity
  PgdDevState* st;   // [2]: read slot par, write slot par ^ 1
  double fconst, beta, gamma, tol;
  int32_t max_iter, max_trials;
};

void launch_pgd_power(const PgdArgs& a, double* v, hipStream_t st);
void launch_pgd_prime(const PgdArgs& a, int par, hipStream_t st);
void launch_pgd_round(const PgdArgs& a, int first, int par, hipStream_t st);

}  // namespace admmbb
