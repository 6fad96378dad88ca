/*
 * admmbb.h — C ABI of the MI355X (gfx950) ADMM-BB robust proton planning library.
 *
 * Problem (Sec. 2.1, scenario objective and robust problem): spot intensities
 * x in R^n minimise
 *
 *     f(x) = sum_s c_s sum_i w_i (a_{s,i}^T x - p_i)^2     subject to lb <= x <= ub
 *
 * where A_s (m voxels x n spots, nonnegative) is the dose-influence matrix of
 * uncertainty scenario s, w_i >= 0 is the weight of voxel i (constant within a
 * structure), p the prescription and c_s the scenario probability (end of
 * Sec. 2.1; c_s = 1 reproduces the equal-probability problem).  The paper's
 * constraint x >= 0 is lb = 0, ub = +inf.
 *
 * Method (Sec. 2.2 and Appendix A): consensus ADMM over scenarios with a
 * Barzilai-Borwein dual step.  Each iteration solves, for every scenario, the
 * regularised WLS subproblem through its normal equations
 *     (A_s^T diag(c_s w) A_s + rho/2 I) x_s = A_s^T diag(c_s w) p + rho/2 (z - y_s/rho).
 * The paper factors each matrix once by Cholesky (Appendix A).  Here the
 * default x-update (ADMM_XUPDATE_DENSE, chosen whenever the matrices fit)
 * caches the inverse of every such matrix in fp32 and applies it with one
 * GEMV per iteration, an exact solve like the paper's; the alternative
 * (ADMM_XUPDATE_CG) runs warm-started conjugate gradients whose every step is
 * one fused pass over the sparse A_s.  Then z = P(mean_s(x_s + y_s/rho)), the BB step
 * beta = -<dd, dy>/||dd||^2 replacing rho in y_s += tau (x_s - z) when
 * positive, and the residual stopping test of Sec. 2.2 combined with a
 * relative-objective-change test (Sec. 2.3).  pgd_solve is the comparison
 * method of Sec. 2.1 (projected gradient with Armijo backtracking).
 *
 * Conventions
 *   - Every function returns admm_status and never throws or aborts across the
 *     ABI.  Negative codes mean the outputs were not written; ADMM_MAX_ITER
 *     means outputs are valid but the stopping test was not met.
 *     admm_last_error() gives a message for the last failure.
 *   - Input arrays are host memory (or, for the CSR arrays, device memory when
 *     admm_problem.mem_kind says so), borrowed only for the duration of the
 *     call; the library copies and repacks what it needs into device memory it
 *     owns.
 *   - Output arrays are caller-allocated host memory.
 *   - One context is used by one host thread at a time.  All device work of a
 *     context is issued on its stream (admm_options.stream; NULL means a
 *     stream the library creates).
 *   - Validation of a problem happens entirely on the host before any device
 *     work, so malformed input is reported without touching the GPU.
 */
#ifndef ADMMBB_H
#define ADMMBB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct admm_ctx admm_ctx; /* opaque, owned by the library */

typedef enum {
  ADMM_OK = 0,
  ADMM_MAX_ITER = 1,     /* outputs valid, stopping test not met */
  ADMM_E_ARG = -1,       /* bad argument (NULL pointer, size, option) */
  ADMM_E_CSR = -2,       /* malformed CSR: row_ptr not monotone, column out of range or not increasing */
  ADMM_E_NEGATIVE = -3,  /* negative matrix value, weight or prescription */
  ADMM_E_NONFINITE = -4, /* NaN or Inf in an input */
  ADMM_E_OOM = -5,       /* device or host allocation failed */
  ADMM_E_HIP = -6,       /* HIP runtime error (no device, launch failure) */
  ADMM_E_DIVERGED = -7,  /* iterates became non-finite */
  ADMM_E_STATE = -8      /* call not valid in the context's current state */
} admm_status;

enum { ADMM_PREC_FP32 = 0, ADMM_PREC_BF16 = 1, ADMM_PREC_FP16 = 2 };

/* One scenario's dose-influence matrix A_s in CSR (Sec. 2.1: A_s in R_+^{m x n}).
 * row_ptr: m+1 nondecreasing offsets, row_ptr[0] = 0, row_ptr[m] = nnz.
 * col: column (spot) indices, strictly increasing within a row, in [0, n).
 * val: entries, finite and >= 0.
 * prob: scenario probability c_s >= 0 (0 is read as 1). */
typedef struct {
  int64_t nnz;
  const int64_t* row_ptr;
  const int32_t* col;
  const float* val;
  double prob;
} admm_csr;

/* Where the CSR arrays (row_ptr, col, val) of a problem live. */
enum { ADMM_MEM_HOST = 0, ADMM_MEM_DEVICE = 1 };

/* One patient: num_scen matrices with the same m, n.
 * w_i = struct_weight[struct_id[i]] >= 0 (weights constant per structure, Sec. 2.1);
 * presc[i] = p_i >= 0 (Sec. 2.1); lb/ub: n bounds each, NULL means 0 / +inf.
 * mem_kind: ADMM_MEM_HOST (0): every array is host memory.  ADMM_MEM_DEVICE
 * (1): row_ptr, col and val of every scenario are device memory of the
 * current device (for example tensors allocated by PyTorch on the GPU), read
 * only during admm_setup / admm_setup_batch, which copy them to host staging
 * buffers (synchronous copies, before any other device work) and then
 * validate and pack them like host input; the caller keeps ownership.  A
 * failed copy (for example nnz larger than the arrays) returns ADMM_E_HIP.  The admm_csr array, struct_id,
 * struct_weight, presc, lb and ub are host memory in both cases. */
typedef struct {
  int32_t m, n, num_scen;
  const admm_csr* A;
  const uint8_t* struct_id;
  int32_t num_struct;
  const double* struct_weight;
  const double* presc;
  const double* lb;
  const double* ub;
  int32_t mem_kind;
} admm_problem;

enum { ADMM_XUPDATE_AUTO = -1, ADMM_XUPDATE_CG = 0, ADMM_XUPDATE_DENSE = 1 };

typedef struct {
  double rho;          /* penalty; <= 0 selects 2 * mean_s mean_j (A_s^T c_s W A_s)_jj */
  double eps_abs;      /* stopping tolerances of Sec. 2.2; default 1e-6 (Sec. 2.3) */
  double eps_rel;      /* default 1e-6 */
  double obj_rel_tol;  /* relative objective change combined with the residual test; default 1e-5; 0 disables */
  int32_t max_iter;    /* default 1000 */
  int32_t bb;          /* 1: Barzilai-Borwein dual step (default), 0: fixed rho */
  int32_t z_mode;      /* 0: z = P(mean(x_s + y_s/rho)) (default); 1: z = P(mean x_s) as printed in Sec. 2.2 */
  double bb_clamp;     /* 0: none (default); c > 0: tau clamped to [rho/c, rho*c] */
  int32_t cg_max;      /* CG steps per ADMM iteration, 1..64; default 8 */
  double cg_eta;       /* CG stops at ||r|| <= eta ||c_s||, eta = max(eta_floor, cg_eta*min(1, r_prim/||x||)); default 0.01 */
  double cg_eta_floor; /* default 1e-8 (a floor of 1e-6 holds the intensities of the fp32 CG solve
                          about 4e-4 from the minimiser on the 13-scenario head-and-neck workload) */
  int32_t precision;   /* ADMM_PREC_*: value type of A_s inside CG; the objective and the
                          per-iteration residual always use the fp32 matrix; default FP32 */
  int32_t precond;     /* 1: Jacobi-preconditioned CG; default 0 */
  int32_t use_graph;   /* 1: capture one iteration in a HIP graph and replay it (default) */
  int32_t check_every; /* host reads the stop flags every k iterations; default 1 */
  int32_t lds_acc;     /* column accumulators of the fused pass in LDS: 0 fp32 atomics, 1 fp64 atomics,
                          2 64-bit fixed point (integer atomics: exact, order-independent sums);
                          -1 = chosen by the set-up autotuner among 1 and 2 */
  int32_t tile_nnz;    /* target nonzeros per workgroup tile; 0 = automatic, per patient
                          (about 2048 tiles each, 8192 .. 4M nonzeros) */
  int32_t pass_threads; /* fused-pass workgroup size 256, 512 or 1024 (1024: chunk-row layout
                          only); 0 = chosen per patient by the set-up autotuner */
  int32_t pass_unroll;  /* 1: row data loaded when the row starts; 2: next row's data in flight during the
                           current row (software pipelined); 0 = chosen by the autotuner */
  int32_t xupdate;     /* x-update of every scenario subproblem:
                          ADMM_XUPDATE_CG: warm-started CG steps with the sparse A_s (cg_max, cg_eta);
                          ADMM_XUPDATE_DENSE: exact solve with a cached inverse of
                            A_s^T c_s W A_s + rho/2 I (fp64 Gram matrix and block Gauss-Jordan sweep at
                            set-up and on every change of rho, fp32 inverse, one GEMV per iteration;
                            the cached-factor solver of Appendix A); needs n <= 8128 and
                            about 20 N n^2 bytes of device memory per patient;
                          ADMM_XUPDATE_AUTO (default): DENSE when every patient has n <= 8128 and the
                            matrices take at most a quarter of the free device memory, else CG.
                          The set-up works on chunks of scenarios whose fp64 matrices take at most
                          8 GiB (environment variable ADMMBB_DENSE_CHUNK_MB overrides the limit). */
  int32_t format;      /* layout of A_s read by the sparse passes (the same length-sorted rows in
                          4-element chunks either way):
                          ADMM_FORMAT_CSR: each row's chunks contiguous, L lanes per row;
                          ADMM_FORMAT_SELL: sliced, the rows of a tile in slices of 64 / L rows with
                            their chunks interleaved so that a wave load reads 64 consecutive chunks
                            (16-bit column indices only, n <= 65535);
                          ADMM_FORMAT_AUTO (default): with the CG x-update both are built and
                            the set-up autotuner picks the faster for each patient's CG pass;
                            with the dense x-update, where the tuner does not run, only the
                            chunk-row one is built */
  int32_t deterministic; /* 1: every sum of an iteration is exact or in a fixed order (64-bit
                          fixed-point column accumulators, lds_acc -1 or 2 required), so runs and
                          resumed runs repeat bit for bit; default 0 (the autotuner may pick fp64
                          LDS atomics, whose sums depend on the order of the additions) */
  int32_t dense_launches; /* dense x-update: 3 (default) = three launches per iteration, the
                          stopping test of an iteration evaluated beside the next iteration's
                          x-update (and after the last one in a launch of its own) and the dual
                          update beside the dual step; 4 = four launches, each iteration
                          complete at its end.  The iterates, scalars and stopping decisions
                          are the same bit for bit; with 3 the device computes one more
                          x-update of a patient that has just stopped, and discards it */
  void* stream;        /* hipStream_t for all device work; NULL = library-owned stream */
} admm_options;

enum { ADMM_FORMAT_AUTO = -1, ADMM_FORMAT_CSR = 0, ADMM_FORMAT_SELL = 1 };

/* Per-iteration record (also the summary returned by solve / iterate). */
typedef struct {
  int32_t iter;      /* ADMM iterations completed */
  int32_t cg_steps;  /* CG steps summed over scenarios: last iteration (trace) or total (summary) */
  int32_t status;    /* admm_status of the patient */
  int32_t pad;
  double obj;        /* f(z) (fp32 matrix, fp64 accumulation) */
  double r_prim, r_dual, eps_prim, eps_dual;
  double tau;        /* dual step used */
  double kkt;        /* scaled KKT residual of the returned point, as admm_kkt computes it:
                        filled by admm_solve (at the point where the stopping test ended the run)
                        and pgd_solve (when x_out is given); -1 where it is not evaluated
                        (admm_iterate, trace records) */
} admm_info;

/* PGD options (Sec. 2.1). alpha <= 0 selects 10 / lambda_max(H) (30 power iterations). */
typedef struct {
  double alpha, beta, gamma; /* initial step, sufficient-decrease constant, shrink factor; defaults 0 / 1e-4 / 0.5 */
  double obj_rel_tol;        /* stop when |f_k - f_{k+1}| <= tol |f_k|; default 1e-5 */
  int32_t max_iter;          /* default 10000 */
  int32_t max_trials;        /* backtracking trials per iteration; default 60 */
  int32_t dense;             /* -1 (default): the dense form when the context holds the dense
                                x-update's matrices, else the sparse passes; 0: sparse passes;
                                1: dense form (ADMM_E_ARG when the context has no dense matrices) */
  int32_t reserved;          /* 0 */
} pgd_options;

/* Fill opts / popts with the defaults documented above. */
admm_status admm_default_options(admm_options* opts);
admm_status pgd_default_options(pgd_options* popts);

/* Validate the problem on the host (n <= 13 600 spots per patient: the sparse
 * pass keeps an n-vector and n column accumulators in the LDS of a workgroup),
 * copy it to the device (length-sorted CSR,
 * optional bf16/fp16 copy of the values with per-row scales), and prepare the
 * ADMM state at z = P(0), y = 0.  On failure *out = NULL and nothing leaks. */
admm_status admm_setup(const admm_problem* prob, const admm_options* opts, admm_ctx** out);

/* Several independent patients in one context: every kernel launch covers all
 * of them (one launch per phase per iteration). */
admm_status admm_setup_batch(const admm_problem* probs, int32_t num_patients, const admm_options* opts,
                             admm_ctx** out);

/* The x-update the context uses (ADMM_XUPDATE_CG or ADMM_XUPDATE_DENSE) and, for
 * DENSE, the device time in ms of the last set-up of the cached inverses
 * (Gram matrices and sweeps of all patients). */
admm_status admm_get_xupdate(const admm_ctx* ctx, int32_t* mode, double* setup_ms);

/* Restart one patient from z = P(z0) (z0 NULL: 0), iteration 0.
 * rho > 0 replaces the penalty of that patient (rho <= 0 keeps it).
 * dual_init = 0: y_s = 0.  dual_init = 1: y_s = -grad f_s(z) for every scenario,
 * the duals for which x_s = z solves every x-update subproblem exactly (from the
 * optimality condition of the subproblem of Sec. 2.2), computed on the GPU. */
admm_status admm_warm_start(admm_ctx* ctx, int32_t patient, const double* z0, double rho, int32_t dual_init);
/* Restart every patient from z = P(0), y = 0, iteration 0. */
admm_status admm_reset(admm_ctx* ctx);

/* Run exactly k ADMM iterations for every patient, without the stopping test.
 * info (one per patient, may be NULL) receives the state after the last one. */
admm_status admm_iterate(admm_ctx* ctx, int32_t k, admm_info* info);

/* Iterate until every patient meets the stopping test or max_iter.
 * z_out: n doubles per patient, concatenated (may be NULL); info: one per patient. */
admm_status admm_solve(admm_ctx* ctx, double* z_out, admm_info* info);

/* Projected gradient descent with Armijo backtracking for one patient, from
 * P(x0) (x0 NULL: 0); x_out: n doubles.
 * Sparse form: x in fp32, one objective pass over the A_s per trial step, host
 * loop.  Dense form: f(x) = x^T (sum_s G_s) x - g0^T x + const from the packed
 * fp64 sum of the Gram matrices, x in fp64, the whole iteration on the device:
 * 8 trial steps per round share one read of sum_s G_s, which also yields the
 * gradient at the accepted point; the accepted step is the first (largest) one
 * that passes the test, as in the sequential backtracking.
 * info: iter = accepted steps, obj = f(x), tau = initial step alpha, status. */
admm_status pgd_solve(admm_ctx* ctx, const pgd_options* popts, int32_t patient, const double* x0, double* x_out,
                      admm_info* info);

/* f(x) with the fp32 matrix and fp64 accumulation; x: n doubles (rounded to fp32). */
admm_status admm_objective(admm_ctx* ctx, int32_t patient, const double* x, double* f_out);

/* grad f(x) (n doubles) and f(x). */
admm_status admm_gradient(admm_ctx* ctx, int32_t patient, const double* x, double* grad_out, double* f_out);

/* Scaled KKT residual ||x - P(x - grad f(x))||_inf / max(1, ||grad f(0) ... g0||_inf), g0 = 2 sum_s c_s A_s^T W p. */
admm_status admm_kkt(admm_ctx* ctx, int32_t patient, const double* x, double* r_out);

/* Single products with the device matrices (fp32 values), for checking:
 *   matvec:  out[m] = A_s v          (v: n floats)
 *   rmatvec: out[n] = A_s^T t        (t: m floats)
 *   normal:  out[n] = (A_s^T diag(c_s w) A_s + rho/2 I) v, rho the patient's penalty;
 *            precision selects the value copy used (ADMM_PREC_*), as inside CG. */
admm_status admm_matvec(admm_ctx* ctx, int32_t patient, int32_t scen, const float* v, float* out);
admm_status admm_rmatvec(admm_ctx* ctx, int32_t patient, int32_t scen, const float* t, float* out);
admm_status admm_normal_apply(admm_ctx* ctx, int32_t patient, int32_t scen, int32_t precision, const float* v,
                              float* out);

/* Dose statistics of a plan x (n doubles, host) for dose-volume evaluation
 * (Sec. 3: dose-volume histograms and D98 / Dmax / D3 / Dmean metrics).
 * Voxel i belongs to group voxel_group[i] < num_groups (<= 256), for example
 * its structure.  For every scenario s and group g, with d = A_s x (fp32
 * matrix, fp64 row sums rounded to fp32) and bin width w = dmax / nbins:
 *   counts[(s*G + g)*nbins + k] = #{i in g : k w <= d_i < (k+1) w}; doses below
 *                                 0 count in bin 0, doses >= dmax in bin nbins-1
 *   sums[s*G + g]  = sum of d_i over the group (fp64)
 *   maxes[s*G + g] = max of d_i over the group (-inf for an empty group)
 * dose_out (may be NULL): the N*m doses, scenario-major, original voxel order.
 * Requires 12 G + 4 G nbins <= 65536 (the per-block histograms live in LDS).
 * Counts and maxima are exact; sums are order-dependent in the last bits. */
admm_status admm_dose_stats(admm_ctx* ctx, int32_t patient, const double* x, const uint8_t* voxel_group,
                            int32_t num_groups, int32_t nbins, double dmax, uint32_t* counts, double* sums,
                            float* maxes, float* dose_out);

/* admm_dose_stats for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, outputs and errors, computed by the same kernels, with
 * no hipMalloc, hipFree or other allocating call.  Its staging (voxel groups,
 * the plan in fp64, histograms, sums, max keys) lives in a fixed 16 MiB array
 * in device memory that each GPU the library runs on holds until the process
 * ends; a call needs m + 4 N G nbins + 12 N G + 8 n bytes of it (each part
 * rounded up to 256 bytes) and fails with ADMM_E_ARG when that exceeds 16 MiB.
 * Every call on a GPU shares that GPU's array and clears what it accumulates
 * into, so calls that overlap on one GPU (from several threads or streams)
 * race; calls in sequence do not. */
admm_status admm_dose_stats_noalloc(admm_ctx* ctx, int32_t patient, const double* x, const uint8_t* voxel_group,
                                    int32_t num_groups, int32_t nbins, double dmax, uint32_t* counts, double* sums,
                                    float* maxes, float* dose_out);

/* Measurement: average device time in ms of one launch of a sparse pass over
 * every scenario of every patient (reps launches back to back, HIP events on
 * the context's stream).  kind 0: forward product A_s z fused with the
 * weighted residual norm (the objective pass); 1: transpose product A_s^T t for
 * a voxel vector t; 2: the fused normal operator A_s^T diag(c_s w) A_s v of a
 * CG step.  Changes no solver state. */
admm_status admm_time_pass(admm_ctx* ctx, int32_t kind, int32_t reps, double* ms_out);

/* Measurement aid, no context: the rate (GB/s, 1e9 bytes) at which the current
 * device streams a buffer of `bytes` (1 MiB .. 16 GiB) through one read pass
 * (16 KiB per workgroup, 1 KiB contiguous per wave load, four loads in flight
 * per lane), averaged over `reps` passes after one warm-up.  The
 * buffer is allocated, filled and freed inside the call on a stream of its
 * own.  ADMM_E_ARG for sizes out of range or reps < 1, ADMM_E_OOM when the
 * buffer does not fit, ADMM_E_HIP on a runtime failure. */
admm_status admm_stream_probe(int64_t bytes, int32_t reps, double* gbs_out);

/* Dose-derived per-spot features for the learned warm start, computed on the GPU
 * from A_s^T applied to voxel indicator vectors.  voxel_class[m]: 0 other,
 * 1 target, 2 organ at risk.  feat: n x ADMM_NUM_DOSE_FEATURES floats, row-major:
 *   0..2  mean / min / max over scenarios of the target share of the spot's dose
 *         (sum_{i in targets} a_ij / sum_i a_ij)
 *   3..4  mean / max over scenarios of the organ-at-risk share
 *   5     log(1 + mean over scenarios of sum_i a_ij)
 *   6     sum_s (A_s^T c_s W p)_j / sum_s (A_s^T c_s W A_s)_jj, the intensity that
 *         would minimise f if spot j acted alone */
#define ADMM_NUM_DOSE_FEATURES 7
admm_status admm_spot_features(admm_ctx* ctx, int32_t patient, const uint8_t* voxel_class, float* feat);

/* Penalty rho in use for a patient. */
admm_status admm_get_rho(const admm_ctx* ctx, int32_t patient, double* rho);

/* Current consensus iterate z (n doubles). */
admm_status admm_get_z(admm_ctx* ctx, int32_t patient, double* z);

/* Checkpoint / resume.  The state that determines the next iterations is
 * z (n), y (N*n, scenario-major), d = x - z of the last iteration (N*n) and
 * ADMM_STATE_SCALARS scalars {iter, tau, f_prev, pending, stopped, status, rho,
 * cg_total, f_cur, r_prim, r_dual, eps_prim, eps_dual, ||x||, ||z||, cg_steps}.
 * Resuming from a saved state in the same or a fresh context with the same
 * problem and options reproduces the following iterations bit for bit when the
 * column sums are exact (lds_acc = 2 or the dense x-update). */
#define ADMM_STATE_SCALARS 16
admm_status admm_get_state(admm_ctx* ctx, int32_t patient, double* z, double* y, double* d, double* scalars);
admm_status admm_set_state(admm_ctx* ctx, int32_t patient, const double* z, const double* y, const double* d,
                           const double* scalars);

/* Per-iteration records of the last solve / iterate calls (up to cap). */
admm_status admm_get_trace(admm_ctx* ctx, int32_t patient, admm_info* buf, int32_t cap, int32_t* count);

/* Fused-pass configuration in use (picked by the set-up autotuner unless fixed
 * in the options), of patient 0 (admm_get_pass_config gives every patient's):
 * workgroup size, rows in flight per lane group, LDS accumulator kind, and the
 * measured average pass time in ms of the chosen configurations summed over
 * the patients (all scenarios, fp32 or the CG value precision). */
admm_status admm_get_tuning(const admm_ctx* ctx, int32_t* threads, int32_t* unroll, int32_t* lds_acc, double* ms);
/* The sparse-pass configuration of one patient of the context for the CG
   operator and the gradient pass (the passes are launched once per patient,
   each with its own; the set-up autotuner of the CG x-update chooses it per
   patient): workgroup size, row pipelining (1 or 2),
   LDS accumulator (0 fp32, 1 fp64, 2 64-bit fixed point), layout
   (ADMM_FORMAT_CSR / ADMM_FORMAT_SELL) and the tuned pass time in ms (0 where
   the tuner did not run).  Any output pointer may be NULL.  ADMM_E_ARG for a
   NULL ctx or a patient outside [0, num_patients). */
admm_status admm_get_pass_config(const admm_ctx* ctx, int32_t patient, int32_t* threads, int32_t* unroll,
                                 int32_t* lds_acc, int32_t* format, double* ms);
/* The configuration of one patient's other sparse products (the forward
   product A_s z with the objective, Sec. 2; admm_matvec; the transpose product
   A_s^T t): workgroup size (512 or 1024) and row pipelining (1 or 2), chosen
   with either x-update as the fastest forward product over the patient's
   matrices unless the options fix them, and that product's time in ms over all
   its scenarios (0 until chosen).  The choice is made once, on the context's
   first admm_objective, admm_matvec, admm_rmatvec, admm_spot_features, sparse
   pgd_solve or admm_time_pass call (the iterations use none of these
   products; until then they run with the options' pass configuration).
   Results do not depend on the choice except the objective's last bits (its
   per-tile sums follow the workgroup size).  Any output pointer may be NULL.
   ADMM_E_ARG for a NULL ctx or a patient outside [0, num_patients). */
admm_status admm_get_forward_config(const admm_ctx* ctx, int32_t patient, int32_t* threads, int32_t* unroll,
                                    double* ms);

/* Layout of A_s the sparse passes of patient 0 read (ADMM_FORMAT_CSR or
 * ADMM_FORMAT_SELL): the one asked for, or under ADMM_FORMAT_AUTO the set-up
 * autotuner's pick (chunk-row with the dense x-update). */
admm_status admm_get_format(const admm_ctx* ctx, int32_t* format);

/* CG steps performed per scenario of a patient since its last reset
 * (num_scen int64 entries): the number of fused CG-pass applications of A_s. */
admm_status admm_get_cg_counts(admm_ctx* ctx, int32_t patient, int64_t* counts);

/* Sizes: num_patients; per patient n, m, num_scen, total nonzeros. */
admm_status admm_get_sizes(const admm_ctx* ctx, int32_t patient, int32_t* n, int32_t* m, int32_t* num_scen,
                           int64_t* nnz);

/* Device timing.  admm_enable_timing(ctx, 1) makes later solve / iterate calls
 * record HIP events on the context stream: around the whole call, and around
 * every launch of the fused CG pass (the dominant kernel, including launches
 * whose scenarios have all converged and exit early).  admm_get_timing returns
 * the total milliseconds of the most recent call and the average duration and
 * count of those pass launches. */
admm_status admm_enable_timing(admm_ctx* ctx, int32_t on);
admm_status admm_get_timing(const admm_ctx* ctx, double* total_ms, double* pass_ms, int32_t* pass_launches);

/* Message of the last failure on ctx (ctx NULL: the last failed setup of this thread). */
const char* admm_last_error(const admm_ctx* ctx);

void admm_destroy(admm_ctx* ctx);

/* Host-only validation of a problem (the checks admm_setup performs first);
 * a problem with mem_kind ADMM_MEM_DEVICE is refused with ADMM_E_ARG (its
 * CSR arrays are not host memory). */
admm_status admm_validate(const admm_problem* prob);

/* ---- Learned warm start: a small network trained and run on the GPU ----
 * Not part of the paper's method.  For the spots of one patient (rows of X,
 * rows x nin, row-major float32):
 *   h1 = relu(X W1^T + b1), h2 = relu(h1 W2^T + b2), y = softplus(h2 . w3 + b3)
 * predicts the spot intensities z0 (>= 0), and lr = mean_rows(h2) . wr + br the
 * log of the penalty scale rho / rho_default.  Loss for training:
 *   L = mean_rows (y - target)^2 + lam (lr - target_log_rho)^2.
 * Parameters (float32, flat): W1[hidden x nin], b1[hidden], W2[hidden x hidden],
 * b2[hidden], w3[hidden], b3, wr[hidden], br. */
typedef struct admm_mlp admm_mlp;
/* He-uniform weights from a splitmix64 stream seeded with `seed`, zero biases. */
admm_status mlp_create(int32_t nin, int32_t hidden, uint64_t seed, void* stream, admm_mlp** out);
void mlp_destroy(admm_mlp* net);
int64_t mlp_num_params(const admm_mlp* net);
admm_status mlp_get_params(admm_mlp* net, float* out);
/* Also clears the Adam moments and step count. */
admm_status mlp_set_params(admm_mlp* net, const float* in);
/* precision: ADMM_PREC_FP32, or ADMM_PREC_BF16 (hidden activations rounded to
 * bf16, fp32 accumulation).  y_out: rows floats (may be NULL). */
admm_status mlp_forward(admm_mlp* net, const float* X, int32_t rows, int32_t precision, float* y_out,
                        float* log_rho_out);
/* Loss and its gradient with respect to every parameter (grad_out: num_params
 * floats, may be NULL); the gradient is kept for mlp_adam_step. */
admm_status mlp_loss_grad(admm_mlp* net, const float* X, const float* target, int32_t rows, float target_log_rho,
                          float lam, double* loss_out, float* grad_out);
/* One Adam update with the last gradient. */
admm_status mlp_adam_step(admm_mlp* net, float lr, float beta1, float beta2, float eps);
const char* mlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ADMMBB_H */
