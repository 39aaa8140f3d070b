/*
 * dualip.h - C ABI of the MI355X (gfx950) ridge-regularized matching-LP dual
 * ascent library.
 *
 * Problem (paper eq. 1):  min_{x in C} c^T x + (gamma/2)||x||^2  s.t.  A x <= b
 *   x        one variable per eligible (user i, item j) pair, user-major
 *   C        product of per-user sets: simplex {x_i >= 0, sum x_i <= z},
 *            simplex {x_i >= 0, sum x_i = z}, box [0,u]^(d_i) (Section 3.3), or
 *            box-cut {0 <= x_i <= u, sum x_i <= z} (Table 1's third kind)
 *   A        m coupling families; family k has one row per item j and
 *            A[(k,j),(i,j)] = a_kij (Definition 1: diagonal per-user blocks);
 *            a family may hold equality rows A_k x = b_k (free duals); plus,
 *            optionally, one global-count row sum_{(i,j)} x_ij <= M (the new
 *            coupling constraint of Section 5: one more dual coordinate)
 * Dual (eq. 2): g(lam) = min_{x in C} c^T x + (gamma/2)||x||^2 + lam^T (A x - b)
 * Primal recovery (eq. 3): x*(lam) = Pi_C(-(A^T lam + c)/gamma)
 * Gradient (eq. 4): grad g(lam) = A x*(lam) - b
 *
 * The three calls mirror the paper's programming model (Table 1):
 *   ObjectiveFunction.calculate -> dl_dual_grad
 *   ProjectionMap               -> dl_project
 *   Maximizer                   -> dl_solve (and the stepwise dl_solver_*)
 * Beyond them: dl_batch_* (many problems per launch), dl_problem_update and
 * dl_solve_warm (recurring solves), dl_item_features and dl_mlp_* (learned
 * warm start).
 *
 * Conventions shared by every entry point
 *   Memory    Arrays marked "device" are caller-owned device pointers on the
 *             problem's device; arrays marked "host" are host memory.  The
 *             library never frees caller memory.  dl_problem_create copies
 *             what it needs, so the caller may free its inputs when it returns.
 *   Streams   Every call is ordered on the stream given at create time
 *             (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream;
 *             NULL = the default stream).  Calls that return host values
 *             synchronise that stream; the others only enqueue work.
 *   Errors    Every call returns a dl_status; on failure dl_last_error()
 *             gives a message (thread-local).  Nothing aborts or throws across
 *             the ABI.  Positive statuses are non-fatal.
 *   Units     lam, grad and A x are in the problem's own units even when
 *             Jacobi scaling is on (the scaling is internal to the solver).
 *   Rows      Dual vectors (lam, grad, A x, solver states) have n_rows =
 *             m*J + g entries: the m*J item rows family-major, then, with a
 *             global-count row (g = 1), its coordinate last.
 *   Threads   A dl_problem or dl_solver must not be used from two threads at
 *             once; distinct objects are independent.
 */
#ifndef DUALIP_H
#define DUALIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DL_OK = 0,
  DL_NOT_CONVERGED = 1, /* solve stopped at its iteration cap; results valid */
  DL_EINVAL = -1,       /* invalid argument or invalid instance data */
  DL_ENOMEM = -2,       /* device or host allocation failed */
  DL_EHIP = -3,         /* a HIP runtime call failed */
  DL_EUNSUPPORTED = -4, /* valid but outside what this build supports */
  DL_DIVERGED = -5,     /* a non-finite value appeared in the dual iterate */
  DL_NUMERIC = -6       /* a non-finite dual objective or certificate */
} dl_status;

/* Per-user simple set (Section 3.3). radius is z for the simplices, u for the box. */
typedef enum { DL_PROJ_SIMPLEX_LE = 0, DL_PROJ_SIMPLEX_EQ = 1, DL_PROJ_BOX = 2, DL_PROJ_BOXCUT = 3 } dl_proj_kind;

/* Storage of c and a in device memory. DL_BF16 rounds (to nearest even) at
 * create time; projection and accumulation stay FP32 / fixed point, the dual
 * objective and gap FP64. */
typedef enum { DL_F32 = 0, DL_BF16 = 1 } dl_storage;

typedef struct dl_problem dl_problem;
typedef struct dl_solver dl_solver;
typedef struct dl_batch dl_batch;

/*
 * User-to-lane mapping of the gradient pass.  DL_LAYOUT_BUCKETED groups users
 * by degree and gives each 2^g lanes so that no lane holds more than a fixed
 * number of elements (the degree bucketing of Section 4.2, generalised).
 * DL_LAYOUT_WAVEFRONT gives every user a full 64-lane wavefront: the plain
 * mapping, kept as the baseline the bucketed layout is measured against.
 * Both compute the same values up to the order of the FP32 sums inside one
 * user's projection.
 */
typedef enum { DL_LAYOUT_BUCKETED = 0, DL_LAYOUT_WAVEFRONT = 1 } dl_layout;

typedef struct {
  int64_t n_users;          /* I >= 0 */
  int32_t n_items;          /* J >= 1 */
  int32_t n_families;       /* m, 1..4 */
  const int64_t* row_ptr;   /* device, I+1: row_ptr[0] = 0, nondecreasing */
  const int32_t* item_idx;  /* device, nnz: strictly increasing within each row, in [0, J) */
  const float* c;           /* device, nnz: linear cost c_ij (finite) */
  const float* a;           /* device, m*nnz family-major (finite), or NULL: every a_kij = 1 */
  const double* b;          /* host, m*J, family-major right-hand side */
  int32_t proj;             /* dl_proj_kind */
  int32_t storage;          /* dl_storage */
  double radius;            /* z (simplex, box-cut sum) or u (box), > 0 */
  double upper;             /* u of the box-cut set {0 <= x <= u, sum x <= z} (DL_PROJ_BOXCUT), > 0 */
  int32_t jacobi;           /* 1: Jacobi row scaling in the solver (Appendix C) */
  int32_t wg_per_cu;        /* gradient-pass workgroups per compute unit, 0 = default (4) */
  int32_t layout;           /* dl_layout: user-to-lane mapping of the gradient pass */
  int32_t eq_families;      /* bit k set: family k holds equality rows A_k x = b_k, whose duals are free
                               (not clamped at 0); the certificate then has no feasible repair: rel_gap
                               is NaN, max_slack is max |A x - b| on those rows (give the last stage a
                               fixed iteration count) */
  void* stream;             /* hipStream_t */
  double global_cap;        /* M of the global-count row (global_count = 1), finite, >= 0 */
  int32_t global_count;     /* 1: add the row sum over all (i,j) of x_ij <= global_cap (Section 5) */
} dl_problem_desc;

/* Facts about a created problem (all host values). */
typedef struct {
  int64_t n_users, nnz;
  int32_t n_items, n_families;
  int32_t n_stored_families;  /* families whose a is not identically 1 */
  int32_t n_workgroups;       /* gradient-pass grid */
  int64_t n_tasks;            /* wavefront tasks per pass */
  double lhat;                /* bound on ||A'||_2^2, A' = DA (exact for m = 1) */
  double bytes_per_pass;      /* algorithmic HBM bytes of one gradient pass */
  double device_bytes;        /* library-owned device memory */
  int32_t max_degree;
  int32_t n_buckets;
  int32_t bucket_glog[8];     /* log2 lanes per user of each degree bucket (7 = long rows) */
  int64_t bucket_users[8];
  float qscale[4];            /* fixed-point step of each family's accumulation is 1/qscale */
  int64_t n_rows;             /* dual coordinates: m*J (+1 with the global-count row) */
  int32_t n_windows;          /* launches per gradient pass: 1, or the histogram row windows */
} dl_problem_info;

/*
 * Creates a problem: validates the CSR instance, reorders users by degree,
 * builds the per-wavefront task table, computes the Jacobi scaling D and the
 * step bound lhat (Appendix C), and copies c and a into library storage.
 * Returns DL_EINVAL for malformed data (non-monotone row_ptr, item out of
 * range or repeated in a row, non-finite c/a/b, radius <= 0, a negative or
 * non-finite global_cap), DL_EUNSUPPORTED when J > 16,383 (16-bit item
 * offsets) or n_rows + J > 40,832 (the duals and one repair factor per item
 * staged in one workgroup's 160 KiB of LDS), DL_ENOMEM or DL_EHIP otherwise.
 * Up to m*J = 13,000 each workgroup accumulates all of A x in LDS in one
 * launch.  Beyond that the histogram rows are cut into n_windows equal windows
 * that fit in LDS beside the duals, and a gradient pass is one launch per
 * window: each recomputes x and keeps the sums of its own rows (the result is
 * bitwise the same; the data is read n_windows times).  Such problems use a
 * multi-family kernel and cannot join a batch.
 * Synchronises the stream before returning.
 */
dl_status dl_problem_create(const dl_problem_desc* desc, dl_problem** out);

/* Frees everything the problem owns. NULL-safe. */
void dl_problem_destroy(dl_problem* prob);

dl_status dl_problem_get_info(const dl_problem* prob, dl_problem_info* out);

/*
 * New day on the same eligibility pattern (the recurring solves of Section 1):
 * replaces c (device, nnz, caller order; nullable = keep) and b (host, m*J;
 * nullable = keep; a global cap is kept).  a, the Jacobi scaling and the step bound are unchanged.
 * DL_EINVAL on non-finite input (c may then be partly replaced).  Synchronises.
 */
dl_status dl_problem_update(dl_problem* prob, const float* c, const double* b);

/*
 * ObjectiveFunction.calculate (Table 1; eqs. 2-4) at lam, gamma > 0.
 *   lambda    device, n_rows: the dual point (used at FP32 in the per-nnz gather)
 *   grad      device, n_rows, nullable: A x*(lam) - b
 *   dual_obj  host, nullable: g(lam) in FP64 (synchronises)
 *   x         device, nnz, nullable: x*(lam) in the caller's CSR order
 */
dl_status dl_dual_grad(dl_problem* prob, const double* lambda, double gamma, double* grad,
                       double* dual_obj, float* x);

/*
 * ProjectionMap (Table 1): x = Pi_C(v) row by row, v and x device arrays of
 * length nnz in the caller's CSR order (v and x may alias).
 */
dl_status dl_project(dl_problem* prob, const float* v, float* x);

/* ----------------------------------------------------------------------- */
/* Maximizer: accelerated projected dual ascent with gamma continuation     */
/* (Sections 4.4 and 6, Appendix C).                                        */
/* ----------------------------------------------------------------------- */
typedef struct {
  int32_t n_stages;        /* >= 1 */
  int32_t check_every;     /* certificate period in the final stage; 0 = only at the end */
  const double* gammas;    /* host, n_stages, each > 0 */
  const int64_t* iters;    /* host, n_stages; the last may be -1: until tol or max_iters */
  double tol;              /* stop when the certified relative gap <= tol (final stage) */
  int64_t max_iters;       /* total iteration cap */
  int32_t reset_momentum;  /* 1: restart the momentum at each stage switch */
  int32_t autotune_rounds; /* > 0: dl_solver_autotune once, after up to 50 iterations of stage 0
                              (dl_batch_solve: the batch's own tuner, at the same point) */
  double step_scale;       /* step = step_scale * gamma / lhat */
} dl_solve_opts;

typedef struct {
  int64_t iters;           /* iterations run */
  int32_t stage;           /* stage index at exit */
  int32_t status;          /* dl_status of the solve */
  double gamma;            /* gamma of the last stage run */
  double dual_obj;         /* g_gamma(lam) */
  double primal_obj;       /* P_gamma(x~) of the feasible repair of x*(lam) */
  double rel_gap;          /* (P_gamma(x~) - g_gamma(lam)) / max(1, |g_gamma(lam)|) */
  double max_slack;        /* max (A x*(lam) - b)^+ */
  double lagr_gap;         /* -lam^T grad g(lam) */
  int64_t n_checks;        /* certificates evaluated */
  double wall_ms;          /* host wall time of the call */
} dl_solve_stats;

/*
 * Runs the whole schedule from lambda0 (device, n_rows, nullable = 0) and writes
 * the final lam (device, n_rows) and stats (host).  The certificate (two extra
 * gradient passes) is evaluated every check_every iterations of the final
 * stage and at the end.  Returns DL_OK, DL_NOT_CONVERGED (cap reached, results
 * valid), DL_DIVERGED (non-finite iterate) or an error.
 */
dl_status dl_solve(dl_problem* prob, const dl_solve_opts* opts, const double* lambda0,
                   double* lambda_out, dl_solve_stats* stats);

/*
 * dl_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same schedule, stopping rule, results and statuses as dl_solve, bitwise,
 * but the solver state (lam', y', A x in FP64 and the two FP32 gather points:
 * 32 bytes per coupling row, plus a flag) lives in one fixed device array of
 * the library (524,544 bytes per device, held until the process ends) instead of
 * memory allocated per call.  The problem's own buffers, made at create time,
 * are used as by dl_solve; the call itself calls no hipMalloc or hipFree.
 *   Limits  n_rows <= 16384 (else DL_EUNSUPPORTED);
 *           opts->autotune_rounds must be 0 (the tuner allocates; DL_EINVAL);
 *           the problem's device must be the current device (DL_EINVAL).
 *   Sharing every call on a device uses that device's one array and leaves
 *           its contents behind (each call starts by setting what it reads):
 *           calls that overlap on one device, from two threads or on two
 *           streams, race and must be serialised by the caller.
 */
dl_status dl_solve_noalloc(dl_problem* prob, const dl_solve_opts* opts, const double* lambda0,
                           double* lambda_out, dl_solve_stats* stats);

/* Stepwise access to the same iteration, for trajectories and timing. */
dl_status dl_solver_create(dl_problem* prob, const double* lambda0, dl_solver** out);
void dl_solver_destroy(dl_solver* s);
/* Starts a stage at gamma with step step_scale*gamma/lhat; reset=1 restarts the momentum. */
dl_status dl_solver_set_stage(dl_solver* s, double gamma, double step_scale, int32_t reset);
/* Enqueues n accelerated iterations (gradient pass + fused update each). No sync. */
dl_status dl_solver_step(dl_solver* s, int64_t n);
/* Current lam (device, n_rows). */
dl_status dl_solver_get_lambda(dl_solver* s, double* lambda_out);

/*
 * Checkpoint / resume of a stepwise solve.  dl_solver_export copies the dual
 * state into state (device, 2*n_rows: the Jacobi-scaled lam' then the momentum
 * point y', in the solver's internal units: opaque) and fills meta (host).
 * dl_solver_import loads both into a solver of a problem with the same data
 * (same layout, scaling and step bound); the next dl_solver_step continues
 * bitwise where the exported solver stood.  DL_EINVAL on a size mismatch or
 * an invalid meta.  Neither call synchronises.
 */
typedef struct {
  double gamma;       /* current stage's gamma */
  double eta;         /* current step */
  double tk;          /* FISTA momentum sequence t_k (>= 1) */
  int64_t iters;      /* iterations taken */
  int64_t m_times_j;  /* size check: n_rows of the exporting problem */
} dl_solver_meta;
dl_status dl_solver_export(dl_solver* s, double* state, dl_solver_meta* meta);
dl_status dl_solver_import(dl_solver* s, const double* state, const dl_solver_meta* meta);
/* Certificate at the current lam and gamma (synchronises). */
dl_status dl_solver_certificate(dl_solver* s, dl_solve_stats* out);

typedef struct {
  int64_t n_grad;          /* timed gradient passes */
  double grad_ms_total;    /* summed HIP-event durations of those passes */
  int64_t n_update;
  double update_ms_total;  /* summed time from each pass's end to the end of its reduction and update */
} dl_timing;
/* Brackets every later gradient pass with HIP events on the stream, and closes
 * each reduction + update with one more (three events per iteration). */
dl_status dl_solver_enable_timing(dl_solver* s, int32_t on);
/* Synchronises and returns the sums since timing was enabled. */
dl_status dl_solver_get_timing(dl_solver* s, dl_timing* out);

/* ----------------------------------------------------------------------- */
/* Many independent instances in one launch per iteration phase.           */
/* ----------------------------------------------------------------------- */
/*
 * Groups n created problems (n >= 1; same device, stream, storage and kernel
 * variant: the same family count class and whether a is stored).  The batch
 * borrows the problems: they must outlive it and must not be used by other
 * calls while a batch solve runs.  DL_EUNSUPPORTED for mixed variants.
 */
dl_status dl_batch_create(int32_t n, dl_problem* const* probs, dl_batch** out);
void dl_batch_destroy(dl_batch* batch); /* NULL-safe; does not destroy the problems */
/*
 * Solves every member with the same schedule as dl_solve, in lockstep: each
 * iteration is one gradient-pass launch over all live members (workgroups
 * dealt by pass cost) plus one update launch.  Members leave the launch when
 * their certified gap reaches tol at a check point of the final stage.
 * With opts->autotune_rounds = r > 0 the workgroup schedule is tuned on the
 * solve's own iterations (no extra passes), from iteration 10 of the first
 * stage that runs at least 10 + 12 (1 + r) iterations: for grids of 4, 2 and
 * 1 workgroups per compute unit, the cost-model split and then r splits
 * re-dealt (between members and inside each) from the previous trial's
 * per-workgroup clock stamps each serve 4 iterations timed with HIP events;
 * the fastest serves the rest of the solve (dl_batch_get_tune reports it).
 * The split never changes a member's iterates: they stay bitwise equal to its
 * solo solve.
 *   lambda0     host array of n device pointers (n_rows of member i each), or NULL (zeros)
 *   lambda_out  host array of n device pointers (n_rows of member i each)
 *   stats       host array of n records (iters and status per member)
 * Returns DL_OK when every member converged, DL_NOT_CONVERGED when some hit
 * the cap (results valid), or an error.
 */
dl_status dl_batch_solve(dl_batch* batch, const dl_solve_opts* opts, const double* const* lambda0,
                         double* const* lambda_out, dl_solve_stats* stats);

/* ----------------------------------------------------------------------- */
/* Workgroup schedule tuning                                               */
/* ----------------------------------------------------------------------- */
typedef struct {
  int32_t n_workgroups;     /* gradient-pass grid kept */
  int32_t rounds;           /* balancing rounds per candidate grid */
  double pass_ms_model;     /* mean pass + partial-sum reduction time, cost-model split, at the kept grid */
  double pass_ms_tuned;     /* the same after balancing (10 passes, the time the grid was chosen on) */
  double imbalance_model;   /* max / mean workgroup time before balancing */
  double imbalance_tuned;   /* the same after */
} dl_tune_result;

/*
 * Tunes the gradient pass's workgroup schedule at the solver's current point
 * (call it after some iterations, so the active sets are realistic): for
 * grids of 1, 2, 4, ... workgroups per compute unit (up to what the problem
 * was created with), the task split is re-balanced `rounds` times from
 * measured per-workgroup times (steady-clock stamps), and the fastest grid and
 * split are kept for every later pass of this problem.  Does not change the
 * solver's iterate.  Synchronises the stream.  A round costs three passes per
 * grid size; each re-deal starts from one noisy measurement, so more rounds
 * give the best-timed split more chances (10M x 10k production rows: 3 rounds
 * leave a workgroup imbalance of 1.05-1.17, 10 rounds 1.02-1.03).
 */
dl_status dl_solver_autotune(dl_solver* s, int32_t rounds, dl_tune_result* out);
/*
 * The tuning of the last dl_batch_solve run on this batch (all zeros when it
 * ran without autotune_rounds).  Here pass_ms_model is the mean time of one
 * whole iteration (scale pass, batched gradient pass, update) over the first
 * trial (cost-model split, 4 workgroups per compute unit), pass_ms_tuned the
 * same over the kept configuration's trial, and n_workgroups the kept grid
 * over the members live when tuned.
 */
dl_status dl_batch_get_tune(const dl_batch* batch, dl_tune_result* out);

/* ----------------------------------------------------------------------- */
/* Learned warm start (not part of the paper's method).                    */
/* ----------------------------------------------------------------------- */
/*
 * Per-item features of a day's instance (family 0), FP32, row-major J x 16:
 *   0 b/n, 1 log1p(n)/10, 2 mean c, 3 std c, 4 max c, 5 min c over the item's
 *   eligible users, 6 lam_prev, 7 [lam_prev > 0], 8 b_prev/n,
 *   9 clip(g_prev/b_prev, -1, 1), 10 10 (b/b_prev - 1), 11 n / mean n, 12-15 0
 * with n the item's eligible-user count (n = 1 in the divisions when 0).
 *   lam_prev  device, J: the previous day's duals
 *   g_prev    device, J: a gradient A x - b at lam_prev; the warm-start
 *             pipeline passes this problem's (today's) gradient there, so
 *             column 9 is today's relative over-subscription at yesterday's
 *             duals
 *   b_prev    host, J: the previous day's right-hand side
 *   feats     device, J*16 output
 * The per-item sums are exact integer (fixed-point) sums: reproducible.
 */
dl_status dl_item_features(dl_problem* prob, const double* lam_prev, const double* g_prev, const double* b_prev,
                           float* feats);

typedef struct dl_mlp dl_mlp;
typedef struct {
  int32_t n_in;        /* must be 16 (features zero-padded to 16) */
  int32_t hidden;      /* H, multiple of 64 in [64, 1024] */
  int64_t max_batch;   /* largest number of rows per call, <= 2^24 */
  void* stream;        /* hipStream_t */
} dl_mlp_desc;

/*
 * MLP 16 -> H -> H -> 1 with ReLU: y = relu(relu(x W1 + b1) W2 + b2) w3 + b3.
 * FP32 master parameters, BF16 copies of W1, W2, w3 and BF16 activations for
 * the matrix-core GEMMs, FP32 accumulation.  Parameters are flat FP32:
 * W1 [16 x H] row-major, b1 [H], W2 [H x H] row-major, b2 [H], w3 [H], b3 [1].
 * Created with zero parameters: set them with dl_mlp_set_params.
 */
dl_status dl_mlp_create(const dl_mlp_desc* desc, dl_mlp** out);
void dl_mlp_destroy(dl_mlp* mlp);  /* NULL-safe */
int64_t dl_mlp_num_params(const dl_mlp* mlp);
/* host, num_params floats; resets the optimiser state (synchronises) */
dl_status dl_mlp_set_params(dl_mlp* mlp, const float* params);
dl_status dl_mlp_get_params(dl_mlp* mlp, float* params);  /* host; synchronises */
/*
 * Input normalisation (host, 16 each): the network sees column k of X as
 * (x - shift[k]) * scale[k] (FP32, then one BF16 rounding); scale 0 removes
 * a column.  Default shift 0, scale 1.  Synchronises.
 */
dl_status dl_mlp_set_input_norm(dl_mlp* mlp, const float* shift, const float* scale);
/* y (device, n) = MLP(X) for X device n x 16, n <= max_batch */
dl_status dl_mlp_forward(dl_mlp* mlp, const float* X, int64_t n, float* y);
/*
 * Warm-start prediction: lam0 (device, n) = max(0, lam_prev + s * MLP(X)) in
 * FP64; rows whose network output is non-finite keep max(0, lam_prev).
 */
dl_status dl_mlp_predict_duals(dl_mlp* mlp, const float* X, int64_t n, const double* lam_prev, double s,
                               double* lam0);
/* grad (device, num_params) = gradient of sum_i dy_i y_i; y (device, n, nullable) */
dl_status dl_mlp_gradients(dl_mlp* mlp, const float* X, const float* dy, int64_t n, float* y, float* grad);
/* One AdamW step (beta 0.9 / 0.999, eps 1e-8, decay wd on W1, W2, w3) on the
 * loss (1/2n) sum (y - target)^2; target device, n.  loss (host, nullable)
 * returns the loss before the step and synchronises. */
dl_status dl_mlp_train_step(dl_mlp* mlp, const float* X, const float* target, int64_t n, float lr, float wd,
                            double* loss);

/*
 * Judged warm start: each candidate start (device pointers, n_rows each; a NULL
 * entry means lam = 0) is clamped to lam >= 0 and scored by the dual value
 * g_{gamma_0}(lam) at the schedule's first gamma; non-finite candidates score
 * -inf.  dl_solve then runs from the best.  chosen (nullable) returns its index,
 * cand_dual (host, n_cand, nullable) the scores.  Pass the cold start (NULL) as
 * one candidate to keep it as the fallback.
 */
dl_status dl_solve_warm(dl_problem* prob, const dl_solve_opts* opts, int32_t n_cand, const double* const* cands,
                        double* lambda_out, dl_solve_stats* stats, int32_t* chosen, double* cand_dual);

/* ----------------------------------------------------------------------- */
/* Measurement                                                             */
/* ----------------------------------------------------------------------- */
/*
 * Sustained read rate of the current device's HBM: the library allocates a
 * buffer of bytes (rounded down to 16-byte words) with hipMalloc, and a
 * streaming kernel reads it reps times with 16-byte loads and nothing else,
 * timed with HIP events on stream (a hipStream_t, NULL = default).  gbps
 * (host) returns bytes read per second / 1e9.  This is the practical ceiling
 * against which the gradient pass's bandwidth is reported (the pass is bound
 * by HBM reads).  DL_ENOMEM when the buffer does not fit.  Synchronises the
 * stream and frees the buffer.  Not part of the paper's method.
 */
dl_status dl_read_bandwidth(int64_t bytes, int32_t reps, void* stream, double* gbps);

/* Message for the last non-OK status on this thread. */
const char* dl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DUALIP_H */
