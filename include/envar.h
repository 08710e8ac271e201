/* envar.h -- C ABI of the MI355X EnVar forward-ensemble library.
 *
 * The library integrates N independent 2D incompressible Navier-Stokes
 * open-cavity simulations in one batch, each driven by its own steady
 * forcing row f_i (eq. forced_NS with f_u(x) steady, Sec. 2), accumulates
 * each member's cost J_i on the fly (eq. Envarcost with the fluctuation
 * energy of eq. kinenergy as observation term), and reduces the control
 * anomalies and costs to a gradient estimate (eq. gradient_EnVar in its
 * scalar-J form, with the finite differences of eq. fdapprox).
 *
 * Conventions shared by every entry point
 *  - The caller owns all memory. Device buffers are plain device pointers
 *    (any allocator); the library never allocates device memory. Sizes come
 *    from envar_state_bytes / envar_workspace_bytes / envar_gradient_bytes.
 *  - Every call is stream ordered on `stream` (a hipStream_t passed as void*,
 *    NULL = the default stream) and asynchronous unless stated otherwise.
 *  - Arrays are row-major FP64. A control row has m = 2 * n_ctrl entries:
 *    f_x over the control cells in row-major cell order, then f_y over the
 *    same cells. The gradient is the Euclidean dJ/df_k (no mass-matrix
 *    scaling).
 *  - Return value: ENVAR_OK or an error code; envar_last_error() returns a
 *    thread-local message for the last failing call on this thread. No C++
 *    exception crosses the ABI. Calls on distinct workspaces are thread safe.
 *
 * Grid (cavity geometry): channel [0, 4] x [0, 1] over a square cavity
 * [x_cav, x_cav + 1] x [-1, 0], uniform spacing h = 1 / inv_h, MAC
 * staggering; bounding box NX = 4 inv_h by NY = 2 inv_h cells. Host field
 * layouts ("oracle layout") are dense row-major: u (NY, NX + 1), v (NY + 1,
 * NX), cell fields (NY, NX). The channel geometry drops the cavity (NY = inv_h).
 */
#ifndef ENVAR_H
#define ENVAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ENVAR_OK = 0,
  ENVAR_EINVAL = 1,      /* bad argument: shape, size, NULL pointer, NaN input */
  ENVAR_ENOMEM = 2,      /* a buffer is smaller than the size the library needs */
  ENVAR_EDIVERGED = 3,   /* >= 1 member produced a non-finite cost; its J is NaN, others are valid */
  ENVAR_EDEVICE = 4,     /* a HIP runtime call failed */
  ENVAR_EBUSY = 5,       /* serving queue is full */
  ENVAR_ECANCELLED = 6,  /* request cancelled before completion */
  ENVAR_ETIMEOUT = 7,    /* envar_wait timed out */
  ENVAR_EUNCONVERGED = 8 /* served request: >= 1 member-step's pressure solve stopped at the pass cap
                            before div_tol; the costs are returned */
};

/* ENVAR_CAVITY_PAPER: the configuration of Sec. 2 (Table tabgeometry) with the boundary
 * conditions of Sec. 4.4 on this grid: a channel of height 1/2 over the unit cavity (NY =
 * inv_h + inv_h / 2), uniform inflow u = 1, a symmetry (slip) top wall, a lower wall that is no-slip
 * for x_cav - 0.4 <= x <= x_cav + 1.75 and slip beyond, no-slip cavity walls; the outlet keeps the
 * convective condition, with the inflow's bulk speed 1. */
enum { ENVAR_CAVITY = 0, ENVAR_CHANNEL = 1, ENVAR_CAVITY_PAPER = 2 };
/* Control regions (cells whose centre lies inside):
 *  COLUMN: x in [x_cav, x_cav + 1], all y (cavity + channel column above it), 2 / h^2 cells
 *  CAVITY: the cavity cells only, 1 / h^2 cells
 *  BOX:    fluid cells with centre in [box[0], box[1]] x [box[2], box[3]] (Sec. 4.1 actuation window) */
enum { ENVAR_REGION_COLUMN = 0, ENVAR_REGION_CAVITY = 1, ENVAR_REGION_BOX = 2 };
/* FP64: every kernel in FP64. MIXED: the multigrid V-cycle (every smoothing,
 * restriction and prolongation) in FP32, wrapped in FP64 iterative refinement
 * of the pressure; the state, the AB2 tendencies, the coarse solve, the cost
 * sums and the least squares stay FP64 (tendencies rounded to FP32 would put
 * rounding noise into every step's divergence and cost a refinement pass). */
enum { ENVAR_FP64 = 0, ENVAR_MIXED = 1 };

/* One forward problem, passed by value-pointer; fields <= 0 take defaults. */
typedef struct {
  int32_t inv_h;       /* 1/h; a multiple of 16 (cavity aligned down to h = 1/4) */
  int32_t geometry;    /* ENVAR_CAVITY | ENVAR_CHANNEL | ENVAR_CAVITY_PAPER */
  int32_t region;      /* ENVAR_REGION_* */
  int32_t precision;   /* ENVAR_FP64 | ENVAR_MIXED */
  double Re;           /* U D / nu with U = inflow centreline speed, D = cavity depth (Sec. 2) */
  double dt;           /* <= 0: 0.064 h */
  double x_cav;        /* <= 0: 1.25 */
  double box[4];       /* x0, x1, y0, y1 for ENVAR_REGION_BOX */
  double penalty;      /* lambda of the penalty lambda h^2 |f|^2; < 0: 1e-3 */
  double div_tol;      /* bound on the divergence after projection: the pressure solve stops when
                          dt * max|b - L phi| <= 0.999 div_tol (the margin covers rounding between
                          the residual and the divergence of the projected velocities);
                          <= 0: 1e-12 FP64, 1e-10 MIXED */
  int32_t max_cycles;  /* cap on V-cycles (FP64) or refinement passes (MIXED) per step; <= 0: 30 */
  int32_t flags;       /* ENVAR_FLAG_* bits, 0 = none */
} envar_problem;

/* envar_problem.flags */
enum {
  /* Record HIP events on the call's stream around the predictor, the first
   * full cycle's finest-level multigrid launches and the projection of a
   * uniform sample of steps (at most ~256), filling the *_us fields of
   * envar_stats (requires stats != NULL). */
  ENVAR_FLAG_TIME_KERNELS = 1,
  /* Launch every step eagerly instead of replaying captured HIP graphs of
   * the steady steps (for comparisons; results are identical). */
  ENVAR_FLAG_NO_GRAPHS = 2,
  /* Tile heights. By default the first call for a (grid, geometry,
   * precision, member count) times 8- and 16-row tiles for the predictor and
   * the projection and 8-, 16- and 32-row tiles for every tiled multigrid
   * level (32 where the cavity rows take whole tiles) on the call's workspace
   * (before the members are initialised) and keeps the fastest for the
   * process. The results do not depend on the choice (the cost partial sums
   * live on fixed 64 x 8 blocks; the multigrid windows reproduce the global
   * red-black sweep). These flags bypass the tuner: */
  ENVAR_FLAG_NO_TUNE = 4,   /* 8-row step tiles, 16-row multigrid tiles */
  ENVAR_FLAG_TILES_8 = 8,   /* 8 rows everywhere */
  ENVAR_FLAG_TILES_16 = 16, /* 16 rows everywhere (step tiles only where the rows align) */
  ENVAR_FLAG_TILES_32 = 32, /* 32-row multigrid tiles where the cavity rows take whole tiles
                               (16 elsewhere), 16-row step tiles where the rows align */
  /* By default the members of a forward (or of a batch) advance in two lanes: member groups of
   * about equal work on two streams (the call's stream and one the library keeps per host
   * thread), each with its own step graphs and cycle cap, so that one group's latency-bound
   * phases overlap with the other's bandwidth-bound kernels. The call stays ordered on its
   * stream (the lanes fork from it and join back). Results do not depend on the lanes. This
   * flag runs every member on the call's stream. */
  ENVAR_FLAG_ONE_LANE = 64,
  /* Pressure passes. A step launches its first passes (V-cycles in FP64, refinement passes in
   * MIXED) level by level, as many as the members needed lately (at least two); the passes
   * beyond, up to max_cycles, run in one launch that gives each member a workgroup of its own and
   * goes through the same per-tile arithmetic, so a member that needs more passes than its batch
   * has lately needed gets them at the cost of one launch per step when no member does. This
   * holds for jobs with 32 <= inv_h <= 256; other batches keep one extra level-by-level pass of
   * headroom. Results do not depend on either choice. */
  ENVAR_FLAG_NO_TAIL = 128,      /* one pass of headroom instead of the per-member launch */
  ENVAR_FLAG_SHORT_GRAPH = 256   /* one level-by-level pass per step, every later one in the
                                    per-member launch (for comparisons; much slower) */
};

/* Per-call statistics (filled only when a non-NULL pointer is passed; then the
 * call synchronises its stream before returning). */
typedef struct {
  double max_resid;        /* max over members and steps of dt * max|b - L phi| after the last cycle */
  double max_div;          /* max over members and steps of max |div_h u^{n+1}| measured after projection */
  double mean_cycles;      /* V-cycles (FP64) or refinement passes (MIXED) per member-step */
  int32_t max_cycles_used; /* largest per-step count */
  int32_t unconverged;     /* member-steps that reached max_cycles without meeting div_tol */
  int32_t diverged;        /* members with a non-finite cost */
  int32_t steps;           /* time steps integrated */
  double cell_steps;       /* fluid cells x steps x members */
  /* ENVAR_FLAG_TIME_KERNELS: mean device time per launch (microseconds) over
   * the sampled steps, and the number of sampled steps */
  double predictor_us;     /* predictor, fused with the previous step's projection and cost sample */
  double pre_us;           /* finest-level pre-smoothing + restriction */
  double post_us;          /* finest-level prolongation + post-smoothing (+ residual norm) */
  double resid_us;         /* FP64 refinement residual (MIXED) */
  double project_us;       /* 0: the projection runs inside the next predictor (one closing launch per forward) */
  double vcycle_us;        /* one full V-cycle (FP64) or refinement pass (MIXED) */
  int32_t timed_steps;
  int32_t timed_members;   /* members active in the timed cycle (all, unless converged before it) */
  /* tile heights in use: predictor and projection 8 | 16, tiled multigrid levels 0..3 8 | 16 | 32 (0 = none) */
  int32_t rows_pred, rows_proj, rows_mg[4];
} envar_stats;

/* Number of control entries m = 2 * n_ctrl for this problem. */
int envar_control_dim(const envar_problem* p, int64_t* m);

/* Fluid cells of the flow grid. */
int envar_cell_count(const envar_problem* p, int64_t* ncells);

/* Device bytes of a resident base state (flow fields, AB2 history, warm-start
 * pressure, cost shift, control map, coarse-grid inverse). */
size_t envar_state_bytes(const envar_problem* p);

/* Device bytes of the workspace of a forward over n_rows members (all member
 * fields and the multigrid hierarchy). The admission footprint of a request. */
size_t envar_workspace_bytes(const envar_problem* p, int32_t n_rows);

/* Build a base state in caller memory `state_dev` (envar_state_bytes) from host
 * arrays in oracle layout: u (NY, NX+1), v (NY+1, NX) and optionally the
 * previous tendencies tu_prev, tv_prev (same shapes; NULL = cold start, the
 * first step then uses T^{-1} = T^0) and a warm-start pressure phi (NY, NX)
 * (NULL = 0). Boundary values are imposed (walls 0, inflow 4y(1-y)).
 * Synchronous (returns after the upload completed). */
int envar_state_init(const envar_problem* p, const double* u, const double* v,
                     const double* tu_prev, const double* tv_prev, const double* phi,
                     void* state_dev, void* stream);

/* Copy a base state back to host arrays in oracle layout (any pointer may be
 * NULL). Synchronous. */
int envar_state_read(const envar_problem* p, const void* state_dev, double* u, double* v,
                     double* tu_prev, double* tv_prev, double* phi);

/* Advance a base state in place by `steps` unforced steps (spin-up). Uses a
 * workspace sized for n_rows = 1. */
int envar_spinup(const envar_problem* p, void* state_dev, int32_t steps, void* ws_dev,
                 size_t ws_bytes, envar_stats* stats, void* stream);

/* The N+1 forward evaluations (Sec. 3.3.1, eq. fdapprox): every row i of
 * controls_dev [n_rows][m] (device, FP64) drives one member from the base state
 * for `horizon` steps; J_dev[i] (device, FP64) receives
 *   J_i = dt h^2 sum_{n=1..K} sum_c |u_c^n - ubar_c|^2 + lambda h^2 |f_i|^2
 * with ubar_c the member's time mean over its K = horizon samples.
 * fields_dev (optional, device, may be NULL): [n_rows][NY*(NX+1) + (NY+1)*NX]
 * receives each member's final u then v in oracle layout.
 * Errors: EINVAL (shape, m mismatch, horizon < 1), ENOMEM (ws_bytes too small),
 * EDIVERGED (only when stats != NULL and a cost is non-finite). */
int envar_forward(const envar_problem* p, const void* state_dev, const double* controls_dev,
                  int32_t n_rows, int64_t m, int32_t horizon, void* ws_dev, size_t ws_bytes,
                  double* J_dev, double* fields_dev, envar_stats* stats, void* stream);

/* One ensemble of a batched forward (envar_forward_batch). */
typedef struct {
  envar_problem problem;     /* its own grid, Re, region, dt; precision must match across the batch */
  const void* state_dev;     /* its base state (envar_state_init) */
  const double* controls_dev;/* [n_rows][m] */
  int32_t n_rows;
  int32_t horizon;           /* its own number of steps */
  int64_t m;
  void* ws_dev;              /* envar_workspace_bytes(&problem, n_rows) bytes */
  size_t ws_bytes;
  double* J_dev;             /* [n_rows] */
  envar_stats* stats;        /* optional (the call then synchronises) */
  double* fields_dev;        /* optional: final u, v of every member, layout as in envar_forward */
} envar_job;

/* Uneven batching: up to 8 ensembles that differ in grid size, Reynolds
 * number, member count and horizon advance together, every kernel launch
 * carrying one segment per ensemble (the N+1 forward evaluations of several
 * EnVar iterations at once, Sec. 5.3). An ensemble leaves the batch when its
 * horizon is reached. Results equal those of separate envar_forward calls
 * (per-member convergence). Errors: EINVAL (njobs outside [1, 8], mixed
 * precisions, bad shapes), ENOMEM, EDIVERGED (stats requested and a cost is
 * non-finite). */
int envar_forward_batch(envar_job* jobs, int32_t njobs, void* stream);

/* Device bytes of the workspace of envar_gradient (the same with or without ENVAR_GRADIENT_PINV). */
size_t envar_gradient_bytes(int32_t n, int64_t m, int32_t precision);

/* Anomaly reduction {delta f_i, J_i} -> g (eq. gradient_EnVar, scalar-J form):
 * rows 1..n of controls_dev [n+1][m] are the perturbed controls and row 0 the
 * centre; X_i = f_i - f_0, dJ_i = J_i - J_0 (J_dev [n+1], device);
 * g_dev [m] (device) receives the minimum-norm least-squares solution
 * g = X^+ dJ = X^T (X X^T)^{-1} dJ (n <= m; n > m uses (X^T X)^{-1} X^T dJ).
 * The Gram X X^T runs on the matrix cores (FP64 MFMA, or FP32 MFMA with
 * precision = ENVAR_MIXED); the n x n solve is an FP64 Cholesky with a
 * relative ridge 1e-12 tr(G)/n (a rank-deficient X, e.g. repeated members, then gives the
 * minimum-norm solution up to that ridge). When the factor fails (a pivot not positive after
 * the ridge), the call does not give up: in mixed precision (n <= m) the system is formed
 * again in FP64 from the control rows, the FP64 gradient's arithmetic; a factor that fails in
 * FP64 is replaced by the eigen-pseudo-inverse of the Gram (cyclic Jacobi, eigenvalues at or
 * below 1e-12 of the largest dropped; systems up to 512). precision | ENVAR_GRADIENT_PINV asks
 * for the pseudo-inverse directly (in mixed precision over the FP64 Gram). Synchronous (the
 * solve is checked on the host).
 * Errors: EINVAL (n < 1, m < 1, min(n, m) > 1024, an unknown precision or flag), ENOMEM,
 * EDIVERGED (a non-finite solution, e.g. from a non-finite cost; a failed factor with no
 * fallback: mixed precision with n > m, or a system above 512; g_dev is then undefined),
 * EDEVICE (a launch failed). */
#define ENVAR_GRADIENT_PINV 16
int envar_gradient(const double* controls_dev, const double* J_dev, int32_t n, int64_t m,
                   int32_t precision, void* ws_dev, size_t ws_bytes, double* g_dev, void* stream);

/* For callers that cannot allocate device memory at call time (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): envar_gradient with its workspace in
 * a library-owned static device array of ENVAR_GRADIENT_STATIC_MAX_BYTES (64 MiB), one copy on
 * every GPU the library runs on, held until the process ends. Arguments, results and errors as
 * envar_gradient; the call allocates nothing (no device or pinned host memory: the solve's
 * status word is read through pageable memory). Problems whose envar_gradient_bytes exceed the
 * array (e.g. n = 64, m = 65,536 fits in both precisions; n = 256, m = 65,536 does not) return
 * ENVAR_ENOMEM before any launch. Every call on one GPU uses the same array: calls that overlap
 * on one GPU (other threads, other streams) race and must be serialised by the caller; nothing
 * in the array needs clearing between calls (every kernel writes what a later one reads). */
#define ENVAR_GRADIENT_STATIC_MAX_BYTES ((size_t)64 << 20)
int envar_gradient_static(const double* controls_dev, const double* J_dev, int32_t n, int64_t m,
                          int32_t precision, double* g_dev, void* stream);

/* ---- Vector-observation EnVar (Sec. 3.3.1, with the observation of Sec. 4.1) ----
 * The observation H q(f) is the velocity fluctuation u' = u - u_bar at four sensors on
 * the cavity lid, x = x_cav + 1/5, 2/5, 3/5, 4/5, y = 0 (the paper places its cavity at
 * x = 0), both components, sampled at the end of steps every, 2 every, ...: eight
 * channels (channel c = 2 s + component of sensor s), each component interpolated
 * bilinearly from its own MAC positions; u_bar is the time mean of the member's own
 * samples; R = I and y = 0. */

/* Forward ensemble as envar_forward, also recording the sensor series into obs_dev
 * [n_rows][8][horizon / every] (FP64, device, caller-owned; samples of the projected
 * velocity, before the fluctuation is formed). Requires the cavity geometry. Errors:
 * EINVAL (bad sizes, every outside [1, horizon], channel geometry), ENOMEM, EDIVERGED. */
int envar_forward_obs(const envar_problem* p, const void* state_dev, const double* controls_dev,
                      int32_t n_rows, int64_t m, int32_t horizon, int32_t every, void* ws_dev,
                      size_t ws_bytes, double* J_dev, double* obs_dev, envar_stats* stats, void* stream);

/* Workspace bytes of envar_gn_step for n members and K samples per channel (0 = invalid). */
size_t envar_gn_bytes(int32_t n, int64_t K);

/* Gauss-Newton step in ensemble space (eq. gradient_EnVar, eq. Hessian_EnVar,
 * eq. update_Newton) from the series of envar_forward_obs: series_dev [n+1][8][K]
 * (row 0 the centre f^(e) + E w, row i the member f^(e) + E w + eps E_i). With d_i the
 * fluctuations of row i: Y_i = (d_i - d_0) / eps, H_GN = Y^T Y + (n - 1) I (Gram on the
 * FP64 matrix cores), dJ/dw = Y^T d_0 + (n - 1) w (w_dev [n], the current weights),
 * dw_dev [n] <- -H_GN^-1 dJ/dw (FP64 Cholesky), hgn_dev [n][n] <- H_GN (input of
 * envar_posterior_var), jw_dev [2] <- (1/2 |d_0|^2, 1/2 (n - 1) |w|^2), the two terms of
 * J(w) in eq. (J_w). All pointers device. Errors: EINVAL (n < 1, n > 1024, K < 1,
 * eps <= 0), ENOMEM, EDEVICE (a launch failed). */
int envar_gn_step(const double* series_dev, int32_t n, int64_t K, double eps, const double* w_dev,
                  void* ws_dev, size_t ws_bytes, double* dw_dev, double* hgn_dev, double* jw_dev,
                  void* stream);

/* Workspace bytes of envar_posterior_var (0 = invalid). */
size_t envar_posterior_bytes(int32_t n);

/* Diagonal of the posterior covariance B_post = E H_GN^-1 E^T (eq.
 * posterior_covariance_matrix) with E_i = (f_i - f_0) / eps from controls_dev [n+1][m]
 * and H_GN from envar_gn_step: var_dev [m] (device). H_GN is inverted in one workgroup
 * by Gauss-Jordan sweeps (n <= 128). Errors: EINVAL (n < 1, n > 128, m < 1, eps <= 0),
 * ENOMEM. */
int envar_posterior_var(const double* controls_dev, int32_t n, int64_t m, double eps,
                        const double* hgn_dev, void* ws_dev, size_t ws_bytes, double* var_dev,
                        void* stream);

/* ---------------------------------------------------------------- EnVar loop over w
 * Minimisation of J(w) (eq. J_w) over the ensemble weights with the ensemble held fixed
 * (Sec. 3.3.3), the vector observation of envar_forward_obs and R = I, y = 0. */
enum { ENVAR_GN = 0, ENVAR_LBFGS = 1 };

typedef struct {
  int32_t method;      /* ENVAR_GN: w += dw (eq. update_Newton, unit step);
                          ENVAR_LBFGS: w += alpha d, d = -H_BFGS^-1 dJ/dw (eq. update_BFGS) */
  int32_t iters;       /* outer iterations (each runs the n + 1 forwards) */
  int32_t memory;      /* L-BFGS pairs kept; <= 0: 5 */
  int32_t max_trials;  /* Armijo trials per search (one centre forward each); <= 0: 10 */
  int32_t every;       /* sensor sampling interval in steps; <= 0: 1 */
  int32_t trial_batch; /* line-search trials evaluated per batched forward (min with n + 1); <= 0: 8 */
  double eps;          /* finite-difference scale of eq. (fdapprox); <= 0: 1e-4 */
  double c1;           /* sufficient-decrease constant; <= 0: 1e-4 */
  double shrink;       /* step reduction per trial, in (0, 1); otherwise 0.5 */
} envar_ens_params;

/* Per-iteration record of envar_ens_iterate (NaN entries after an early stop). */
typedef struct {
  double J;        /* J(w) at the start of the iteration = J_obs + J_prior */
  double J_obs;    /* 1/2 |d_0|^2 */
  double J_prior;  /* 1/2 (n - 1) |w|^2 */
  double gnorm;    /* |dJ/dw| (eq. gradient_EnVar) */
  double alpha;    /* accepted step: 1 for Gauss-Newton; 0 = no sufficient decrease, loop stopped */
  int32_t trials;      /* line-search trials up to the accepted one (0 for Gauss-Newton) */
  int32_t trial_rows;  /* forward rows the search ran (>= trials: trials are batched) */
} envar_ens_record;

/* Workspace bytes of envar_ens_iterate (0 = invalid). */
size_t envar_ens_bytes(const envar_problem* p, int32_t n, int64_t m, int32_t horizon, int32_t every);

/* Each iteration builds on the device the centre f = f^(e) + E w and the members
 * f + eps E_i (eq. fdapprox), runs their n + 1 forwards recording the lid sensors, forms
 * dJ/dw and H_GN as envar_gn_step does, and updates w by the chosen method; the L-BFGS pair
 * (s, y) of consecutive iterates is stored when s.y > 0, and the direction comes from the
 * two-loop recursion with the initial scaling s.y / y.y of the newest pair. The line search
 * takes the first of 1, shrink, shrink^2, ... meeting J(w + alpha d) <= J(w) + c1 alpha g.d;
 * when none does, that record has alpha = 0, w keeps its value and the loop stops. The trial
 * steps run trial_batch at a time as rows of one forward (each row's result does not depend on
 * its batch), which gives the same accepted step as trying them one at a time.
 * fe_dev [m] = f^(e), E_dev [n][m] (row i = E_i), w_dev [n] (in: w_0, out: the final w), all
 * device; records (host, `iters` entries) may be NULL. Needs the cavity geometry.
 * Synchronous: the update decisions read J and dJ/dw on the host. Errors: EINVAL (bad
 * sizes, unknown method, no cavity), ENOMEM, EDIVERGED (non-finite gradient). */
int envar_ens_iterate(const envar_problem* p, const void* state_dev, const double* fe_dev,
                      const double* E_dev, int32_t n, int64_t m, int32_t horizon,
                      const envar_ens_params* params, double* w_dev, void* ws_dev, size_t ws_bytes,
                      envar_ens_record* records, void* stream);

/* ---------------------------------------------------------------- eigen-ensemble
 * The deterministic ensemble of Sec. 3.3.2: the N leading eigenvectors of the prior covariance
 * B_ij = sigma_i sigma_j exp(-(x_i - x_j)^2 / a_x^2 - (y_i - y_j)^2 / a_y^2) of eq. (covarianceB)
 * (c_xy = infinity, the value of Sec. 4.2) over the control cells, as members
 * E = U_N Sigma_N^(1/2) sqrt(N - 1) (eq. eigenvm1). With M_f = h^2 I the M_f-orthonormal
 * eigenvectors are U = V / h with Sigma = h^2 mu (V, mu: the orthonormal eigenpairs of the matrix
 * B), so E = V_N mu_N^(1/2) sqrt(N - 1). */
enum { ENVAR_TAPER_NONE = 0, ENVAR_TAPER_ELLIPSE = 1 };

typedef struct {
  double a_x, a_y;      /* correlation lengths; <= 0: 0.07 (Sec. 4.2) */
  double sigma2_max;    /* largest variance sigma_i^2; <= 0: 0.01 (Sec. 4.2) */
  double tol;           /* stop when |B v_k - mu_k v_k| <= tol mu_1 for every k < N; <= 0: 1e-10 */
  int32_t taper;        /* ENVAR_TAPER_ELLIPSE: sigma_i^2 = sigma2_max (1 - r^2)^2 inside the ellipse
                           inscribed in the bounding rectangle of the control cells (r = 1 on the
                           ellipse), 0 outside; ENVAR_TAPER_NONE: sigma2_max on every control cell */
  int32_t component;    /* forcing component the members drive: 0 = x, 1 = y (Sec. 4.1: y only) */
  int32_t oversample;   /* subspace vectors beyond N; <= 0: max(8, N / 2); N + oversample <= 512 */
  int32_t max_iters;    /* subspace iterations; <= 0: 500 */
  uint64_t seed;        /* start block */
} envar_eigen_params;

typedef struct {
  int32_t iters;      /* subspace iterations run */
  int32_t converged;  /* 1 when every kept residual met tol */
  int32_t block;      /* subspace size b = N + oversample (reduced to the cells with sigma > 0) */
  int32_t reserved;
  double max_resid;   /* max over k < N of |B v_k - mu_k v_k| / mu_1 at exit */
  double orth_err;    /* max |V V^T - I| of the kept directions */
} envar_eigen_info;

/* Workspace bytes of envar_eigen_ensemble (0 = invalid). */
size_t envar_eigen_bytes(const envar_problem* p, int32_t N, const envar_eigen_params* params);

/* E_dev [N][m] (device): row k the k-th member, nonzero only in params->component (the other
 * component's half of the row is 0); mu_dev [N] (device): the eigenvalues mu_k of B, decreasing.
 * The sign of each member, and the basis inside an eigenspace of a repeated eigenvalue, are not
 * fixed; E E^T is. Block subspace iteration on the matrix cores (B applied through the separable
 * kernel on the region's bounding rectangle); info (host) may be NULL. Synchronous. Errors: EINVAL
 * (N < 2, N above the number of cells with sigma > 0 or above 448, bad lengths), ENOMEM. An
 * iteration limit reached before tol is not an error: info->converged = 0. */
int envar_eigen_ensemble(const envar_problem* p, int32_t N, const envar_eigen_params* params, double* E_dev,
                         double* mu_dev, void* ws_dev, size_t ws_bytes, envar_eigen_info* info, void* stream);

/* Workspace bytes of envar_recon_error. */
size_t envar_recon_bytes(int32_t N, int64_t m);

/* Reconstruction error of App. A (eq. reconstruction_error): the share of |f|^2 outside the span of
 * the members, |f - V V^T f|^2 / |f|^2 with V the normalised rows of E_dev [N][m] (orthogonal rows,
 * as envar_eigen_ensemble returns; M_f = h^2 I cancels). f_dev [m], out_dev [1], all device.
 * Errors: EINVAL (N < 1, m < 1), ENOMEM. */
int envar_recon_error(const double* E_dev, int32_t N, int64_t m, const double* f_dev, void* ws_dev,
                      size_t ws_bytes, double* out_dev, void* stream);

/* Line search and iteration parameters of envar_iterate (Armijo, eq. update_BFGS). */
typedef struct {
  int32_t iters;          /* descent iterations */
  int32_t max_trials;     /* Armijo backtracking trials per search; <= 0: 8 */
  double c1;              /* sufficient-decrease constant; <= 0: 1e-4 */
  double shrink;          /* step reduction per trial; <= 0: 0.5 */
  double alpha0;          /* first trial step; <= 0: max|perturb| / max|g| */
  int32_t search_every;   /* 0: search at the first iteration only and reuse that step */
  int32_t reserved;
} envar_ls_params;

/* Per-iteration record of envar_iterate. */
typedef struct {
  double J0;       /* centre cost at the start of the iteration */
  double gnorm;    /* |g| */
  double alpha;    /* accepted step (0 = line search failed, loop stopped) */
  double J_trial;  /* cost at the accepted trial (NaN when the step was reused without a trial) */
} envar_iter_record;

/* Fixed-ensemble descent (Fig. envar_loop, Sec. 3.3.3): each iteration runs
 * the N+1 forwards of f and f + perturb_i, forms g, and moves f <- f - alpha g.
 * f_dev [m] (device, in/out), perturb_dev [n][m] (device, held fixed).
 * ws_dev must hold envar_iterate_bytes. records (host, `iters` entries) may be
 * NULL. When a line search finds no sufficient decrease the loop stops: that
 * record has alpha = 0 and f is left unchanged. Synchronous (the step
 * decisions read costs on the host). */
size_t envar_iterate_bytes(const envar_problem* p, int32_t n, int64_t m);
int envar_iterate(const envar_problem* p, const void* state_dev, double* f_dev,
                  const double* perturb_dev, int32_t n, int64_t m, int32_t horizon,
                  const envar_ls_params* ls, void* ws_dev, size_t ws_bytes,
                  envar_iter_record* records, void* stream);

/* ---------------------------------------------------------------- serving
 * Continuous batching of forward-solve requests from concurrent EnVar
 * optimisations (each request is one set of N+1 forward evaluations,
 * Sec. 3.3.1). A worker thread owns a HIP stream; admitted requests join the
 * running batch at the next step boundary and leave it at their own horizon,
 * so requests that arrive while others are on the GPU overlap with them in
 * the same merged launches. Device memory comes from one caller-provided
 * pool: a request is admitted (FIFO) when its footprint
 * (envar_request_bytes) fits next to the resident ones. */
typedef struct envar_server envar_server;

typedef struct {
  int32_t max_jobs;    /* ensembles per merged launch, 1..8 */
  int32_t precision;   /* ENVAR_FP64 | ENVAR_MIXED for every request */
  int32_t max_queue;   /* pending (not yet admitted) requests; <= 0: 1024 */
  int32_t flags;       /* ENVAR_FLAG_NO_GRAPHS to disable graph replay */
} envar_server_config;

typedef struct {
  envar_problem problem;   /* its grid, Re, region (precision is the server's) */
  const void* state_dev;   /* resident base state; must stay valid until the request completes */
  const double* controls;  /* HOST [n_rows][m]; copied at submission */
  int32_t n_rows;
  int32_t horizon;
  int64_t m;
} envar_request;

typedef struct {
  double submit_s;    /* host clock, seconds since envar_server_create */
  double start_s;     /* admitted into the batch */
  double done_s;      /* costs available on the host */
  double latency_s;   /* done_s - submit_s */
  double queue_s;     /* start_s - submit_s */
  double cell_steps;  /* fluid cells x horizon x n_rows */
  int32_t status;     /* ENVAR_OK, ENVAR_EDIVERGED (some J non-finite), ENVAR_EUNCONVERGED (see
                         `unconverged`), ENVAR_EDEVICE (a HIP call of the worker failed; the server
                         stops) or ENVAR_ECANCELLED */
  int32_t peak_jobs;  /* largest batch this request shared launches with */
  double max_div;     /* largest max|div_h u| after projection over the request's member-steps */
  double mean_cycles; /* refinement passes (MIXED) or V-cycles (FP64) per member-step */
  int32_t unconverged;/* member-steps whose pressure solve stopped at the pass cap before div_tol.
                         A member that meets div_tol within the cap at every step does the same
                         arithmetic in any batch (it skips the passes after its own convergence);
                         the cap follows the batch's recent needs with one pass of headroom and is
                         lifted to max_cycles after a cut, so a cut member's result can depend on
                         the requests it shared launches with */
  int32_t reserved;
} envar_request_stats;

/* Pool bytes one request occupies while resident. */
size_t envar_request_bytes(const envar_problem* p, int32_t n_rows);

/* Start a server over the caller's device pool (pool_dev, pool_bytes). */
int envar_server_create(const envar_server_config* cfg, void* pool_dev, size_t pool_bytes, envar_server** out);

/* Queue a request; returns at once with a ticket. Errors: EINVAL (shape),
 * ENOMEM (footprint larger than the whole pool), EBUSY (queue full). */
int envar_submit(envar_server* srv, const envar_request* req, uint64_t* ticket);

/* Wait up to timeout_s (< 0: forever) for a ticket; copies its n_rows costs
 * into J_host (may be NULL) and fills stats (may be NULL). Each ticket can be
 * waited on once. Returns the request's status (the costs and stats are copied
 * for EDIVERGED and EUNCONVERGED too). Errors: EINVAL (unknown ticket),
 * ETIMEOUT, ECANCELLED, EDEVICE. */
int envar_wait(envar_server* srv, uint64_t ticket, double timeout_s, double* J_host, envar_request_stats* stats);

/* Stop the worker (pending requests complete as ENVAR_ECANCELLED) and free
 * the server. The pool is not touched after return. */
int envar_server_destroy(envar_server* srv);

/* Thread-local message of the last failing call. */
const char* envar_last_error(void);

/* Plain device-to-device streaming copy of `bytes` (a multiple of 16,
 * 16-byte aligned buffers): the measured HBM ceiling beside the kernels'
 * roofline, and the reference workload that calibrates memory-traffic
 * counters. Not part of the method. */
int envar_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream);

/* Library version string. */
const char* envar_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ENVAR_H */
