/*
 * ffolio.h - C interface of the MI355X (gfx950) first-order portfolio solver.
 *
 * The library solves the two models of "FlashFolio: A GPU-Accelerated Solver for
 * Portfolio Optimization" (Jiang, Lu, Peng, Yang; arXiv 2604.22625):
 *
 *   single-period (Section 2.1, eq. 1-3):
 *     max_w  GMV a^T w - l1 GMV^2 w^T S w - l2 GMV s^T|w - w0| - l3 GMV q^T|w - w0|^d
 *     s.t.   L <= A w <= U,   ||w||_1 <= 1
 *
 *   multi-period (Section 2.2, eq. 4-6), decisions w_1..w_{T-1}, w_0 and w_T given:
 *     max    sum_{t=1..T} GMV a_t^T w_t - l1 GMV^2 (w_t - w_T)^T S (w_t - w_T)
 *                         - l2 GMV s_t^T|w_t - w_{t-1}| - l3 GMV q_t^T|w_t - w_{t-1}|^d
 *     s.t.   L <= A w_t <= U,  ||w_t||_1 <= 1   for t = 1..T-1
 *
 * with the factor risk model S = F Omega F^T + diag(delta^2) (Section 3.2).  The
 * paper states the problems but not its iteration; this library runs a restarted,
 * reflected Halpern primal-dual hybrid gradient method on the splitting
 *   g(W) = sum_t [-a_t^T w_t + g1 sum_i delta_i^2 (w_ti - c_i)^2 + I{||w_t||_1 <= 1}],
 *   h    = I_[L,U](A w_t) + g1 ||F_c^T (w_t - c)||^2 + sum_t cost_t(u_t),
 * with g1 = l1 GMV, F_c = F chol(Omega), c = 0 or w_T, and trades u_t = w_t - w_{t-1}.
 * Every step of that iteration runs in HIP kernels on the device.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers to contiguous row-major float64 data,
 *    owned by the caller.  The library never frees or retains them beyond the call.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on it; the
 *    call returns after the solve has finished (it reads the final status back).
 *  - On FFO_EINVAL nothing has been launched and the outputs are untouched.
 *  - The library keeps a per-device workspace cache (grown on demand, freed by
 *    ffo_release or at process exit).  Calls on different host threads must use
 *    different streams; calls that overlap on one device share no state.
 *  - ffo_last_error() returns a thread-local message for the last non-OK status.
 */
#ifndef FFOLIO_H
#define FFOLIO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFO_OK = 0,
  FFO_EINVAL = 1,          /* bad size, pointer or scalar; nothing launched            */
  FFO_ENOMEM = 2,          /* device workspace allocation failed                      */
  FFO_EDEVICE = 3,         /* a HIP call or a device-side consistency check failed    */
  FFO_NOT_CONVERGED = 4,   /* max_iter reached; outputs hold the last iterate         */
  FFO_NUMERIC = 5,         /* NaN/Inf met in an FP64 check; outputs hold the last
                              finite restart point                                    */
  FFO_INFEASIBLE = 6,      /* the exposure bounds and the budget admit no portfolio:
                              y_out's exposure part holds a certificate (see ffo_solve) */
  FFO_TIMEOUT = 7          /* time_limit_s reached; outputs hold the last iterate     */
} ffo_status;

typedef enum {
  FFO_FP64 = 0,            /* every vector and matrix in float64                      */
  FFO_FP32 = 1,            /* per-asset iterates stored in float32 as offsets from their
                              float64 restart anchors; the scaled constraint slice and
                              per-asset data copies in float32; every reduction, the
                              budget multipliers, checks, restarts and the KKT residual
                              in float64 against the float64 inputs                  */
  FFO_FP32_BF16K = 2       /* batched solver only: as FP32, with the scaled constraint
                              rows rounded to bfloat16 (to nearest even, through float)
                              for the iteration and the checks alike, so the solve
                              converges on the rounded problem; its weights differ from
                              the FP64 solution by a few 1e-3 of max |w| (the caller
                              states that error).  ffo_solve and ffo_adjoint return
                              FFO_EINVAL                                              */
} ffo_precision;

typedef struct {
  double tol_rel_kkt;      /* stop when the relative KKT error <= tol (default 1e-6)  */
  int64_t max_iter;        /* iteration cap (default 1000000)                          */
  double time_limit_s;     /* wall-clock cap per solve (default 360, paper Sec. 4.1)  */
  int32_t check_every;     /* iterations between FP64 checks (default 64)             */
  int32_t precision;       /* ffo_precision (default FFO_FP64)                        */
  double restart_suff;     /* restart when residual <= suff * residual at restart (0.2) */
  double restart_nec;      /* ... or <= nec * that and no longer decreasing (0.8)     */
  double restart_art;      /* ... or the epoch is >= art * total iterations (0.36)    */
  double reflection;       /* rho of the reflected Halpern step, in [0, 1] (1.0)      */
  int32_t workgroups;      /* workgroups of the persistent solve kernel, 0 = auto     */
  int32_t verbose;         /* 1: one summary line per solve to stderr; 2: also per-check progress (device
                              printf) and, in the batched team form, one line per instance */
  int32_t deterministic;   /* 1: partial sums exchanged through per-workgroup slots and
                              added in a fixed order, so repeated solves are bitwise
                              identical (slower); 0 (default): device-scope atomic adds,
                              whose order varies from run to run                     */
  int32_t speculative;     /* 1: one exchange per iteration (the multiplier's affine
                              correction); 0: separate statistics and row exchanges;
                              -1 (default): 1 for single-period, 0 for multi-period   */
  int32_t breakpoint_lists;/* 1 (default): publish breakpoint lists with the statistics so
                              that most multiplier brackets close without extra exchanges;
                              0: multisection exchanges only (same solution)           */
  int32_t infeasibility_check; /* 1 (default): at every check, test the exposure-dual
                              displacement for an infeasibility certificate and stop with
                              FFO_INFEASIBLE when one is found; 0: never               */
  int32_t batched_form;    /* ffo_solve_batched only.  1: the team form (each instance runs
                              the solve kernel's loop on its own team of workgroups);
                              2: the lockstep form (every unconverged instance advances one
                              iteration per step, the products over the shared rows run as
                              float64 matrix-core GEMMs; FFO_FP64 only); 0 (default): the
                              lockstep form when it applies (FFO_FP64, m + k <= 160),
                              else the team form                                      */
  int32_t autotune;        /* lockstep form only.  1 (default): on the first solve of a shape
                              the library times a few tile sizes and kernel arrangements and
                              keeps the fastest for later solves of that shape; -1: fixed
                              defaults (the element passes as kernels of their own); 0:
                              fixed defaults with the element passes fused into the two
                              matrix-core kernels.  The choice changes
                              speed and the rounding order of some sums, not the method;
                              deterministic = 1 keeps the fixed defaults (-1 unless 0 is
                              given)                                                   */
} ffo_options;

typedef struct {
  int32_t status;          /* ffo_status of the solve                                  */
  int64_t iters;           /* PDHG iterations run                                      */
  int64_t restarts;        /* restarts taken                                           */
  double rel_kkt;          /* max(rel_pri, rel_dual, rel_gap) at the returned point    */
  double rel_pri;          /* ||A W - clip(A W, L, U)|| / (1 + ||clip(A W, L, U)||)    */
  double rel_dual;         /* distance of Y to the conjugate's domain / (1 + ||Y||)   */
  double rel_gap;          /* |Phi - Psi| / (|Phi| + |Psi|)                            */
  double fixed_point_res;  /* ||z - T(z)|| in the PDHG metric at the last check        */
  double primal_obj;       /* Phi(W) = -(paper objective)/GMV, without the multi-period
                              constant a_T^T w_T                                       */
  double dual_obj;         /* Psi(Y), the closed-form dual of the splitting            */
  double omega;            /* final primal weight                                      */
  double ms_setup;         /* setup time (scaling, factorisation), milliseconds        */
  double ms_iter;          /* iteration time, milliseconds                             */
} ffo_info;

/* Fill `opt` with the defaults listed above. */
void ffo_default_options(ffo_options* opt);

/*
 * Solve one single-period (T == 0) or multi-period (T >= 2) instance.
 *
 * Sizes: n >= 1 assets, k >= 0 factors, m >= 0 exposure rows; P = 1 if T == 0 else
 * T-1 decision periods; T' = 1 if T == 0 else T trades.
 *   alpha    [P][n]    expected returns a_t (paper eq. 1 / eq. 4)
 *   F        [n][k]    factor loadings (the paper's beta, Section 3.2)
 *   Omega    [k][k]    factor covariance, symmetric positive semidefinite
 *   delta    [n]       specific volatilities, S = F Omega F^T + diag(delta^2)
 *   s, q     [T'][n]   spread and impact coefficients, >= 0 (eq. 1 / eq. 4)
 *   d                  impact exponent, 1 < d <= 2 (Section 2.1)
 *   A        [m][n]    exposure matrix; L, U [m] its bounds (+-inf allowed, L <= U)
 *   w0       [n]       initial portfolio
 *   GMV > 0, lambda1, lambda2, lambda3 >= 0   (lambda1 > 0 and delta > 0 required)
 *   w_target [n]       terminal portfolio w_T; must be NULL iff T == 0
 *   opt                options (NULL = defaults)
 *   stream             hipStream_t
 * Outputs (caller-allocated device memory):
 *   w_out    [P][n]    the solution W
 *   y_out    optional, [P*m + P*k + T'*n]: the dual point (y_A [P][m], y_F [P][k],
 *            y_C [T'][n]) of the splitting in the header comment, so that the dual
 *            objective can be evaluated independently.  y_F is expressed in the basis
 *            F_c = F C with C the lower-triangular Cholesky factor of Omega (when Omega
 *            is only semidefinite: C = V diag(sqrt(max(lambda, 0))) from a Jacobi
 *            eigendecomposition Omega = V diag(lambda) V^T).  NULL to skip
 *   info     host pointer, filled on every status except FFO_EINVAL
 * Returns FFO_OK when the relative KKT error reached opt->tol_rel_kkt.
 * FFO_INFEASIBLE (with opt->infeasibility_check): every period has the same feasible set
 * {w : L <= A w <= U, ||w||_1 <= 1}; the solve found y in R^m with
 *   sum_j max(U_j y_j, L_j y_j) + max_i |(A^T y)_i| < 0,
 * which proves that set empty (for feasible w, y^T A w is at most the first term and at
 * least minus the second).  y_out's y_A part then holds the tested y for every period
 * (at least one of them is such a certificate); w_out holds the last iterate.
 */
ffo_status ffo_solve(int64_t n, int64_t k, int64_t m, int64_t T,
                     const double* alpha, const double* F, const double* Omega,
                     const double* delta, const double* s, const double* q, double d,
                     const double* A, const double* L, const double* U, const double* w0,
                     double GMV, double lambda1, double lambda2, double lambda3,
                     const double* w_target, const ffo_options* opt, void* stream,
                     double* w_out, double* y_out, ffo_info* info);

/*
 * Warm-started solve: as ffo_solve, but the iteration starts from the caller's point
 * instead of (w0 in every period, duals 0) (paper Section 4.1 starts every solve at w0;
 * a warm start serves rolling re-solves, date to date, of nearby problems).
 *   w_init     [P][n]  starting weights (device; NULL: w0 in every period)
 *   y_init     [P*m + P*k + T'*n]  starting duals in ffo_solve's y_out layout (device;
 *                      NULL: zero), e.g. the y_out of a previous solve with the same Omega
 *   omega_init starting primal weight (e.g. the previous ffo_info.omega; 0: 1)
 * The Halpern anchor is the starting point, so a start at a solution of the same problem
 * stops at the first check.  Non-finite w_init / y_init values give FFO_EINVAL.
 * Everything else (arguments, outputs, statuses) as in ffo_solve.
 */
ffo_status ffo_solve_warm(int64_t n, int64_t k, int64_t m, int64_t T,
                          const double* alpha, const double* F, const double* Omega,
                          const double* delta, const double* s, const double* q, double d,
                          const double* A, const double* L, const double* U, const double* w0,
                          double GMV, double lambda1, double lambda2, double lambda3,
                          const double* w_target, const double* w_init, const double* y_init,
                          double omega_init, const ffo_options* opt, void* stream,
                          double* w_out, double* y_out, ffo_info* info);

/*
 * Allocation-free solve, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, outputs and statuses as ffo_solve; it runs the same kernels, but its
 * workspace is one static device array of 32 MiB per GPU (held until the process ends)
 * instead of the library's cache, and it calls no hipMalloc, hipFree or other allocating
 * routine (the first call on a device takes the array's device address and creates three
 * timing events).  A problem whose workspace exceeds 32 MiB (about the constraint rows,
 * (m+k) x n doubles, plus a dozen vectors of P*n doubles; n = 5000 with m + k = 140 uses
 * 7 MB) returns FFO_EINVAL before any device work.  Every call on a GPU shares that
 * GPU's array and the library's static host staging area, so calls are serialised by a
 * lock; calls that overlap on one GPU from different processes are not supported.  The
 * result is read back through a synchronous copy into static (pageable) host memory.
 */
ffo_status ffo_solve_noalloc(int64_t n, int64_t k, int64_t m, int64_t T,
                             const double* alpha, const double* F, const double* Omega,
                             const double* delta, const double* s, const double* q, double d,
                             const double* A, const double* L, const double* U, const double* w0,
                             double GMV, double lambda1, double lambda2, double lambda3,
                             const double* w_target, const ffo_options* opt, void* stream,
                             double* w_out, double* y_out, ffo_info* info);

/*
 * Adjoint form: gradients of a loss l(W*) of the solution with respect to the expected
 * returns, the spread coefficients and the factor loadings (A, L, U, Omega, delta, q
 * held fixed).  The problem arguments are those of the ffo_solve call that produced
 *   w_star [P][n] and y_star [P*m + P*k + T'*n]   (its w_out and y_out, device)
 * and grad_w [P][n] = dl/dW* (device).  omega: the solve's final primal weight
 * (ffo_info.omega; 0 selects 1), a conditioning hint only: the adjoint iteration first
 * runs with weight 1/omega for at most 100000 iterations and, if that does not converge,
 * again from the start with weight omega (ffo_info.iters counts both).  Outputs (device,
 * caller-allocated): grad_alpha [P][n], grad_s [T'][n], grad_F [n][k] (may be NULL iff
 * k == 0).  Method: the solution is a fixed point z* = T(z*) of the iteration; with
 * J = dT/dz at z* (every nonsmooth piece frozen as T(z*) finds it: budget supports,
 * clipped exposure rows, the spread dead zones) the adjoint lambda = J^T lambda + g,
 * g = (dl/dz*, 0), is solved by the same restarted reflected Halpern iteration, and the
 * gradients are lambda^T dT/dtheta.  opt->tol_rel_kkt is the relative residual
 * ||J^T lambda + g - lambda|| / ||g|| to reach (default 1e-9 when opt is NULL);
 * opt->precision must be FFO_FP64.  Statuses as in ffo_solve (FFO_NOT_CONVERGED: the
 * gradients hold the last iterate's values).
 */
ffo_status ffo_adjoint(int64_t n, int64_t k, int64_t m, int64_t T,
                       const double* alpha, const double* F, const double* Omega,
                       const double* delta, const double* s, const double* q, double d,
                       const double* A, const double* L, const double* U, const double* w0,
                       double GMV, double lambda1, double lambda2, double lambda3,
                       const double* w_target, const double* w_star, const double* y_star,
                       const double* grad_w, double omega, const ffo_options* opt, void* stream,
                       double* grad_alpha, double* grad_s, double* grad_F, ffo_info* info);

/*
 * Batched form: B independent single-period instances (paper eq. 1-3) that share one
 * asset universe of n_max assets; instance b uses assets [0, n_b[b]).  Shared (device):
 *   F [n_max][k], Omega [k][k], delta [n_max], A [m][n_max]
 * Packed per instance (device), instance b at [offs[b], offs[b+1]):
 *   alpha, s, q, w0   [N], N = offs[B]          L, U   [B][m]
 * Host: n_b [B] (1 <= n_b <= n_max), offs [B+1] (offs[0] = 0, running sum of n_b),
 * infos [B] (one record per instance).  d, GMV, lambda1..3 as in ffo_solve (shared).
 * Output (device): w_out [N], packed like alpha.
 * Every instance runs the same restarted Halpern PDHG as ffo_solve, to its own relative
 * KKT tolerance, in one of two forms (opt->batched_form):
 *   lockstep: every unconverged instance advances one iteration per step; a step is a
 *     few kernels replayed from a captured graph: the products over the shared rows as
 *     float64 matrix-core GEMMs with ragged columns, then per-instance passes (budget
 *     multiplier, dual prox, Halpern step); converged instances are compacted out at
 *     every check; tile sizes come from the library's autotuner (opt->autotune).  The
 *     default for FFO_FP64 with m + k <= 160, B <= 65536, n_max <= 2^22.
 *   teams: each instance runs the solve kernel's loop on a team of workgroups sized to
 *     its asset count (spare resident workgroups go to the teams with the most assets per
 *     workgroup, down to 128 assets each; constraint slice and per-asset state in LDS when
 *     every team of the launch fits); all teams of a launch are resident at once and
 *     never wait for each
 *     other (batches larger than the resident grid run in several launches, largest
 *     instances first).  Every precision.
 * opt->precision: FFO_FP64, FFO_FP32 or FFO_FP32_BF16K (the last two: team form);
 * opt->workgroups is ignored; statuses as in ffo_solve.
 * Returns FFO_OK if every instance converged, else the most severe instance status
 * (FFO_EDEVICE > FFO_NUMERIC > FFO_TIMEOUT > FFO_NOT_CONVERGED); infos[b].status holds
 * each instance's own status.  FFO_EINVAL is returned before any device work.
 */
ffo_status ffo_solve_batched(int64_t B, const int64_t* n_b, int64_t n_max, int64_t k, int64_t m,
                             const double* F, const double* Omega, const double* delta, const double* A,
                             const int64_t* offs, const double* alpha, const double* s, const double* q,
                             const double* w0, const double* L, const double* U, double d, double GMV,
                             double lambda1, double lambda2, double lambda3, const ffo_options* opt,
                             void* stream, double* w_out, ffo_info* infos);

/* Many unrelated markets in one launch (paper Section 2.1, eq. 1-3, and Section 2.2,
 * eq. 4-6, per instance): instance b has its own n[b] assets, loadings, factor covariance,
 * specific vols, costs, exposure rows, bounds and (T > 0) terminal target, with k factors,
 * m exposure rows and T shared by all.  Each instance gets ffo_solve's setup (its own
 * scaled rows and scales), then one team of workgroups runs the solve kernel's loop for
 * it, as in ffo_solve_batched's team form: teams sized to n[b] (spare resident workgroups
 * go to the teams with the most assets per workgroup, down to 128 assets each; at most
 * 2048 assets per workgroup, fewer when T periods of staging would not fit in LDS),
 * constraint slice and state in LDS when every team of a launch fits, several launches
 * when the minimal teams exceed the resident grid.
 * Host: n [B] (1 <= n[b] <= 2^24), infos [B], and the arrays of B device pointers, with
 * P = T - 1 decisions and T trades (P = T = 1 when T = 0):
 *   alpha: [P][n[b]];  s, q: [T][n[b]];  delta, w0: [n[b]];  F: [n[b]][k];  Omega: [k][k];
 *   A: [m][n[b]];  L, U: [m];  w_target: [n[b]] (w_target itself NULL iff T == 0);
 *   w_out: [P][n[b]]   (F, Omega may be NULL when k = 0; A, L, U when m = 0).
 * d, GMV, lambda1..3 as in ffo_solve, shared.  1 <= B <= 2^16; T = 0 or 2 <= T <= 4096.
 * opt->precision: FFO_FP64 or FFO_FP32; opt->speculative as in ffo_solve (by default on
 * for T = 0, off otherwise); opt->workgroups, opt->batched_form and opt->breakpoint_lists
 * are ignored; statuses as in ffo_solve.  Every instance stops at its own relative KKT
 * tolerance; infos[b] holds its record.
 * Returns FFO_OK if every instance converged, else the most severe instance status
 * (FFO_EDEVICE > FFO_NUMERIC > FFO_INFEASIBLE > FFO_TIMEOUT > FFO_NOT_CONVERGED).
 * FFO_EINVAL is returned before any device work for bad sizes, null pointers or options,
 * or a working set beyond LDS, and after the one value check for non-finite values,
 * L > U or an Omega that is not positive semidefinite.
 */
ffo_status ffo_solve_many(int64_t B, const int64_t* n, int64_t k, int64_t m, int64_t T, const double* const* alpha,
                          const double* const* F, const double* const* Omega, const double* const* delta,
                          const double* const* s, const double* const* q, const double* const* A,
                          const double* const* L, const double* const* U, const double* const* w0,
                          const double* const* w_target, double d, double GMV, double lambda1, double lambda2,
                          double lambda3, const ffo_options* opt, void* stream, double* const* w_out,
                          ffo_info* infos);

/*
 * Risk-model construction (paper Section 3.2): the inputs S = beta Sigma_f beta^T + D of
 * the solvers from a window of daily returns.
 *   R      [days][n]  asset returns (device)
 *   Fr     [days][p]  factor returns (device), 1 <= p <= 8 (the paper: p = 6)
 *   mask   [days][n]  optional (device, NULL = all observed): nonzero where R holds an
 *                     observation; unobserved entries are never read (they may be NaN)
 *   min_obs           assets with fewer observed days get no loadings (the paper: at
 *                     least two months of history)
 * Outputs (device, caller-allocated):
 *   beta   [n][p]     least-squares loadings of r_i ~ Fr beta_i over the asset's observed
 *                     days (no intercept), 0 for assets without loadings
 *   Sigma_f [p][p]    (Fr - mean)^T (Fr - mean) / (days - 1) over the whole window
 *   D      [n]        sample variance (centred, 1/(count - 1)) of the residuals
 *                     r_ki - beta_i^T f_k over the observed days (of the returns themselves
 *                     for assets without loadings; 0 with fewer than two observations)
 *   valid  [n]        1 where loadings were estimated (enough observations and a
 *                     nonsingular Gram matrix), else 0
 * These feed ffo_solve as F = beta, Omega = Sigma_f, delta = sqrt(D).  Observed entries
 * must be finite.  Statuses: FFO_EINVAL (sizes, pointers), FFO_ENOMEM, FFO_EDEVICE.
 */
ffo_status ffo_risk_model(int64_t days, int64_t n, int64_t p, const double* R, const double* Fr,
                          const uint8_t* mask, int64_t min_obs, void* stream, double* beta,
                          double* Sigma_f, double* D, int32_t* valid);

/* Thread-local description of the last non-OK status ("" if none). */
const char* ffo_last_error(void);

/* Free the cached device workspaces of every device.  Safe to call at any time when
 * no solve is running. */
void ffo_release(void);

/* Library version string. */
const char* ffo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FFOLIO_H */
