// Internal structures shared by the host library and the solve kernels.
// Not part of the public C interface (see include/ffolio.h).
#pragma once
#include <stdint.h>

namespace ffo {

// Exchange buffer modes of the persistent kernel.
// Exchange modes: device-scope atomic adds, per-workgroup slots summed in a fixed order,
// or (a single-workgroup team) LDS only.
enum XMode : int32_t { XM_ATOMIC = 0, XM_GATHER = 1, XM_LOCAL = 2 };
// Atomic exchange over several copies of the slot: at most XG_MAX copies; barrier
// words XGSTRIDE apart, one cache line each: bar[0], the group counters
// bar[XGSTRIDE * (1 + g)] and the group release flags bar[XGSTRIDE * (1 + XG_MAX + g)].
constexpr int XG_MAX = 8;
constexpr int XGSTRIDE = 32;
constexpr int BAR_WORDS = XGSTRIDE * (1 + 2 * XG_MAX);

// Status codes written by the device (mirror ffo_status).
enum DevStatus : int32_t {
  DS_RUNNING = -1, DS_OK = 0, DS_NOT_CONVERGED = 4, DS_NUMERIC = 5, DS_INFEASIBLE = 6, DS_TIMEOUT = 7,
  DS_BARRIER = 100  // a bounded wait expired (device consistency failure)
};

// Problem in scaled form (every pointer is device memory).
//   K~ = diag(dr) [A; G^T] diag(dc)   rows 0..m-1 exposure, m..m+k-1 factor (G = F C)
//   trade rows (per asset) carry drC[t][i] * dc[i] * (+-1)
struct DevProblem {
  int32_t n, k, m, P, Tp, nr, multi, ldk;
  int32_t kscaled;      // 1: K holds diag(dr) K diag(dc); 0: K holds K diag(dc), rows scaled by dr on use
  const double* K;      // [nr][ldk] constraint rows (see kscaled)
  const float* Kf;      // the same rows rounded to float (FP32 form reading rows from device memory), or null
  const uint16_t* Kb;   // the same rows as bfloat16 bit patterns (PREC_BF16K), or null
  const double* dr;     // [nr]
  const double* dc;     // [n]
  const double* drC;    // [Tp][n]
  const double* alpha;  // [P][n]
  const double* arisk;  // [n]  2 g1 delta^2
  const double* cvec;   // [n]  risk centre (0 or w_T)
  const double* ca;     // [Tp][n] g2 s
  const double* cb;     // [Tp][n] g3 q
  const double* w0;     // [n]
  const double* wT;     // [n] (multi-period) or nullptr
  const double* L;      // [m]
  const double* U;      // [m]
  const double* bF;     // [k] G^T c (unscaled)
  const double* crisk;  // [1] g1 * sum_i delta_i^2 c_i^2
  double g1, d;
  double g2;            // spread weight (the adjoint differentiates through ca = g2 s)
};

// Per-(t,i) state arrays (device memory, each workgroup touches only its own assets).
struct DevState {
  double *xs, *x0s, *Txs;             // [P][n] iterate, Halpern anchor (= last restart point), T(z)
  double *ysC, *ys0C, *TysC;          // [Tp][n] trade duals, same roles
                                      // (xs, Txs, ysC, TysC hold float offsets from the anchor
                                      //  in the FP32 form)
  double *bb, *aa;                    // [P][n] prox inputs b and a of the current step
  double *vpow;                       // [P][n] power-iteration vector, later scratch
  double *xbuf;                       // exchange buffer (see kernel)
  double *blist;                      // [2][nwg][P][LIST_W] breakpoint lists (see kernel)
  unsigned long long* bar;            // barrier counter (zeroed by the host)
  double* info;                       // [INFO_LEN] result record written by workgroup 0
  int32_t* status;                    // [1]
  double* w_out;                      // [P][n] unscaled solution
  double* y_out;                      // optional dual output
  const double* w_init;               // optional [P][n] unscaled starting weights (else w0)
  const double* y_init;               // optional unscaled starting duals, y_out layout (else 0)
};

struct DevControl {
  double tol, time_limit_s, r_suff, r_nec, r_art, rho, eta_safety;
  int64_t max_iter;
  int32_t check_every, xmode, nwg, vmax, npow, verbose;
  int32_t lds_k;        // 1 if the constraint slice is staged in LDS
  int32_t lds_state;    // 1 if the per-asset state lives in LDS (else device memory)
  int32_t spec;         // 1: one speculative exchange per iteration; 0: two-phase
  int32_t nw;           // assets per workgroup (max)
  int32_t prec;         // PREC_FP64 or PREC_FP32: stored type of the iterates and LDS copies
  uint32_t spin_limit;
  double wall_hz;       // rate of the device wall clock
  int32_t lists;        // 1: publish breakpoint lists with the statistics (blist non-null)
  int32_t infeas;       // 1: test the exposure-dual displacement for an infeasibility certificate
  double omega0;        // starting primal weight (> 0)
  int32_t xgroups;      // atomic exchange: copies of the slot (workgroup w adds into copy w % xgroups)
};

// Breakpoint lists: per workgroup and period, a count and LIST_CAP entries
// (|b|, 1/a, global asset index, sign(b)/(a dc)).
constexpr int LIST_CAP = 8;
constexpr int LIST_W = 1 + 4 * LIST_CAP;

// PREC_BF16K: the FP32 form reading rows rounded to bfloat16 (batched kernel only).
enum Prec { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16K = 2 };

// Adjoint of the solve operator at a solution (device memory; see adjoint_body).
struct AdjState {
  const double* w_star;                 // [P][n] solution W*
  const double* y_star;                 // [P*m + P*k + Tp*n] its duals (unscaled, solve layout)
  const double* grad_w;                 // [P][n] dl/dW*
  double *xs, *xbar, *bb, *sx;          // [P][n] x*, xbar, prox input b, support signs / a
  double *lx, *lx0, *Tlx;               // [P][n] adjoint primal part, anchor, its image
  double *ysC, *lyC, *lyC0, *TlyC;      // [Tp][n] y_C*, adjoint trade part, anchor, image
  double *nC, *gsf;                     // [Tp][n] trade prox derivative factors
  double *tsg, *trho;                   // [Tp][n] sign(z) outside the spread dead zone (else 0), |prox(z)|
  double *grad_alpha;                   // [P][n]
  double *grad_s;                       // [Tp][n]
  double *grad_G;                       // [n][k] gradient w.r.t. G = F C
  double *xbuf;                         // exchange buffer
  unsigned long long* bar;
  double* info;                         // [INFO_LEN]
  int32_t* status;
};
int launch_adjoint(const DevProblem& p, const AdjState& a, const DevControl& c, double omega, void* stream,
                   size_t lds_bytes);
size_t adjoint_lds_bytes(const DevProblem& p, const DevControl& c);
int adjoint_vmax(const DevProblem& p);
// grad_F = grad_G C^T (n x k times k x k).
int launch_grad_F(int n, int k, const double* grad_G, const double* C, double* grad_F, void* stream);

enum InfoIdx {
  IX_ITERS = 0, IX_RESTARTS, IX_RELKKT, IX_RELPRI, IX_RELDUAL, IX_RELGAP, IX_FPR, IX_POBJ,
  IX_DOBJ, IX_OMEGA, IX_ETA, IX_NORMK, IX_SPEC_MISS, IX_EXCHANGES, IX_CHECKS, IX_T_WAIT,
  IX_T_ITER, IX_T_CHECK, IX_T_POWER, IX_MS_ROUNDS, IX_T_PHA, IX_T_PHB, IX_T_PHC, IX_T_PHD,
  IX_T_PRE, IX_T_READ, IX_T_B1, IX_T_B2, IX_T_B3, IX_T_B1S, IX_MISS_IN, IX_MISS_OUT, IX_T_GATHER, IX_GATHERS,
  INFO_LEN = 34
};

// Launch the persistent solve kernel (defined in solve_kernel.hip).
int launch_solve(const DevProblem& p, const DevState& s, const DevControl& c, void* stream,
                 size_t lds_bytes);
size_t solve_lds_bytes(const DevProblem& p, const DevControl& c);
// Batched launch: workgroup b of the grid runs rank wg_rank[b] of team wg_team[b]; team t
// solves problem dp[t] with state ds[t] and control dc[t] (device arrays).  All teams use
// the same instantiation (kl, sl, prec) and the same dynamic LDS size.
int launch_solve_batch(const DevProblem* dp, const DevState* ds, const DevControl* dc, const int* wg_team,
                       const int* wg_rank, int nblocks, int kl, int sl, int prec, void* stream, size_t lds_bytes);
// Resident workgroups per CU of the batched kernel at the given dynamic LDS size.
int solve_batch_occupancy(int kl, int sl, int prec, size_t lds_bytes);
int solve_vmax(const DevProblem& p);

// Setup kernels (setup_kernels.hip).
// Batched form: shared rows K diag(dc) of the n_max-asset universe (unscaled by rows),
// per-instance row scales drs [B][nr] over each prefix of nb[b] columns (nb on the
// device), shared arisk / cvec (zero) / drC (one), packed cost coefficients ca, cb [N].
int launch_setup_batch(int64_t B, const int64_t* nb_dev, int64_t n_max, int64_t k, int64_t m, int ldk,
                       const double* F, const double* Cfac, const double* A, const double* delta, int64_t N,
                       const double* s, const double* q, double g1, double g2, double g3, double* Kbuf,
                       double* drs, double* dc, double* drC, double* arisk, double* cvec, double* ca, double* cb,
                       void* stream);
// Kf[i] = (float)K[i] for i < count (FP32 form).
int launch_to_float(const double* K, float* Kf, int64_t count, void* stream);
// Kb[i] = bfloat16(K[i]) (round to nearest even, through float), then K[i] = Kb[i] exactly,
// so that every reader of K sees the rounded rows.
int launch_to_bf16(double* K, uint16_t* Kb, int64_t count, void* stream);
int launch_setup(int64_t n, int64_t k, int64_t m, int64_t P, int64_t Tp, int ldk,
                 const double* F, const double* Cfac, const double* A, const double* delta,
                 const double* s, const double* q, const double* wT, double g1, double g2,
                 double g3, double* Kbuf, double* dr, double* dc, double* drC, double* arisk,
                 double* cvec, double* ca, double* cb, double* bF, double* crisk_dev,
                 void* stream);

// ---------------------------------------------------------------------------------
// Lockstep batched form (lockstep.hip): every unconverged instance advances by one
// iteration per step; K~^T Y and K~ Xbar over the shared rows run as FP64 MFMA GEMMs.
// Instances sit in "slots" 0..nact-1 (sorted by decreasing n_b, compacted at checks);
// slots form groups of 16 (the MFMA tile height).
constexpr int LS_EW = 1024;   // assets per element tile of the lockstep form's elementwise passes

struct LsInst {
  double omega, eta, mu, r0, rprev, lam;   // primal weight, step, last multiplier, restart refs, power est.
  double kvr;                              // power iteration: sum of squares of the row products
  int64_t it, kk, restarts, checks;        // iterations, iterations since restart, restarts, checks
  int32_t done, status;                    // status: DevStatus (DS_RUNNING while active)
  int32_t mu_passes, mu_passes_sum;        // multiplier passes in the last step, and in all (diagnostic)
};

struct LsShared {
  int32_t B, nr, m, k, n_max, ldk, nrp;     // nrp: nr rounded up to 16
  int32_t ch;                               // assets per K~ xbar chunk (multiple of 16)
  int32_t gpt;                              // slot groups per K~^T y tile
  int32_t nchunk;                           // ceil(n_max / ch)
  int32_t lds_cap;                          // largest n_b whose (b, 1/a) pair fits in LDS
  int32_t nr4;                              // ceil(nr / 4)
  int64_t N;                                // total assets of the batch
  double g1, d, tol, rho, time_limit_s, wall_hz, r_suff, r_nec, r_art;
  int64_t max_iter;
  const double* KD;     // [nr][ldk]   K diag(dc) (rows unscaled), zero beyond n_max
  const double* KDT;    // [n_max][nrp] its transpose, zero-padded rows
  const double* drs;    // [B][nr]     per-instance row scales
  const double *dc, *arisk, *drC;           // [n_max]
  const double *alpha, *ca, *cb, *w0;       // packed [N]
  const double *L, *U;                      // [B][m]
  const int64_t* offs;                      // [B+1]
  const int32_t* nb;                        // [B]
  double *x, *x0, *yC, *yC0, *xbar, *R, *Tx, *TyC, *gb, *ga;   // packed [N]
  double *y, *y0, *Ty, *yh, *yhT;           // [B][nrp]
  double* part;                             // [nchunk][B][nrp] partial row sums (by slot)
  LsInst* inst;                             // [B]
  int32_t* act;                             // [B] slot -> instance
  int32_t* cnt;                             // [0] nact, [1] K~^T y tiles, [2] K~ x tiles, [3] groups,
                                            // [4] element tiles
  int32_t* tileA;                           // [2][...] (asset block, first group)
  int32_t* tileC;                           // [3][...] (chunk, first group, end group)
  int32_t* tileE;                           // [2][...] (slot, element chunk) of the elementwise passes
  int32_t* eoff;                            // [B] first element tile of each slot
  double* estat;                            // [tiles][8] per-tile sums of the first pass
  double* estat2;                           // [64-asset blocks][B][8] the same sums, fused form
  double* w_out;                            // packed [N]
  double* info;                             // [B][INFO_LEN]
  int32_t* status;                          // [B]
  unsigned long long* clock0;               // wall clock at the start
};

// Lockstep launchers (lockstep.hip); each returns a hipError_t value (0 = success).
// Phases of one iteration: kty (R = K~^T y over the rows), primal (prox inputs over
// element tiles, the multiplier per instance, then T(x), xbar and the trade duals over
// element tiles; check = 1: keep T(z) for the check), kx (partial K~ xbar), dual (row
// duals; check = 1 keeps T(y)).  A check then runs kty on T(y), kx on T(x),
// check (KKT, restarts, Halpern/restart apply) and compact.
int ls_launch_init(const LsShared& S, void* stream);
int ls_launch_kty(const LsShared& S, const double* yin, double* Rout, int grid, void* stream);
int ls_launch_primal(const LsShared& S, int check, int threads, int gridE, void* stream);
int ls_launch_kx(const LsShared& S, const double* xin, int grid, void* stream);
int ls_launch_dual(const LsShared& S, int mode, void* stream);
// Fused form of kty + primal + kx: prox inputs in the K~^T y epilogue, the multiplier,
// then T(x), xbar, trade duals and Halpern in the K~ xbar staging loop.
int ls_launch_step_fused(const LsShared& S, int check, int threads, int gA, int gC, void* stream);
int ls_launch_check(const LsShared& S, int threads, void* stream);
int ls_launch_compact(const LsShared& S, void* stream);
int ls_launch_power(const LsShared& S, int step, void* stream);   // step 0: rows, 1: assets
int ls_launch_transpose(const LsShared& S, double* KDT, void* stream);
// Instance b's current iterate, unscaled: w [n_b], y [nr + n_b] (rows, then trades).
int ls_launch_export(const LsShared& S, int b, int n_b, double* w, double* y, void* stream);
size_t ls_primal_lds(const LsShared& S);

// Risk-model construction (riskmodel.hip): workspace bytes and the launches of the
// partial sums, the per-asset solves and the factor covariance (1 <= p <= 8).
size_t rm_workspace_bytes(int64_t days, int64_t n, int64_t p);
int launch_risk_model(int days, int n, int p, const double* R, const double* Fr, const uint8_t* mask, int min_obs,
                      double* part, double* beta, double* Sf, double* D, int32_t* valid, void* stream);

}  // namespace ffo
