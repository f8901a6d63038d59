// Host side of the C interface declared in include/ffolio.h.
//
// ffo_solve: validate sizes/pointers/scalars on the host (FFO_EINVAL before any HIP
// call), factor Omega = C C^T on the host (Cholesky, or a Jacobi eigendecomposition
// when Omega is only semidefinite), assemble and scale the constraint rows with the
// setup kernels, run the persistent solve kernel, and read back status and info.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ffolio.h"
#include "internal.h"

namespace {

thread_local std::string g_err;

ffo_status fail(ffo_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(FFO_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Workspace {
  void* base = nullptr;
  size_t bytes = 0;
  void* host = nullptr;      // pinned host staging
  size_t host_bytes = 0;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};

std::mutex g_mu;
std::map<std::tuple<int, void*, int>, Workspace> g_ws;

// Grow-only device workspace for (device, stream, kind); kind 0 = ffo_solve, 1 = batched.
ffo_status get_workspace(int dev, void* stream, size_t bytes, size_t host_bytes, Workspace** out, int kind = 0) {
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace& w = g_ws[std::make_tuple(dev, stream, kind)];
  if (w.bytes < bytes) {
    if (w.base) hipFree(w.base);
    w.base = nullptr;
    w.bytes = 0;
    if (hipMalloc(&w.base, bytes) != hipSuccess) return fail(FFO_ENOMEM, "hipMalloc of the solver workspace failed");
    w.bytes = bytes;
  }
  if (w.host_bytes < host_bytes) {
    if (w.host) hipHostFree(w.host);
    w.host = nullptr;
    w.host_bytes = 0;
    if (hipHostMalloc(&w.host, host_bytes, hipHostMallocDefault) != hipSuccess)
      return fail(FFO_ENOMEM, "hipHostMalloc of the staging buffer failed");
    w.host_bytes = host_bytes;
  }
  for (auto& e : w.ev)
    if (!e && hipEventCreate(&e) != hipSuccess) return fail(FFO_EDEVICE, "hipEventCreate failed");
  *out = &w;
  return FFO_OK;
}

// C with C C^T = Om (k x k, row-major).  Cholesky first; if a pivot is not positive,
// cyclic Jacobi eigendecomposition and C = V diag(sqrt(max(lambda, 0))).  Returns false
// if Om is not symmetric or has an eigenvalue below -1e-10 * max|lambda|.  work: host
// scratch of 2 k^2 doubles.
bool factor_omega(int k, const double* Om, double* C, double* work) {
  double amax = 0.0;
  for (int i = 0; i < k * k; ++i) {
    if (!std::isfinite(Om[i])) return false;
    amax = std::max(amax, std::fabs(Om[i]));
  }
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < i; ++j)
      if (std::fabs(Om[i * k + j] - Om[j * k + i]) > 1e-12 * std::max(1.0, amax)) return false;
  double* Lc = work;   // [k*k]
  std::fill(Lc, Lc + (size_t)k * k, 0.0);
  bool ok = true;
  for (int j = 0; j < k && ok; ++j) {
    double d = Om[j * k + j];
    for (int p = 0; p < j; ++p) d -= Lc[j * k + p] * Lc[j * k + p];
    if (!(d > 1e-14 * std::max(amax, 1e-300))) { ok = false; break; }
    const double r = std::sqrt(d);
    Lc[j * k + j] = r;
    for (int i = j + 1; i < k; ++i) {
      double v = Om[i * k + j];
      for (int p = 0; p < j; ++p) v -= Lc[i * k + p] * Lc[j * k + p];
      Lc[i * k + j] = v / r;
    }
  }
  if (ok) {
    std::copy(Lc, Lc + (size_t)k * k, C);
    return true;
  }
  // Jacobi eigendecomposition
  double* a = work;                   // [k*k]
  double* v = work + (size_t)k * k;   // [k*k]
  std::copy(Om, Om + (size_t)k * k, a);
  std::fill(v, v + (size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) v[i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j) off += a[i * k + j] * a[i * k + j];
    if (off <= 1e-30 * std::max(amax * amax, 1e-300)) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = a[p * k + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (a[q * k + q] - a[p * k + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < k; ++r) {
          const double arp = a[r * k + p], arq = a[r * k + q];
          a[r * k + p] = c * arp - s * arq;
          a[r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = a[p * k + r], aqr = a[q * k + r];
          a[p * k + r] = c * apr - s * aqr;
          a[q * k + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = v[r * k + p], vrq = v[r * k + q];
          v[r * k + p] = c * vrp - s * vrq;
          v[r * k + q] = s * vrp + c * vrq;
        }
      }
  }
  double lmax = 0.0;
  for (int i = 0; i < k; ++i) lmax = std::max(lmax, std::fabs(a[i * k + i]));
  for (int i = 0; i < k; ++i)
    if (a[i * k + i] < -1e-10 * std::max(lmax, 1e-300)) return false;
  for (int r = 0; r < k; ++r)
    for (int j = 0; j < k; ++j) C[r * k + j] = v[r * k + j] * std::sqrt(std::max(a[j * k + j], 0.0));
  return true;
}

// Elementwise device checks of the array values (finite data, delta > 0, s, q >= 0,
// L <= U); flag[0] receives a bit mask of the failures.
__global__ void k_validate(int64_t n, int64_t Pn, int64_t Tpn, int64_t nk, int64_t m, const double* alpha,
                           const double* F, const double* delta, const double* s, const double* q,
                           const double* L, const double* U, const double* w0, const double* wT,
                           int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < Pn; e += stride)
    if (!isfinite(alpha[e])) bad |= 1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nk; e += stride)
    if (!isfinite(F[e])) bad |= 2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += stride) {
    if (!(delta[e] > 0.0) || !isfinite(delta[e])) bad |= 4;
    if (w0 && !isfinite(w0[e])) bad |= 8;
    if (wT && !isfinite(wT[e])) bad |= 8;
  }
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < Tpn; e += stride)
    if (!(s[e] >= 0.0) || !(q[e] >= 0.0) || !isfinite(s[e]) || !isfinite(q[e])) bad |= 16;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += stride)
    if (!(L[e] <= U[e]) || isnan(L[e]) || isnan(U[e]) || L[e] == INFINITY || U[e] == -INFINITY) bad |= 32;
  if (bad) atomicOr(flag, bad);
}

// Packed per-instance vectors of the batched form: alpha, w0 finite; s, q >= 0 finite
// (N entries); L <= U (Bm entries).
__global__ void k_validate_packed(int64_t N, int64_t Bm, const double* alpha, const double* s, const double* q,
                                  const double* w0, const double* L, const double* U, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N; e += stride) {
    if (!isfinite(alpha[e])) bad |= 1;
    if (!isfinite(w0[e])) bad |= 8;
    if (!(s[e] >= 0.0) || !(q[e] >= 0.0) || !isfinite(s[e]) || !isfinite(q[e])) bad |= 16;
  }
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < Bm; e += stride)
    if (!(L[e] <= U[e]) || isnan(L[e]) || isnan(U[e]) || L[e] == INFINITY || U[e] == -INFINITY) bad |= 32;
  if (bad) atomicOr(flag, bad);
}

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

// Host-only checks of the problem arguments shared by ffo_solve and ffo_adjoint.
ffo_status check_problem_args(int64_t n, int64_t k, int64_t m, int64_t T, const double* alpha, const double* F,
                              const double* Omega, const double* delta, const double* s, const double* q, double d,
                              const double* A, const double* L, const double* U, const double* w0, double GMV,
                              double lambda1, double lambda2, double lambda3, const double* w_target) {
  if (n < 1) return fail(FFO_EINVAL, "n must be >= 1");
  if (k < 0 || k > 128) return fail(FFO_EINVAL, "k must lie in [0, 128]");
  if (m < 0 || m > 4096) return fail(FFO_EINVAL, "m must lie in [0, 4096]");
  if (!(T == 0 || T >= 2)) return fail(FFO_EINVAL, "T must be 0 (single-period) or >= 2");
  if (T > 4096) return fail(FFO_EINVAL, "T must be <= 4096");
  const int64_t Tp = T == 0 ? 1 : T;
  if (n * Tp > (int64_t)1 << 30) return fail(FFO_EINVAL, "n * T too large");
  if (!alpha || !delta || !s || !q || !w0) return fail(FFO_EINVAL, "null array pointer");
  if (k > 0 && (!F || !Omega)) return fail(FFO_EINVAL, "F and Omega must be non-null when k > 0");
  if (m > 0 && (!A || !L || !U)) return fail(FFO_EINVAL, "A, L and U must be non-null when m > 0");
  if ((T == 0) != (w_target == nullptr)) return fail(FFO_EINVAL, "w_target must be NULL iff T == 0");
  if (!(d > 1.0 && d <= 2.0)) return fail(FFO_EINVAL, "d must lie in (1, 2]");
  if (!(GMV > 0.0) || !std::isfinite(GMV)) return fail(FFO_EINVAL, "GMV must be positive and finite");
  if (!(lambda1 > 0.0) || !std::isfinite(lambda1)) return fail(FFO_EINVAL, "lambda1 must be positive and finite");
  if (!(lambda2 >= 0.0) || !(lambda3 >= 0.0) || !std::isfinite(lambda2) || !std::isfinite(lambda3))
    return fail(FFO_EINVAL, "lambda2 and lambda3 must be nonnegative and finite");
  if (!std::isfinite(lambda1 * GMV)) return fail(FFO_EINVAL, "lambda1 * GMV must be finite");
  return FFO_OK;
}

ffo_status check_options(const ffo_options& opt) {
  if (!(opt.tol_rel_kkt > 0.0)) return fail(FFO_EINVAL, "tol_rel_kkt must be positive");
  if (opt.max_iter < 1) return fail(FFO_EINVAL, "max_iter must be >= 1");
  if (opt.check_every < 1) return fail(FFO_EINVAL, "check_every must be >= 1");
  if (!(opt.time_limit_s > 0.0)) return fail(FFO_EINVAL, "time_limit_s must be positive");
  if (!(opt.reflection >= 0.0 && opt.reflection <= 1.0)) return fail(FFO_EINVAL, "reflection must lie in [0, 1]");
  if (opt.workgroups < 0 || opt.workgroups > 4096) return fail(FFO_EINVAL, "workgroups must lie in [0, 4096]");
  if (opt.deterministic != 0 && opt.deterministic != 1) return fail(FFO_EINVAL, "deterministic must be 0 or 1");
  if (opt.speculative < -1 || opt.speculative > 1) return fail(FFO_EINVAL, "speculative must be -1, 0 or 1");
  if (opt.breakpoint_lists != 0 && opt.breakpoint_lists != 1) return fail(FFO_EINVAL, "breakpoint_lists must be 0 or 1");
  if (opt.infeasibility_check != 0 && opt.infeasibility_check != 1)
    return fail(FFO_EINVAL, "infeasibility_check must be 0 or 1");
  return FFO_OK;
}

std::string bad_values(int flag) {
  std::string why;
  if (flag & 1) why += " alpha not finite;";
  if (flag & 2) why += " F not finite;";
  if (flag & 4) why += " delta must be positive and finite;";
  if (flag & 8) why += " w0/w_target not finite;";
  if (flag & 16) why += " s and q must be nonnegative and finite;";
  if (flag & 32) why += " need L <= U (no NaN, L < +inf, U > -inf);";
  if (flag & 64) why += " warm-start data not finite;";
  return "invalid input values:" + why;
}

void fill_info(ffo_info* info, ffo_status st, const double* hinfo, double ms_setup, double ms_iter) {
  info->status = st;
  info->iters = (int64_t)hinfo[ffo::IX_ITERS];
  info->restarts = (int64_t)hinfo[ffo::IX_RESTARTS];
  info->rel_kkt = hinfo[ffo::IX_RELKKT];
  info->rel_pri = hinfo[ffo::IX_RELPRI];
  info->rel_dual = hinfo[ffo::IX_RELDUAL];
  info->rel_gap = hinfo[ffo::IX_RELGAP];
  info->fixed_point_res = hinfo[ffo::IX_FPR];
  info->primal_obj = hinfo[ffo::IX_POBJ];
  info->dual_obj = hinfo[ffo::IX_DOBJ];
  info->omega = hinfo[ffo::IX_OMEGA];
  info->ms_setup = ms_setup;
  info->ms_iter = ms_iter;
}

ffo_status status_of(int32_t hstat) {
  switch (hstat) {
    case ffo::DS_OK: return FFO_OK;
    case ffo::DS_NOT_CONVERGED: return FFO_NOT_CONVERGED;
    case ffo::DS_NUMERIC: return FFO_NUMERIC;
    case ffo::DS_TIMEOUT: return FFO_TIMEOUT;
    case ffo::DS_INFEASIBLE: return FFO_INFEASIBLE;
    default: return FFO_EDEVICE;
  }
}

// Fill `words` 32-bit words with `value` (used instead of hipMemsetAsync so that a caller
// may record the solve's stream work into a graph).
__global__ void k_fill(uint32_t* p, int64_t words, uint32_t value) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < words; e += stride) p[e] = value;
}

// Copies of the atomic exchange slot for a grid of nwg workgroups (see the kernel's
// exchange): one per group of workgroups, so that fewer read-modify-writes meet on each
// word.  Below 32 workgroups the extra reads of the copies cost more than they save.
int xgroups_for(int nwg) { return nwg >= 32 ? ffo::XG_MAX : 1; }

// Default workgroup count of the plain and adjoint kernels: every phase of an iteration
// is a latency chain, and with the grouped exchange its cost grows slowly with the grid,
// so from n = 2000 on each workgroup takes 16 assets (up to one per compute unit);
// smaller problems keep 64 per workgroup.
int default_workgroups(int64_t n, int cus) {
  const int64_t per = n >= 2000 ? 16 : 64;
  return (int)std::max<int64_t>(1, std::min<int64_t>(cus, (n + per - 1) / per));
}

hipError_t fill(void* p, size_t bytes, uint32_t value, hipStream_t hs) {
  const int64_t words = (int64_t)(bytes / 4);
  if (words == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (words + 255) / 256);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, hs, (uint32_t*)p, words, value);
  return hipGetLastError();
}

// Finite-value check of an optional caller array (warm-start data); sets `bit` in flag.
__global__ void k_check_finite(const double* x, int64_t cnt, int bit, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt; e += stride)
    if (!isfinite(x[e])) bad = bit;
  if (bad) atomicOr(flag, bad);
}

// Device and host memory for one ffo_solve call that the caller (not the workspace
// cache) provides; events may be null (no timing).
struct Fixed {
  char* dev;
  size_t dev_bytes;
  char* host;
  size_t host_bytes;
  hipEvent_t* ev;   // [3] or null
};

// The single-instance solve behind ffo_solve and ffo_solve_warm.  w_init / y_init
// (device, optional): starting weights [P][n] and duals (y_out layout); omega0 > 0: the
// starting primal weight.  fx: caller-provided memory, or null for the workspace cache.
ffo_status solve_impl(int64_t n, int64_t k, int64_t m, int64_t T, const double* alpha, const double* F,
                      const double* Omega, const double* delta, const double* s, const double* q, double d,
                      const double* A, const double* L, const double* U, const double* w0, double GMV,
                      double lambda1, double lambda2, double lambda3, const double* w_target,
                      const double* w_init, const double* y_init, double omega0, const ffo_options* opt_in,
                      void* stream, double* w_out, double* y_out, ffo_info* info, const Fixed* fx) {
  g_err.clear();
  ffo_options opt;
  ffo_default_options(&opt);
  if (opt_in) opt = *opt_in;
  // ---- host-only validation (no device work before this point) ----
  if (ffo_status st = check_problem_args(n, k, m, T, alpha, F, Omega, delta, s, q, d, A, L, U, w0, GMV, lambda1,
                                         lambda2, lambda3, w_target))
    return st;
  if (!w_out) return fail(FFO_EINVAL, "null array pointer");
  if (ffo_status st = check_options(opt)) return st;
  if (opt.precision != FFO_FP64 && opt.precision != FFO_FP32)
    return fail(FFO_EINVAL, "ffo_solve takes FFO_FP64 or FFO_FP32");
  const int64_t P = T == 0 ? 1 : T - 1, Tp = T == 0 ? 1 : T;

  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  int wall_khz = 0;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
    wall_khz = 100000;

  // ---- sizes and launch shape ----
  const int nr = (int)(m + k);
  const int ldk = (int)((n + 63) / 64 * 64);
  ffo::DevProblem p{};
  p.n = (int)n; p.k = (int)k; p.m = (int)m; p.P = (int)P; p.Tp = (int)Tp; p.nr = nr;
  p.multi = T > 0 ? 1 : 0; p.ldk = ldk; p.kscaled = 1;
  const int cus = std::max(1, prop.multiProcessorCount);
  int nwg = opt.workgroups > 0 ? opt.workgroups : default_workgroups(n, cus);
  nwg = std::max(1, std::min<int>(nwg, (int)n));
  nwg = std::min(nwg, cus);  // one workgroup per compute unit keeps the cooperative grid resident
  int nw = (int)((n + nwg - 1) / nwg);
  nwg = (int)((n + nw - 1) / nw);
  ffo::DevControl c{};
  c.tol = opt.tol_rel_kkt; c.time_limit_s = opt.time_limit_s;
  c.r_suff = opt.restart_suff; c.r_nec = opt.restart_nec; c.r_art = opt.restart_art;
  c.rho = opt.reflection; c.eta_safety = 0.95; c.max_iter = opt.max_iter;
  c.check_every = opt.check_every; c.nwg = nwg; c.npow = 40;
  c.verbose = opt.verbose; c.nw = nw; c.spin_limit = 1u << 26; c.wall_hz = (double)wall_khz * 1e3;
  c.prec = opt.precision == FFO_FP32 ? ffo::PREC_FP32 : ffo::PREC_FP64;
  c.xmode = opt.deterministic ? ffo::XM_GATHER : ffo::XM_ATOMIC;
  c.xgroups = xgroups_for(nwg);
  c.vmax = ffo::solve_vmax(p);
  c.spec = opt.speculative < 0 ? (P == 1 ? 1 : 0) : (opt.speculative ? 1 : 0);
  c.lists = opt.breakpoint_lists ? 1 : 0;
  c.infeas = opt.infeasibility_check ? 1 : 0;
  c.omega0 = omega0;
  // LDS placement: constraint slice and per-asset state in LDS when they fit, the slice
  // first (it is read twice per iteration, by K~^T y and K~ xbar; T=10, n=2000: 69 -> 50 us
  // per iteration against state first).  With the automatic workgroup count, more
  // workgroups (smaller slices) are taken while that lets the constraint slice move into
  // LDS.
  const size_t lds_cap = (size_t)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
  size_t lds = 0;
  if (opt.workgroups == 0) {
    for (int g = nwg; g <= std::min<int64_t>(cus, n); g = std::max(g + 1, g * 5 / 4)) {
      const int w = (int)((n + g - 1) / g);
      ffo::DevControl t = c;
      t.nw = w; t.nwg = (int)((n + w - 1) / w); t.lds_k = 1; t.lds_state = 0;
      t.prec = ffo::PREC_FP64;   // the same grid for both forms: the FP32 slice is smaller, not the work
      if (ffo::solve_lds_bytes(p, t) <= lds_cap) { nw = w; nwg = t.nwg; break; }
    }
    c.nw = nw;
    c.nwg = nwg;
  }
  {
    const int order[4][2] = {{1, 1}, {1, 0}, {0, 1}, {0, 0}};
    bool placed = false;
    for (const auto& o : order) {
      c.lds_k = o[0];
      c.lds_state = o[1];
      lds = ffo::solve_lds_bytes(p, c);
      if (lds <= lds_cap) { placed = true; break; }
    }
    if (!placed) return fail(FFO_EINVAL, "problem too large for the per-workgroup working set (reduce m + k or T)");
  }
  // ---- workspace layout ----
  const size_t Pn = (size_t)P * n, Tpn = (size_t)Tp * n;
  size_t off = 0;
  auto carve = [&](size_t cnt, size_t elt) { const size_t o = off; off = align_up(off + cnt * elt); return o; };
  const size_t oK = carve((size_t)std::max(nr, 1) * ldk, 8), odr = carve(std::max(nr, 1), 8), odc = carve(n, 8);
  const bool f32rows = c.prec == ffo::PREC_FP32 && !c.lds_k;   // FP32 form reading rows from device memory
  const size_t oKf = carve(f32rows ? (size_t)std::max(nr, 1) * ldk : 1, 4);
  const size_t odrC = carve(Tpn, 8), oar = carve(n, 8), ocv = carve(n, 8), oca = carve(Tpn, 8), ocb = carve(Tpn, 8);
  const size_t obF = carve(std::max<int64_t>(k, 1), 8), ocr = carve(1, 8), oC = carve(std::max<int64_t>(k * k, 1), 8);
  size_t ost[6];
  for (auto& o : ost) o = carve(Pn, 8);
  size_t osc[3];
  for (auto& o : osc) o = carve(Tpn, 8);
  const size_t nxbuf = (size_t)std::max(2 * nwg, 3 * ffo::XG_MAX) * c.vmax;
  const size_t oxb = carve(nxbuf, 8), obar = carve(ffo::BAR_WORDS, 8);
  const size_t oblist = carve(c.lists ? (size_t)2 * nwg * P * ffo::LIST_W : 1, 8);
  const size_t oinfo = carve(ffo::INFO_LEN, 8), ostat = carve(1, 4), oflag = carve(1, 4);
  const size_t total = off;
  // host staging: Omega, its factor, the factorisation's work space, info, two flags
  const size_t kk = (size_t)std::max<int64_t>(k * k, 1);
  size_t hoff = 0;
  auto hcarve = [&](size_t bytes) { const size_t o = hoff; hoff = align_up(hoff + bytes); return o; };
  const size_t hOm_o = hcarve(kk * 8), hC_o = hcarve(kk * 8), hW_o = hcarve(2 * kk * 8);
  const size_t hI_o = hcarve(ffo::INFO_LEN * 8), hF_o = hcarve(8);
  const size_t host_bytes = hoff;

  char* B = nullptr;
  char* H = nullptr;
  hipEvent_t* ev = nullptr;
  if (fx) {
    if (total > fx->dev_bytes)
      return fail(FFO_EINVAL, "problem needs " + std::to_string(total) + " bytes of device scratch, more than the " +
                                  std::to_string(fx->dev_bytes) + " available");
    if (host_bytes > fx->host_bytes) return fail(FFO_EINVAL, "k too large for the host staging area");
    B = fx->dev;
    H = fx->host;
    ev = fx->ev;
  } else {
    Workspace* ws = nullptr;
    if (ffo_status st = get_workspace(dev, stream, total, host_bytes, &ws)) return st;
    B = (char*)ws->base;
    H = (char*)ws->host;
    ev = ws->ev;
  }
  auto D = [&](size_t o) { return (double*)(B + o); };
  hipStream_t hs = (hipStream_t)stream;
  double* hOm = (double*)(H + hOm_o);
  double* hC = (double*)(H + hC_o);
  double* hW = (double*)(H + hW_o);
  double* hinfo = (double*)(H + hI_o);
  int* hflag = (int*)(H + hF_o);

  if (ev) HIPCHK(hipEventRecord(ev[0], hs));
  // ---- value validation on the device + Omega to the host (one synchronisation) ----
  HIPCHK(fill(B + oflag, 4, 0u, hs));
  hipLaunchKernelGGL(k_validate, dim3(64), dim3(256), 0, hs, n, (int64_t)Pn, (int64_t)Tpn, n * k, m, alpha, F,
                     delta, s, q, L, U, w0, w_target, (int*)(B + oflag));
  if (w_init)
    hipLaunchKernelGGL(k_check_finite, dim3(64), dim3(256), 0, hs, w_init, (int64_t)Pn, 64, (int*)(B + oflag));
  if (y_init)
    hipLaunchKernelGGL(k_check_finite, dim3(64), dim3(256), 0, hs, y_init, (int64_t)(P * m + P * k) + (int64_t)Tpn,
                       64, (int*)(B + oflag));
  HIPCHK(hipGetLastError());
  if (k > 0) HIPCHK(hipMemcpyAsync(hOm, Omega, (size_t)k * k * 8, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipMemcpyAsync(hflag, B + oflag, 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  if (*hflag) return fail(FFO_EINVAL, bad_values(*hflag));
  if (k > 0 && !factor_omega((int)k, hOm, hC, hW)) return fail(FFO_EINVAL, "Omega must be symmetric positive semidefinite");
  if (k > 0) HIPCHK(hipMemcpyAsync(D(oC), hC, (size_t)k * k * 8, hipMemcpyHostToDevice, hs));

  // ---- setup kernels ----
  const double g1 = lambda1 * GMV, g2 = lambda2, g3 = lambda3;
  if (ffo::launch_setup(n, k, m, P, Tp, ldk, F, D(oC), A, delta, s, q, w_target, g1, g2, g3, D(oK), D(odr),
                        D(odc), D(odrC), D(oar), D(ocv), D(oca), D(ocb), D(obF), D(ocr), stream))
    return fail(FFO_EDEVICE, "setup kernel launch failed");
  p.K = D(oK); p.dr = D(odr); p.dc = D(odc); p.drC = D(odrC); p.alpha = alpha; p.arisk = D(oar);
  p.cvec = D(ocv); p.ca = D(oca); p.cb = D(ocb); p.w0 = w0; p.wT = w_target; p.L = L; p.U = U;
  p.bF = D(obF); p.g1 = g1; p.d = d; p.g2 = g2;
  p.crisk = D(ocr);
  if (f32rows) {
    if (ffo::launch_to_float(D(oK), (float*)(B + oKf), (int64_t)nr * ldk, stream))
      return fail(FFO_EDEVICE, "setup kernel launch failed");
    p.Kf = (const float*)(B + oKf);
  }

  ffo::DevState sv{};
  sv.xs = D(ost[0]); sv.x0s = D(ost[1]); sv.Txs = D(ost[2]);
  sv.bb = D(ost[3]); sv.aa = D(ost[4]); sv.vpow = D(ost[5]);
  sv.ysC = D(osc[0]); sv.ys0C = D(osc[1]); sv.TysC = D(osc[2]);
  sv.xbuf = D(oxb); sv.bar = (unsigned long long*)(B + obar);
  sv.blist = c.lists ? D(oblist) : nullptr;
  sv.info = D(oinfo); sv.status = (int32_t*)(B + ostat); sv.w_out = w_out; sv.y_out = y_out;
  sv.w_init = w_init; sv.y_init = y_init;
  HIPCHK(fill(B + oxb, nxbuf * 8, 0u, hs));
  HIPCHK(fill(B + obar, 8 * ffo::BAR_WORDS, 0u, hs));
  HIPCHK(fill(B + oinfo, ffo::INFO_LEN * 8, 0u, hs));
  HIPCHK(fill(B + ostat, 4, 0xffffffffu, hs));
  if (ev) HIPCHK(hipEventRecord(ev[1], hs));
  if (int e = ffo::launch_solve(p, sv, c, stream, lds))
    return fail(FFO_EDEVICE, std::string("cooperative launch of the solve kernel failed: ") +
                                 hipGetErrorString((hipError_t)e));
  if (ev) HIPCHK(hipEventRecord(ev[2], hs));
  HIPCHK(hipMemcpyAsync(hinfo, B + oinfo, ffo::INFO_LEN * 8, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipMemcpyAsync(hflag, B + ostat, 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  const int32_t hstat = *hflag;
  float ms_setup = 0.f, ms_iter = 0.f;
  if (ev) {
    hipEventElapsedTime(&ms_setup, ev[0], ev[1]);
    hipEventElapsedTime(&ms_iter, ev[1], ev[2]);
  }
  const ffo_status st = status_of(hstat);
  switch (st) {
    case FFO_OK: break;
    case FFO_NOT_CONVERGED: g_err = "iteration limit reached"; break;
    case FFO_NUMERIC: g_err = "NaN or Inf in an FP64 check"; break;
    case FFO_TIMEOUT: g_err = "time limit reached"; break;
    case FFO_INFEASIBLE:
      g_err = "infeasible: no portfolio meets the exposure bounds within the budget (certificate in y_out)";
      break;
    default: g_err = "solve kernel ended without a result (bounded wait expired)"; break;
  }
  if (info) fill_info(info, st, hinfo, ms_setup, ms_iter);
  if (opt.verbose)
    std::fprintf(stderr,
                 "[ffo] status %d iters %.0f restarts %.0f spec_miss %.0f ms_rounds %.0f exchanges %.0f checks %.0f "
                 "normK %.4f nwg %d nw %d lds_k %d lds_state %d spec %d | t_power %.3f ms t_iter %.3f ms "
                 "t_check %.3f ms t_wait(wg0) %.3f ms | A %.3f B %.3f C %.3f D %.3f pre %.3f read %.3f ms "
                 "| B1 %.3f (stats %.3f) B2 %.3f (gather %.3f in %.0f iterations) B3 %.3f ms | multisect in %.0f out %.0f\n",
                 (int)st, hinfo[ffo::IX_ITERS], hinfo[ffo::IX_RESTARTS], hinfo[ffo::IX_SPEC_MISS],
                 hinfo[ffo::IX_MS_ROUNDS], hinfo[ffo::IX_EXCHANGES], hinfo[ffo::IX_CHECKS], hinfo[ffo::IX_NORMK], nwg,
                 nw, c.lds_k, c.lds_state, c.spec, hinfo[ffo::IX_T_POWER] * 1e3, hinfo[ffo::IX_T_ITER] * 1e3,
                 hinfo[ffo::IX_T_CHECK] * 1e3, hinfo[ffo::IX_T_WAIT] * 1e3, hinfo[ffo::IX_T_PHA] * 1e3,
                 hinfo[ffo::IX_T_PHB] * 1e3, hinfo[ffo::IX_T_PHC] * 1e3, hinfo[ffo::IX_T_PHD] * 1e3,
                 hinfo[ffo::IX_T_PRE] * 1e3, hinfo[ffo::IX_T_READ] * 1e3, hinfo[ffo::IX_T_B1] * 1e3,
                 hinfo[ffo::IX_T_B1S] * 1e3, hinfo[ffo::IX_T_B2] * 1e3, hinfo[ffo::IX_T_GATHER] * 1e3,
                 hinfo[ffo::IX_GATHERS], hinfo[ffo::IX_T_B3] * 1e3, hinfo[ffo::IX_MISS_IN], hinfo[ffo::IX_MISS_OUT]);
  return st;
}

// ---- lockstep batched form (kernels in lockstep.hip) ----

// Tunables of the lockstep form: slot groups per K~^T y tile, assets per K~ x chunk,
// threads of the per-instance workgroups.  They change the speed, and the rounding of
// some sums, never the method.
struct LsTune {
  int gpt = 2, ch = 256, threads = 512, fused = 0;
};

// Autotuned choices, cached per shape for the life of the process.
std::mutex g_tune_mu;
std::map<std::tuple<int64_t, int64_t, int64_t, int64_t, int>, LsTune> g_tune;

struct LsBuffers {
  hipStream_t ps = nullptr;   // private stream (graph capture needs a non-null stream)
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};
std::map<std::tuple<int, void*>, LsBuffers> g_ls;

ffo_status ls_buffers(int dev, void* stream, LsBuffers** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  LsBuffers& b = g_ls[std::make_tuple(dev, stream)];
  if (!b.ps && hipStreamCreateWithFlags(&b.ps, hipStreamNonBlocking) != hipSuccess)
    return fail(FFO_EDEVICE, "hipStreamCreateWithFlags failed");
  for (auto& e : b.ev)
    if (!e && hipEventCreate(&e) != hipSuccess) return fail(FFO_EDEVICE, "hipEventCreate failed");
  *out = &b;
  return FFO_OK;
}

// One lockstep iteration (check = 0) or the checked iteration and the check (check = 1)
// on stream ps; grids from the tile capacities.
hipError_t ls_enqueue_iter(const ffo::LsShared& S, const LsTune& tu, int gA, int gC, int check, hipStream_t ps) {
  const int gE = (int)std::min<int64_t>(2048, (S.N + ffo::LS_EW - 1) / ffo::LS_EW + S.B);
  int e = 0;
  if (tu.fused) {
    e = ffo::ls_launch_step_fused(S, check, tu.threads, gA, gC, ps);
  } else {
    e = ffo::ls_launch_kty(S, S.yh, S.R, gA, ps);
    if (!e) e = ffo::ls_launch_primal(S, check, tu.threads, gE, ps);
    if (!e) e = ffo::ls_launch_kx(S, S.xbar, gC, ps);
  }
  if (!e) e = ffo::ls_launch_dual(S, check ? 1 : 0, ps);
  if (check) {
    if (!e) e = ffo::ls_launch_kty(S, S.yhT, S.R, gA, ps);
    if (!e) e = ffo::ls_launch_kx(S, S.Tx, gC, ps);
    if (!e) e = ffo::ls_launch_check(S, tu.threads, ps);
    if (!e) e = ffo::ls_launch_compact(S, ps);
  }
  return (hipError_t)e;
}

// Graph of `iters` iterations (the last one checked when `check`).
hipError_t ls_graph(const ffo::LsShared& S, const LsTune& tu, int gA, int gC, int iters, bool check, hipStream_t ps,
                    hipGraphExec_t* exec) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(ps, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int it = 0; it < iters && le == hipSuccess; ++it)
    le = ls_enqueue_iter(S, tu, gA, gC, check && it == iters - 1 ? 1 : 0, ps);
  e = hipStreamEndCapture(ps, &g);
  if (le != hipSuccess) { if (g) hipGraphDestroy(g); return le; }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return e;
}

// Initial state, slot lists, and the power iteration for every instance's step size.
hipError_t ls_start(const ffo::LsShared& S, const LsTune& tu, int gA, int gC, const int32_t* hact, int32_t* hcnt,
                    hipStream_t ps) {
  hipError_t e = hipMemcpyAsync(S.act, hact, (size_t)S.B * 4, hipMemcpyHostToDevice, ps);
  if (e != hipSuccess) return e;
  hcnt[0] = S.B; hcnt[1] = hcnt[2] = hcnt[3] = hcnt[4] = 0;
  if ((e = hipMemcpyAsync(S.cnt, hcnt, 20, hipMemcpyHostToDevice, ps)) != hipSuccess) return e;
  int r = ffo::ls_launch_init(S, ps);
  if (!r) r = ffo::ls_launch_compact(S, ps);
  for (int pw = 0; pw < 40 && !r; ++pw) {
    r = ffo::ls_launch_kx(S, S.xbar, gC, ps);
    if (!r) r = ffo::ls_launch_dual(S, 2, ps);
    if (!r) r = ffo::ls_launch_kty(S, S.yhT, S.R, gA, ps);
    if (!r) r = ffo::ls_launch_power(S, 1, ps);
  }
  if (!r) r = ffo::ls_launch_power(S, 2, ps);
  return (hipError_t)r;
}

ffo_status batched_lockstep(int64_t B, const int64_t* n_b, int64_t n_max, int64_t k, int64_t m, const double* F,
                            const double* Omega, const double* delta, const double* A, const int64_t* offs,
                            const double* alpha, const double* s, const double* q, const double* w0,
                            const double* L, const double* U, double d, double GMV, double lambda1, double lambda2,
                            double lambda3, const ffo_options& opt, void* stream, double* w_out, ffo_info* infos) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  int wall_khz = 0;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
    wall_khz = 100000;
  const int nr = (int)(m + k);
  const int ldk = (int)((n_max + 63) / 64 * 64);
  const int nrp = (nr + 15) / 16 * 16;
  const int64_t N = offs[B];
  const int ce = opt.check_every;
  const size_t lds_total = (size_t)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);

  // slots: instances by decreasing n_b (ties by index)
  std::vector<int32_t> order(B);
  for (int64_t b = 0; b < B; ++b) order[b] = (int32_t)b;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return n_b[a] > n_b[b]; });

  // tunables: cached per shape, tuned on first use unless the deterministic mode asks
  // for the fixed defaults
  const auto key = std::make_tuple(B, n_max, (int64_t)nr, N, ce);
  LsTune tu;
  if (opt.autotune == 0) tu.fused = 1;
  bool tuned = opt.deterministic != 0 || opt.autotune <= 0;
  if (!tuned) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) { tu = it->second; tuned = true; }
  }
  // capacities for the largest tunables (gpt = 1, ch = 128)
  const int64_t Gmax = (B + 15) / 16;
  const int64_t nab = (n_max + 63) / 64;
  const int64_t maxA = nab * Gmax, nchunk_max = (n_max + 127) / 128, maxC = Gmax * nchunk_max;
  int64_t maxE = 0;
  for (int64_t b = 0; b < B; ++b) maxE += (n_b[b] + ffo::LS_EW - 1) / ffo::LS_EW;
  const int gA = (int)std::min<int64_t>(maxA, 2048), gC = (int)std::min<int64_t>(maxC, 2048);

  // ---- workspace ----
  size_t off = 0;
  auto carve = [&](size_t cnt, size_t elt) { const size_t o = off; off = align_up(off + cnt * elt); return o; };
  const size_t oK = carve((size_t)nr * ldk, 8), oKT = carve((size_t)n_max * nrp, 8), odrs = carve((size_t)B * nr, 8);
  const size_t odc = carve(n_max, 8), odrC = carve(n_max, 8), oar = carve(n_max, 8), ocv = carve(n_max, 8);
  const size_t oca = carve(N, 8), ocb = carve(N, 8), onb64 = carve(B, 8), onb32 = carve(B, 4), ooffs = carve(B + 1, 8);
  const size_t oC = carve(std::max<int64_t>(k * k, 1), 8);
  size_t ov[10];
  for (auto& o : ov) o = carve(N, 8);
  size_t orow[5];
  for (auto& o : orow) o = carve((size_t)B * nrp, 8);
  const size_t opart = carve((size_t)nchunk_max * B * nrp, 8);
  const size_t oinst = carve(B, sizeof(ffo::LsInst)), oact = carve(B, 4), ocnt = carve(8, 4);
  const size_t otA = carve((size_t)3 * maxA, 4), otC = carve((size_t)3 * maxC, 4);
  const size_t otE = carve((size_t)2 * maxE, 4), oeoff = carve(B, 4), oest = carve((size_t)8 * maxE, 8);
  const size_t oest2 = carve((size_t)8 * nab * B, 8);
  const size_t oinfo = carve((size_t)B * ffo::INFO_LEN, 8), ostat = carve(B, 4), oclk = carve(1, 8), oflag = carve(1, 4);
  // the hand-off of the last instances to the plain kernel: warm start and a contiguous
  // copy of the instance's exposure rows
  const size_t ohw = carve(n_max, 8), ohy = carve((size_t)nr + n_max, 8);
  const size_t ohA = carve((size_t)std::max<int64_t>(m, 1) * n_max, 8);
  const size_t total = off;
  size_t hoff = 0;
  auto hcarve = [&](size_t bytes) { const size_t o = hoff; hoff = align_up(hoff + bytes); return o; };
  const size_t kk2 = (size_t)std::max<int64_t>(k * k, 1);
  const size_t hOm_o = hcarve(kk2 * 8), hC_o = hcarve(kk2 * 8), hW_o = hcarve(2 * kk2 * 8), hflag_o = hcarve(4);
  const size_t hnb_o = hcarve((size_t)B * 8), hnb32_o = hcarve((size_t)B * 4), hoffs_o = hcarve((size_t)(B + 1) * 8);
  const size_t hact_o = hcarve((size_t)B * 4), hcnt_o = hcarve(32), hinfo_o = hcarve((size_t)B * ffo::INFO_LEN * 8);
  const size_t hstat_o = hcarve((size_t)B * 4), hinst_o = hcarve((size_t)B * sizeof(ffo::LsInst));
  Workspace* ws = nullptr;
  if (ffo_status st = get_workspace(dev, stream, total, hoff, &ws, 3)) return st;
  LsBuffers* lb = nullptr;
  if (ffo_status st = ls_buffers(dev, stream, &lb)) return st;
  char* Bd = (char*)ws->base;
  char* Hb = (char*)ws->host;
  auto D = [&](size_t o) { return (double*)(Bd + o); };
  hipStream_t hs = (hipStream_t)stream, ps = lb->ps;
  double* hOm = (double*)(Hb + hOm_o);
  double* hC = (double*)(Hb + hC_o);
  int* hflag = (int*)(Hb + hflag_o);
  int32_t* hact = (int32_t*)(Hb + hact_o);
  int32_t* hcnt = (int32_t*)(Hb + hcnt_o);

  // ---- validation, Omega, setup (on the caller's stream) ----
  HIPCHK(hipEventRecord(ws->ev[0], hs));
  std::memcpy(Hb + hnb_o, n_b, (size_t)B * 8);
  std::memcpy(Hb + hoffs_o, offs, (size_t)(B + 1) * 8);
  for (int64_t b = 0; b < B; ++b) ((int32_t*)(Hb + hnb32_o))[b] = (int32_t)n_b[b];
  for (int64_t b = 0; b < B; ++b) hact[b] = order[b];
  HIPCHK(hipMemcpyAsync(Bd + onb64, Hb + hnb_o, (size_t)B * 8, hipMemcpyHostToDevice, hs));
  HIPCHK(hipMemcpyAsync(Bd + onb32, Hb + hnb32_o, (size_t)B * 4, hipMemcpyHostToDevice, hs));
  HIPCHK(hipMemcpyAsync(Bd + ooffs, Hb + hoffs_o, (size_t)(B + 1) * 8, hipMemcpyHostToDevice, hs));
  HIPCHK(fill(Bd + oflag, 4, 0u, hs));
  hipLaunchKernelGGL(k_validate, dim3(64), dim3(256), 0, hs, n_max, (int64_t)0, (int64_t)0, n_max * k, (int64_t)0,
                     (const double*)nullptr, F, delta, (const double*)nullptr, (const double*)nullptr,
                     (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, (const double*)nullptr,
                     (int*)(Bd + oflag));
  hipLaunchKernelGGL(k_validate_packed, dim3(64), dim3(256), 0, hs, N, B * m, alpha, s, q, w0, L, U, (int*)(Bd + oflag));
  HIPCHK(hipGetLastError());
  if (k > 0) HIPCHK(hipMemcpyAsync(hOm, Omega, (size_t)k * k * 8, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipMemcpyAsync(hflag, Bd + oflag, 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  if (*hflag) return fail(FFO_EINVAL, bad_values(*hflag));
  if (k > 0 && !factor_omega((int)k, hOm, hC, (double*)(Hb + hW_o)))
    return fail(FFO_EINVAL, "Omega must be symmetric positive semidefinite");
  if (k > 0) HIPCHK(hipMemcpyAsync(D(oC), hC, (size_t)k * k * 8, hipMemcpyHostToDevice, hs));
  const double g1 = lambda1 * GMV;
  if (ffo::launch_setup_batch(B, (const int64_t*)(Bd + onb64), n_max, k, m, ldk, F, D(oC), A, delta, N, s, q, g1,
                              lambda2, lambda3, D(oK), D(odrs), D(odc), D(odrC), D(oar), D(ocv), D(oca), D(ocb), hs))
    return fail(FFO_EDEVICE, "setup kernel launch failed");

  ffo::LsShared S{};
  S.B = (int)B; S.nr = nr; S.m = (int)m; S.k = (int)k; S.n_max = (int)n_max; S.ldk = ldk; S.nrp = nrp;
  S.nr4 = (nr + 3) / 4;
  S.g1 = g1; S.d = d; S.tol = opt.tol_rel_kkt; S.rho = opt.reflection; S.time_limit_s = opt.time_limit_s;
  S.wall_hz = (double)wall_khz * 1e3; S.r_suff = opt.restart_suff; S.r_nec = opt.restart_nec;
  S.r_art = opt.restart_art; S.max_iter = opt.max_iter;
  S.KD = D(oK); S.KDT = D(oKT); S.drs = D(odrs); S.dc = D(odc); S.arisk = D(oar); S.drC = D(odrC);
  S.alpha = alpha; S.ca = D(oca); S.cb = D(ocb); S.w0 = w0; S.L = m ? L : nullptr; S.U = m ? U : nullptr;
  S.offs = (const int64_t*)(Bd + ooffs); S.nb = (const int32_t*)(Bd + onb32);
  S.x = D(ov[0]); S.x0 = D(ov[1]); S.yC = D(ov[2]); S.yC0 = D(ov[3]); S.xbar = D(ov[4]); S.R = D(ov[5]);
  S.Tx = D(ov[6]); S.TyC = D(ov[7]); S.gb = D(ov[8]); S.ga = D(ov[9]);
  S.y = D(orow[0]); S.y0 = D(orow[1]); S.Ty = D(orow[2]); S.yh = D(orow[3]); S.yhT = D(orow[4]);
  S.part = D(opart); S.inst = (ffo::LsInst*)(Bd + oinst); S.act = (int32_t*)(Bd + oact);
  S.cnt = (int32_t*)(Bd + ocnt); S.tileA = (int32_t*)(Bd + otA); S.tileC = (int32_t*)(Bd + otC);
  S.tileE = (int32_t*)(Bd + otE); S.eoff = (int32_t*)(Bd + oeoff); S.estat = D(oest); S.N = N;
  S.estat2 = D(oest2);
  S.w_out = w_out; S.info = D(oinfo); S.status = (int32_t*)(Bd + ostat);
  S.clock0 = (unsigned long long*)(Bd + oclk);
  // (b, 1/a) pairs of an instance in LDS up to this many assets (else device memory)
  S.lds_cap = (int)std::min<int64_t>(n_max, (int64_t)((lds_total - 16 * 12 * 8 - 512) / 16));
  if (ffo::ls_launch_transpose(S, D(oKT), hs)) return fail(FFO_EDEVICE, "transpose kernel launch failed");
  HIPCHK(fill(Bd + oinfo, (size_t)B * ffo::INFO_LEN * 8, 0u, hs));
  HIPCHK(hipEventRecord(lb->ev[0], hs));
  HIPCHK(hipStreamWaitEvent(ps, lb->ev[0], 0));

  auto apply = [&](LsTune& t) {
    if (t.fused) t.ch = 128;   // the fused K~ x kernel runs 128-asset chunks
    S.gpt = t.gpt; S.ch = t.ch; S.nchunk = (int)((n_max + t.ch - 1) / t.ch);
  };
  // ---- autotuning: time 16 plain iterations per candidate (coordinate descent over the
  // per-instance threads, the chunk size and the groups per tile), then start afresh ----
  int tuned_candidates = 0;
  if (!tuned) {
    const int cand_threads[3] = {256, 512, 512}, cand_ch[3] = {128, 256, 256}, cand_gpt[3] = {1, 2, 4};
    auto time_of = [&](LsTune t, float* ms) -> hipError_t {
      apply(t);
      hipError_t e = ls_start(S, t, gA, gC, hact, hcnt, ps);
      if (e != hipSuccess) return e;
      hipGraphExec_t ex = nullptr;
      if ((e = ls_graph(S, t, gA, gC, 16, false, ps, &ex)) != hipSuccess) return e;
      float best = 1e30f;
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        hipEventRecord(lb->ev[1], ps);
        e = hipGraphLaunch(ex, ps);
        hipEventRecord(lb->ev[2], ps);
        if (e == hipSuccess) e = hipEventSynchronize(lb->ev[2]);
        float t1 = 0.f;
        hipEventElapsedTime(&t1, lb->ev[1], lb->ev[2]);
        best = std::min(best, t1);
      }
      hipGraphExecDestroy(ex);
      *ms = best;
      ++tuned_candidates;
      return e;
    };
    LsTune cur;
    float cur_ms = 0.f;
    HIPCHK(time_of(cur, &cur_ms));
    const int cand_fused[3] = {0, 1, 1};
    for (int dim = 0; dim < 4; ++dim) {
      const int* cand = dim == 0 ? cand_fused : dim == 1 ? cand_threads : dim == 2 ? cand_ch : cand_gpt;
      for (int ci = 0; ci < 3; ++ci) {
        LsTune t = cur;
        int& f = dim == 0 ? t.fused : dim == 1 ? t.threads : dim == 2 ? t.ch : t.gpt;
        if (f == cand[ci]) continue;
        f = cand[ci];
        float ms = 0.f;
        HIPCHK(time_of(t, &ms));
        if (ms < 0.95f * cur_ms) { cur = t; cur_ms = ms; }
      }
    }
    tu = cur;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = tu;
  }
  apply(tu);

  // ---- the solve: start, then replays of one checked graph ----
  HIPCHK(hipEventRecord(ws->ev[1], ps));
  HIPCHK(ls_start(S, tu, gA, gC, hact, hcnt, ps));
  hipGraphExec_t ex = nullptr;
  HIPCHK(ls_graph(S, tu, gA, gC, ce, true, ps, &ex));
  const int64_t max_replays = (opt.max_iter + ce - 1) / ce + 1;
  // When at most kHandoff instances remain, each step still pays every kernel's launch
  // and latency for a handful of assets (about 41 us per step against ~12 us for an
  // iteration of the plain kernel), so the last ones finish on the plain kernel, warm
  // started from their current iterate and primal weight.
  constexpr int64_t kHandoff = 4;
  int64_t replays = 0;
  bool handoff = false;
  hipError_t le = hipSuccess;
  for (; replays < max_replays; ++replays) {
    le = hipGraphLaunch(ex, ps);
    if (le != hipSuccess) break;
    le = hipMemcpyAsync(hcnt, S.cnt, 4, hipMemcpyDeviceToHost, ps);
    if (le != hipSuccess) break;
    le = hipStreamSynchronize(ps);
    if (le != hipSuccess || hcnt[0] == 0) { ++replays; break; }
    if (B > kHandoff && hcnt[0] <= kHandoff) { ++replays; handoff = true; break; }
  }
  hipGraphExecDestroy(ex);
  if (le != hipSuccess) return fail(FFO_EDEVICE, std::string("lockstep replay failed: ") + hipGetErrorString(le));
  // the hand-off: every remaining instance in turn on the plain kernel (same stream)
  std::vector<std::pair<int64_t, ffo_info>> handed;
  if (handoff) {
    const int nleft = hcnt[0];
    ffo::LsInst* hinst = (ffo::LsInst*)(Hb + hinst_o);
    HIPCHK(hipMemcpyAsync(hact, S.act, (size_t)nleft * 4, hipMemcpyDeviceToHost, ps));
    HIPCHK(hipMemcpyAsync(hinst, S.inst, (size_t)B * sizeof(ffo::LsInst), hipMemcpyDeviceToHost, ps));
    HIPCHK(hipStreamSynchronize(ps));
    for (int j = 0; j < nleft; ++j) {
      const int64_t b = hact[j], o = offs[b], nb = n_b[b];
      const ffo::LsInst I = hinst[b];
      if (ffo::ls_launch_export(S, (int)b, (int)nb, D(ohw), D(ohy), ps)) return fail(FFO_EDEVICE, "export launch failed");
      if (m > 0)
        HIPCHK(hipMemcpy2DAsync(D(ohA), (size_t)nb * 8, A, (size_t)n_max * 8, (size_t)nb * 8, (size_t)m,
                                hipMemcpyDeviceToDevice, ps));
      ffo_options o2 = opt;
      o2.max_iter = std::max<int64_t>(1, opt.max_iter - I.it);
      o2.workgroups = 0;
      o2.verbose = 0;
      ffo_info ib{};
      const ffo_status sb = solve_impl(nb, k, m, 0, alpha + o, F, Omega, delta, s + o, q + o, d, D(ohA),
                                       m ? L + (size_t)b * m : nullptr, m ? U + (size_t)b * m : nullptr, w0 + o, GMV,
                                       lambda1, lambda2, lambda3, nullptr, D(ohw), D(ohy), I.omega, &o2, ps,
                                       w_out + o, nullptr, &ib, nullptr);
      if (sb == FFO_EINVAL || sb == FFO_ENOMEM || sb == FFO_EDEVICE) return sb;
      ib.iters += I.it;
      ib.restarts += I.restarts;
      handed.emplace_back(b, ib);
    }
  }
  HIPCHK(hipEventRecord(ws->ev[2], ps));
  double* hinfo = (double*)(Hb + hinfo_o);
  int32_t* hstat = (int32_t*)(Hb + hstat_o);
  HIPCHK(hipMemcpyAsync(hinfo, S.info, (size_t)B * ffo::INFO_LEN * 8, hipMemcpyDeviceToHost, ps));
  HIPCHK(hipMemcpyAsync(hstat, S.status, (size_t)B * 4, hipMemcpyDeviceToHost, ps));
  HIPCHK(hipStreamSynchronize(ps));
  float ms_setup = 0.f, ms_iter = 0.f;
  hipEventElapsedTime(&ms_setup, ws->ev[0], ws->ev[1]);
  hipEventElapsedTime(&ms_iter, ws->ev[1], ws->ev[2]);
  ffo_status worst = FFO_OK;
  auto rank = [](ffo_status x) {
    return x == FFO_EDEVICE ? 5 : x == FFO_NUMERIC ? 4 : x == FFO_INFEASIBLE ? 3 : x == FFO_TIMEOUT ? 2
           : x == FFO_NOT_CONVERGED ? 1 : 0;
  };
  for (int64_t b = 0; b < B; ++b) {
    const ffo_status st = status_of(hstat[b]);
    fill_info(&infos[b], st, hinfo + (size_t)b * ffo::INFO_LEN, ms_setup, ms_iter);
  }
  for (const auto& h : handed) {   // instances finished by the plain kernel
    infos[h.first] = h.second;
    infos[h.first].ms_setup = ms_setup;
    infos[h.first].ms_iter = ms_iter;
  }
  for (int64_t b = 0; b < B; ++b)
    if (rank((ffo_status)infos[b].status) > rank(worst)) worst = (ffo_status)infos[b].status;
  if (opt.verbose) {
    double passes = 0.0, iters = 0.0, pmax = 0.0;
    for (int64_t b = 0; b < B; ++b) {
      const double* h = hinfo + (size_t)b * ffo::INFO_LEN;
      passes += h[ffo::IX_MS_ROUNDS];
      iters += h[ffo::IX_ITERS];
      pmax = std::max(pmax, h[ffo::IX_MS_ROUNDS] / std::max(1.0, h[ffo::IX_ITERS]));
    }
    std::fprintf(stderr, "[ffo lockstep] B %lld replays %lld (x %d iterations) tune fused %d threads %d ch %d gpt %d "
                         "(%d candidates timed) | setup+tune %.3f ms solve %.3f ms | multiplier passes per "
                         "iteration %.2f (instance max %.2f) | %d finished on the plain kernel\n",
                 (long long)B, (long long)replays, ce, tu.fused, tu.threads, tu.ch, tu.gpt, tuned_candidates,
                 ms_setup, ms_iter, passes / std::max(1.0, iters), pmax, (int)handed.size());
  }
  if (worst == FFO_NOT_CONVERGED) g_err = "iteration limit reached for at least one instance";
  else if (worst == FFO_TIMEOUT) g_err = "time limit reached for at least one instance";
  else if (worst == FFO_NUMERIC) g_err = "NaN or Inf in an FP64 check of at least one instance";
  else if (worst == FFO_EDEVICE) g_err = "an instance ended without a result";
  return worst;
}

// ---- the team form: sizing, LDS placement, launches, results (ffo_solve_batched and
// ffo_solve_many) ----

// Instances in decreasing size, cut into launches whose minimal teams (ceil(n / nw_max)
// workgroups) fit the resident grid of W workgroups; a launch's spare workgroups go to
// the team with the most assets per workgroup while each keeps at least nw_min.
struct TeamPlan {
  std::vector<int64_t> order;                        // instances by decreasing n
  std::vector<int> g;                                // team size per instance
  std::vector<std::pair<int64_t, int64_t>> chunks;   // launches: [first, last) into order
};

TeamPlan plan_teams(int64_t B, const int64_t* n_b, int W, int nw_max, int nw_min) {
  TeamPlan tp;
  tp.order.resize(B);
  for (int64_t b = 0; b < B; ++b) tp.order[b] = b;
  std::stable_sort(tp.order.begin(), tp.order.end(), [&](int64_t a, int64_t b) { return n_b[a] > n_b[b]; });
  tp.g.assign(B, 1);
  {
    int64_t first = 0, used = 0;
    for (int64_t r = 0; r < B; ++r) {
      const int64_t need = (n_b[tp.order[r]] + nw_max - 1) / nw_max;
      if (used + need > W && r > first) {
        tp.chunks.push_back({first, r});
        first = r;
        used = 0;
      }
      used += need;
    }
    tp.chunks.push_back({first, B});
  }
  for (const auto& ch : tp.chunks) {
    int64_t used = 0;
    for (int64_t r = ch.first; r < ch.second; ++r) {
      tp.g[tp.order[r]] = (int)((n_b[tp.order[r]] + nw_max - 1) / nw_max);
      used += tp.g[tp.order[r]];
    }
    while (used < W) {
      int64_t best = -1;
      double bv = 0.0;
      for (int64_t r = ch.first; r < ch.second; ++r) {
        const int64_t b = tp.order[r];
        const double per = (double)n_b[b] / tp.g[b];
        if ((double)n_b[b] / (tp.g[b] + 1) >= nw_min && per > bv) { bv = per; best = b; }
      }
      if (best < 0) break;
      tp.g[best]++;
      used++;
    }
  }
  return tp;
}

// LDS placement per launch, in ffo_solve's order (constraint slice and per-asset state,
// slice only, state only, neither): the first that fits every team of the launch and
// keeps the launch resident; bfloat16 rows always stay in device memory.  Sets the
// teams' lds_k / lds_state and returns each launch's placement and LDS bytes.
void place_teams(const TeamPlan& tp, const ffo::DevProblem* hP, ffo::DevControl* hCt, int prec, size_t lds_lim,
                 int cus, std::vector<int>& ckl, std::vector<int>& csl, std::vector<size_t>& clds) {
  const size_t nc = tp.chunks.size();
  ckl.assign(nc, 0);
  csl.assign(nc, 0);
  clds.assign(nc, 0);
  for (size_t ci = 0; ci < nc; ++ci) {
    const auto& ch = tp.chunks[ci];
    int nb = 0;
    for (int64_t r = ch.first; r < ch.second; ++r) nb += tp.g[tp.order[r]];
    const int cand[4][2] = {{1, 1}, {1, 0}, {0, 1}, {0, 0}};
    for (const auto& o : cand) {
      if (o[0] && prec == ffo::PREC_BF16K) continue;
      size_t need = 0;
      for (int64_t r = ch.first; r < ch.second; ++r) {
        ffo::DevControl t = hCt[tp.order[r]];
        t.lds_k = o[0];
        t.lds_state = o[1];
        need = std::max(need, ffo::solve_lds_bytes(hP[tp.order[r]], t));
      }
      const bool last = o[0] == 0 && o[1] == 0;
      if (last || (need <= lds_lim && ffo::solve_batch_occupancy(o[0], o[1], prec, need) * cus >= nb)) {
        ckl[ci] = o[0];
        csl[ci] = o[1];
        clds[ci] = need;
        break;
      }
    }
    for (int64_t r = ch.first; r < ch.second; ++r) {
      hCt[tp.order[r]].lds_k = ckl[ci];
      hCt[tp.order[r]].lds_state = csl[ci];
    }
  }
}

// One cooperative launch of the team kernel per launch of the plan, in stream order.
// ht_all / hr_all: host staging of W team and rank entries per launch; dteam / drank:
// the device tables (W entries), rewritten before each launch.
ffo_status launch_teams(const TeamPlan& tp, int W, const std::vector<int>& ckl, const std::vector<int>& csl,
                        const std::vector<size_t>& clds, int prec, const ffo::DevProblem* dP,
                        const ffo::DevState* dS, const ffo::DevControl* dCt, int* dteam, int* drank, int* ht_all,
                        int* hr_all, void* stream) {
  hipStream_t hs = (hipStream_t)stream;
  for (size_t ci = 0; ci < tp.chunks.size(); ++ci) {
    int* ht = ht_all + ci * W;
    int* hr = hr_all + ci * W;
    int nb = 0;
    for (int64_t r = tp.chunks[ci].first; r < tp.chunks[ci].second; ++r) {
      const int64_t b = tp.order[r];
      for (int w = 0; w < tp.g[b]; ++w) { ht[nb] = (int)b; hr[nb] = w; ++nb; }
    }
    HIPCHK(hipMemcpyAsync(dteam, ht, (size_t)nb * 4, hipMemcpyHostToDevice, hs));
    HIPCHK(hipMemcpyAsync(drank, hr, (size_t)nb * 4, hipMemcpyHostToDevice, hs));
    if (int e = ffo::launch_solve_batch(dP, dS, dCt, dteam, drank, nb, ckl[ci], csl[ci], prec, stream, clds[ci]))
      return fail(FFO_EDEVICE, std::string("cooperative launch of the batched solve kernel failed: ") +
                                   hipGetErrorString((hipError_t)e));
  }
  return FFO_OK;
}

// Statuses and infos of every instance after the team launches; returns the most severe
// status (FFO_EDEVICE > FFO_NUMERIC > FFO_INFEASIBLE > FFO_TIMEOUT > FFO_NOT_CONVERGED).
// verbose: the slowest instance's phase times on stderr (verbose >= 2: every instance's).
ffo_status collect_teams(int64_t B, const int64_t* n_b, const double* hinfo, const int32_t* hstat, float ms_setup,
                         float ms_iter, const ffo::DevControl* hCt, int verbose, ffo_info* infos) {
  ffo_status worst = FFO_OK;
  auto rank = [](ffo_status x) {
    return x == FFO_EDEVICE ? 5 : x == FFO_NUMERIC ? 4 : x == FFO_INFEASIBLE ? 3 : x == FFO_TIMEOUT ? 2
           : x == FFO_NOT_CONVERGED ? 1 : 0;
  };
  for (int64_t b = 0; b < B; ++b) {
    const ffo_status st = status_of(hstat[b]);
    fill_info(&infos[b], st, hinfo + (size_t)b * ffo::INFO_LEN, ms_setup, ms_iter);
    if (rank(st) > rank(worst)) worst = st;
  }
  if (verbose) {
    int64_t slow = 0;
    for (int64_t b = 1; b < B; ++b)
      if (hinfo[(size_t)b * ffo::INFO_LEN + ffo::IX_T_ITER] > hinfo[(size_t)slow * ffo::INFO_LEN + ffo::IX_T_ITER]) slow = b;
    auto show = [&](const char* what, int64_t b) {
      const double* h = hinfo + (size_t)b * ffo::INFO_LEN;
      std::fprintf(stderr,
                   "[ffo batch] %s instance %lld: n %lld team %d xmode %d iters %.0f spec_miss %.0f exchanges %.0f "
                   "| t_iter %.3f ms t_check %.3f ms t_wait %.3f ms | A %.3f B %.3f C %.3f D %.3f pre %.3f read %.3f "
                   "| B1 %.3f (stats %.3f) B2 %.3f B3 %.3f ms\n",
                   what, (long long)b, (long long)n_b[b], hCt[b].nwg, hCt[b].xmode, h[ffo::IX_ITERS],
                   h[ffo::IX_SPEC_MISS], h[ffo::IX_EXCHANGES], h[ffo::IX_T_ITER] * 1e3, h[ffo::IX_T_CHECK] * 1e3,
                   h[ffo::IX_T_WAIT] * 1e3, h[ffo::IX_T_PHA] * 1e3, h[ffo::IX_T_PHB] * 1e3, h[ffo::IX_T_PHC] * 1e3,
                   h[ffo::IX_T_PHD] * 1e3, h[ffo::IX_T_PRE] * 1e3, h[ffo::IX_T_READ] * 1e3, h[ffo::IX_T_B1] * 1e3,
                   h[ffo::IX_T_B1S] * 1e3, h[ffo::IX_T_B2] * 1e3, h[ffo::IX_T_B3] * 1e3);
    };
    show("slowest", slow);
    if (verbose >= 2)
      for (int64_t b = 0; b < B; ++b) show("every", b);
  }
  if (worst == FFO_NOT_CONVERGED) g_err = "iteration limit reached for at least one instance";
  else if (worst == FFO_TIMEOUT) g_err = "time limit reached for at least one instance";
  else if (worst == FFO_NUMERIC) g_err = "NaN or Inf in an FP64 check of at least one instance";
  else if (worst == FFO_INFEASIBLE) g_err = "at least one instance is infeasible";
  else if (worst == FFO_EDEVICE) g_err = "a team ended without a result (bounded wait expired)";
  return worst;
}

// ---- memory of the allocation-free entry point (ffo_solve_noalloc) ----
// One static device array per GPU (each device holds its own copy of `scratch` for the
// life of the process).  Host code never passes `scratch` itself to a kernel or a copy:
// its device address comes from hipGetSymbolAddress, once per device, with that device
// current, and is kept in g_static[dev].ptr.
constexpr size_t kScratchBytes = (size_t)32 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

// host staging of that entry point: Omega, its factor and the factorisation's work space
// (k <= 128), the info record and the flags, in static host memory (no allocation)
constexpr size_t kStaticHostBytes = (size_t)4 * 128 * 128 * 8 + 16384;
alignas(256) unsigned char g_static_host[kStaticHostBytes];

struct StaticSlot {
  bool ready = false;
  void* ptr = nullptr;       // device address of `scratch` on this device
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};
constexpr int kMaxDevices = 64;
StaticSlot g_static[kMaxDevices];
std::mutex g_static_mu;      // serialises the entry point (one static host staging area)

// Set-up of the current device for the allocation-free entry point: the device address
// of `scratch` and three timing events, taken once per device.
ffo_status static_slot(int dev, StaticSlot** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FFO_EDEVICE, "device index beyond the static slots");
  StaticSlot& sl = g_static[dev];
  if (!sl.ready) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(FFO_EDEVICE, std::string("hipGetSymbolAddress of the static scratch failed: ") +
                                   hipGetErrorString(e));
    for (auto& ev : sl.ev)
      if (!ev && hipEventCreate(&ev) != hipSuccess) return fail(FFO_EDEVICE, "hipEventCreate failed");
    sl.ptr = ptr;
    sl.ready = true;
  }
  *out = &sl;
  return FFO_OK;
}

}  // namespace

extern "C" {

void ffo_default_options(ffo_options* o) {
  if (!o) return;
  o->tol_rel_kkt = 1e-6;
  o->max_iter = 1000000;
  o->time_limit_s = 360.0;
  o->check_every = 64;
  o->precision = FFO_FP64;
  o->restart_suff = 0.2;
  o->restart_nec = 0.8;
  o->restart_art = 0.36;
  o->reflection = 1.0;
  o->workgroups = 0;
  o->verbose = 0;
  o->deterministic = 0;
  o->speculative = -1;
  o->breakpoint_lists = 1;
  o->infeasibility_check = 1;
  o->batched_form = 0;
  o->autotune = 1;
}

const char* ffo_last_error(void) { return g_err.c_str(); }

const char* ffo_version(void) { return "ffolio 0.1 (gfx950)"; }

void ffo_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ws) {
    if (kv.second.base) hipFree(kv.second.base);
    if (kv.second.host) hipHostFree(kv.second.host);
    for (auto& e : kv.second.ev)
      if (e) hipEventDestroy(e);
  }
  g_ws.clear();
  for (auto& kv : g_ls) {
    for (auto& e : kv.second.ev)
      if (e) hipEventDestroy(e);
    if (kv.second.ps) hipStreamDestroy(kv.second.ps);
  }
  g_ls.clear();
}

ffo_status ffo_solve(int64_t n, int64_t k, int64_t m, int64_t T, const double* alpha, const double* F,
                     const double* Omega, const double* delta, const double* s, const double* q, double d,
                     const double* A, const double* L, const double* U, const double* w0, double GMV,
                     double lambda1, double lambda2, double lambda3, const double* w_target,
                     const ffo_options* opt_in, void* stream, double* w_out, double* y_out, ffo_info* info) {
  return solve_impl(n, k, m, T, alpha, F, Omega, delta, s, q, d, A, L, U, w0, GMV, lambda1, lambda2, lambda3,
                    w_target, nullptr, nullptr, 0.0, opt_in, stream, w_out, y_out, info, nullptr);
}

ffo_status ffo_solve_noalloc(int64_t n, int64_t k, int64_t m, int64_t T, const double* alpha, const double* F,
                             const double* Omega, const double* delta, const double* s, const double* q, double d,
                             const double* A, const double* L, const double* U, const double* w0, double GMV,
                             double lambda1, double lambda2, double lambda3, const double* w_target,
                             const ffo_options* opt_in, void* stream, double* w_out, double* y_out, ffo_info* info) {
  g_err.clear();
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_static_mu);
  StaticSlot* sl = nullptr;
  if (ffo_status st = static_slot(dev, &sl)) return st;
  const Fixed fx{(char*)sl->ptr, kScratchBytes, (char*)g_static_host, kStaticHostBytes, sl->ev};
  return solve_impl(n, k, m, T, alpha, F, Omega, delta, s, q, d, A, L, U, w0, GMV, lambda1, lambda2, lambda3,
                    w_target, nullptr, nullptr, 0.0, opt_in, stream, w_out, y_out, info, &fx);
}

ffo_status ffo_risk_model(int64_t days, int64_t n, int64_t p, const double* R, const double* Fr, const uint8_t* mask,
                          int64_t min_obs, void* stream, double* beta, double* Sigma_f, double* D, int32_t* valid) {
  g_err.clear();
  if (days < 2 || days > ((int64_t)1 << 20)) return fail(FFO_EINVAL, "days must lie in [2, 2^20]");
  if (n < 1 || n > ((int64_t)1 << 26)) return fail(FFO_EINVAL, "n must lie in [1, 2^26]");
  if (days * n > ((int64_t)1 << 34)) return fail(FFO_EINVAL, "days * n too large");
  if (p < 1 || p > 8) return fail(FFO_EINVAL, "p must lie in [1, 8]");
  if (min_obs < 0 || min_obs > days) return fail(FFO_EINVAL, "min_obs must lie in [0, days]");
  if (!R || !Fr || !beta || !Sigma_f || !D || !valid) return fail(FFO_EINVAL, "null array pointer");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  Workspace* ws = nullptr;
  if (ffo_status st = get_workspace(dev, stream, ffo::rm_workspace_bytes(days, n, p), 256, &ws, 4)) return st;
  if (ffo::launch_risk_model((int)days, (int)n, (int)p, R, Fr, mask, (int)min_obs, (double*)ws->base, beta, Sigma_f,
                             D, valid, stream))
    return fail(FFO_EDEVICE, "risk-model kernel launch failed");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return FFO_OK;
}


ffo_status ffo_solve_warm(int64_t n, int64_t k, int64_t m, int64_t T, const double* alpha, const double* F,
                          const double* Omega, const double* delta, const double* s, const double* q, double d,
                          const double* A, const double* L, const double* U, const double* w0, double GMV,
                          double lambda1, double lambda2, double lambda3, const double* w_target,
                          const double* w_init, const double* y_init, double omega_init, const ffo_options* opt_in,
                          void* stream, double* w_out, double* y_out, ffo_info* info) {
  g_err.clear();
  if (!(omega_init >= 0.0) || !std::isfinite(omega_init))
    return fail(FFO_EINVAL, "omega_init must be finite and >= 0 (0: the default start)");
  return solve_impl(n, k, m, T, alpha, F, Omega, delta, s, q, d, A, L, U, w0, GMV, lambda1, lambda2, lambda3,
                    w_target, w_init, y_init, omega_init, opt_in, stream, w_out, y_out, info, nullptr);
}

ffo_status ffo_adjoint(int64_t n, int64_t k, int64_t m, int64_t T, const double* alpha, const double* F,
                       const double* Omega, const double* delta, const double* s, const double* q, double d,
                       const double* A, const double* L, const double* U, const double* w0, double GMV,
                       double lambda1, double lambda2, double lambda3, const double* w_target,
                       const double* w_star, const double* y_star, const double* grad_w, double omega,
                       const ffo_options* opt_in, void* stream, double* grad_alpha, double* grad_s,
                       double* grad_F, ffo_info* info) {
  g_err.clear();
  ffo_options opt;
  ffo_default_options(&opt);
  opt.tol_rel_kkt = 1e-9;
  if (opt_in) opt = *opt_in;
  // ---- host-only validation ----
  if (ffo_status st = check_problem_args(n, k, m, T, alpha, F, Omega, delta, s, q, d, A, L, U, w0, GMV, lambda1,
                                         lambda2, lambda3, w_target))
    return st;
  if (!w_star || !y_star || !grad_w || !grad_alpha || !grad_s) return fail(FFO_EINVAL, "null array pointer");
  if (k > 0 && !grad_F) return fail(FFO_EINVAL, "grad_F must be non-null when k > 0");
  if (ffo_status st = check_options(opt)) return st;
  if (opt.precision != FFO_FP64) return fail(FFO_EINVAL, "ffo_adjoint runs in FFO_FP64");
  if (!(omega >= 0.0) || !std::isfinite(omega)) return fail(FFO_EINVAL, "omega must be finite and >= 0 (0: default)");
  const int64_t P = T == 0 ? 1 : T - 1, Tp = T == 0 ? 1 : T;

  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  int wall_khz = 0;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
    wall_khz = 100000;
  const int nr = (int)(m + k);
  const int ldk = (int)((n + 63) / 64 * 64);
  ffo::DevProblem p{};
  p.n = (int)n; p.k = (int)k; p.m = (int)m; p.P = (int)P; p.Tp = (int)Tp; p.nr = nr;
  p.multi = T > 0 ? 1 : 0; p.ldk = ldk; p.kscaled = 1;
  const int cus = std::max(1, prop.multiProcessorCount);
  int nwg = opt.workgroups > 0 ? opt.workgroups : default_workgroups(n, cus);
  nwg = std::max(1, std::min<int>(nwg, (int)n));
  nwg = std::min(nwg, cus);
  const int nw = (int)((n + nwg - 1) / nwg);
  nwg = (int)((n + nw - 1) / nw);
  ffo::DevControl c{};
  c.tol = opt.tol_rel_kkt; c.time_limit_s = opt.time_limit_s;
  c.r_suff = opt.restart_suff; c.r_nec = opt.restart_nec; c.r_art = opt.restart_art;
  c.rho = opt.reflection; c.eta_safety = 0.95; c.max_iter = opt.max_iter;
  c.check_every = opt.check_every; c.xmode = ffo::XM_ATOMIC; c.nwg = nwg; c.npow = 40;
  c.xgroups = xgroups_for(nwg);
  c.verbose = opt.verbose; c.nw = nw; c.spin_limit = 1u << 26; c.wall_hz = (double)wall_khz * 1e3;
  c.prec = ffo::PREC_FP64; c.spec = 0; c.lds_state = 0;
  c.vmax = ffo::adjoint_vmax(p);
  const size_t lds_cap = (size_t)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
  c.lds_k = 1;
  size_t lds = ffo::adjoint_lds_bytes(p, c);
  if (lds > lds_cap) {
    c.lds_k = 0;
    lds = ffo::adjoint_lds_bytes(p, c);
    if (lds > lds_cap) return fail(FFO_EINVAL, "problem too large for the per-workgroup working set (reduce m + k or T)");
  }
  // ---- workspace layout ----
  const size_t Pn = (size_t)P * n, Tpn = (size_t)Tp * n;
  size_t off = 0;
  auto carve = [&](size_t cnt, size_t elt) { const size_t o = off; off = align_up(off + cnt * elt); return o; };
  const size_t oK = carve((size_t)std::max(nr, 1) * ldk, 8), odr = carve(std::max(nr, 1), 8), odc = carve(n, 8);
  const size_t odrC = carve(Tpn, 8), oar = carve(n, 8), ocv = carve(n, 8), oca = carve(Tpn, 8), ocb = carve(Tpn, 8);
  const size_t obF = carve(std::max<int64_t>(k, 1), 8), ocr = carve(1, 8), oC = carve(std::max<int64_t>(k * k, 1), 8);
  size_t ost[7];
  for (auto& o : ost) o = carve(Pn, 8);
  size_t osc[8];
  for (auto& o : osc) o = carve(Tpn, 8);
  const size_t ogG = carve((size_t)n * std::max<int64_t>(k, 1), 8);
  const size_t oxb = carve((size_t)3 * ffo::XG_MAX * c.vmax, 8), obar = carve(ffo::BAR_WORDS, 8);
  const size_t oinfo = carve(ffo::INFO_LEN, 8), ostat = carve(1, 4), oflag = carve(1, 4);
  const size_t total = off;
  const size_t hk = align_up((size_t)std::max<int64_t>(k * k, 1) * 8);
  const size_t host_bytes = 2 * hk + align_up(ffo::INFO_LEN * 8) + 4096;
  Workspace* ws = nullptr;
  if (ffo_status st = get_workspace(dev, stream, total, host_bytes, &ws, 2)) return st;
  char* B = (char*)ws->base;
  auto D = [&](size_t o) { return (double*)(B + o); };
  hipStream_t hs = (hipStream_t)stream;
  double* hOm = (double*)ws->host;
  double* hC = hOm + hk / 8;
  double* hinfo_buf = hC + hk / 8;
  int* hflag = (int*)(hinfo_buf + align_up(ffo::INFO_LEN * 8) / 8);

  HIPCHK(hipEventRecord(ws->ev[0], hs));
  HIPCHK(hipMemsetAsync(B + oflag, 0, 4, hs));
  hipLaunchKernelGGL(k_validate, dim3(64), dim3(256), 0, hs, n, (int64_t)Pn, (int64_t)Tpn, n * k, m, alpha, F,
                     delta, s, q, L, U, w0, w_target, (int*)(B + oflag));
  HIPCHK(hipGetLastError());
  if (k > 0) HIPCHK(hipMemcpyAsync(hOm, Omega, (size_t)k * k * 8, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipMemcpyAsync(hflag, B + oflag, 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  if (*hflag) return fail(FFO_EINVAL, bad_values(*hflag));
  std::vector<double> fwork((size_t)2 * std::max<int64_t>(k * k, 1));
  if (k > 0 && !factor_omega((int)k, hOm, hC, fwork.data()))
    return fail(FFO_EINVAL, "Omega must be symmetric positive semidefinite");
  if (k > 0) HIPCHK(hipMemcpyAsync(D(oC), hC, (size_t)k * k * 8, hipMemcpyHostToDevice, hs));
  const double g1 = lambda1 * GMV, g2 = lambda2, g3 = lambda3;
  if (ffo::launch_setup(n, k, m, P, Tp, ldk, F, D(oC), A, delta, s, q, w_target, g1, g2, g3, D(oK), D(odr),
                        D(odc), D(odrC), D(oar), D(ocv), D(oca), D(ocb), D(obF), D(ocr), stream))
    return fail(FFO_EDEVICE, "setup kernel launch failed");
  p.K = D(oK); p.dr = D(odr); p.dc = D(odc); p.drC = D(odrC); p.alpha = alpha; p.arisk = D(oar);
  p.cvec = D(ocv); p.ca = D(oca); p.cb = D(ocb); p.w0 = w0; p.wT = w_target; p.L = L; p.U = U;
  p.bF = D(obF); p.g1 = g1; p.d = d; p.g2 = g2; p.crisk = D(ocr);
  ffo::AdjState a{};
  a.w_star = w_star; a.y_star = y_star; a.grad_w = grad_w;
  a.xs = D(ost[0]); a.xbar = D(ost[1]); a.bb = D(ost[2]); a.sx = D(ost[3]);
  a.lx = D(ost[4]); a.lx0 = D(ost[5]); a.Tlx = D(ost[6]);
  a.ysC = D(osc[0]); a.lyC = D(osc[1]); a.lyC0 = D(osc[2]); a.TlyC = D(osc[3]); a.nC = D(osc[4]); a.gsf = D(osc[5]);
  a.tsg = D(osc[6]); a.trho = D(osc[7]);
  a.grad_alpha = grad_alpha; a.grad_s = grad_s; a.grad_G = D(ogG);
  a.xbuf = D(oxb); a.bar = (unsigned long long*)(B + obar); a.info = D(oinfo); a.status = (int32_t*)(B + ostat);
  HIPCHK(hipEventRecord(ws->ev[1], hs));
  // The transposed step swaps the roles of the primal and dual steps, and its natural
  // weight is usually the reciprocal of the solve's (about 20x fewer iterations on the
  // T = 10, n = 2000 market), but not always: that weight runs first under an iteration
  // cap, and if it does not converge the solve's own weight runs from scratch.
  const int64_t first_cap = std::min<int64_t>(opt.max_iter, 100000);
  const double weights[2] = {omega > 0.0 ? 1.0 / omega : 1.0, omega > 0.0 ? omega : 1.0};
  int32_t st_dev = -1;
  int64_t used = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    ffo::DevControl ca = c;
    ca.max_iter = attempt == 0 ? first_cap : std::max<int64_t>(1, opt.max_iter - used);
    HIPCHK(fill(B + oxb, (size_t)3 * ffo::XG_MAX * c.vmax * 8, 0u, hs));
    HIPCHK(fill(B + obar, 8 * ffo::BAR_WORDS, 0u, hs));
    HIPCHK(fill(B + oinfo, ffo::INFO_LEN * 8, 0u, hs));
    HIPCHK(hipMemsetAsync(B + ostat, 0xff, 4, hs));
    if (int e = ffo::launch_adjoint(p, a, ca, weights[attempt], stream, lds))
      return fail(FFO_EDEVICE, std::string("cooperative launch of the adjoint kernel failed: ") +
                                   hipGetErrorString((hipError_t)e));
    HIPCHK(hipMemcpyAsync(hflag, B + ostat, 4, hipMemcpyDeviceToHost, hs));
    HIPCHK(hipMemcpyAsync(hinfo_buf, B + oinfo, ffo::INFO_LEN * 8, hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    st_dev = *hflag;
    used += (int64_t)hinfo_buf[ffo::IX_ITERS];
    if (st_dev != ffo::DS_NOT_CONVERGED || attempt == 1 || weights[0] == weights[1] || used >= opt.max_iter) break;
  }
  if (k > 0 && ffo::launch_grad_F((int)n, (int)k, D(ogG), D(oC), grad_F, stream))
    return fail(FFO_EDEVICE, "grad_F kernel launch failed");
  HIPCHK(hipEventRecord(ws->ev[2], hs));
  HIPCHK(hipMemcpyAsync(hinfo_buf, B + oinfo, ffo::INFO_LEN * 8, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipMemcpyAsync(hflag, B + ostat, 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  float ms_setup = 0.f, ms_iter = 0.f;
  hipEventElapsedTime(&ms_setup, ws->ev[0], ws->ev[1]);
  hipEventElapsedTime(&ms_iter, ws->ev[1], ws->ev[2]);
  hinfo_buf[ffo::IX_ITERS] = (double)used;   // both attempts
  const ffo_status st = status_of(*hflag);
  if (st == FFO_NOT_CONVERGED) g_err = "adjoint iteration limit reached";
  else if (st == FFO_NUMERIC) g_err = "NaN or Inf in the adjoint iteration";
  else if (st == FFO_TIMEOUT) g_err = "time limit reached";
  else if (st == FFO_EDEVICE) g_err = "adjoint kernel ended without a result (bounded wait expired)";
  if (info) fill_info(info, st, hinfo_buf, ms_setup, ms_iter);
  if (opt.verbose)
    std::fprintf(stderr, "[ffo adjoint] status %d iters %.0f restarts %.0f residual %.3e exchanges %.0f nwg %d lds_k %d "
                         "| setup %.3f ms adjoint %.3f ms\n",
                 (int)st, hinfo_buf[ffo::IX_ITERS], hinfo_buf[ffo::IX_RESTARTS], hinfo_buf[ffo::IX_RELKKT],
                 hinfo_buf[ffo::IX_EXCHANGES], nwg, c.lds_k, ms_setup, ms_iter);
  return st;
}

ffo_status ffo_solve_batched(int64_t B, const int64_t* n_b, int64_t n_max, int64_t k, int64_t m,
                             const double* F, const double* Omega, const double* delta, const double* A,
                             const int64_t* offs, const double* alpha, const double* s, const double* q,
                             const double* w0, const double* L, const double* U, double d, double GMV,
                             double lambda1, double lambda2, double lambda3, const ffo_options* opt_in,
                             void* stream, double* w_out, ffo_info* infos) {
  g_err.clear();
  ffo_options opt;
  ffo_default_options(&opt);
  if (opt_in) opt = *opt_in;
  // ---- host-only validation (no device work before this point) ----
  if (B < 1 || B > (1 << 20)) return fail(FFO_EINVAL, "B must lie in [1, 2^20]");
  if (!n_b || !offs || !infos) return fail(FFO_EINVAL, "null host array (n_b, offs or infos)");
  if (n_max < 1 || n_max > (1 << 24)) return fail(FFO_EINVAL, "n_max must lie in [1, 2^24]");
  if (k < 0 || k > 128) return fail(FFO_EINVAL, "k must lie in [0, 128]");
  if (m < 0 || m > 4096) return fail(FFO_EINVAL, "m must lie in [0, 4096]");
  if (offs[0] != 0) return fail(FFO_EINVAL, "offs[0] must be 0");
  for (int64_t b = 0; b < B; ++b) {
    if (n_b[b] < 1 || n_b[b] > n_max) return fail(FFO_EINVAL, "every n_b must lie in [1, n_max]");
    if (offs[b + 1] - offs[b] != n_b[b]) return fail(FFO_EINVAL, "offs must be the running sum of n_b");
  }
  const int64_t N = offs[B];
  if (N > ((int64_t)1 << 31)) return fail(FFO_EINVAL, "sum of n_b too large");
  if (!alpha || !delta || !s || !q || !w0 || !w_out) return fail(FFO_EINVAL, "null array pointer");
  if (k > 0 && (!F || !Omega)) return fail(FFO_EINVAL, "F and Omega are required when k > 0");
  if (m > 0 && (!A || !L || !U)) return fail(FFO_EINVAL, "A, L and U are required when m > 0");
  if (!(d > 1.0 && d <= 2.0)) return fail(FFO_EINVAL, "d must lie in (1, 2]");
  if (!(GMV > 0.0) || !std::isfinite(GMV)) return fail(FFO_EINVAL, "GMV must be positive and finite");
  if (!(lambda1 > 0.0) || !std::isfinite(lambda1)) return fail(FFO_EINVAL, "lambda1 must be positive and finite");
  if (!(lambda2 >= 0.0) || !(lambda3 >= 0.0) || !std::isfinite(lambda2) || !std::isfinite(lambda3))
    return fail(FFO_EINVAL, "lambda2 and lambda3 must be nonnegative and finite");
  if (!std::isfinite(lambda1 * GMV)) return fail(FFO_EINVAL, "lambda1 * GMV must be finite");
  if (!(opt.tol_rel_kkt > 0.0)) return fail(FFO_EINVAL, "tol_rel_kkt must be positive");
  if (opt.max_iter < 1) return fail(FFO_EINVAL, "max_iter must be >= 1");
  if (opt.check_every < 1) return fail(FFO_EINVAL, "check_every must be >= 1");
  if (!(opt.time_limit_s > 0.0)) return fail(FFO_EINVAL, "time_limit_s must be positive");
  if (!(opt.reflection >= 0.0 && opt.reflection <= 1.0)) return fail(FFO_EINVAL, "reflection must lie in [0, 1]");
  if (opt.precision != FFO_FP64 && opt.precision != FFO_FP32 && opt.precision != FFO_FP32_BF16K)
    return fail(FFO_EINVAL, "ffo_solve_batched takes FFO_FP64, FFO_FP32 or FFO_FP32_BF16K");
  if (opt.batched_form < 0 || opt.batched_form > 2) return fail(FFO_EINVAL, "batched_form must be 0, 1 or 2");
  if (opt.autotune < -1 || opt.autotune > 1) return fail(FFO_EINVAL, "autotune must be -1, 0 or 1");
  {
    const bool ls_ok = opt.precision == FFO_FP64 && m + k >= 1 && m + k <= 160 && B <= 65536 && n_max <= (1 << 22);
    if (opt.batched_form == 2 && !ls_ok)
      return fail(FFO_EINVAL, "the lockstep batched form needs FFO_FP64, 1 <= m + k <= 160, B <= 65536 and "
                              "n_max <= 2^22");
    if (opt.batched_form == 2 || (opt.batched_form == 0 && ls_ok))
      return batched_lockstep(B, n_b, n_max, k, m, F, Omega, delta, A, offs, alpha, s, q, w0, L, U, d, GMV, lambda1,
                              lambda2, lambda3, opt, stream, w_out, infos);
  }

  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  int wall_khz = 0;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
    wall_khz = 100000;
  const int cus = std::max(1, prop.multiProcessorCount);
  const int nr = (int)(m + k);
  const int ldk = (int)((n_max + 63) / 64 * 64);
  const int prec = opt.precision == FFO_FP32 ? ffo::PREC_FP32
                   : (opt.precision == FFO_FP32_BF16K ? ffo::PREC_BF16K : ffo::PREC_FP64);

  // ---- control and team sizing ----
  ffo::DevProblem p0{};
  p0.k = (int)k; p0.m = (int)m; p0.P = 1; p0.Tp = 1; p0.nr = nr; p0.multi = 0; p0.ldk = ldk; p0.kscaled = 0;
  ffo::DevControl c0{};
  c0.tol = opt.tol_rel_kkt; c0.time_limit_s = opt.time_limit_s;
  c0.r_suff = opt.restart_suff; c0.r_nec = opt.restart_nec; c0.r_art = opt.restart_art;
  c0.rho = opt.reflection; c0.eta_safety = 0.95; c0.max_iter = opt.max_iter; c0.check_every = opt.check_every;
  c0.npow = 40; c0.verbose = opt.verbose; c0.spin_limit = 1u << 26; c0.wall_hz = (double)wall_khz * 1e3;
  c0.prec = prec; c0.spec = 1; c0.lds_k = 0; c0.lds_state = 0; c0.infeas = opt.infeasibility_check ? 1 : 0;
  c0.vmax = ffo::solve_vmax(p0);
  const int NW_MAX = 2048;   // assets per workgroup at most (bounds the LDS staging)
  // extra workgroups only while a team keeps at least this many assets each (ten n = 5000
  // instances: 25 workgroups per team at 128, 0.28 s per batch, against 19 and 0.34 s at 256)
  const int NW_MIN = 128;
  size_t lds_cap = 0;
  {
    ffo::DevProblem pp = p0;
    ffo::DevControl cc = c0;
    pp.n = NW_MAX; cc.nw = NW_MAX; cc.nwg = 1; cc.xmode = ffo::XM_LOCAL;
    lds_cap = ffo::solve_lds_bytes(pp, cc);
  }
  if (lds_cap > std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024))
    return fail(FFO_EINVAL, "m + k too large for the batched working set");
  const int occ = ffo::solve_batch_occupancy(0, 0, prec, lds_cap);
  if (occ < 1) return fail(FFO_EDEVICE, "the batched solve kernel cannot be resident");
  const int W = occ * cus;
  // instances in decreasing size, cut into launches whose minimal teams fit the resident grid
  const TeamPlan tp = plan_teams(B, n_b, W, NW_MAX, NW_MIN);
  const std::vector<int>& g = tp.g;
  const auto& chunks = tp.chunks;

  // ---- workspace layout ----
  size_t off = 0;
  auto carve = [&](size_t cnt, size_t elt) { const size_t o = off; off = align_up(off + cnt * elt); return o; };
  const size_t oK = carve((size_t)std::max(nr, 1) * ldk, 8), odc = carve(n_max, 8), odrC = carve(n_max, 8);
  const bool f32rows = prec == ffo::PREC_FP32;   // the batched kernel reads rows from device memory
  const bool bf16rows = prec == ffo::PREC_BF16K;
  const size_t oKf = carve(f32rows ? (size_t)std::max(nr, 1) * ldk : 1, 4);
  const size_t oKb = carve(bf16rows ? (size_t)std::max(nr, 1) * ldk : 1, 2);
  const size_t oar = carve(n_max, 8), ocv = carve(n_max, 8), obF = carve(std::max<int64_t>(k, 1), 8);
  const size_t ocr = carve(1, 8), oC = carve(std::max<int64_t>(k * k, 1), 8), onb = carve(B, 8);
  const size_t odrs = carve((size_t)B * std::max(nr, 1), 8), oca = carve(N, 8), ocb = carve(N, 8);
  size_t ost[9];
  for (auto& o : ost) o = carve(N, 8);
  const size_t oxb = carve((size_t)B * 3 * c0.vmax, 8), obar = carve(B, 8);
  const size_t oinfo = carve((size_t)B * ffo::INFO_LEN, 8), ostat = carve(B, 4), oflag = carve(1, 4);
  const size_t oP = carve(B, sizeof(ffo::DevProblem)), oS = carve(B, sizeof(ffo::DevState));
  const size_t oCt = carve(B, sizeof(ffo::DevControl)), oteam = carve(W, 4), orank = carve(W, 4);
  const size_t total = off;
  size_t hoff = 0;
  auto hcarve = [&](size_t bytes) { const size_t o = hoff; hoff = align_up(hoff + bytes); return o; };
  const size_t hOm_o = hcarve((size_t)std::max<int64_t>(k * k, 1) * 8), hC_o = hcarve((size_t)std::max<int64_t>(k * k, 1) * 8);
  const size_t hflag_o = hcarve(4), hinfo_o = hcarve((size_t)B * ffo::INFO_LEN * 8), hstat_o = hcarve((size_t)B * 4);
  const size_t hP_o = hcarve((size_t)B * sizeof(ffo::DevProblem)), hS_o = hcarve((size_t)B * sizeof(ffo::DevState));
  const size_t hCt_o = hcarve((size_t)B * sizeof(ffo::DevControl)), hnb_o = hcarve((size_t)B * 8);
  const size_t hteam_o = hcarve((size_t)W * 4 * chunks.size()), hrank_o = hcarve((size_t)W * 4 * chunks.size());
  const size_t host_bytes = hoff;

  Workspace* ws = nullptr;
  if (ffo_status st = get_workspace(dev, stream, total, host_bytes, &ws, 1)) return st;
  char* Bd = (char*)ws->base;
  char* Hb = (char*)ws->host;
  auto D = [&](size_t o) { return (double*)(Bd + o); };
  hipStream_t hs = (hipStream_t)stream;
  double* hOm = (double*)(Hb + hOm_o);
  double* hC = (double*)(Hb + hC_o);
  int* hflag = (int*)(Hb + hflag_o);

  // ---- device value checks (one synchronisation, with the Omega copy) ----
  HIPCHK(hipEventRecord(ws->ev[0], hs));
  std::memcpy(Hb + hnb_o, n_b, (size_t)B * 8);
  HIPCHK(hipMemcpyAsync(Bd + onb, Hb + hnb_o, (size_t)B * 8, hipMemcpyHostToDevice, hs));
  HIPCHK(hipMemsetAsync(Bd + oflag, 0, 4, hs));
  hipLaunchKernelGGL(k_validate, dim3(64), dim3(256), 0, hs, n_max, (int64_t)0, (int64_t)0, n_max * k, (int64_t)0,
                     (const double*)nullptr, F, delta, (const double*)nullptr, (const double*)nullptr,
                     (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, (const double*)nullptr,
                     (int*)(Bd + oflag));
  hipLaunchKernelGGL(k_validate_packed, dim3(64), dim3(256), 0, hs, N, B * m, alpha, s, q, w0, L, U,
                     (int*)(Bd + oflag));
  HIPCHK(hipGetLastError());
  if (k > 0) HIPCHK(hipMemcpyAsync(hOm, Omega, (size_t)k * k * 8, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipMemcpyAsync(hflag, Bd + oflag, 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  if (*hflag) return fail(FFO_EINVAL, bad_values(*hflag));
  std::vector<double> fwork((size_t)2 * std::max<int64_t>(k * k, 1));
  if (k > 0 && !factor_omega((int)k, hOm, hC, fwork.data()))
    return fail(FFO_EINVAL, "Omega must be symmetric positive semidefinite");
  if (k > 0) HIPCHK(hipMemcpyAsync(D(oC), hC, (size_t)k * k * 8, hipMemcpyHostToDevice, hs));

  // ---- setup: shared rows and per-instance scales ----
  const double g1 = lambda1 * GMV, g2 = lambda2, g3 = lambda3;
  if (ffo::launch_setup_batch(B, (const int64_t*)(Bd + onb), n_max, k, m, ldk, F, D(oC), A, delta, N, s, q, g1, g2, g3,
                              D(oK), D(odrs), D(odc), D(odrC), D(oar), D(ocv), D(oca), D(ocb), stream))
    return fail(FFO_EDEVICE, "setup kernel launch failed");
  if (f32rows && ffo::launch_to_float(D(oK), (float*)(Bd + oKf), (int64_t)nr * ldk, stream))
    return fail(FFO_EDEVICE, "setup kernel launch failed");
  if (bf16rows && ffo::launch_to_bf16(D(oK), (uint16_t*)(Bd + oKb), (int64_t)nr * ldk, stream))
    return fail(FFO_EDEVICE, "setup kernel launch failed");
  HIPCHK(hipMemsetAsync(Bd + obF, 0, (size_t)std::max<int64_t>(k, 1) * 8, hs));
  HIPCHK(hipMemsetAsync(Bd + ocr, 0, 8, hs));
  HIPCHK(hipMemsetAsync(Bd + oxb, 0, (size_t)B * 3 * c0.vmax * 8, hs));
  HIPCHK(hipMemsetAsync(Bd + obar, 0, (size_t)B * 8, hs));
  HIPCHK(hipMemsetAsync(Bd + oinfo, 0, (size_t)B * ffo::INFO_LEN * 8, hs));
  HIPCHK(hipMemsetAsync(Bd + ostat, 0xff, (size_t)B * 4, hs));

  // ---- per-instance problem, state and control ----
  ffo::DevProblem* hP = (ffo::DevProblem*)(Hb + hP_o);
  ffo::DevState* hS = (ffo::DevState*)(Hb + hS_o);
  ffo::DevControl* hCt = (ffo::DevControl*)(Hb + hCt_o);
  for (int64_t b = 0; b < B; ++b) {
    const int64_t o = offs[b];
    ffo::DevProblem p = p0;
    p.n = (int)n_b[b];
    p.K = D(oK); p.Kf = f32rows ? (const float*)(Bd + oKf) : nullptr;
    p.Kb = bf16rows ? (const uint16_t*)(Bd + oKb) : nullptr; p.dr = D(odrs) + (size_t)b * nr; p.dc = D(odc); p.drC = D(odrC); p.alpha = alpha + o;
    p.arisk = D(oar); p.cvec = D(ocv); p.ca = D(oca) + o; p.cb = D(ocb) + o; p.w0 = w0 + o; p.wT = nullptr;
    p.L = m ? L + (size_t)b * m : nullptr; p.U = m ? U + (size_t)b * m : nullptr;
    p.bF = D(obF); p.crisk = D(ocr); p.g1 = g1; p.d = d; p.g2 = g2;
    hP[b] = p;
    ffo::DevState sv{};
    sv.xs = D(ost[0]) + o; sv.x0s = D(ost[1]) + o; sv.Txs = D(ost[2]) + o;
    sv.bb = D(ost[3]) + o; sv.aa = D(ost[4]) + o; sv.vpow = D(ost[5]) + o;
    sv.ysC = D(ost[6]) + o; sv.ys0C = D(ost[7]) + o; sv.TysC = D(ost[8]) + o;
    sv.xbuf = D(oxb) + (size_t)b * 3 * c0.vmax; sv.bar = (unsigned long long*)(Bd + obar) + b;
    sv.info = D(oinfo) + (size_t)b * ffo::INFO_LEN; sv.status = (int32_t*)(Bd + ostat) + b;
    sv.w_out = w_out + o; sv.y_out = nullptr;
    hS[b] = sv;
    ffo::DevControl c = c0;
    c.nwg = g[b];
    c.nw = (int)((n_b[b] + g[b] - 1) / g[b]);
    c.xmode = g[b] == 1 ? ffo::XM_LOCAL : ffo::XM_ATOMIC;
    hCt[b] = c;
  }
  std::vector<int> ckl, csl;
  std::vector<size_t> clds;
  place_teams(tp, hP, hCt, prec, std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024), cus, ckl, csl, clds);
  HIPCHK(hipMemcpyAsync(Bd + oP, hP, (size_t)B * sizeof(ffo::DevProblem), hipMemcpyHostToDevice, hs));
  HIPCHK(hipMemcpyAsync(Bd + oS, hS, (size_t)B * sizeof(ffo::DevState), hipMemcpyHostToDevice, hs));
  HIPCHK(hipMemcpyAsync(Bd + oCt, hCt, (size_t)B * sizeof(ffo::DevControl), hipMemcpyHostToDevice, hs));
  HIPCHK(hipEventRecord(ws->ev[1], hs));
  if (ffo_status st = launch_teams(tp, W, ckl, csl, clds, prec, (const ffo::DevProblem*)(Bd + oP),
                                   (const ffo::DevState*)(Bd + oS), (const ffo::DevControl*)(Bd + oCt),
                                   (int*)(Bd + oteam), (int*)(Bd + orank), (int*)(Hb + hteam_o),
                                   (int*)(Hb + hrank_o), stream))
    return st;
  HIPCHK(hipEventRecord(ws->ev[2], hs));
  double* hinfo = (double*)(Hb + hinfo_o);
  int32_t* hstat = (int32_t*)(Hb + hstat_o);
  HIPCHK(hipMemcpyAsync(hinfo, Bd + oinfo, (size_t)B * ffo::INFO_LEN * 8, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipMemcpyAsync(hstat, Bd + ostat, (size_t)B * 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  float ms_setup = 0.f, ms_iter = 0.f;
  hipEventElapsedTime(&ms_setup, ws->ev[0], ws->ev[1]);
  hipEventElapsedTime(&ms_iter, ws->ev[1], ws->ev[2]);
  if (opt.verbose)
    std::fprintf(stderr,
                 "[ffo batch] B %lld launches %zu resident %d (occupancy %d) lds %zu | first launch: slice in LDS %d, "
                 "state in LDS %d, %zu bytes | setup %.3f ms solve %.3f ms\n",
                 (long long)B, chunks.size(), W, occ, lds_cap, ckl[0], csl[0], clds[0], ms_setup, ms_iter);
  return collect_teams(B, n_b, hinfo, hstat, ms_setup, ms_iter, hCt, opt.verbose, infos);
}

ffo_status ffo_solve_many(int64_t B, const int64_t* n, int64_t k, int64_t m, int64_t T, const double* const* alpha,
                          const double* const* F, const double* const* Omega, const double* const* delta,
                          const double* const* s, const double* const* q, const double* const* A,
                          const double* const* L, const double* const* U, const double* const* w0,
                          const double* const* w_target, double d, double GMV, double lambda1, double lambda2,
                          double lambda3, const ffo_options* opt_in, void* stream, double* const* w_out,
                          ffo_info* infos) {
  g_err.clear();
  ffo_options opt;
  ffo_default_options(&opt);
  if (opt_in) opt = *opt_in;
  // ---- host-only validation (no device work before this point) ----
  if (B < 1 || B > (1 << 16)) return fail(FFO_EINVAL, "B must lie in [1, 2^16]");
  if (!n || !alpha || !delta || !s || !q || !w0 || !w_out || !infos)
    return fail(FFO_EINVAL, "null host array (n, alpha, delta, s, q, w0, w_out or infos)");
  if (k > 0 && (!F || !Omega)) return fail(FFO_EINVAL, "F and Omega are required when k > 0");
  if (m > 0 && (!A || !L || !U)) return fail(FFO_EINVAL, "A, L and U are required when m > 0");
  if (!(T == 0 || (T >= 2 && T <= 4096))) return fail(FFO_EINVAL, "T must be 0 (single-period) or in [2, 4096]");
  if ((T > 0) != (w_target != nullptr)) return fail(FFO_EINVAL, "w_target must be NULL iff T == 0");
  for (int64_t b = 0; b < B; ++b) {
    if (ffo_status st = check_problem_args(n[b], k, m, T, alpha[b], k ? F[b] : nullptr, k ? Omega[b] : nullptr,
                                           delta[b], s[b], q[b], d, m ? A[b] : nullptr, m ? L[b] : nullptr,
                                           m ? U[b] : nullptr, w0[b], GMV, lambda1, lambda2, lambda3,
                                           T ? w_target[b] : nullptr))
      return fail(st, "instance " + std::to_string(b) + ": " + g_err);
    if (!w_out[b]) return fail(FFO_EINVAL, "instance " + std::to_string(b) + ": null w_out");
    if (n[b] > (1 << 24)) return fail(FFO_EINVAL, "instance " + std::to_string(b) + ": n must be <= 2^24");
  }
  if (ffo_status st = check_options(opt)) return st;
  if (opt.precision != FFO_FP64 && opt.precision != FFO_FP32)
    return fail(FFO_EINVAL, "ffo_solve_many takes FFO_FP64 or FFO_FP32");

  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  int wall_khz = 0;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
    wall_khz = 100000;
  const int cus = std::max(1, prop.multiProcessorCount);
  const int nr = (int)(m + k);
  const int prec = opt.precision == FFO_FP32 ? ffo::PREC_FP32 : ffo::PREC_FP64;
  const int64_t P = T == 0 ? 1 : T - 1, Tp = T == 0 ? 1 : T;

  // ---- control and team sizing, as in the team form of ffo_solve_batched ----
  ffo::DevProblem p0{};
  p0.k = (int)k; p0.m = (int)m; p0.P = (int)P; p0.Tp = (int)Tp; p0.nr = nr; p0.multi = T > 0 ? 1 : 0;
  p0.kscaled = 1;
  ffo::DevControl c0{};
  c0.tol = opt.tol_rel_kkt; c0.time_limit_s = opt.time_limit_s;
  c0.r_suff = opt.restart_suff; c0.r_nec = opt.restart_nec; c0.r_art = opt.restart_art;
  c0.rho = opt.reflection; c0.eta_safety = 0.95; c0.max_iter = opt.max_iter; c0.check_every = opt.check_every;
  c0.npow = 40; c0.verbose = opt.verbose; c0.spin_limit = 1u << 26; c0.wall_hz = (double)wall_khz * 1e3;
  // the speculative single exchange as in ffo_solve: on for single-period problems by
  // default, off for multi-period ones, unless opt->speculative says otherwise
  c0.spec = opt.speculative < 0 ? (P == 1 ? 1 : 0) : (opt.speculative ? 1 : 0);
  c0.prec = prec; c0.lds_k = 0; c0.lds_state = 0; c0.infeas = opt.infeasibility_check ? 1 : 0;
  c0.vmax = ffo::solve_vmax(p0);
  // assets per workgroup at most: 2048 as in the team form of ffo_solve_batched, halved
  // while a workgroup's staging for P periods does not fit in LDS (multi-period)
  const int NW_MIN = 128;
  const size_t lds_lim = std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
  int NW_MAX = 2048;
  size_t lds_cap = 0;
  for (;; NW_MAX /= 2) {
    ffo::DevProblem pp = p0;
    ffo::DevControl cc = c0;
    pp.n = NW_MAX; cc.nw = NW_MAX; cc.nwg = 1; cc.xmode = ffo::XM_LOCAL;
    lds_cap = ffo::solve_lds_bytes(pp, cc);
    if (lds_cap <= lds_lim || NW_MAX <= 16) break;
  }
  if (lds_cap > lds_lim) return fail(FFO_EINVAL, "m + k or T too large for the batched working set");
  const int occ = ffo::solve_batch_occupancy(0, 0, prec, lds_cap);
  if (occ < 1) return fail(FFO_EDEVICE, "the batched solve kernel cannot be resident");
  const int W = occ * cus;
  const TeamPlan tp = plan_teams(B, n, W, NW_MAX, NW_MIN);

  // ---- workspace: each instance's scaled rows, scales, costs and state, as ffo_solve's ----
  struct Inst {
    int ldk;
    size_t K, Kf, dr, dc, drC, ar, cv, ca, cb, bF, cr, C, st[9];
  };
  std::vector<Inst> io(B);
  size_t off = 0;
  auto carve = [&](size_t cnt, size_t elt) { const size_t o = off; off = align_up(off + cnt * elt); return o; };
  for (int64_t b = 0; b < B; ++b) {
    Inst& r = io[b];
    const size_t nb = (size_t)n[b];
    r.ldk = (int)((n[b] + 63) / 64 * 64);
    r.K = carve((size_t)std::max(nr, 1) * r.ldk, 8);
    r.Kf = carve(prec == ffo::PREC_FP32 ? (size_t)std::max(nr, 1) * r.ldk : 1, 4);
    r.dr = carve(std::max(nr, 1), 8); r.dc = carve(nb, 8); r.drC = carve(Tp * nb, 8); r.ar = carve(nb, 8);
    r.cv = carve(nb, 8); r.ca = carve(Tp * nb, 8); r.cb = carve(Tp * nb, 8);
    r.bF = carve(std::max<int64_t>(k, 1), 8); r.cr = carve(1, 8); r.C = carve(std::max<int64_t>(k * k, 1), 8);
    for (int j = 0; j < 9; ++j) r.st[j] = carve((j < 6 ? P : Tp) * nb, 8);   // 6 primal [P][n], 3 trade [T][n]
  }
  const size_t oxb = carve((size_t)B * 3 * c0.vmax, 8), obar = carve(B, 8);
  const size_t oinfo = carve((size_t)B * ffo::INFO_LEN, 8), ostat = carve(B, 4), oflag = carve(1, 4);
  const size_t oP = carve(B, sizeof(ffo::DevProblem)), oS = carve(B, sizeof(ffo::DevState));
  const size_t oCt = carve(B, sizeof(ffo::DevControl)), oteam = carve(W, 4), orank = carve(W, 4);
  const size_t total = off;
  const size_t kk = (size_t)std::max<int64_t>(k * k, 1);
  size_t hoff = 0;
  auto hcarve = [&](size_t bytes) { const size_t o = hoff; hoff = align_up(hoff + bytes); return o; };
  const size_t hOm_o = hcarve((size_t)B * kk * 8), hC_o = hcarve(kk * 8), hWk_o = hcarve(2 * kk * 8);
  const size_t hflag_o = hcarve(4), hinfo_o = hcarve((size_t)B * ffo::INFO_LEN * 8), hstat_o = hcarve((size_t)B * 4);
  const size_t hP_o = hcarve((size_t)B * sizeof(ffo::DevProblem)), hS_o = hcarve((size_t)B * sizeof(ffo::DevState));
  const size_t hCt_o = hcarve((size_t)B * sizeof(ffo::DevControl));
  const size_t hteam_o = hcarve((size_t)W * 4 * tp.chunks.size()), hrank_o = hcarve((size_t)W * 4 * tp.chunks.size());
  const size_t host_bytes = hoff;

  Workspace* ws = nullptr;
  if (ffo_status st = get_workspace(dev, stream, total, host_bytes, &ws, 5)) return st;
  char* Bd = (char*)ws->base;
  char* Hb = (char*)ws->host;
  auto D = [&](size_t o) { return (double*)(Bd + o); };
  hipStream_t hs = (hipStream_t)stream;
  int* hflag = (int*)(Hb + hflag_o);

  // ---- device value checks of every instance, and the Omegas to the host (one synchronisation) ----
  HIPCHK(hipEventRecord(ws->ev[0], hs));
  HIPCHK(fill(Bd + oflag, 4, 0u, hs));
  for (int64_t b = 0; b < B; ++b) {
    hipLaunchKernelGGL(k_validate, dim3(64), dim3(256), 0, hs, n[b], P * n[b], Tp * n[b], n[b] * k, m, alpha[b],
                       k ? F[b] : nullptr, delta[b], s[b], q[b], m ? L[b] : nullptr, m ? U[b] : nullptr, w0[b],
                       T ? w_target[b] : (const double*)nullptr, (int*)(Bd + oflag));
    if (k > 0)
      HIPCHK(hipMemcpyAsync(Hb + hOm_o + (size_t)b * kk * 8, Omega[b], (size_t)k * k * 8, hipMemcpyDeviceToHost, hs));
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hflag, Bd + oflag, 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  if (*hflag) return fail(FFO_EINVAL, bad_values(*hflag));

  // ---- setup of every instance (ffo_solve's kernels), problem, state and control records ----
  const double g1 = lambda1 * GMV, g2 = lambda2, g3 = lambda3;
  ffo::DevProblem* hP = (ffo::DevProblem*)(Hb + hP_o);
  ffo::DevState* hS = (ffo::DevState*)(Hb + hS_o);
  ffo::DevControl* hCt = (ffo::DevControl*)(Hb + hCt_o);
  for (int64_t b = 0; b < B; ++b) {
    const Inst& r = io[b];
    if (k > 0) {
      double* hC = (double*)(Hb + hC_o);
      if (!factor_omega((int)k, (double*)(Hb + hOm_o + (size_t)b * kk * 8), hC, (double*)(Hb + hWk_o)))
        return fail(FFO_EINVAL, "instance " + std::to_string(b) + ": Omega must be symmetric positive semidefinite");
      // the copy reads the host staging at once (pageable order: the stream waits for it)
      HIPCHK(hipMemcpyAsync(D(r.C), hC, (size_t)k * k * 8, hipMemcpyHostToDevice, hs));
      HIPCHK(hipStreamSynchronize(hs));
    }
    if (ffo::launch_setup(n[b], k, m, P, Tp, r.ldk, k ? F[b] : nullptr, D(r.C), m ? A[b] : nullptr, delta[b], s[b],
                          q[b], T ? w_target[b] : nullptr, g1, g2, g3, D(r.K), D(r.dr), D(r.dc), D(r.drC), D(r.ar),
                          D(r.cv), D(r.ca), D(r.cb), D(r.bF), D(r.cr), stream))
      return fail(FFO_EDEVICE, "setup kernel launch failed");
    if (prec == ffo::PREC_FP32 && ffo::launch_to_float(D(r.K), (float*)(Bd + r.Kf), (int64_t)nr * r.ldk, stream))
      return fail(FFO_EDEVICE, "setup kernel launch failed");
    ffo::DevProblem p = p0;
    p.n = (int)n[b]; p.ldk = r.ldk;
    p.K = D(r.K); p.Kf = prec == ffo::PREC_FP32 ? (const float*)(Bd + r.Kf) : nullptr;
    p.dr = D(r.dr); p.dc = D(r.dc); p.drC = D(r.drC); p.alpha = alpha[b]; p.arisk = D(r.ar); p.cvec = D(r.cv);
    p.ca = D(r.ca); p.cb = D(r.cb); p.w0 = w0[b]; p.wT = T ? w_target[b] : nullptr;
    p.L = m ? L[b] : nullptr; p.U = m ? U[b] : nullptr;
    p.bF = D(r.bF); p.crisk = D(r.cr); p.g1 = g1; p.d = d; p.g2 = g2;
    hP[b] = p;
    ffo::DevState sv{};
    sv.xs = D(r.st[0]); sv.x0s = D(r.st[1]); sv.Txs = D(r.st[2]);
    sv.bb = D(r.st[3]); sv.aa = D(r.st[4]); sv.vpow = D(r.st[5]);
    sv.ysC = D(r.st[6]); sv.ys0C = D(r.st[7]); sv.TysC = D(r.st[8]);
    sv.xbuf = D(oxb) + (size_t)b * 3 * c0.vmax; sv.bar = (unsigned long long*)(Bd + obar) + b;
    sv.info = D(oinfo) + (size_t)b * ffo::INFO_LEN; sv.status = (int32_t*)(Bd + ostat) + b;
    sv.w_out = w_out[b]; sv.y_out = nullptr;
    hS[b] = sv;
    ffo::DevControl c = c0;
    c.nwg = tp.g[b];
    c.nw = (int)((n[b] + tp.g[b] - 1) / tp.g[b]);
    c.xmode = tp.g[b] == 1 ? ffo::XM_LOCAL : ffo::XM_ATOMIC;
    hCt[b] = c;
  }
  HIPCHK(fill(Bd + oxb, (size_t)B * 3 * c0.vmax * 8, 0u, hs));
  HIPCHK(fill(Bd + obar, (size_t)B * 8, 0u, hs));
  HIPCHK(fill(Bd + oinfo, (size_t)B * ffo::INFO_LEN * 8, 0u, hs));
  HIPCHK(fill(Bd + ostat, (size_t)B * 4, 0xffffffffu, hs));

  // ---- LDS placement, records to the device, one cooperative launch per chunk ----
  std::vector<int> ckl, csl;
  std::vector<size_t> clds;
  place_teams(tp, hP, hCt, prec, lds_lim, cus, ckl, csl, clds);
  HIPCHK(hipMemcpyAsync(Bd + oP, hP, (size_t)B * sizeof(ffo::DevProblem), hipMemcpyHostToDevice, hs));
  HIPCHK(hipMemcpyAsync(Bd + oS, hS, (size_t)B * sizeof(ffo::DevState), hipMemcpyHostToDevice, hs));
  HIPCHK(hipMemcpyAsync(Bd + oCt, hCt, (size_t)B * sizeof(ffo::DevControl), hipMemcpyHostToDevice, hs));
  HIPCHK(hipEventRecord(ws->ev[1], hs));
  if (ffo_status st = launch_teams(tp, W, ckl, csl, clds, prec, (const ffo::DevProblem*)(Bd + oP),
                                   (const ffo::DevState*)(Bd + oS), (const ffo::DevControl*)(Bd + oCt),
                                   (int*)(Bd + oteam), (int*)(Bd + orank), (int*)(Hb + hteam_o),
                                   (int*)(Hb + hrank_o), stream))
    return st;
  HIPCHK(hipEventRecord(ws->ev[2], hs));
  double* hinfo = (double*)(Hb + hinfo_o);
  int32_t* hstat = (int32_t*)(Hb + hstat_o);
  HIPCHK(hipMemcpyAsync(hinfo, Bd + oinfo, (size_t)B * ffo::INFO_LEN * 8, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipMemcpyAsync(hstat, Bd + ostat, (size_t)B * 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  float ms_setup = 0.f, ms_iter = 0.f;
  hipEventElapsedTime(&ms_setup, ws->ev[0], ws->ev[1]);
  hipEventElapsedTime(&ms_iter, ws->ev[1], ws->ev[2]);
  if (opt.verbose)
    std::fprintf(stderr,
                 "[ffo many] B %lld launches %zu resident %d (occupancy %d) | first launch: slice in LDS %d, state in "
                 "LDS %d, %zu bytes | setup %.3f ms solve %.3f ms\n",
                 (long long)B, tp.chunks.size(), W, occ, ckl[0], csl[0], clds[0], ms_setup, ms_iter);
  return collect_teams(B, n, hinfo, hstat, ms_setup, ms_iter, hCt, opt.verbose, infos);
}

// Extra diagnostics of the last solve on this thread's (device, stream): not part of the
// stable interface; used by the benchmark to report exchanges and speculation misses.
int ffo_debug_last_info(void* stream, double* out16) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find(std::make_tuple(dev, stream, 0));
  if (it == g_ws.end() || !it->second.host) return 1;
  std::memcpy(out16, it->second.host, ffo::INFO_LEN * sizeof(double));
  return 0;
}

}  // extern "C"
