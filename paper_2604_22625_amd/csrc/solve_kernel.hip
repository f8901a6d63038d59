// Persistent PDHG solve kernel for gfx950 (CDNA4).
//
// Method (the paper fixes the problem, not the iteration): a restarted, reflected
// Halpern PDHG on the splitting described in include/ffolio.h, in diagonally scaled
// variables xs = W / dc, ys = Y / dr.  One iteration computes T(z) for z = (xs, ys):
//
//   x+ = prox_{tau g}(xs - tau K~^T ys)      per asset: weighted L1-ball solve with a
//                                            global multiplier mu_t per period
//   y+ = prox_{sigma h~*}(ys + sigma K~ (2 x+ - xs))
//
// then z <- (k+1)/(k+2) ((1+rho) T(z) - rho z) + 1/(k+2) z0 (Halpern anchoring with
// reflection), with adaptive restarts on the fixed-point residual and a primal weight
// omega (tau = eta/omega, sigma = eta*omega, eta = safety/||K~|| from a power
// iteration run at the start of the kernel).
//
// Work split: workgroup w owns a contiguous slice of assets for every period.  Its
// slice of the constraint rows and its per-asset state stay in LDS when they fit (else
// in device memory, touched only by this workgroup); the exposure and factor duals
// (P x (m+k) numbers) are replicated in every workgroup and updated redundantly from
// the same exchanged totals, so all workgroups hold bit-identical copies and take
// identical control decisions.
//
// Exchange: each workgroup publishes partial sums with device-scope (sc1) stores or
// atomic adds, then arrives at a counter barrier; readers fetch totals with
// device-scope loads.  No L2 writeback/invalidate fences are needed because every
// exchanged word is accessed only through device-coherent operations.  Every wait is
// bounded (spin_limit): on expiry the kernel records DS_BARRIER and all workgroups exit.
//
// The L1-ball multiplier mu_t is exact.  Speculative mode (one period): a predicted
// bracket [lo, hi] is tested in the same exchange that carries the two affine pieces
// of K~ x_bar(mu); if the root lies in the bracket and no breakpoint |b_i| falls
// inside it, mu and K~ x_bar follow in closed form (one exchange per iteration).
// Two-phase mode (many periods): a small exchange settles mu_t, a second one carries
// K~ x_bar.  Misses fall back to a 32-candidate multisection that isolates a
// breakpoint-free piece.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include "internal.h"

namespace ffo {
namespace {

constexpr int TB = 256;
constexpr int NWAVE = TB / 64;
constexpr int MSC = 32;          // multisection candidates per round
constexpr int MS_ROUNDS = 40;

__device__ __forceinline__ double ldd(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void std_(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void addd(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

// Per-(t, li) array view: element (t, li) at b[t * ld + off + li].
struct Arr {
  double* b;
  int ld, off;
  __device__ __forceinline__ double& operator()(int t, int li) const { return b[(size_t)t * ld + off + li]; }
};

// ---------------------------------------------------------------------------------
// Workgroup context and the exchange primitive
// ---------------------------------------------------------------------------------
struct Ctx {
  int wg, nwg, tid;
  int i0, nwa;            // owned assets [i0, i0 + nwa)
  unsigned long long epoch;
  double* xbuf;
  double* xmax;
  unsigned long long* bar;
  int vmax, xmode, P;
  uint32_t spin_limit;
  double* tot;            // LDS [vmax]
  double* red;            // LDS reduction scratch [256]
  int* flag;              // LDS flag word
  long long t_wait;       // device-clock ticks spent waiting (thread 0)
};

// Contribution j of this workgroup to the current exchange.  In gather mode every
// index in [0, V) must be written each exchange; in atomic mode zeros may be skipped.
__device__ __forceinline__ void put(const Ctx& c, int j, double v) {
  if (c.xmode == XM_GATHER) {
    std_(&c.xbuf[((size_t)(c.epoch & 1) * c.nwg + c.wg) * c.vmax + j], v);
  } else if (v != 0.0) {
    addd(&c.xbuf[(size_t)(c.epoch % 3) * c.vmax + j], v);
  }
}

// This workgroup's maximum for period t in the current exchange.
__device__ __forceinline__ void put_max(const Ctx& c, int t, double v) {
  std_(&c.xmax[((size_t)(c.epoch & 1) * c.nwg + c.wg) * c.P + t], v);
}

// Maximum over workgroups for period t of the exchange that just completed (all threads
// call; loads are spread over the threads and combined through LDS).
__device__ double get_max(const Ctx& c, int t) {
  const size_t par = (size_t)((c.epoch - 1) & 1);
  double m = 0.0;
  for (int w = c.tid; w < c.nwg; w += TB) m = fmax(m, ldd(&c.xmax[(par * c.nwg + w) * c.P + t]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  if ((c.tid & 63) == 0) c.red[200 + (c.tid >> 6)] = m;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < NWAVE; ++w) r = fmax(r, c.red[200 + w]);
  __syncthreads();
  return r;
}

// Barrier + reduction of the V published values into c.tot (LDS).  Returns false when
// the bounded wait expired.
__device__ bool xsync(Ctx& c, int V) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's device-scope stores/atomics are complete
  __syncthreads();
  if (c.tid == 0) {
    const long long t0 = wall_clock64();
    const unsigned long long target = (c.epoch + 1) * (unsigned long long)c.nwg;
    __hip_atomic_fetch_add(c.bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    int ok = 1;
    while (__hip_atomic_load(c.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > c.spin_limit) { ok = 0; break; }
    }
    *c.flag = ok;
    c.t_wait += wall_clock64() - t0;
  }
  __syncthreads();
  if (!*c.flag) return false;
  if (c.xmode == XM_GATHER) {
    const double* base = c.xbuf + (size_t)(c.epoch & 1) * c.nwg * c.vmax;
    for (int j = c.tid; j < V; j += TB) {
      double s = 0.0;
      for (int w = 0; w < c.nwg; ++w) s += ldd(&base[(size_t)w * c.vmax + j]);
      c.tot[j] = s;
    }
  } else {
    const double* base = c.xbuf + (size_t)(c.epoch % 3) * c.vmax;
    for (int j = c.tid; j < V; j += TB) c.tot[j] = ldd(&base[j]);
    // clear the slot used two exchanges from now (its last readers passed this barrier)
    double* z = c.xbuf + (size_t)((c.epoch + 2) % 3) * c.vmax;
    const int per = (c.vmax + c.nwg - 1) / c.nwg;
    const int j0 = c.wg * per, j1 = min(c.vmax, j0 + per);
    for (int j = j0 + c.tid; j < j1; j += TB) std_(&z[j], 0.0);
  }
  __syncthreads();
  c.epoch++;
  return true;
}

// Fixed-order workgroup sum of NV per-thread values; result in out[0..NV) (LDS),
// valid for every thread after the call.  Uses red[0 .. NWAVE*NV).
template <int NV>
__device__ void wg_sum(const Ctx& c, double (&v)[NV], double* out) {
  const int lane = c.tid & 63, wave = c.tid >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double x = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) c.red[wave * NV + q] = x;
  }
  __syncthreads();
  if (c.tid < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) s += c.red[w * NV + c.tid];
    out[c.tid] = s;
  }
  __syncthreads();
}

__device__ double wg_max(const Ctx& c, double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
  if ((c.tid & 63) == 0) c.red[128 + (c.tid >> 6)] = x;
  __syncthreads();
  double m = 0.0;
  for (int w = 0; w < NWAVE; ++w) m = fmax(m, c.red[128 + w]);
  __syncthreads();
  return m;
}

// ---------------------------------------------------------------------------------
// Per-workgroup problem and state views
// ---------------------------------------------------------------------------------
struct S {
  const DevProblem* p;
  const double* Kl;     // LDS slice [nr][nw] or nullptr (then read global K)
  int nw, i0;
  // state
  Arr xs, x0s, Txs, xL, bb, aa, xb;         // [P]
  Arr ysC, ys0C, TysC, ysCL;                // [Tp]
  // constants
  Arr alpha;                                // [P]
  Arr ca, cb, drC;                          // [Tp]
  Arr dc, arisk, cvec, w0, wT;              // [1]
  __device__ __forceinline__ double Kat(int j, int li) const {
    return Kl ? Kl[j * nw + li] : p->K[(size_t)j * p->ldk + i0 + li];
  }
};

// (K~^T y)_ti over the exposure and factor rows for owned (t, li).
__device__ __forceinline__ double kty_rows(const S& v, const double* y, int t, int li) {
  const int nr = v.p->nr;
  const double* yt = y + t * nr;
  double s = 0.0;
  for (int j = 0; j < nr; ++j) s = fma(v.Kat(j, li), yt[j], s);
  return s;
}

// Trade-row adjoint for asset li, period t: dc (drC_t yC_t - drC_{t+1} yC_{t+1}).
__device__ __forceinline__ double kty_trade(const S& v, const Arr& yC, int t, int li) {
  double r = v.drC(t, li) * yC(t, li);
  if (v.p->multi) r -= v.drC(t + 1, li) * yC(t + 1, li);
  return v.dc(0, li) * r;
}

// Trade row t of K~ applied to a scaled primal x for asset li.
__device__ __forceinline__ double kx_trade(const S& v, const Arr& x, int t, int li) {
  double d;
  if (!v.p->multi || t == 0) d = x(0, li);
  else if (t == v.p->P) d = -x(v.p->P - 1, li);
  else d = x(t, li) - x(t - 1, li);
  return v.drC(t, li) * v.dc(0, li) * d;
}

// Offset b_C of trade row t: w0 for the first trade, -w_T for the last (multi-period).
__device__ __forceinline__ double trade_offset(const S& v, int t, int li) {
  if (t == 0) return v.w0(0, li);
  if (v.p->multi && t == v.p->P) return -v.wT(0, li);
  return 0.0;
}

// Unscaled trade u_t of W = dc * x for asset li.
__device__ __forceinline__ double trade_of(const S& v, const Arr& x, int t, int li) {
  const double dci = v.dc(0, li);
  if (!v.p->multi || t == 0) return dci * x(0, li) - v.w0(0, li);
  if (t == v.p->P) return v.wT(0, li) - dci * x(v.p->P - 1, li);
  return dci * (x(t, li) - x(t - 1, li));
}

// prox of t'(a|x| + b|x|^d) at z (closed forms for d = 2 and d = 3/2; Newton with a
// bisection safeguard otherwise).
__device__ __forceinline__ double prox_cost(double z, double tp, double a, double b, double d) {
  const double r = fmax(fabs(z) - tp * a, 0.0);
  if (r <= 0.0) return 0.0;
  const double tb = tp * b;
  double rho;
  if (d == 2.0) {
    rho = r / (1.0 + 2.0 * tb);
  } else if (d == 1.5) {
    const double cc = 1.5 * tb;
    const double u = 2.0 * r / (cc + sqrt(cc * cc + 4.0 * r));
    rho = u * u;
  } else {
    double lo = 0.0, hi = r;
    rho = r;
    for (int it = 0; it < 100; ++it) {
      const double f = rho + tb * d * pow(rho, d - 1.0) - r;
      if (f > 0.0) hi = rho; else lo = rho;
      const double fp = 1.0 + tb * d * (d - 1.0) * pow(rho, d - 2.0);
      double nx = rho - f / fp;
      if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
      if (fabs(nx - rho) <= 1e-16 * r) { rho = nx; break; }
      rho = nx;
    }
  }
  return z > 0.0 ? rho : -rho;
}

// c*(e) for one entry (a = g2 s, b = g3 q).
__device__ __forceinline__ double conj_cost(double e, double a, double b, double d) {
  const double r = fabs(e) - a;
  if (r <= 0.0) return 0.0;
  if (b <= 0.0) return INFINITY;
  const double u = pow(r / (b * d), 1.0 / (d - 1.0));
  return (d - 1.0) / d * r * u;
}

// Rows product for (t, j) over the owned assets: sum_li K~[j][li] x[t][li] (x in LDS).
__device__ __forceinline__ double rows_dot(const Ctx& c, const S& V, const double* x, int nw, int t, int j) {
  double a = 0.0;
  for (int li = 0; li < c.nwa; ++li) a = fma(V.Kat(j, li), x[t * nw + li], a);
  return a;
}

// ---------------------------------------------------------------------------------
// Exact L1-budget multiplier
// ---------------------------------------------------------------------------------
// S_t(mu) = sum_i max(|b_ti| - mu, 0) / a_ti with signed b in bb and 1/a in aa.

// Publish [S(0), S(lo), A0(lo), cnt(lo), S(hi), A0(hi), cnt(hi), 0] for period t at
// payload offset off and this workgroup's max |b| (all threads must call).
__device__ void period_stats(Ctx& c, const Arr& bb, const Arr& aa, double l, double h, int t, int off) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double mx = 0.0;
  for (int li = c.tid; li < c.nwa; li += TB) {
    const double ab = fabs(bb(t, li)), ia = aa(t, li);
    v[0] = fma(ab, ia, v[0]);
    mx = fmax(mx, ab);
    if (ab > l) { v[1] = fma(ab - l, ia, v[1]); v[2] += ia; v[3] += 1.0; }
    if (ab > h) { v[4] = fma(ab - h, ia, v[4]); v[5] += ia; v[6] += 1.0; }
  }
  const double m = wg_max(c, mx);
  wg_sum<8>(c, v, c.red + 64);
  if (c.tid == 0) {
    for (int q = 0; q < 8; ++q) put(c, off + q, c.red[64 + q]);
    put_max(c, t, m);
  }
  __syncthreads();
}

// From exchanged statistics st[8] and the global max: 1 = mu exact from the bracket,
// 2 = mu = 0 but the bracket was not [0,0], 0 = multisection needed with the root inside
// the tested bracket (breakpoints inside it), 3 = multisection needed with the root
// outside it.  On 0 and 3, lo/hi are replaced by a bracket with S(lo) >= 1 >= S(hi).
__device__ int bracket_decide(const double* st, double maxb, double& lo, double& hi, double& mu) {
  const double S0 = st[0];
  const double Slo = st[1], clo = st[3];
  const double Shi = st[4], A0hi = st[5], chi = st[6];
  if (S0 <= 1.0) { mu = 0.0; return hi == 0.0 ? 1 : 2; }
  const bool inside = hi > 0.0 && Shi <= 1.0 && Slo >= 1.0;
  if (inside && clo == chi && A0hi > 0.0) {
    const double m_ = hi - (1.0 - Shi) / A0hi;
    mu = fmin(fmax(m_, lo), hi);
    return 1;
  }
  double nlo = 0.0, nhi = maxb;
  if (lo > 0.0 && Slo >= 1.0) nlo = fmax(nlo, lo);
  if (hi > 0.0 && Shi >= 1.0) nlo = fmax(nlo, hi);
  if (hi > 0.0 && Shi <= 1.0) nhi = fmin(nhi, hi);
  if (lo > 0.0 && Slo <= 1.0) nhi = fmin(nhi, lo);
  if (!(nhi >= nlo)) { nlo = 0.0; nhi = maxb; }
  lo = nlo;
  hi = nhi;
  return inside ? 0 : 3;
}

// Multisection for the periods with need[t] != 0 (caller synchronised; S(lo) >= 1 >= S(hi)).
// absb/inva: LDS staging [P][nw] of |b| and 1/a for the owned assets.
__device__ bool multisect(Ctx& c, int P, const double* absb, const double* inva, int nw,
                          int* need, double* lo, double* hi, double* mu, int* rounds_out) {
  for (int round = 0; round < MS_ROUNDS; ++round) {
    int any = 0;
    for (int t = 0; t < P; ++t) any |= need[t];
    if (!any) return true;
    if (c.tid == 0) ++*rounds_out;
    for (int e = c.tid; e < P * MSC; e += TB) {
      const int t = e / MSC, q = e % MSC;
      double S = 0.0, A0 = 0.0, cnt = 0.0;
      if (need[t]) {
        const double cq = lo[t] + (hi[t] - lo[t]) * (double)q / (double)(MSC - 1);
        for (int li = 0; li < c.nwa; ++li) {
          const double ab = absb[t * nw + li];
          if (ab > cq) {
            const double ia = inva[t * nw + li];
            S = fma(ab - cq, ia, S);
            A0 += ia;
            cnt += 1.0;
          }
        }
      }
      put(c, 3 * e + 0, S);
      put(c, 3 * e + 1, A0);
      put(c, 3 * e + 2, cnt);
    }
    if (!xsync(c, 3 * P * MSC)) return false;
    if (c.tid == 0) {
      for (int t = 0; t < P; ++t) {
        if (!need[t]) continue;
        const double* T0 = c.tot + 3 * t * MSC;
        int qs = 0;
        for (int q = 0; q < MSC; ++q)
          if (T0[3 * q] >= 1.0) qs = q;
        const double cq = lo[t] + (hi[t] - lo[t]) * (double)qs / (double)(MSC - 1);
        if (qs == MSC - 1) { mu[t] = hi[t]; need[t] = 0; continue; }
        const double cn = lo[t] + (hi[t] - lo[t]) * (double)(qs + 1) / (double)(MSC - 1);
        const bool linear = T0[3 * qs + 2] == T0[3 * (qs + 1) + 2];
        const bool tiny = (cn - cq) <= 4.0 * 2.220446049250313e-16 * fabs(cn);
        if (linear || tiny || round == MS_ROUNDS - 1) {
          const double m_ = T0[3 * qs + 1] > 0.0 ? cq + (T0[3 * qs] - 1.0) / T0[3 * qs + 1] : cq;
          mu[t] = fmin(fmax(m_, cq), cn);
          need[t] = 0;
        } else {
          lo[t] = cq;
          hi[t] = cn;
        }
      }
    }
    __syncthreads();
  }
  return true;
}

// Bracket policy after a decision r (see bracket_decide): width kept on a hit, shrunk
// when breakpoints fell inside, grown when the root was outside.
__device__ __forceinline__ double adapt_width(int r, double w) {
  if (r == 1 || r == 2) return w;
  if (r == 0) return fmax(w * 0.7, 1e-13);
  return fmin(w * 1.6, 0.5);
}

// Next bracket around the trend prediction mu + (mu - mu_prev).
__device__ __forceinline__ void next_bracket(double mu, double mprev, double w, double& lo, double& hi) {
  if (mu <= 0.0) { lo = 0.0; hi = 0.0; return; }
  const double ctr = fmax(mu + (mu - mprev), 0.5 * mu);
  lo = fmax(ctr - w * mu, 0.0);
  hi = ctr + w * mu;
}

// ---------------------------------------------------------------------------------
// The kernel
// ---------------------------------------------------------------------------------
struct Scal {   // uniform scalars kept in LDS (identical in every workgroup)
  double omega, eta, r0, rprev;
  long long it, kk, restarts, spec_miss, checks;
  int done, status, restart, ms_rounds;
};

__global__ __launch_bounds__(TB) void k_solve(DevProblem p, DevState s, DevControl ctl) {
  extern __shared__ double lds[];
  const int P = p.P, nr = p.nr, n = p.n, Tp = p.Tp, nw = ctl.nw;
  Ctx c;
  c.wg = blockIdx.x;
  c.nwg = gridDim.x;
  c.tid = threadIdx.x;
  c.i0 = c.wg * nw;
  c.nwa = max(0, min(nw, n - c.i0));
  c.epoch = 0;
  c.xbuf = s.xbuf;
  c.xmax = s.xmax;
  c.bar = s.bar;
  c.vmax = ctl.vmax;
  c.xmode = ctl.xmode;
  c.P = P;
  c.spin_limit = ctl.spin_limit;
  c.t_wait = 0;

  // LDS layout (doubles); must match solve_lds_bytes
  double* ptr = lds;
  double* Kl = nullptr;
  if (ctl.lds_k) { Kl = ptr; ptr += (size_t)nr * nw; }
  double* ys = ptr;   ptr += P * nr;
  double* ys0 = ptr;  ptr += P * nr;
  double* Tys = ptr;  ptr += P * nr;
  double* ysL = ptr;  ptr += P * nr;
  double* Kx = ptr;   ptr += P * nr;          // K~ xbar rows (exchanged)
  double* xv1 = ptr;  ptr += P * nw;          // staging (also multisection |b|)
  double* xv2 = ptr;  ptr += P * nw;          // staging (also multisection 1/a)
  double* tot = ptr;  ptr += ctl.vmax;
  double* red = ptr;  ptr += 256;
  double* lo = ptr;   ptr += P;
  double* hi = ptr;   ptr += P;
  double* mu = ptr;   ptr += P;
  double* mpv = ptr;  ptr += P;               // previous mu (trend)
  double* wid = ptr;  ptr += P;               // relative bracket width
  double* dlo = ptr;  ptr += P;               // dual-inner bracket
  double* dhi = ptr;  ptr += P;
  double* dmu = ptr;  ptr += P;
  double* dmp = ptr;  ptr += P;
  double* dwd = ptr;  ptr += P;
  double* mxb = ptr;  ptr += P;
  S V;
  V.p = &p;
  V.nw = nw;
  V.i0 = c.i0;
  if (ctl.lds_state) {
    Arr a{nullptr, nw, 0};
    auto take = [&](int rows) { Arr r{ptr, nw, 0}; ptr += (size_t)rows * nw; return r; };
    (void)a;
    V.xs = take(P); V.x0s = take(P); V.Txs = take(P); V.xL = take(P); V.bb = take(P); V.aa = take(P);
    V.xb = take(P);
    V.ysC = take(Tp); V.ys0C = take(Tp); V.TysC = take(Tp); V.ysCL = take(Tp);
    V.alpha = take(P); V.ca = take(Tp); V.cb = take(Tp); V.drC = take(Tp);
    V.dc = take(1); V.arisk = take(1); V.cvec = take(1); V.w0 = take(1); V.wT = take(1);
  } else {
    auto g = [&](const double* b) { return Arr{(double*)b, n, c.i0}; };
    V.xs = g(s.xs); V.x0s = g(s.x0s); V.Txs = g(s.Txs); V.xL = g(s.xL); V.bb = g(s.bb); V.aa = g(s.aa);
    V.xb = g(s.vpow);
    V.ysC = g(s.ysC); V.ys0C = g(s.ys0C); V.TysC = g(s.TysC); V.ysCL = g(s.ysCL);
    V.alpha = g(p.alpha); V.ca = g(p.ca); V.cb = g(p.cb); V.drC = g(p.drC);
    V.dc = g(p.dc); V.arisk = g(p.arisk); V.cvec = g(p.cvec); V.w0 = g(p.w0);
    V.wT = g(p.wT ? p.wT : p.w0);
  }
  Scal* sc = (Scal*)ptr; ptr += (sizeof(Scal) + 7) / 8;
  int* iflag = (int*)ptr; ptr += 1;
  int* need = (int*)ptr;
  c.tot = tot;
  c.red = red;
  c.flag = iflag;
  V.Kl = Kl;

  if (Kl) {
    for (int e = c.tid; e < nr * nw; e += TB) {
      const int j = e / nw, li = e % nw;
      Kl[e] = li < c.nwa ? p.K[(size_t)j * p.ldk + c.i0 + li] : 0.0;
    }
  }
  if (ctl.lds_state) {
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      V.alpha(t, li) = p.alpha[(size_t)t * n + c.i0 + li];
    }
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const size_t ix = (size_t)t * n + c.i0 + li;
      V.ca(t, li) = p.ca[ix]; V.cb(t, li) = p.cb[ix]; V.drC(t, li) = p.drC[ix];
    }
    for (int li = c.tid; li < c.nwa; li += TB) {
      const int i = c.i0 + li;
      V.dc(0, li) = p.dc[i]; V.arisk(0, li) = p.arisk[i]; V.cvec(0, li) = p.cvec[i];
      V.w0(0, li) = p.w0[i]; V.wT(0, li) = p.wT ? p.wT[i] : 0.0;
    }
  }
  for (int e = c.tid; e < P * nr; e += TB) { ys[e] = 0.0; ys0[e] = 0.0; Tys[e] = 0.0; ysL[e] = 0.0; Kx[e] = 0.0; }
  if (c.tid == 0) {
    sc->omega = 1.0; sc->it = 0; sc->kk = 0; sc->restarts = 0; sc->spec_miss = 0; sc->checks = 0;
    sc->r0 = -1.0; sc->rprev = INFINITY; sc->done = 0; sc->status = DS_RUNNING; sc->restart = 0;
    sc->ms_rounds = 0;
    for (int t = 0; t < P; ++t) {
      lo[t] = 0.0; hi[t] = 0.0; mu[t] = 0.0; mpv[t] = 0.0; wid[t] = 1e-3;
      dlo[t] = 0.0; dhi[t] = 0.0; dmu[t] = 0.0; dmp[t] = 0.0; dwd[t] = 1e-3;
      need[t] = 0;
    }
  }
  __syncthreads();
  // initial primal point w0 in every period, duals zero
  for (int e = c.tid; e < P * c.nwa; e += TB) {
    const int t = e / c.nwa, li = e % c.nwa, i = c.i0 + li;
    const double x = V.w0(0, li) / V.dc(0, li);
    V.xs(t, li) = x; V.x0s(t, li) = x; V.xL(t, li) = x; V.Txs(t, li) = x;
    V.xb(t, li) = 1.0 + 0.25 * (double)((i * 7919 + t * 104729) % 1000) / 1000.0;   // power vector
  }
  for (int e = c.tid; e < Tp * c.nwa; e += TB) {
    const int t = e / c.nwa, li = e % c.nwa;
    V.ysC(t, li) = 0.0; V.ys0C(t, li) = 0.0; V.TysC(t, li) = 0.0; V.ysCL(t, li) = 0.0;
  }
  __syncthreads();
  const long long t_start = wall_clock64();
  long long t_check = 0;

  // ------------------------------------------------------------- power iteration
  // lambda ~ ||K~ v||^2 / ||v||^2 ; v <- K~^T K~ v / (lambda ||v||)  (v kept in xb)
  double lam = 0.0;
  for (int pw = 0; pw < ctl.npow; ++pw) {
    double loc[2] = {0.0, 0.0};
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double x = V.xb(t, li);
      xv1[t * nw + li] = x;
      loc[0] = fma(x, x, loc[0]);
    }
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double u = kx_trade(V, V.xb, t, li);
      loc[1] = fma(u, u, loc[1]);
    }
    wg_sum<2>(c, loc, red + 64);
    if (c.tid == 0) { put(c, 0, red[64]); put(c, 1, red[65]); }
    for (int e = c.tid; e < P * nr; e += TB) put(c, 2 + e, rows_dot(c, V, xv1, nw, e / nr, e % nr));
    if (!xsync(c, 2 + P * nr)) goto barrier_fail;
    {
      const double vv = tot[0];
      double kv = tot[1];
      for (int e = 0; e < P * nr; ++e) kv = fma(tot[2 + e], tot[2 + e], kv);
      lam = vv > 0.0 ? kv / vv : 0.0;
      const double scale = (lam > 0.0 && vv > 0.0) ? 1.0 / (lam * sqrt(vv)) : 1.0;
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double r = kty_rows(V, tot + 2, t, li);
        double uc = kx_trade(V, V.xb, t, li) * V.drC(t, li) * V.dc(0, li);
        if (p.multi) uc -= kx_trade(V, V.xb, t + 1, li) * V.drC(t + 1, li) * V.dc(0, li);
        xv2[t * nw + li] = (r + uc) * scale;
      }
      __syncthreads();
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        V.xb(t, li) = xv2[t * nw + li];
      }
      __syncthreads();
    }
  }
  if (c.tid == 0) sc->eta = ctl.eta_safety / sqrt(fmax(lam, 1e-300));
  __syncthreads();
  const long long t_loop = wall_clock64();

  // ------------------------------------------------------------- main loop
  while (true) {
    const double omega = sc->omega, eta = sc->eta;
    const double tau = eta / omega, sigma = eta * omega;
    const bool check = ((sc->it + 1) % ctl.check_every == 0) || (sc->it + 1 >= ctl.max_iter);

    // Phase A: prox inputs (signed b and 1/a) for owned (t, li).
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double R = kty_rows(V, ys, t, li) + kty_trade(V, V.ysC, t, li);
      const double v = V.xs(t, li) - tau * R;
      const double dci = V.dc(0, li);
      const double a = 1.0 / (tau * dci * dci) + V.arisk(0, li);
      V.bb(t, li) = v / (tau * dci) + V.alpha(t, li) + V.arisk(0, li) * V.cvec(0, li);
      V.aa(t, li) = 1.0 / a;
    }
    __syncthreads();

    // Phase B: the multiplier mu_t and K~ xbar.
    {
      const int oP1 = 8 * P, oP2 = oP1 + P * nr;
      const int VE1 = ctl.spec ? oP2 + P * nr : 8 * P;
      for (int t = 0; t < P; ++t) period_stats(c, V.bb, V.aa, lo[t], hi[t], t, 8 * t);
      if (ctl.spec) {
        // affine pieces at hi: P1 = K~ (2 xhat_s(hi) - xs), P2 = K~ d xhat_s / d mu
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double b = V.bb(t, li), ab = fabs(b), ia = V.aa(t, li), dci = V.dc(0, li);
          const double h = hi[t];
          const double xh = ab > h ? sgn(b) * (ab - h) * ia / dci : 0.0;
          xv1[t * nw + li] = 2.0 * xh - V.xs(t, li);
          xv2[t * nw + li] = ab > h ? -sgn(b) * ia / dci : 0.0;
        }
        __syncthreads();
        for (int e = c.tid; e < P * nr; e += TB) {
          const int t = e / nr, j = e % nr;
          double a1 = 0.0, a2 = 0.0;
          for (int li = 0; li < c.nwa; ++li) {
            const double kv = V.Kat(j, li);
            a1 = fma(kv, xv1[t * nw + li], a1);
            a2 = fma(kv, xv2[t * nw + li], a2);
          }
          put(c, oP1 + e, a1);
          put(c, oP2 + e, a2);
        }
      }
      if (!xsync(c, VE1)) goto barrier_fail;
      for (int t = 0; t < P; ++t) {
        const double mb = get_max(c, t);
        if (c.tid == 0) mxb[t] = mb;
      }
      __syncthreads();
      if (c.tid == 0) {
        int anyfb = 0, anymiss = 0;
        for (int t = 0; t < P; ++t) {
          double l = lo[t], h = hi[t], m_ = 0.0;
          const int r = bracket_decide(tot + 8 * t, mxb[t], l, h, m_);
          wid[t] = adapt_width(r, wid[t]);
          mpv[t] = mu[t];
          if (r == 1) {
            mu[t] = m_;
            need[t] = 0;
          } else if (r == 2) {
            mu[t] = 0.0;
            need[t] = 0;
            anyfb = 1;
          } else {
            lo[t] = l; hi[t] = h;
            need[t] = 1;
            anyfb = 1;
            anymiss = 1;
          }
        }
        // speculative mode recomputes K~ xbar after any miss; two-phase always does
        *iflag = ctl.spec ? anyfb : 1;
        if (anymiss || (ctl.spec && anyfb)) sc->spec_miss++;
      }
      __syncthreads();
      const int redo = *iflag;
      if (!redo) {
        for (int e = c.tid; e < P * nr; e += TB) {
          const int t = e / nr;
          Kx[e] = tot[oP1 + e] + 2.0 * (mu[t] - hi[t]) * tot[oP2 + e];
        }
        __syncthreads();
      } else {
        int any = 0;
        for (int t = 0; t < P; ++t) any |= need[t];
        if (any) {
          for (int e = c.tid; e < P * c.nwa; e += TB) {
            const int t = e / c.nwa, li = e % c.nwa;
            xv1[t * nw + li] = fabs(V.bb(t, li));
            xv2[t * nw + li] = V.aa(t, li);
          }
          __syncthreads();
          if (!multisect(c, P, xv1, xv2, nw, need, lo, hi, mu, &sc->ms_rounds)) goto barrier_fail;
        }
        // exact K~ xbar for every period
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double b = V.bb(t, li), ab = fabs(b);
          const double xh = ab > mu[t] ? sgn(b) * (ab - mu[t]) * V.aa(t, li) / V.dc(0, li) : 0.0;
          xv1[t * nw + li] = 2.0 * xh - V.xs(t, li);
        }
        __syncthreads();
        for (int e = c.tid; e < P * nr; e += TB) put(c, e, rows_dot(c, V, xv1, nw, e / nr, e % nr));
        if (!xsync(c, P * nr)) goto barrier_fail;
        for (int e = c.tid; e < P * nr; e += TB) Kx[e] = tot[e];
        __syncthreads();
      }
      if (c.tid == 0)
        for (int t = 0; t < P; ++t) next_bracket(mu[t], mpv[t], wid[t], lo[t], hi[t]);
      __syncthreads();
    }

    // Phase C: T(z).  Primal: xhat; trades and rows: dual prox.
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double b = V.bb(t, li), ab = fabs(b);
      const double xh = ab > mu[t] ? sgn(b) * (ab - mu[t]) * V.aa(t, li) / V.dc(0, li) : 0.0;
      V.Txs(t, li) = xh;
      V.xb(t, li) = 2.0 * xh - V.xs(t, li);
    }
    __syncthreads();
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double kc = kx_trade(V, V.xb, t, li);
      const double vs = V.ysC(t, li) + sigma * kc;
      const double drc = V.drC(t, li);
      const double bc = trade_offset(V, t, li);
      const double z = vs / (sigma * drc) - bc;
      const double pr = prox_cost(z, 1.0 / (sigma * drc * drc), V.ca(t, li), V.cb(t, li), p.d);
      V.TysC(t, li) = vs - sigma * drc * bc - sigma * drc * pr;
    }
    for (int e = c.tid; e < P * nr; e += TB) {
      const int j = e % nr;
      const double vs = ys[e] + sigma * Kx[e];
      double ny;
      if (j < p.m) {
        const double sd = sigma * p.dr[j];
        ny = vs - sd * fmin(fmax(vs / sd, p.L[j]), p.U[j]);
      } else {
        const double drj = p.dr[j];
        ny = 2.0 * p.g1 * (vs - sigma * drj * p.bF[j - p.m]) / (sigma * drj * drj + 2.0 * p.g1);
      }
      Tys[e] = ny;
    }
    __syncthreads();

    // Checks (FP64): fixed-point residual, relative KKT at T(z), restart decisions.
    if (check) {
      const long long tc0 = wall_clock64();
      // C1 = [16 scalars][P budgets][P*nr K~ Txs][8P dual-inner stats]
      const int oB = 16, oR = 16 + P, oD = oR + P * nr, VC1 = oD + 8 * P;
      double v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double tx = V.Txs(t, li), dx = V.xs(t, li) - tx, dl = tx - V.xL(t, li);
        v[0] = fma(omega * dx, dx, v[0]);
        v[1] = fma(dl, dl, v[1]);
        const double w = V.dc(0, li) * tx, wc = w - V.cvec(0, li);
        v[3] += -V.alpha(t, li) * w + 0.5 * V.arisk(0, li) * wc * wc;
        if (!isfinite(tx)) v[9] += 1.0;
        xv1[t * nw + li] = tx;
      }
      for (int e = c.tid; e < Tp * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double ty = V.TysC(t, li), dy = V.ysC(t, li) - ty, dl = ty - V.ysCL(t, li);
        v[0] = fma(dy / omega, dy, v[0]);
        v[2] = fma(dl, dl, v[2]);
        const double au = fabs(trade_of(V, V.Txs, t, li));
        const double ca = V.ca(t, li), cb = V.cb(t, li);
        v[4] += ca * au + cb * pow(au, p.d);
        const double yc = V.drC(t, li) * ty;   // unscaled trade dual
        v[5] += conj_cost(yc, ca, cb, p.d);
        if (t == 0) v[6] += yc * V.w0(0, li);
        if (p.multi && t == P) v[6] -= yc * V.wT(0, li);
        v[7] = fma(yc, yc, v[7]);
        if (cb <= 0.0 && fabs(yc) > ca) { const double ex = fabs(yc) - ca; v[10] = fma(ex, ex, v[10]); }
        if (!isfinite(ty)) v[9] += 1.0;
      }
      wg_sum<12>(c, v, red + 64);
      if (c.tid == 0) {
        double rows_fp = 0.0, rows_dl = 0.0, rows_y2 = 0.0, rows_dom = 0.0, tflag = 0.0;
        if (c.wg == 0) {
          for (int e = 0; e < P * nr; ++e) {
            const int j = e % nr;
            const double dy = ys[e] - Tys[e], dl = Tys[e] - ysL[e];
            rows_fp += dy * dy / omega;
            rows_dl += dl * dl;
            const double yu = p.dr[j] * Tys[e];
            rows_y2 += yu * yu;
            if (j < p.m) {
              if (isinf(p.L[j]) && yu < 0.0) rows_dom += yu * yu;
              if (isinf(p.U[j]) && yu > 0.0) rows_dom += yu * yu;
            }
          }
          const double el = (double)(wall_clock64() - t_start) / ctl.wall_hz;
          tflag = el > ctl.time_limit_s ? 1.0 : 0.0;
        }
        const double vals[16] = {red[64] + rows_fp, red[65], red[66] + rows_dl, red[67], red[68], red[69],
                                 red[70], red[71] + rows_y2, tflag, red[73], red[74] + rows_dom, 0, 0, 0, 0, 0};
        for (int q = 0; q < 16; ++q) put(c, q, vals[q]);
      }
      __syncthreads();
      for (int t = 0; t < P; ++t) {
        double bv[1] = {0.0};
        for (int li = c.tid; li < c.nwa; li += TB) bv[0] += fabs(V.dc(0, li) * xv1[t * nw + li]);
        wg_sum<1>(c, bv, red + 64);
        if (c.tid == 0) put(c, oB + t, red[64]);
        __syncthreads();
      }
      for (int e = c.tid; e < P * nr; e += TB) put(c, oR + e, rows_dot(c, V, xv1, nw, e / nr, e % nr));
      // dual inner problem: b' = alpha + arisk c - R' (signed, in bb), 1/a' in aa,
      // R' = unscaled K^T Y at T(y).
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double R = (kty_rows(V, Tys, t, li) + kty_trade(V, V.TysC, t, li)) / V.dc(0, li);
        V.bb(t, li) = V.alpha(t, li) + V.arisk(0, li) * V.cvec(0, li) - R;
        V.aa(t, li) = 1.0 / V.arisk(0, li);
      }
      __syncthreads();
      for (int t = 0; t < P; ++t) period_stats(c, V.bb, V.aa, dlo[t], dhi[t], t, oD + 8 * t);
      if (!xsync(c, VC1)) goto barrier_fail;
      double c1s[16];
      for (int q = 0; q < 16; ++q) c1s[q] = tot[q];
      double phi = c1s[3] + c1s[4];
      double pres2 = 0.0, clip2 = 0.0;
      for (int t = 0; t < P; ++t) {
        for (int j = 0; j < nr; ++j) {
          const double val = tot[oR + t * nr + j] / p.dr[j];   // unscaled (A W)_j or (G^T W)_l
          if (j < p.m) {
            const double cl = fmin(fmax(val, p.L[j]), p.U[j]);
            pres2 += (val - cl) * (val - cl);
            clip2 += cl * cl;
          } else {
            const double g = val - p.bF[j - p.m];
            phi += p.g1 * g * g;
          }
        }
        const double ex = fmax(tot[oB + t] - 1.0, 0.0);
        pres2 += ex * ex;
      }
      for (int t = 0; t < P; ++t) {
        const double mb = get_max(c, t);
        if (c.tid == 0) mxb[t] = mb;
      }
      __syncthreads();
      if (c.tid == 0) {
        int anyd = 0;
        for (int t = 0; t < P; ++t) {
          double l = dlo[t], h = dhi[t], m_ = 0.0;
          const int r = bracket_decide(tot + oD + 8 * t, mxb[t], l, h, m_);
          dwd[t] = adapt_width(r, dwd[t]);
          dmp[t] = dmu[t];
          if (r == 1 || r == 2) { dmu[t] = m_; need[t] = 0; }
          else { dlo[t] = l; dhi[t] = h; need[t] = 1; anyd = 1; }
        }
        *iflag = anyd;
      }
      __syncthreads();
      if (*iflag) {
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          xv1[t * nw + li] = fabs(V.bb(t, li));
          xv2[t * nw + li] = V.aa(t, li);
        }
        __syncthreads();
        if (!multisect(c, P, xv1, xv2, nw, need, dlo, dhi, dmu, &sc->ms_rounds)) goto barrier_fail;
      }
      if (c.tid == 0)
        for (int t = 0; t < P; ++t) next_bracket(dmu[t], dmp[t], dwd[t], dlo[t], dhi[t]);
      __syncthreads();
      // C2: inner value sum (a'/2 w^2 - b' w), w = sign(b') max(|b'| - mu', 0) / a'
      {
        double iv[1] = {0.0};
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double b = V.bb(t, li), ab = fabs(b), ia = V.aa(t, li);
          const double w = ab > dmu[t] ? sgn(b) * (ab - dmu[t]) * ia : 0.0;
          iv[0] += 0.5 * w * w / ia - b * w;
        }
        wg_sum<1>(c, iv, red + 64);
        if (c.tid == 0) put(c, 0, red[64]);
        if (!xsync(c, 1)) goto barrier_fail;
      }
      double psi = tot[0] + (double)P * p.crisk[0] - c1s[6] - c1s[5];
      for (int t = 0; t < P; ++t)
        for (int j = 0; j < nr; ++j) {
          const double yu = p.dr[j] * Tys[t * nr + j];
          if (j < p.m) {
            if (yu > 0.0) psi -= (isinf(p.U[j]) ? INFINITY : p.U[j] * yu);
            else if (yu < 0.0) psi -= (isinf(p.L[j]) ? INFINITY : p.L[j] * yu);
          } else {
            psi -= yu * p.bF[j - p.m];
            psi -= yu * yu / (4.0 * p.g1);
          }
        }
      const double rel_pri = sqrt(pres2) / (1.0 + sqrt(clip2));
      const double rel_dual = sqrt(c1s[10]) / (1.0 + sqrt(c1s[7]));
      const double den = fabs(phi) + fabs(psi);
      const double rel_gap = den > 0.0 ? fabs(phi - psi) / den : 0.0;
      const double relkkt = fmax(rel_pri, fmax(rel_dual, rel_gap));
      const double fpr = sqrt(c1s[0]);
      const bool nonfinite = c1s[9] > 0.0 || !isfinite(phi) || !isfinite(relkkt);
      if (c.tid == 0) {
        sc->checks++;
        sc->restart = 0;
        if (c.wg == 0) {
          s.info[IX_RELKKT] = relkkt; s.info[IX_RELPRI] = rel_pri; s.info[IX_RELDUAL] = rel_dual;
          s.info[IX_RELGAP] = rel_gap; s.info[IX_FPR] = fpr; s.info[IX_POBJ] = phi; s.info[IX_DOBJ] = psi;
          if (ctl.verbose)
            printf("[ffo] it %lld kkt %.3e pri %.3e gap %.3e fpr %.3e omega %.3e restarts %lld miss %lld\n",
                   sc->it + 1, relkkt, rel_pri, rel_gap, fpr, omega, sc->restarts, sc->spec_miss);
        }
        if (nonfinite) { sc->done = 1; sc->status = DS_NUMERIC; }
        else if (relkkt <= ctl.tol) { sc->done = 1; sc->status = DS_OK; }
        else if (c1s[8] > 0.0) { sc->done = 1; sc->status = DS_TIMEOUT; }
        else if (sc->it + 1 >= ctl.max_iter) { sc->done = 1; sc->status = DS_NOT_CONVERGED; }
        else {
          if (sc->r0 < 0.0) sc->r0 = fpr;
          const bool rs = (fpr <= ctl.r_suff * sc->r0) ||
                          (fpr <= ctl.r_nec * sc->r0 && fpr > sc->rprev) ||
                          ((double)(sc->kk + 1) >= ctl.r_art * (double)(sc->it + 1));
          sc->rprev = fpr;
          if (rs) {
            const double dxn = sqrt(c1s[1]), dyn = sqrt(c1s[2]);
            if (dxn > 1e-300 && dyn > 1e-300)
              sc->omega = exp(0.5 * log(dyn / dxn) + 0.5 * log(sc->omega));
            sc->r0 = fpr;
            sc->rprev = INFINITY;
            sc->restarts++;
            sc->restart = 1;
            // a restart jumps the iterate: drop the multiplier trend
            for (int t = 0; t < P; ++t) { mpv[t] = mu[t]; next_bracket(mu[t], mu[t], wid[t], lo[t], hi[t]); }
          }
        }
      }
      __syncthreads();
      t_check += wall_clock64() - tc0;
      if (sc->done) {
        const bool bad = sc->status == DS_NUMERIC;
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          s.w_out[(size_t)t * n + c.i0 + li] = V.dc(0, li) * (bad ? V.xL(t, li) : V.Txs(t, li));
        }
        if (s.y_out) {
          double* yA = s.y_out;
          double* yF = s.y_out + (size_t)P * p.m;
          double* yC = s.y_out + (size_t)P * nr;
          if (c.wg == 0)
            for (int e = c.tid; e < P * nr; e += TB) {
              const int t = e / nr, j = e % nr;
              const double yu = p.dr[j] * (bad ? ysL[e] : Tys[e]);
              if (j < p.m) yA[(size_t)t * p.m + j] = yu; else yF[(size_t)t * p.k + (j - p.m)] = yu;
            }
          for (int e = c.tid; e < Tp * c.nwa; e += TB) {
            const int t = e / c.nwa, li = e % c.nwa;
            yC[(size_t)t * n + c.i0 + li] = V.drC(t, li) * (bad ? V.ysCL(t, li) : V.TysC(t, li));
          }
        }
        break;
      }
      if (sc->restart) {
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double x = V.Txs(t, li);
          V.xs(t, li) = x; V.x0s(t, li) = x; V.xL(t, li) = x;
        }
        for (int e = c.tid; e < Tp * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double y = V.TysC(t, li);
          V.ysC(t, li) = y; V.ys0C(t, li) = y; V.ysCL(t, li) = y;
        }
        for (int e = c.tid; e < P * nr; e += TB) { const double y = Tys[e]; ys[e] = y; ys0[e] = y; ysL[e] = y; }
        __syncthreads();
        if (c.tid == 0) { sc->kk = 0; sc->it++; }
        __syncthreads();
        continue;
      }
    }

    // Phase D: reflected Halpern step
    {
      const double kk = (double)sc->kk;
      const double a1 = (kk + 1.0) / (kk + 2.0), a0 = 1.0 / (kk + 2.0), rho = ctl.rho;
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        V.xs(t, li) = a1 * ((1.0 + rho) * V.Txs(t, li) - rho * V.xs(t, li)) + a0 * V.x0s(t, li);
      }
      for (int e = c.tid; e < Tp * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        V.ysC(t, li) = a1 * ((1.0 + rho) * V.TysC(t, li) - rho * V.ysC(t, li)) + a0 * V.ys0C(t, li);
      }
      for (int e = c.tid; e < P * nr; e += TB) ys[e] = a1 * ((1.0 + rho) * Tys[e] - rho * ys[e]) + a0 * ys0[e];
      __syncthreads();
      if (c.tid == 0) { sc->kk++; sc->it++; }
      __syncthreads();
    }
  }

  if (c.wg == 0 && c.tid == 0) {
    const long long t_end = wall_clock64();
    s.info[IX_ITERS] = (double)sc->it;
    s.info[IX_RESTARTS] = (double)sc->restarts;
    s.info[IX_OMEGA] = sc->omega;
    s.info[IX_ETA] = sc->eta;
    s.info[IX_NORMK] = ctl.eta_safety / sc->eta;
    s.info[IX_SPEC_MISS] = (double)sc->spec_miss;
    s.info[IX_EXCHANGES] = (double)c.epoch;
    s.info[IX_CHECKS] = (double)sc->checks;
    s.info[IX_T_WAIT] = (double)c.t_wait / ctl.wall_hz;
    s.info[IX_T_ITER] = (double)(t_end - t_loop) / ctl.wall_hz;
    s.info[IX_T_CHECK] = (double)t_check / ctl.wall_hz;
    s.info[IX_T_POWER] = (double)(t_loop - t_start) / ctl.wall_hz;
    s.info[IX_MS_ROUNDS] = (double)sc->ms_rounds;
    s.status[0] = sc->status;
  }
  return;

barrier_fail:
  if (c.tid == 0) __hip_atomic_store(s.status, (int32_t)DS_BARRIER, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return;
}

}  // namespace

int solve_vmax(const DevProblem& p) {
  const int P = p.P, nr = p.nr;
  int v = 8 * P + 2 * P * nr;                     // speculative exchange
  v = std::max(v, 16 + P + P * nr + 8 * P);       // check exchange
  v = std::max(v, 3 * P * MSC);                   // multisection round
  v = std::max(v, 2 + P * nr);                    // power iteration
  return (v + 63) / 64 * 64;
}

size_t solve_state_doubles(const DevProblem& p, int nw) {
  const size_t P = p.P, Tp = p.Tp;
  return (8 * P + 7 * Tp + 5) * (size_t)nw;
}

size_t solve_lds_bytes(const DevProblem& p, const DevControl& c) {
  const size_t P = p.P, nr = p.nr, nw = c.nw;
  size_t d = 0;
  if (c.lds_k) d += nr * nw;
  d += 5 * P * nr + 2 * P * nw + (size_t)c.vmax + 256 + 11 * P;
  if (c.lds_state) d += solve_state_doubles(p, c.nw);
  d += (sizeof(Scal) + 7) / 8 + 1 + (P + 1) / 2 + 1;
  return d * sizeof(double);
}

int launch_solve(const DevProblem& p, const DevState& s, const DevControl& c, void* stream, size_t lds) {
  void* args[] = {(void*)&p, (void*)&s, (void*)&c};
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_solve, dim3(c.nwg), dim3(TB), args,
                                            (unsigned int)lds, (hipStream_t)stream);
  return e == hipSuccess ? 0 : (int)e;
}

}  // namespace ffo
