// Lockstep batched form of the solver: B single-period instances (paper Section 2.1,
// eq. 1-3) on one shared asset universe, every unconverged instance advancing by one
// iteration of the same restarted, reflected Halpern PDHG per step.
//
// Instance b uses assets [0, n_b) of the universe, so its scaled constraint rows are
// K~_b = diag(dr_b) K diag(dc) restricted to those columns, with K = [A; (F C)^T] shared.
// The two products of an iteration over all instances are therefore matrix products
// with the shared rows:
//   R  = Yhat KD          (B x nr)(nr x n_max),  Yhat[b] = dr_b * y_b     (K~^T y)
//   KX = Xbar KD^T        (B x n_max)(n_max x nr), then times dr_b        (K~ xbar)
// ragged in n (instance b only has its first n_b columns).  Both run on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64: 16 instances x 16 assets or rows per tile), so the
// arithmetic stays in float64.  Everything per instance - the exact L1-budget multiplier,
// the trade duals, the Halpern step, the float64 checks and restarts - runs in one
// workgroup per instance, whose (b, 1/a) pairs sit in LDS.
//
// Instances live in slots (sorted by decreasing n_b; a slot group of 16 is one MFMA tile
// height); at every check the finished instances are compacted out of the slot list and
// the tile lists are rebuilt, so later steps only touch unconverged instances.  The host
// records the kernels of check_every iterations plus the check in one hipGraph and
// replays it until no instance is left.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <cmath>
#include "internal.h"
#include "cost_math.h"

namespace ffo {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 on gfx950 (lane layout checked on the device): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register j of lane l is
// D[4 j + l / 16][l % 16].
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

// Fixed-order sum of NV values over the workgroup; every thread gets the totals.
// red: LDS scratch of (blockDim / 64) * NV doubles.
template <int NV>
__device__ __forceinline__ void bsum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double t = wsum(v[q]);
    if (lane == 0) red[w * NV + q] = t;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i * NV + q];
    v[q] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ unsigned long long wall_clock() { return (unsigned long long)wall_clock64(); }

constexpr int RED_DOUBLES = 16 * 12;   // bsum scratch (up to 16 waves x 12 values)

// Exact multiplier of the weighted L1-ball problem min sum_i (a_i/2 w_i^2 - b_i w_i)
// s.t. sum |w_i| <= 1: mu = 0 if S(0) = sum |b_i|/a_i <= 1, else the root of
// S(mu) = sum max(|b_i| - mu, 0)/a_i = 1.  S is convex, decreasing and piecewise linear,
// so Newton steps converge monotonically from the left and stop exactly when the set
// {|b_i| > mu} no longer changes (the same closed form as on that set); a step from a
// point right of the root lands left of it.  The start is mu_prev (the previous
// iteration's multiplier), whose S and slope the caller summed in its first pass.
// sb / sa: signed b and 1/a (LDS or device memory).  Returns the number of passes.
__device__ int l1_multiplier(const double* sb, const double* sa, int n, double S0, double A0, double C0,
                             double mp, double Sp, double Ap, double Cp, double* red, double& mu) {
  mu = 0.0;
  if (!(S0 > 1.0)) return 0;
  double m, Sm, Am, Cm;
  if (mp > 0.0 && Ap > 0.0) { m = mp; Sm = Sp; Am = Ap; Cm = Cp; }
  else { m = 0.0; Sm = S0; Am = A0; Cm = C0; }
  int passes = 0;
  for (; passes < 100; ++passes) {
    double mn = m + (Sm - 1.0) / Am;
    if (!(mn > 0.0)) mn = 0.0;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double ab = fabs(sb[i]);
      if (ab > mn) { const double ia = sa[i]; v[0] = fma(ab - mn, ia, v[0]); v[1] += ia; v[2] += 1.0; }
    }
    bsum<3>(v, red);
    const bool from_left = Sm >= 1.0;
    if ((from_left && v[2] == Cm) || mn == m) { m = mn; break; }
    m = mn; Sm = v[0]; Am = v[1]; Cm = v[2];
    if (!(Am > 0.0)) { m = 0.0; Sm = S0; Am = A0; Cm = C0; }
  }
  mu = m;
  return passes + 1;
}

// ---------------------------------------------------------------------------------
// Initial state: x = w0 / dc (w0 in every instance, paper Section 4.1), duals zero, the
// power-iteration vector in xbar.
__global__ __launch_bounds__(256) void k_init(LsShared S) {
  const int slot = blockIdx.x;
  if (slot >= S.B) return;
  const int b = S.act[slot];
  const int64_t o = S.offs[b];
  const int n = S.nb[b];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double x = S.w0[o + i] / S.dc[i];
    S.x[o + i] = x;
    S.x0[o + i] = x;
    S.yC[o + i] = 0.0;
    S.yC0[o + i] = 0.0;
    S.xbar[o + i] = 1.0 + 0.25 * (double)(((int64_t)i * 7919) % 1000) / 1000.0;
  }
  for (int r = threadIdx.x; r < S.nrp; r += blockDim.x) {
    const size_t e = (size_t)b * S.nrp + r;
    S.y[e] = 0.0; S.y0[e] = 0.0; S.Ty[e] = 0.0; S.yh[e] = 0.0; S.yhT[e] = 0.0;
  }
  if (threadIdx.x == 0) {
    LsInst I{};
    I.omega = 1.0; I.eta = 0.0; I.mu = 0.0; I.r0 = -1.0; I.rprev = INFINITY; I.lam = 0.0; I.kvr = 0.0;
    I.it = 0; I.kk = 0; I.restarts = 0; I.checks = 0; I.done = 0; I.status = DS_RUNNING;
    S.inst[b] = I;
    S.status[b] = DS_RUNNING;
  }
}

// ---------------------------------------------------------------------------------
// Slot compaction and tile lists (one workgroup of 1024 threads).  Finished instances
// leave the slot list (stable, so slots stay sorted by decreasing n_b); then
//   K~^T y tiles: (asset block of 64, first group, end group) for every asset block
//     and every run of gpt groups whose largest instance reaches that block;
//   K~ x tiles: (chunk of ch assets, group) for every chunk the group's largest
//     instance reaches.
constexpr int CT = 1024;

__device__ int block_excl_scan(int v, int* sh, int& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < CT; o <<= 1) {
    const int a = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  total = sh[CT - 1];
  const int incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(CT) void k_compact(LsShared S) {
  __shared__ int sh[CT];
  const int t = threadIdx.x;
  const int nold = S.cnt[0];
  int base = 0;
  for (int c0 = 0; c0 < nold; c0 += CT) {
    const int idx = c0 + t;
    const int b = idx < nold ? S.act[idx] : -1;
    const int keep = (b >= 0 && !S.inst[b].done) ? 1 : 0;
    int tot = 0;
    const int pos = block_excl_scan(keep, sh, tot);
    if (keep) S.act[base + pos] = b;
    base += tot;
    __syncthreads();
  }
  const int nact = base;
  const int G = (nact + 15) / 16;
  auto nfirst = [&](int g) { return S.nb[S.act[16 * g]]; };
  // K~^T y tiles
  const int nab = G > 0 ? (nfirst(0) + 63) / 64 : 0;
  int tA = 0;
  for (int a0 = 0; a0 < nab; a0 += CT) {
    const int ab = a0 + t;
    int Gab = 0, nt = 0;
    if (ab < nab) {
      int lo = 0, hi = G;   // groups with n_first > 64 ab form a prefix
      while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (nfirst(mid) > 64 * ab) lo = mid + 1; else hi = mid;
      }
      Gab = lo;
      nt = (Gab + S.gpt - 1) / S.gpt;
    }
    int tot = 0;
    const int pos = block_excl_scan(nt, sh, tot);
    for (int q = 0; q < nt; ++q) {
      const int e = tA + pos + q;
      S.tileA[3 * e] = ab;
      S.tileA[3 * e + 1] = q * S.gpt;
      S.tileA[3 * e + 2] = min(Gab, (q + 1) * S.gpt);
    }
    tA += tot;
    __syncthreads();
  }
  // K~ x tiles
  int tC = 0;
  for (int g0 = 0; g0 < G; g0 += CT) {
    const int g = g0 + t;
    const int nc = g < G ? (nfirst(g) + S.ch - 1) / S.ch : 0;
    int tot = 0;
    const int pos = block_excl_scan(nc, sh, tot);
    for (int q = 0; q < nc; ++q) {
      S.tileC[2 * (tC + pos + q)] = q;
      S.tileC[2 * (tC + pos + q) + 1] = g;
    }
    tC += tot;
    __syncthreads();
  }
  if (t == 0) { S.cnt[0] = nact; S.cnt[1] = tA; S.cnt[2] = tC; S.cnt[3] = G; }
}

// ---------------------------------------------------------------------------------
// R[b][i] = sum_r yin[b][r] KD[r][i] for the slots of each tile's groups and the tile's
// 64 assets (four waves of 16).  The wave keeps its 16 columns of KD in registers and
// runs over the tile's groups; per group one MFMA per 4 rows.
template <int NR4>
__global__ __launch_bounds__(256) void k_kty(LsShared S, const double* __restrict__ yin, double* __restrict__ Rout) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nact = S.cnt[0], ntile = S.cnt[1];
  const int rq = lane >> 4, cl = lane & 15;
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int ab = S.tileA[3 * tile], g0 = S.tileA[3 * tile + 1], g1 = S.tileA[3 * tile + 2];
    const int i = ab * 64 + wave * 16 + cl;
    double kb[NR4];
#pragma unroll
    for (int q = 0; q < NR4; ++q) {
      const int r = 4 * q + rq;
      kb[q] = (q < S.nr4 && r < S.nr && i < S.n_max) ? S.KD[(size_t)r * S.ldk + i] : 0.0;
    }
    for (int g = g0; g < g1; ++g) {
      const int sa = 16 * g + cl;               // A-operand row: slot
      const int ba = sa < nact ? S.act[sa] : -1;
      const double* yrow = yin + (size_t)(ba < 0 ? 0 : ba) * S.nrp;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NR4; ++q) {
        const int r = 4 * q + rq;
        const double a = (ba >= 0 && q < S.nr4 && r < S.nr) ? yrow[r] : 0.0;
        acc = mfma(a, kb[q], acc);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int s = 16 * g + 4 * j + rq;
        if (s < nact) {
          const int b = S.act[s];
          if (i < S.nb[b]) Rout[S.offs[b] + i] = acc[j];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// Partial row sums part[c][s][r] = sum_{i in chunk c, i < n_b} KD[r][i] xin[b][i] for the
// 16 slots s of the tile's group; wave w owns row block w (16 rows), the chunk's inputs
// are staged in LDS (row stride ch + 1).
template <int NRB>
__global__ __launch_bounds__(64 * NRB) void k_kx(LsShared S, const double* __restrict__ xin) {
  extern __shared__ double xs[];   // [16][ch + 1]
  const int lane = threadIdx.x & 63, rb = threadIdx.x >> 6;
  const int nact = S.cnt[0], ntile = S.cnt[2];
  const int ch = S.ch, ld = ch + 1;
  const int rq = lane >> 4, cl = lane & 15;
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int c = S.tileC[2 * tile], g = S.tileC[2 * tile + 1];
    const int i0 = c * ch;
    for (int e = threadIdx.x; e < 16 * ch; e += blockDim.x) {
      const int sl = e / ch, ii = e - sl * ch;
      const int s = 16 * g + sl;
      double v = 0.0;
      if (s < nact) {
        const int b = S.act[s];
        if (i0 + ii < S.nb[b]) v = xin[S.offs[b] + i0 + ii];
      }
      xs[sl * ld + ii] = v;
    }
    __syncthreads();
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const int r = rb * 16 + cl;   // B-operand column: row of KD
    const int iend = min(ch, S.n_max - i0);
    for (int kk = 0; kk < iend; kk += 4) {
      const int ii = kk + rq;
      const double a = ii < iend ? xs[cl * ld + ii] : 0.0;      // A[slot cl][asset rq]
      const double bo = ii < iend ? S.KDT[(size_t)(i0 + ii) * S.nrp + r] : 0.0;
      acc = mfma(a, bo, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = 16 * g + 4 * j + rq;
      if (s < nact) S.part[((size_t)c * S.B + s) * S.nrp + rb * 16 + cl] = acc[j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------
// Row duals per slot (one wave per slot, lanes over rows).  The group's chunks of
// partial sums are added in chunk order: Kx = dr_b * sum_c part[c][s][r] = (K~_b xbar)_r.
// mode 0: T(y) and the reflected Halpern step (y, yh = dr y); then it, kk advance.
// mode 1: T(y) kept in Ty and yhT = dr T(y) (a check follows).
// mode 2: power iteration: u = Kx, yhT = dr u (input of K~^T u), inst.kvr = ||u||^2.
__global__ __launch_bounds__(256) void k_dual(LsShared S, int mode) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = blockIdx.x;
  const int nact = S.cnt[0];
  if (g >= S.cnt[3]) return;
  const int nch = (S.nb[S.act[16 * g]] + S.ch - 1) / S.ch;
  for (int sl = wave; sl < 16; sl += 4) {
    const int s = 16 * g + sl;
    if (s >= nact) break;
    const int b = S.act[s];
    const LsInst I = S.inst[b];
    const double sigma = I.eta * I.omega;
    const double kk = (double)I.kk;
    const double a1 = (kk + 1.0) / (kk + 2.0), a0 = 1.0 / (kk + 2.0), rho = S.rho;
    double kv = 0.0;
    for (int r = lane; r < S.nr; r += 64) {
      double sum = 0.0;
      for (int c = 0; c < nch; ++c) sum += S.part[((size_t)c * S.B + s) * S.nrp + r];
      const double dr = S.drs[(size_t)b * S.nr + r];
      const double kx = dr * sum;
      const size_t e = (size_t)b * S.nrp + r;
      if (mode == 2) {
        S.yhT[e] = dr * kx;
        kv = fma(kx, kx, kv);
        continue;
      }
      const double vs = S.y[e] + sigma * kx;
      double ty;
      if (r < S.m) {
        const double sd = sigma * dr;
        ty = vs - sd * fmin(fmax(vs / sd, S.L[(size_t)b * S.m + r]), S.U[(size_t)b * S.m + r]);
      } else {
        ty = 2.0 * S.g1 * vs / (sigma * dr * dr + 2.0 * S.g1);   // G^T c = 0 (single period)
      }
      if (mode == 1) {
        S.Ty[e] = ty;
        S.yhT[e] = dr * ty;
      } else {
        const double yn = a1 * ((1.0 + rho) * ty - rho * S.y[e]) + a0 * S.y0[e];
        S.y[e] = yn;
        S.yh[e] = dr * yn;
      }
    }
    if (mode == 2) {
      kv = wsum(kv);
      if (lane == 0) S.inst[b].kvr = kv;
    } else if (mode == 0 && lane == 0) {
      S.inst[b].kk = I.kk + 1;
      S.inst[b].it = I.it + 1;
    }
  }
}

// ---------------------------------------------------------------------------------
// Primal step per instance (one workgroup per slot): prox inputs from R = K~^T y,
// the exact budget multiplier, T(x), xbar = 2 T(x) - x, the trade duals T(y_C), and
// (check == 0) the reflected Halpern step on x and y_C, or (check == 1) T(x), T(y_C)
// kept for the check.
__global__ void k_primal(LsShared S, int check) {
  extern __shared__ double lds[];
  double* red = lds;
  const int slot = blockIdx.x;
  if (slot >= S.cnt[0]) return;
  const int b = S.act[slot];
  const int64_t o = S.offs[b];
  const int n = S.nb[b];
  const bool in_lds = n <= S.lds_cap;
  double* sb = in_lds ? lds + RED_DOUBLES : S.gb + o;
  double* sa = in_lds ? lds + RED_DOUBLES + n : S.ga + o;
  const LsInst I = S.inst[b];
  const double tau = I.eta / I.omega, sigma = I.eta * I.omega;
  const double mp = I.mu;
  // pass 1: signed b and 1/a, S and its slope at 0 and at the previous multiplier
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // S0, A0, C0, S(mp), A(mp), C(mp)
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double dci = S.dc[i];
    const double Ry = S.R[o + i] + dci * S.drC[i] * S.yC[o + i];
    const double v = S.x[o + i] - tau * Ry;
    const double a = 1.0 / (tau * dci * dci) + S.arisk[i];
    const double bv = v / (tau * dci) + S.alpha[o + i];
    const double ia = 1.0 / a, ab = fabs(bv);
    sb[i] = bv;
    sa[i] = ia;
    if (ab > 0.0) { acc[0] = fma(ab, ia, acc[0]); acc[1] += ia; acc[2] += 1.0; }
    if (ab > mp) { acc[3] = fma(ab - mp, ia, acc[3]); acc[4] += ia; acc[5] += 1.0; }
  }
  bsum<6>(acc, red);
  double mu = 0.0;
  const int passes = l1_multiplier(sb, sa, n, acc[0], acc[1], acc[2], mp, acc[3], acc[4], acc[5], red, mu);
  // pass 2
  const double kk = (double)I.kk;
  const double a1 = (kk + 1.0) / (kk + 2.0), a0 = 1.0 / (kk + 2.0), rho = S.rho;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double bv = sb[i], ia = sa[i], dci = S.dc[i], ab = fabs(bv);
    const double xh = ab > mu ? sgn(bv) * (ab - mu) * ia / dci : 0.0;
    const double xo = S.x[o + i];
    const double xb = 2.0 * xh - xo;
    S.xbar[o + i] = xb;
    const double drc = S.drC[i];
    const double yco = S.yC[o + i], w0 = S.w0[o + i];
    const double vs = yco + sigma * (drc * dci * xb);
    const double z = vs / (sigma * drc) - w0;
    const double pr = prox_cost(z, 1.0 / (sigma * drc * drc), S.ca[o + i], S.cb[o + i], S.d);
    const double ty = vs - sigma * drc * w0 - sigma * drc * pr;
    if (check) {
      S.Tx[o + i] = xh;
      S.TyC[o + i] = ty;
    } else {
      S.x[o + i] = a1 * ((1.0 + rho) * xh - rho * xo) + a0 * S.x0[o + i];
      S.yC[o + i] = a1 * ((1.0 + rho) * ty - rho * yco) + a0 * S.yC0[o + i];
    }
  }
  if (threadIdx.x == 0) {
    S.inst[b].mu = mu;
    S.inst[b].mu_passes = passes;
  }
}

// ---------------------------------------------------------------------------------
// Power iteration, asset part (one workgroup per slot): with u = K~ v (rows in kvr,
// trade rows u_C = drC dc v), lambda = ||u||^2 / ||v||^2 and
// v <- K~^T u / (lambda ||v||) = (R + drC dc u_C) / (lambda ||v||), R = K~^T u over the
// rows.  step 2 sets the step size eta = 0.95 / sqrt(lambda).
__global__ __launch_bounds__(256) void k_power(LsShared S, int step) {
  __shared__ double red[RED_DOUBLES];
  const int slot = blockIdx.x;
  if (slot >= S.cnt[0]) return;
  const int b = S.act[slot];
  if (step == 2) {
    if (threadIdx.x == 0) S.inst[b].eta = 0.95 / sqrt(fmax(S.inst[b].lam, 1e-300));
    return;
  }
  const int64_t o = S.offs[b];
  const int n = S.nb[b];
  double v2[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = S.xbar[o + i];
    const double uc = S.drC[i] * S.dc[i] * v;
    v2[0] = fma(v, v, v2[0]);
    v2[1] = fma(uc, uc, v2[1]);
  }
  bsum<2>(v2, red);
  const double vv = v2[0];
  const double lam = vv > 0.0 ? (S.inst[b].kvr + v2[1]) / vv : 0.0;
  const double scale = (lam > 0.0 && vv > 0.0) ? 1.0 / (lam * sqrt(vv)) : 1.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = S.xbar[o + i];
    const double dd = S.drC[i] * S.dc[i];
    S.xbar[o + i] = (S.R[o + i] + dd * dd * v) * scale;
  }
  if (threadIdx.x == 0) S.inst[b].lam = lam;
}

// ---------------------------------------------------------------------------------
// Check per instance (one workgroup per slot), all in float64: fixed-point residual,
// relative KKT at T(z) (primal residual of the exposure box and the budget, dual-domain
// distance, gap between Phi and the closed-form dual Psi), then the decision (done /
// restart with the primal-weight update / continue) and its application (the Halpern
// step of this iteration, or the restart to T(z)).  Inputs: Tx, TyC, Ty from the
// check-mode steps, R = K~^T T(y) over the rows, part = partial sums of K T(x) (with
// KD = K diag(dc), so K T(x) = A w and G^T w unscaled).
__global__ void k_check(LsShared S) {
  extern __shared__ double lds[];
  double* red = lds;
  __shared__ int s_dec;
  const int slot = blockIdx.x;
  if (slot >= S.cnt[0]) return;
  const int b = S.act[slot];
  const int64_t o = S.offs[b];
  const int n = S.nb[b];
  const bool in_lds = n <= S.lds_cap;
  double* sb = in_lds ? lds + RED_DOUBLES : S.gb + o;
  double* sa = in_lds ? lds + RED_DOUBLES + n : S.ga + o;
  const LsInst I = S.inst[b];
  const double omega = I.omega;
  const int g = slot / 16;
  const int nch = (S.nb[S.act[16 * g]] + S.ch - 1) / S.ch;
  // assets: v[0] fpr^2, v[1] |dx|^2, v[2] |dy|^2, v[3] phi (linear + quadratic),
  // v[4] costs, v[5] conjugates, v[6] y_C . w0, v[7] |y|^2, v[8] budget, v[9] non-finite,
  // v[10] dual-domain violation^2, v[11] S'(0) of the dual inner problem
  double v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double dci = S.dc[i];
    const double tx = S.Tx[o + i], dx = S.x[o + i] - tx, dl = tx - S.x0[o + i];
    v[0] = fma(omega * dx, dx, v[0]);
    v[1] = fma(dl, dl, v[1]);
    const double w = dci * tx, ar = S.arisk[i];
    v[3] += -S.alpha[o + i] * w + 0.5 * ar * w * w;
    v[8] += fabs(w);
    const double ty = S.TyC[o + i], dy = S.yC[o + i] - ty, dly = ty - S.yC0[o + i];
    v[0] = fma(dy / omega, dy, v[0]);
    v[2] = fma(dly, dly, v[2]);
    const double w0 = S.w0[o + i], ca = S.ca[o + i], cb = S.cb[o + i];
    const double au = fabs(w - w0);
    v[4] += ca * au + cb * pow(au, S.d);
    const double drc = S.drC[i];
    const double yc = drc * ty;
    v[5] += conj_cost(yc, ca, cb, S.d);
    v[6] += yc * w0;
    v[7] = fma(yc, yc, v[7]);
    if (cb <= 0.0 && fabs(yc) > ca) { const double ex = fabs(yc) - ca; v[10] = fma(ex, ex, v[10]); }
    if (!isfinite(tx) || !isfinite(ty)) v[9] += 1.0;
    // dual inner problem at T(y): b' = alpha - (K^T T(y))_i (unscaled), weights a' = arisk
    const double Ry = (S.R[o + i] + dci * drc * ty) / dci;
    const double bp = S.alpha[o + i] - Ry;
    sb[i] = bp;
    sa[i] = 1.0 / ar;
    v[11] = fma(fabs(bp), 1.0 / ar, v[11]);
  }
  // rows: r[0] primal residual^2, r[1] clip^2, r[2] factor risk, r[3] row part of Psi,
  // plus the row duals' share of v[0], v[2], v[7], v[10] (added below)
  double rw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int r = threadIdx.x; r < S.nr; r += blockDim.x) {
    double val = 0.0;
    for (int c = 0; c < nch; ++c) val += S.part[((size_t)c * S.B + slot) * S.nrp + r];
    const size_t e = (size_t)b * S.nrp + r;
    const double dr = S.drs[(size_t)b * S.nr + r];
    const double ty = S.Ty[e], dy = S.y[e] - ty, dl = ty - S.y0[e];
    rw[4] = fma(dy / omega, dy, rw[4]);
    rw[5] = fma(dl, dl, rw[5]);
    const double yu = dr * ty;
    rw[6] = fma(yu, yu, rw[6]);
    if (r < S.m) {
      const double Lj = S.L[(size_t)b * S.m + r], Uj = S.U[(size_t)b * S.m + r];
      const double cl = fmin(fmax(val, Lj), Uj);
      rw[0] = fma(val - cl, val - cl, rw[0]);
      rw[1] = fma(cl, cl, rw[1]);
      if (yu > 0.0) rw[3] -= (isinf(Uj) ? INFINITY : Uj * yu);
      else if (yu < 0.0) rw[3] -= (isinf(Lj) ? INFINITY : Lj * yu);
      if (isinf(Lj) && yu < 0.0) rw[7] = fma(yu, yu, rw[7]);
      if (isinf(Uj) && yu > 0.0) rw[7] = fma(yu, yu, rw[7]);
    } else {
      rw[2] = fma(S.g1 * val, val, rw[2]);
      rw[3] -= yu * yu / (4.0 * S.g1);
    }
    if (!isfinite(ty)) v[9] += 1.0;
  }
  bsum<12>(v, red);
  bsum<8>(rw, red);
  v[0] += rw[4]; v[2] += rw[5]; v[7] += rw[6]; v[10] += rw[7];
  // dual inner problem: min_{||w||_1 <= 1} sum (a'/2 w^2 - b' w) by the same multiplier
  // (its weights are a' = arisk, so 1/a' = sa)
  double cnt0[2] = {0.0, 0.0};   // A'(0), count(0)
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (fabs(sb[i]) > 0.0) { cnt0[0] += sa[i]; cnt0[1] += 1.0; }
  bsum<2>(cnt0, red);
  double mud = 0.0;
  l1_multiplier(sb, sa, n, v[11], cnt0[0], cnt0[1], 0.0, 0.0, 0.0, 0.0, red, mud);
  double iv[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double bp = sb[i], ab = fabs(bp), ia = sa[i];
    const double w = ab > mud ? sgn(bp) * (ab - mud) * ia : 0.0;
    iv[0] += 0.5 * w * w / ia - bp * w;
  }
  bsum<1>(iv, red);
  const double phi = v[3] + v[4] + rw[2];
  const double psi = iv[0] - v[6] - v[5] + rw[3];
  const double ex = fmax(v[8] - 1.0, 0.0);
  const double rel_pri = sqrt(rw[0] + ex * ex) / (1.0 + sqrt(rw[1]));
  const double rel_dual = sqrt(v[10]) / (1.0 + sqrt(v[7]));
  const double den = fabs(phi) + fabs(psi);
  const double rel_gap = den > 0.0 ? fabs(phi - psi) / den : 0.0;
  const double relkkt = fmax(rel_pri, fmax(rel_dual, rel_gap));
  const double fpr = sqrt(v[0]);
  const bool nonfinite = v[9] > 0.0 || !isfinite(phi) || !isfinite(psi) || !isfinite(rel_gap) || !isfinite(relkkt);
  // decision (thread 0), applied by every thread: 0 continue, 1 restart, 2 done
  if (threadIdx.x == 0) {
    LsInst J = I;
    J.checks++;
    int dec = 0;
    const double el = (double)(wall_clock() - S.clock0[0]) / S.wall_hz;
    if (nonfinite) { J.status = DS_NUMERIC; dec = 2; }
    else if (relkkt <= S.tol) { J.status = DS_OK; dec = 2; }
    else if (el > S.time_limit_s) { J.status = DS_TIMEOUT; dec = 2; }
    else if (J.it + 1 >= S.max_iter) { J.status = DS_NOT_CONVERGED; dec = 2; }
    else {
      if (J.r0 < 0.0) J.r0 = fpr;
      const bool rs = (fpr <= S.r_suff * J.r0) || (fpr <= S.r_nec * J.r0 && fpr > J.rprev) ||
                      ((double)(J.kk + 1) >= S.r_art * (double)(J.it + 1));
      J.rprev = fpr;
      if (rs) {
        const double dxn = sqrt(v[1]), dyn = sqrt(v[2]);
        if (dxn > 1e-300 && dyn > 1e-300) J.omega = exp(0.5 * log(dyn / dxn) + 0.5 * log(J.omega));
        J.r0 = fpr;
        J.rprev = INFINITY;
        J.restarts++;
        dec = 1;
      }
    }
    double* inf = S.info + (size_t)b * INFO_LEN;
    inf[IX_RELKKT] = relkkt; inf[IX_RELPRI] = rel_pri; inf[IX_RELDUAL] = rel_dual; inf[IX_RELGAP] = rel_gap;
    inf[IX_FPR] = fpr; inf[IX_POBJ] = phi; inf[IX_DOBJ] = psi;
    if (dec == 2) {
      J.done = 1;
      J.it = J.it + 1;
      inf[IX_ITERS] = (double)J.it;
      inf[IX_RESTARTS] = (double)J.restarts;
      inf[IX_OMEGA] = J.omega;
      inf[IX_ETA] = J.eta;
      inf[IX_NORMK] = 0.95 / J.eta;
      inf[IX_CHECKS] = (double)J.checks;
      inf[IX_T_ITER] = el;
      S.status[b] = J.status;
    }
    S.inst[b] = J;
    s_dec = dec;
  }
  __syncthreads();
  const int dec = s_dec;
  const double kk = (double)I.kk;
  const double a1 = (kk + 1.0) / (kk + 2.0), a0 = 1.0 / (kk + 2.0), rho = S.rho;
  if (dec == 2) {
    const bool bad = S.inst[b].status == DS_NUMERIC;
    for (int i = threadIdx.x; i < n; i += blockDim.x) S.w_out[o + i] = S.dc[i] * (bad ? S.x0[o + i] : S.Tx[o + i]);
    return;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double tx = S.Tx[o + i], ty = S.TyC[o + i];
    if (dec == 1) {
      S.x[o + i] = tx; S.x0[o + i] = tx;
      S.yC[o + i] = ty; S.yC0[o + i] = ty;
    } else {
      S.x[o + i] = a1 * ((1.0 + rho) * tx - rho * S.x[o + i]) + a0 * S.x0[o + i];
      S.yC[o + i] = a1 * ((1.0 + rho) * ty - rho * S.yC[o + i]) + a0 * S.yC0[o + i];
    }
  }
  for (int r = threadIdx.x; r < S.nr; r += blockDim.x) {
    const size_t e = (size_t)b * S.nrp + r;
    const double dr = S.drs[(size_t)b * S.nr + r];
    const double ty = S.Ty[e];
    const double yn = dec == 1 ? ty : a1 * ((1.0 + rho) * ty - rho * S.y[e]) + a0 * S.y0[e];
    S.y[e] = yn;
    if (dec == 1) S.y0[e] = ty;
    S.yh[e] = dr * yn;
  }
  if (threadIdx.x == 0) {
    S.inst[b].kk = dec == 1 ? 0 : I.kk + 1;
    S.inst[b].it = I.it + 1;
  }
}

// KDT[i][r] = KD[r][i] (rows padded to nrp with zeros).
__global__ __launch_bounds__(256) void k_transpose(LsShared S, double* KDT) {
  const int64_t total = (int64_t)S.n_max * S.nrp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / S.nrp), r = (int)(e % S.nrp);
    KDT[e] = r < S.nr ? S.KD[(size_t)r * S.ldk + i] : 0.0;
  }
}

__global__ __launch_bounds__(64) void k_clock(unsigned long long* c) {
  if (threadIdx.x == 0) c[0] = wall_clock();
}

}  // namespace

size_t ls_primal_lds(const LsShared& S) {
  return (size_t)(RED_DOUBLES + 2 * (size_t)S.lds_cap) * sizeof(double);
}

int ls_launch_init(const LsShared& S, void* stream) {
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, (hipStream_t)stream, S.clock0);
  hipLaunchKernelGGL(k_init, dim3(S.B), dim3(256), 0, (hipStream_t)stream, S);
  return (int)hipGetLastError();
}

int ls_launch_compact(const LsShared& S, void* stream) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(CT), 0, (hipStream_t)stream, S);
  return (int)hipGetLastError();
}

int ls_launch_kty(const LsShared& S, const double* yin, double* Rout, int grid, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (S.nr4 <= 8) hipLaunchKernelGGL(k_kty<8>, dim3(grid), dim3(256), 0, st, S, yin, Rout);
  else if (S.nr4 <= 16) hipLaunchKernelGGL(k_kty<16>, dim3(grid), dim3(256), 0, st, S, yin, Rout);
  else if (S.nr4 <= 24) hipLaunchKernelGGL(k_kty<24>, dim3(grid), dim3(256), 0, st, S, yin, Rout);
  else if (S.nr4 <= 32) hipLaunchKernelGGL(k_kty<32>, dim3(grid), dim3(256), 0, st, S, yin, Rout);
  else return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int ls_launch_kx(const LsShared& S, const double* xin, int grid, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const size_t lds = (size_t)16 * (S.ch + 1) * sizeof(double);
  const int nrb = S.nrp / 16;   // one wave per block of 16 rows
  if (nrb <= 2) hipLaunchKernelGGL(k_kx<2>, dim3(grid), dim3(64 * nrb), lds, st, S, xin);
  else if (nrb <= 5) hipLaunchKernelGGL(k_kx<5>, dim3(grid), dim3(64 * nrb), lds, st, S, xin);
  else if (nrb <= 8) hipLaunchKernelGGL(k_kx<8>, dim3(grid), dim3(64 * nrb), lds, st, S, xin);
  else if (nrb <= 16) hipLaunchKernelGGL(k_kx<16>, dim3(grid), dim3(64 * nrb), lds, st, S, xin);
  else return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int ls_launch_dual(const LsShared& S, int mode, void* stream) {
  hipLaunchKernelGGL(k_dual, dim3((S.B + 15) / 16), dim3(256), 0, (hipStream_t)stream, S, mode);
  return (int)hipGetLastError();
}

int ls_launch_primal(const LsShared& S, int check, int threads, void* stream) {
  hipLaunchKernelGGL(k_primal, dim3(S.B), dim3(threads), ls_primal_lds(S), (hipStream_t)stream, S, check);
  return (int)hipGetLastError();
}

int ls_launch_check(const LsShared& S, int threads, void* stream) {
  hipLaunchKernelGGL(k_check, dim3(S.B), dim3(threads), ls_primal_lds(S), (hipStream_t)stream, S);
  return (int)hipGetLastError();
}

int ls_launch_power(const LsShared& S, int step, void* stream) {
  hipLaunchKernelGGL(k_power, dim3(S.B), dim3(256), 0, (hipStream_t)stream, S, step);
  return (int)hipGetLastError();
}

int ls_launch_transpose(const LsShared& S, double* KDT, void* stream) {
  const int64_t total = (int64_t)S.n_max * S.nrp;
  const int grid = (int)std::min<int64_t>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(k_transpose, dim3(std::max(grid, 1)), dim3(256), 0, (hipStream_t)stream, S, KDT);
  return (int)hipGetLastError();
}

}  // namespace ffo
