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
template <class PT>
__device__ int l1_multiplier(PT sb, PT sa, int n, double S0, double A0, double C0, double mp, double Sp, double Ap,
                             double Cp, double* red, double& mu) {
  mu = 0.0;
  if (!(S0 > 1.0)) return 0;
  double m, Sm, Am, Cm;
  if (mp > 0.0 && Ap > 0.0) { m = mp; Sm = Sp; Am = Ap; Cm = Cp; }
  else { m = 0.0; Sm = S0; Am = A0; Cm = C0; }
  const int nt = blockDim.x;
  int passes = 0;
  for (; passes < 100; ++passes) {
    double mn = m + (Sm - 1.0) / Am;
    if (!(mn > 0.0)) mn = 0.0;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i0 = threadIdx.x; i0 < n; i0 += 4 * nt) {   // four pairs per thread and step
      double bq[4], aq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * nt;
        bq[u] = i < n ? sb[i] : 0.0;
        aq[u] = i < n ? sa[i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double ab = fabs(bq[u]);
        if (ab > mn) { v[0] = fma(ab - mn, aq[u], v[0]); v[1] += aq[u]; v[2] += 1.0; }
      }
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

typedef __attribute__((address_space(3))) double ldbl;

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
constexpr int EW = LS_EW;   // assets per element tile (256 threads x 4)

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
  // K~ x tiles: chunks of ch assets, runs of gpt groups that reach the chunk
  const int nchk = G > 0 ? (nfirst(0) + S.ch - 1) / S.ch : 0;
  int tC = 0;
  for (int c0 = 0; c0 < nchk; c0 += CT) {
    const int c = c0 + t;
    int Gc = 0, nt = 0;
    if (c < nchk) {
      int lo = 0, hi = G;
      while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (nfirst(mid) > c * S.ch) lo = mid + 1; else hi = mid;
      }
      Gc = lo;
      nt = (Gc + S.gpt - 1) / S.gpt;
    }
    int tot = 0;
    const int pos = block_excl_scan(nt, sh, tot);
    for (int q = 0; q < nt; ++q) {
      const int e = tC + pos + q;
      S.tileC[3 * e] = c;
      S.tileC[3 * e + 1] = q * S.gpt;
      S.tileC[3 * e + 2] = min(Gc, (q + 1) * S.gpt);
    }
    tC += tot;
    __syncthreads();
  }
  // element tiles of the elementwise passes: (slot, chunk of EW assets), slot-major
  int tE = 0;
  for (int s0 = 0; s0 < nact; s0 += CT) {
    const int sl = s0 + t;
    const int ne = sl < nact ? (S.nb[S.act[sl]] + EW - 1) / EW : 0;
    int tot = 0;
    const int pos = block_excl_scan(ne, sh, tot);
    if (sl < nact) S.eoff[sl] = tE + pos;
    for (int q = 0; q < ne; ++q) {
      S.tileE[2 * (tE + pos + q)] = sl;
      S.tileE[2 * (tE + pos + q) + 1] = q;
    }
    tE += tot;
    __syncthreads();
  }
  if (t == 0) { S.cnt[0] = nact; S.cnt[1] = tA; S.cnt[2] = tC; S.cnt[3] = G; S.cnt[4] = tE; }
}

// ---------------------------------------------------------------------------------
// R[b][i] = sum_r yin[b][r] KD[r][i] for the slots of each tile's groups and the tile's
// 64 assets (four waves of 16).  The wave keeps its 16 columns of KD in registers and
// runs over the tile's groups; per group one MFMA per 4 rows.
constexpr int GPT_MAX = 4;

// PRE: instead of R, the epilogue forms the prox inputs of the primal step from R (as
// k_pre does) and writes per-(asset block, slot) sums of S and its slope to estat2.
template <int NR4, bool PRE>
__global__ __launch_bounds__(256) void k_kty(LsShared S, const double* __restrict__ yin, double* __restrict__ Rout) {
  extern __shared__ double ys[];   // [gpt * 16][nrp + 1] dual rows of the tile's slots
  __shared__ int s_b[GPT_MAX * 16], s_n[GPT_MAX * 16];
  __shared__ int64_t s_o[GPT_MAX * 16];
  __shared__ double s_tau[GPT_MAX * 16], s_mp[GPT_MAX * 16];
  __shared__ double s_st[4][16][6];   // per wave and slot of the group: the six sums
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nact = S.cnt[0], ntile = S.cnt[1];
  const int rq = lane >> 4, cl = lane & 15;
  const int ld = S.nrp + 1;
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int ab = S.tileA[3 * tile], g0 = S.tileA[3 * tile + 1], g1 = S.tileA[3 * tile + 2];
    const int ns = (g1 - g0) * 16;
    const int i = ab * 64 + wave * 16 + cl;
    double kb[NR4];
#pragma unroll
    for (int q = 0; q < NR4; ++q) {
      const int r = 4 * q + rq;
      kb[q] = (q < S.nr4 && r < S.nr && i < S.n_max) ? S.KD[(size_t)r * S.ldk + i] : 0.0;
    }
    double dci = 1.0, drci = 1.0, ari = 1.0;
    if (PRE && i < S.n_max) { dci = S.dc[i]; drci = S.drC[i]; ari = S.arisk[i]; }
    if (threadIdx.x < ns) {
      const int sl = 16 * g0 + threadIdx.x;
      const int b = sl < nact ? S.act[sl] : -1;
      s_b[threadIdx.x] = b;
      s_n[threadIdx.x] = b >= 0 ? S.nb[b] : 0;
      s_o[threadIdx.x] = b >= 0 ? S.offs[b] : 0;
      if (PRE) {
        s_tau[threadIdx.x] = b >= 0 ? S.inst[b].eta / S.inst[b].omega : 1.0;
        s_mp[threadIdx.x] = b >= 0 ? S.inst[b].mu : 0.0;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ns * S.nrp; e += blockDim.x) {
      const int sl = e / S.nrp, r = e - sl * S.nrp;
      const int b = s_b[sl];
      ys[sl * ld + r] = (b >= 0 && r < S.nr) ? yin[(size_t)b * S.nrp + r] : 0.0;
    }
    __syncthreads();
    for (int g = g0; g < g1; ++g) {
      const double* yr = ys + ((g - g0) * 16 + cl) * ld;   // A-operand row: slot 16 g + cl
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NR4; ++q) {
        const double a = q < S.nr4 ? yr[4 * q + rq] : 0.0;
        acc = mfma(a, kb[q], acc);
      }
      if (!PRE) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int sl = (g - g0) * 16 + 4 * j + rq;   // output row: slot 16 g + 4 j + rq
          if (i < s_n[sl]) Rout[s_o[sl] + i] = acc[j];
        }
        continue;
      }
      double yc[4], xv[4], al[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int sl = (g - g0) * 16 + 4 * j + rq;
        const bool in = i < s_n[sl];
        const int64_t oi = s_o[sl] + i;
        yc[j] = in ? S.yC[oi] : 0.0;
        xv[j] = in ? S.x[oi] : 0.0;
        al[j] = in ? S.alpha[oi] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int sl = (g - g0) * 16 + 4 * j + rq;
        double st[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (i < s_n[sl]) {
          const double tau = s_tau[sl], mp = s_mp[sl];
          const double Ry = acc[j] + dci * drci * yc[j];
          const double v = xv[j] - tau * Ry;
          const double a = 1.0 / (tau * dci * dci) + ari;
          const double bv = v / (tau * dci) + al[j];
          const double ia = 1.0 / a, abv = fabs(bv);
          const int64_t oi = s_o[sl] + i;
          S.gb[oi] = bv;
          S.ga[oi] = ia;
          if (abv > 0.0) { st[0] = abv * ia; st[1] = ia; st[2] = 1.0; }
          if (abv > mp) { st[3] = (abv - mp) * ia; st[4] = ia; st[5] = 1.0; }
        }
        // sum over the 16 assets of this wave (lanes with the same rq), fixed order
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          double x = st[q];
          x += __shfl_xor(x, 1, 64);
          x += __shfl_xor(x, 2, 64);
          x += __shfl_xor(x, 4, 64);
          x += __shfl_xor(x, 8, 64);
          if (cl == 0) s_st[wave][4 * j + rq][q] = x;
        }
      }
      __syncthreads();
      if (threadIdx.x < 16 * 6) {
        const int sl16 = threadIdx.x / 6, q = threadIdx.x % 6;
        const int s = 16 * g + sl16;
        if (s < nact) {
          const double t = s_st[0][sl16][q] + s_st[1][sl16][q] + s_st[2][sl16][q] + s_st[3][sl16][q];
          S.estat2[((size_t)ab * S.B + s) * 8 + q] = t;
        }
      }
      __syncthreads();
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------
// Partial row sums part[c][s][r] = sum_{i in chunk c, i < n_b} KD[r][i] xin[b][i] for the
// 16 slots s of the tile's group; wave w owns row block w (16 rows), the chunk's inputs
// are staged in LDS (row stride ch + 1).
// POST: the staged inputs are formed here from the prox inputs (as k_post does): T(x),
// xbar = 2 T(x) - x (the A operand), the trade duals and the Halpern step, or (check)
// T(x), T(y_C) kept.
// XB (more than NRB row blocks): wave rb takes blocks rb, rb + NRB, ..., loading each
// block's rows over the chunk per group instead of keeping one block in registers.
template <int NRB, int CH, bool POST, bool XB = false>
__global__ __launch_bounds__(64 * NRB) void k_kx(LsShared S, const double* __restrict__ xin, int check) {
  __shared__ double xs[16 * (CH + 1)];   // the group's inputs over the chunk, row stride CH + 1
  __shared__ int64_t s_off[16];
  __shared__ int s_n[16];
  __shared__ double s_sig[16], s_mu[16], s_a1[16], s_a0[16];
  const int lane = threadIdx.x & 63, rb = threadIdx.x >> 6;
  const int nact = S.cnt[0], ntile = S.cnt[2];
  constexpr int ld = CH + 1;
  const int rq = lane >> 4, cl = lane & 15;
  const int r = rb * 16 + cl;   // B-operand column: row of KD
  const int nt = blockDim.x;
  const double rho = S.rho;
  const int nrb_all = S.nrp / 16;
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int c = S.tileC[3 * tile], g0 = S.tileC[3 * tile + 1], g1 = S.tileC[3 * tile + 2];
    const int i0 = c * CH;
    // this wave's block of 16 rows over the chunk, kept in registers for all groups
    double bk[XB ? 1 : CH / 4];
    if constexpr (!XB) {
#pragma unroll
      for (int q = 0; q < CH / 4; ++q) {
        const int ii = i0 + 4 * q + rq;
        bk[q] = ii < S.n_max ? S.KDT[(size_t)ii * S.nrp + r] : 0.0;
      }
    }
    for (int g = g0; g < g1; ++g) {
      if (threadIdx.x < 16) {
        const int s = 16 * g + threadIdx.x;
        const int b = s < nact ? S.act[s] : -1;
        s_n[threadIdx.x] = b >= 0 ? S.nb[b] : 0;
        s_off[threadIdx.x] = b >= 0 ? S.offs[b] : 0;
        if (POST && b >= 0) {
          const LsInst I = S.inst[b];
          const double kk = (double)I.kk;
          s_sig[threadIdx.x] = I.eta * I.omega;
          s_mu[threadIdx.x] = I.mu;
          s_a1[threadIdx.x] = (kk + 1.0) / (kk + 2.0);
          s_a0[threadIdx.x] = 1.0 / (kk + 2.0);
        }
      }
      __syncthreads();
      if (!POST) {
        for (int e = threadIdx.x; e < 16 * CH; e += nt) {
          const int sl = e / CH, ii = e - sl * CH;
          xs[sl * ld + ii] = i0 + ii < s_n[sl] ? xin[s_off[sl] + i0 + ii] : 0.0;
        }
      } else {
        for (int e0 = threadIdx.x; e0 < 16 * CH; e0 += 4 * nt) {
          double bvv[4], iav[4], dcv[4], xo[4], drc[4], yco[4], w0v[4], cav[4], cbv[4], x0v[4], y0v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * nt;
            const int sl = e / CH, ii = e - sl * CH;
            const bool in = e < 16 * CH && i0 + ii < s_n[sl];
            const int64_t oi = in ? s_off[sl] + i0 + ii : 0;
            const int i = i0 + ii;
            bvv[u] = in ? S.gb[oi] : 0.0;
            iav[u] = in ? S.ga[oi] : 0.0;
            dcv[u] = in ? S.dc[i] : 1.0;
            xo[u] = in ? S.x[oi] : 0.0;
            drc[u] = in ? S.drC[i] : 1.0;
            yco[u] = in ? S.yC[oi] : 0.0;
            w0v[u] = in ? S.w0[oi] : 0.0;
            cav[u] = in ? S.ca[oi] : 0.0;
            cbv[u] = in ? S.cb[oi] : 0.0;
            x0v[u] = in && !check ? S.x0[oi] : 0.0;
            y0v[u] = in && !check ? S.yC0[oi] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * nt;
            if (e >= 16 * CH) break;
            const int sl = e / CH, ii = e - sl * CH;
            double xb = 0.0;
            if (i0 + ii < s_n[sl]) {
              const int64_t oi = s_off[sl] + i0 + ii;
              const double mu = s_mu[sl], sigma = s_sig[sl];
              const double bv = bvv[u], ia = iav[u], dci = dcv[u], abv = fabs(bv);
              const double xh = abv > mu ? sgn(bv) * (abv - mu) * ia / dci : 0.0;
              xb = 2.0 * xh - xo[u];
              const double dr = drc[u];
              const double vs = yco[u] + sigma * (dr * dci * xb);
              const double z = vs / (sigma * dr) - w0v[u];
              const double pr = prox_cost(z, 1.0 / (sigma * dr * dr), cav[u], cbv[u], S.d);
              const double ty = vs - sigma * dr * w0v[u] - sigma * dr * pr;
              if (check) {
                S.Tx[oi] = xh;
                S.TyC[oi] = ty;
              } else {
                const double a1 = s_a1[sl], a0 = s_a0[sl];
                S.x[oi] = a1 * ((1.0 + rho) * xh - rho * xo[u]) + a0 * x0v[u];
                S.yC[oi] = a1 * ((1.0 + rho) * ty - rho * yco[u]) + a0 * y0v[u];
              }
            }
            xs[sl * ld + ii] = xb;
          }
        }
      }
      __syncthreads();
      if constexpr (!XB) {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < CH / 4; ++q) acc = mfma(xs[cl * ld + 4 * q + rq], bk[q], acc);   // A[slot cl][asset]
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s = 16 * g + 4 * j + rq;
          if (s < nact) S.part[((size_t)c * S.B + s) * S.nrp + r] = acc[j];
        }
      }
      if constexpr (XB) {
#pragma unroll 1
        for (int rb2 = rb; rb2 < nrb_all; rb2 += NRB) {
          const int r2 = rb2 * 16 + cl;
          d4 acc2 = {0.0, 0.0, 0.0, 0.0};
          // sixteen steps' rows at a time (a whole block's would not fit the registers)
#pragma unroll 1
          for (int q0 = 0; q0 < CH / 4; q0 += 16) {
            double bk2[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
              const int ii = i0 + 4 * (q0 + q) + rq;
              bk2[q] = ii < S.n_max ? S.KDT[(size_t)ii * S.nrp + r2] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) acc2 = mfma(xs[cl * ld + 4 * (q0 + q) + rq], bk2[q], acc2);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int s = 16 * g + 4 * j + rq;
            if (s < nact) S.part[((size_t)c * S.B + s) * S.nrp + r2] = acc2[j];
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------
// Row duals per slot (one workgroup per slot, threads over rows).  The group's chunks of
// partial sums are added in chunk order: Kx = dr_b * sum_c part[c][s][r] = (K~_b xbar)_r.
// mode 0: T(y) and the reflected Halpern step (y, yh = dr y); then it, kk advance.
// mode 1: T(y) kept in Ty and yhT = dr T(y) (a check follows).
// mode 2: power iteration: u = Kx, yhT = dr u (input of K~^T u), inst.kvr = ||u||^2.
__global__ __launch_bounds__(128) void k_dual(LsShared S, int mode) {
  __shared__ double red[2];
  const int slot = blockIdx.x;
  if (slot >= S.cnt[0]) return;
  const int b = S.act[slot];
  const int g = slot / 16;
  const int nch = (S.nb[S.act[16 * g]] + S.ch - 1) / S.ch;
  const LsInst I = S.inst[b];
  const double sigma = I.eta * I.omega;
  const double kk = (double)I.kk;
  const double a1 = (kk + 1.0) / (kk + 2.0), a0 = 1.0 / (kk + 2.0), rho = S.rho;
  double kv = 0.0;
  for (int r = threadIdx.x; r < S.nr; r += blockDim.x) {
    const double* pc = S.part + (size_t)slot * S.nrp + r;
    const size_t cstride = (size_t)S.B * S.nrp;
    double sum = 0.0;
    int c = 0;
    for (; c + 8 <= nch; c += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pc[(size_t)(c + u) * cstride];
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += v[u];
    }
    for (; c < nch; ++c) sum += pc[(size_t)c * cstride];
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
      const double Lr = S.L[(size_t)b * S.m + r], Ur = S.U[(size_t)b * S.m + r];
      ty = vs - sd * fmin(fmax(vs / sd, Lr), Ur);
      if (isinf(Ur) && ty > 0.0) ty = 0.0;   // an infinite side fixes the dual's sign exactly
      if (isinf(Lr) && ty < 0.0) ty = 0.0;
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
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = kv;
    __syncthreads();
    if (threadIdx.x == 0) S.inst[b].kvr = red[0] + (blockDim.x > 64 ? red[1] : 0.0);
  } else if (mode == 0 && threadIdx.x == 0) {
    S.inst[b].kk = I.kk + 1;
    S.inst[b].it = I.it + 1;
  }
}

// ---------------------------------------------------------------------------------
// Primal step, in three kernels:
//   k_pre  (element tiles): prox inputs b, 1/a from R = K~^T y and the tile's sums of
//          S and its slope at 0 and at the previous multiplier;
//   k_mu   (one workgroup per instance): the exact budget multiplier;
//   k_post (element tiles): T(x), xbar = 2 T(x) - x, the trade duals T(y_C), and either
//          the reflected Halpern step on x and y_C (check == 0) or T(x), T(y_C) kept for
//          the check.
__global__ __launch_bounds__(256) void k_pre(LsShared S) {
  __shared__ double red[RED_DOUBLES];
  const int ntile = S.cnt[4];
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int slot = S.tileE[2 * tile], ec = S.tileE[2 * tile + 1];
    const int b = S.act[slot];
    const int64_t o = S.offs[b];
    const int n = S.nb[b];
    const double eta = S.inst[b].eta, omega = S.inst[b].omega, mp = S.inst[b].mu;
    const double tau = eta / omega;
    const int iend = min(n, (ec + 1) * EW);
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // S0, A0, C0, S(mp), A(mp), C(mp)
    double Rv[4], yc[4], xv[4], al[4], dcv[4], drc[4], ar[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = ec * EW + threadIdx.x + u * 256;
      const bool in = i < iend;
      Rv[u] = in ? S.R[o + i] : 0.0;
      yc[u] = in ? S.yC[o + i] : 0.0;
      xv[u] = in ? S.x[o + i] : 0.0;
      al[u] = in ? S.alpha[o + i] : 0.0;
      dcv[u] = in ? S.dc[i] : 1.0;
      drc[u] = in ? S.drC[i] : 1.0;
      ar[u] = in ? S.arisk[i] : 1.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = ec * EW + threadIdx.x + u * 256;
      if (i < iend) {
        const double dci = dcv[u];
        const double Ry = Rv[u] + dci * drc[u] * yc[u];
        const double v = xv[u] - tau * Ry;
        const double a = 1.0 / (tau * dci * dci) + ar[u];
        const double bv = v / (tau * dci) + al[u];
        const double ia = 1.0 / a, ab = fabs(bv);
        S.gb[o + i] = bv;
        S.ga[o + i] = ia;
        if (ab > 0.0) { acc[0] = fma(ab, ia, acc[0]); acc[1] += ia; acc[2] += 1.0; }
        if (ab > mp) { acc[3] = fma(ab - mp, ia, acc[3]); acc[4] += ia; acc[5] += 1.0; }
      }
    }
    bsum<6>(acc, red);
    if (threadIdx.x < 6) S.estat[(size_t)tile * 8 + threadIdx.x] = acc[threadIdx.x];
  }
}

__global__ __launch_bounds__(512) void k_mu(LsShared S, int fused) {
  extern __shared__ double lds[];
  double* red = lds;
  const int slot = blockIdx.x;
  if (slot >= S.cnt[0]) return;
  const int b = S.act[slot];
  const int64_t o = S.offs[b];
  const int n = S.nb[b];
  const double mp = S.inst[b].mu;
  // the first pass's sums for this instance, added in tile order: element tiles (split
  // form) or 64-asset blocks (fused form)
  double acc[6];
  if (!fused) {
    const int t0 = S.eoff[slot], nt = (n + EW - 1) / EW;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      double v = 0.0;
      for (int t = 0; t < nt; ++t) v += S.estat[(size_t)(t0 + t) * 8 + q];
      acc[q] = v;
    }
  } else {
    const int nab = (n + 63) / 64;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < nab; t += blockDim.x) {   // per thread in block order, then
#pragma unroll                                              // a fixed-order workgroup sum
      for (int q = 0; q < 6; ++q) v[q] += S.estat2[((size_t)t * S.B + slot) * 8 + q];
    }
    bsum<6>(v, red);
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[q] = v[q];
  }
  // the (b, 1/a) pairs move to LDS when they fit (every multiplier pass reads them)
  const bool in_lds = n <= S.lds_cap;
  double mu = 0.0;
  int passes = 0;
  if (acc[0] > 1.0) {
    const double* gb = S.gb + o;
    const double* ga = S.ga + o;
    if (in_lds) {
      ldbl* sb = (ldbl*)(lds + RED_DOUBLES);
      ldbl* sa = sb + n;
      const int nt = blockDim.x;
      // sixteen pairs per thread and step: the copy of an 8000-asset instance is one or
      // two round trips to memory instead of four to eight
      for (int i0 = threadIdx.x; i0 < n; i0 += 16 * nt) {
        double bq[16], aq[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int i = i0 + u * nt;
          bq[u] = i < n ? gb[i] : 0.0;
          aq[u] = i < n ? ga[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int i = i0 + u * nt;
          if (i < n) { sb[i] = bq[u]; sa[i] = aq[u]; }
        }
      }
      __syncthreads();
      passes = l1_multiplier((const ldbl*)sb, (const ldbl*)sa, n, acc[0], acc[1], acc[2], mp, acc[3], acc[4],
                             acc[5], red, mu);
    } else {
      passes = l1_multiplier(gb, ga, n, acc[0], acc[1], acc[2], mp, acc[3], acc[4], acc[5], red, mu);
    }
  }
  if (threadIdx.x == 0) {
    S.inst[b].mu = mu;
    S.inst[b].mu_passes = passes;
    S.inst[b].mu_passes_sum += passes;
  }
}

__global__ __launch_bounds__(256) void k_post(LsShared S, int check) {
  const int ntile = S.cnt[4];
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int slot = S.tileE[2 * tile], ec = S.tileE[2 * tile + 1];
    const int b = S.act[slot];
    const int64_t o = S.offs[b];
    const int n = S.nb[b];
    const LsInst I = S.inst[b];
    const double sigma = I.eta * I.omega, mu = I.mu;
    const double kk = (double)I.kk;
    const double a1 = (kk + 1.0) / (kk + 2.0), a0 = 1.0 / (kk + 2.0), rho = S.rho;
    const int iend = min(n, (ec + 1) * EW);
    double bvv[4], iav[4], dcv[4], xo[4], drc[4], yco[4], w0v[4], cav[4], cbv[4], x0v[4], y0v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = ec * EW + threadIdx.x + u * 256;
      const bool in = i < iend;
      bvv[u] = in ? S.gb[o + i] : 0.0;
      iav[u] = in ? S.ga[o + i] : 0.0;
      dcv[u] = in ? S.dc[i] : 1.0;
      xo[u] = in ? S.x[o + i] : 0.0;
      drc[u] = in ? S.drC[i] : 1.0;
      yco[u] = in ? S.yC[o + i] : 0.0;
      w0v[u] = in ? S.w0[o + i] : 0.0;
      cav[u] = in ? S.ca[o + i] : 0.0;
      cbv[u] = in ? S.cb[o + i] : 0.0;
      x0v[u] = in && !check ? S.x0[o + i] : 0.0;
      y0v[u] = in && !check ? S.yC0[o + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = ec * EW + threadIdx.x + u * 256;
      if (i < iend) {
        const double bv = bvv[u], ia = iav[u], dci = dcv[u], ab = fabs(bv);
        const double xh = ab > mu ? sgn(bv) * (ab - mu) * ia / dci : 0.0;
        const double xb = 2.0 * xh - xo[u];
        S.xbar[o + i] = xb;
        const double dr = drc[u];
        const double vs = yco[u] + sigma * (dr * dci * xb);
        const double z = vs / (sigma * dr) - w0v[u];
        const double pr = prox_cost(z, 1.0 / (sigma * dr * dr), cav[u], cbv[u], S.d);
        const double ty = vs - sigma * dr * w0v[u] - sigma * dr * pr;
        if (check) {
          S.Tx[o + i] = xh;
          S.TyC[o + i] = ty;
        } else {
          S.x[o + i] = a1 * ((1.0 + rho) * xh - rho * xo[u]) + a0 * x0v[u];
          S.yC[o + i] = a1 * ((1.0 + rho) * ty - rho * yco[u]) + a0 * y0v[u];
        }
      }
    }
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
__global__ __launch_bounds__(512) void k_check(LsShared S) {
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
      inf[IX_MS_ROUNDS] = (double)J.mu_passes_sum;   // multiplier passes over the elements
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

// The current iterate of instance b in unscaled coordinates, as a warm start of the
// plain solver: w [n_b] = dc x, and the duals in its y layout [m rows][k rows][n_b
// trades] (row r: dr_r y_r; trade i: drC_i yC_i).
__global__ void k_export(LsShared S, int b, double* __restrict__ w, double* __restrict__ y) {
  const int64_t o = S.offs[b];
  const int n = S.nb[b];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    w[i] = S.dc[i] * S.x[o + i];
    y[S.nr + i] = S.drC[i] * S.yC[o + i];
  }
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < S.nr; r += gridDim.x * blockDim.x)
    y[r] = S.drs[(size_t)b * S.nr + r] * S.y[(size_t)b * S.nrp + r];
}

int ls_launch_export(const LsShared& S, int b, int n_b, double* w, double* y, void* stream) {
  const int grid = std::max(1, std::min(256, (n_b + 255) / 256));
  hipLaunchKernelGGL(k_export, dim3(grid), dim3(256), 0, (hipStream_t)stream, S, b, w, y);
  return (int)hipGetLastError();
}

int ls_launch_compact(const LsShared& S, void* stream) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(CT), 0, (hipStream_t)stream, S);
  return (int)hipGetLastError();
}

template <bool PRE>
static int launch_kty_t(const LsShared& S, const double* yin, double* Rout, int grid, hipStream_t st) {
  const size_t lds = (size_t)GPT_MAX * 16 * (S.nrp + 1) * sizeof(double);
  if (S.gpt > GPT_MAX) return (int)hipErrorInvalidValue;
  if (S.nr4 <= 8) hipLaunchKernelGGL((k_kty<8, PRE>), dim3(grid), dim3(256), lds, st, S, yin, Rout);
  else if (S.nr4 <= 16) hipLaunchKernelGGL((k_kty<16, PRE>), dim3(grid), dim3(256), lds, st, S, yin, Rout);
  else if (S.nr4 <= 24) hipLaunchKernelGGL((k_kty<24, PRE>), dim3(grid), dim3(256), lds, st, S, yin, Rout);
  else if (S.nr4 <= 32) hipLaunchKernelGGL((k_kty<32, PRE>), dim3(grid), dim3(256), lds, st, S, yin, Rout);
  else if (S.nr4 <= 40) hipLaunchKernelGGL((k_kty<40, PRE>), dim3(grid), dim3(256), lds, st, S, yin, Rout);
  else return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int ls_launch_kty(const LsShared& S, const double* yin, double* Rout, int grid, void* stream) {
  return launch_kty_t<false>(S, yin, Rout, grid, (hipStream_t)stream);
}

template <bool POST>
static int launch_kx_t(const LsShared& S, const double* xin, int check, int grid, hipStream_t st) {
  const int nrb = S.nrp / 16;   // one wave per block of 16 rows, at most 8 waves (the
                                // waves of k_kx<8, ...> loop over further blocks)
  const dim3 blk(64 * std::min(nrb, 8));
  if (POST && S.ch != 128) return (int)hipErrorInvalidValue;   // the fused form runs 128-asset chunks
  if (POST) {
    if (nrb <= 2) hipLaunchKernelGGL((k_kx<2, 128, true>), dim3(grid), blk, 0, st, S, xin, check);
    else if (nrb <= 5) hipLaunchKernelGGL((k_kx<5, 128, true>), dim3(grid), blk, 0, st, S, xin, check);
    else if (nrb <= 8) hipLaunchKernelGGL((k_kx<8, 128, true>), dim3(grid), blk, 0, st, S, xin, check);
    else if (nrb <= 10) hipLaunchKernelGGL((k_kx<8, 128, true, true>), dim3(grid), blk, 0, st, S, xin, check);
    else return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
  }
  if (S.ch == 256 && nrb <= 2) hipLaunchKernelGGL((k_kx<2, 256, POST>), dim3(grid), blk, 0, st, S, xin, check);
  else if (S.ch == 256 && nrb <= 5) hipLaunchKernelGGL((k_kx<5, 256, POST>), dim3(grid), blk, 0, st, S, xin, check);
  else if (S.ch == 256 && nrb <= 8) hipLaunchKernelGGL((k_kx<8, 256, POST>), dim3(grid), blk, 0, st, S, xin, check);
  else if (S.ch == 256 && nrb <= 10) hipLaunchKernelGGL((k_kx<8, 256, POST, true>), dim3(grid), blk, 0, st, S, xin, check);
  else if (S.ch == 128 && nrb <= 2) hipLaunchKernelGGL((k_kx<2, 128, POST>), dim3(grid), blk, 0, st, S, xin, check);
  else if (S.ch == 128 && nrb <= 5) hipLaunchKernelGGL((k_kx<5, 128, POST>), dim3(grid), blk, 0, st, S, xin, check);
  else if (S.ch == 128 && nrb <= 8) hipLaunchKernelGGL((k_kx<8, 128, POST>), dim3(grid), blk, 0, st, S, xin, check);
  else if (S.ch == 128 && nrb <= 10) hipLaunchKernelGGL((k_kx<8, 128, POST, true>), dim3(grid), blk, 0, st, S, xin, check);
  else return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int ls_launch_kx(const LsShared& S, const double* xin, int grid, void* stream) {
  return launch_kx_t<false>(S, xin, 0, grid, (hipStream_t)stream);
}

int ls_launch_step_fused(const LsShared& S, int check, int threads, int gA, int gC, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  int e = launch_kty_t<true>(S, S.yh, nullptr, gA, st);
  if (e) return e;
  hipLaunchKernelGGL(k_mu, dim3(S.B), dim3(threads), ls_primal_lds(S), st, S, 1);
  if ((e = (int)hipGetLastError())) return e;
  return launch_kx_t<true>(S, nullptr, check, gC, st);
}

int ls_launch_dual(const LsShared& S, int mode, void* stream) {
  hipLaunchKernelGGL(k_dual, dim3(S.B), dim3(S.nr <= 64 ? 64 : 128), 0, (hipStream_t)stream, S, mode);
  return (int)hipGetLastError();
}

int ls_launch_primal(const LsShared& S, int check, int threads, int gridE, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_pre, dim3(gridE), dim3(256), 0, st, S);
  hipLaunchKernelGGL(k_mu, dim3(S.B), dim3(threads), ls_primal_lds(S), st, S, 0);
  hipLaunchKernelGGL(k_post, dim3(gridE), dim3(256), 0, st, S, check);
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
