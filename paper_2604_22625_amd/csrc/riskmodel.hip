// Risk-model construction of paper Section 3.2 on the device: from a window of daily
// factor returns Fr [days][p] and asset returns R [days][n] (with an optional observation
// mask), per-asset least-squares loadings beta_i (r_i ~ Fr beta_i over the asset's
// observed days, no intercept, only for assets with at least min_obs observations), the
// factor covariance Sigma_f (centred, 1/(days-1)) and the specific variances D_ii (the
// centred sample variance of the residuals over the observed days).
//
// The work is one pass over R, which dominates the bytes (days x n doubles), so the
// kernels are laid out for streaming it: lanes run over 64 consecutive assets (every
// load of a day's returns is one 512-byte coalesced row segment), the four waves of a
// workgroup take interleaved days of a 64-day chunk, and a grid over (asset block, day
// chunk) keeps every compute unit busy.  Each asset has its own Gram matrix (the mask
// selects its days), so this is a batch of small normal-equation systems, not a GEMM:
// per asset the pass accumulates the p(p+1)/2 Gram entries, the p cross products, the
// sum and sum of squares of its returns, its observation count and the p factor sums;
// a second kernel adds the day chunks in order, solves the p x p system by Cholesky and
// forms D from the sums (sum theta^2 = sum r^2 - 2 beta^T c + beta^T G beta).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <cmath>
#include "internal.h"

namespace ffo {
namespace {

constexpr int RM_CHUNK = 64;   // days per partial-sum tile

template <int P>
struct RmDim {
  static constexpr int G = P * (P + 1) / 2;    // Gram entries (upper triangle, row-major)
  static constexpr int NV = G + P + 3 + P;     // + cross, sum r, sum r^2, count, factor sums
};

template <int P>
__global__ __launch_bounds__(256) void k_rm_partial(int days, int n, const double* __restrict__ R,
                                                    const double* __restrict__ Fr, const uint8_t* __restrict__ mask,
                                                    double* __restrict__ part) {
  constexpr int NV = RmDim<P>::NV, G = RmDim<P>::G;
  __shared__ double fs[RM_CHUNK * P];
  __shared__ double red[4 * NV * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int k0 = blockIdx.y * RM_CHUNK, k1 = min(days, k0 + RM_CHUNK);
  for (int e = threadIdx.x; e < (k1 - k0) * P; e += blockDim.x) fs[e] = Fr[(size_t)k0 * P + e];
  __syncthreads();
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const bool col = i < n;
  for (int k = k0 + wave; k < k1; k += 16) {   // four days per step, loads first
    double rv[4];
    bool ob[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + 4 * u;
      const bool in = col && kk < k1;
      ob[u] = in && (mask == nullptr || mask[(size_t)kk * n + i] != 0);
      rv[u] = ob[u] ? R[(size_t)kk * n + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!ob[u]) continue;
      const double* f = fs + (k + 4 * u - k0) * P;
      const double r = rv[u];
      int g = 0;
#pragma unroll
      for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = a; b < P; ++b) { acc[g] = fma(f[a], f[b], acc[g]); ++g; }
#pragma unroll
      for (int a = 0; a < P; ++a) acc[G + a] = fma(f[a], r, acc[G + a]);
      acc[G + P] += r;
      acc[G + P + 1] = fma(r, r, acc[G + P + 1]);
      acc[G + P + 2] += 1.0;
#pragma unroll
      for (int a = 0; a < P; ++a) acc[G + P + 3 + a] += f[a];
    }
  }
  // the four waves' sums, added in wave order
#pragma unroll
  for (int v = 0; v < NV; ++v) red[(wave * NV + v) * 64 + lane] = acc[v];
  __syncthreads();
  if (wave == 0 && col) {
    double* out = part + (size_t)blockIdx.y * NV * n;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double s = red[(0 * NV + v) * 64 + lane] + red[(1 * NV + v) * 64 + lane] +
                       red[(2 * NV + v) * 64 + lane] + red[(3 * NV + v) * 64 + lane];
      out[(size_t)v * n + i] = s;
    }
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_rm_solve(int n, int nchunk, int min_obs, const double* __restrict__ part,
                                                  double* __restrict__ beta, double* __restrict__ D,
                                                  int32_t* __restrict__ valid) {
  constexpr int NV = RmDim<P>::NV, G = RmDim<P>::G;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    const double* pc = part + (size_t)c * NV * n;
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] += pc[(size_t)v * n + i];
  }
  const double cnt = s[G + P + 2];
  double b[P];
#pragma unroll
  for (int a = 0; a < P; ++a) b[a] = 0.0;
  bool ok = cnt >= (double)min_obs && cnt >= (double)(P + 1);
  if (ok) {
    // Cholesky of the Gram matrix (lower factor Lc, row-major), then two triangular solves
    double A[P][P], Lc[P][P];
    {
      int g = 0;
#pragma unroll
      for (int a = 0; a < P; ++a)
#pragma unroll
        for (int c2 = a; c2 < P; ++c2) { A[a][c2] = s[g]; A[c2][a] = s[g]; ++g; }
    }
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
      for (int c2 = 0; c2 < P; ++c2) Lc[a][c2] = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      double dj = A[j][j];
#pragma unroll
      for (int q = 0; q < j; ++q) dj -= Lc[j][q] * Lc[j][q];
      if (!(dj > 1e-300)) ok = false;
      const double rj = ok ? sqrt(dj) : 1.0;
      Lc[j][j] = rj;
#pragma unroll
      for (int r2 = j + 1; r2 < P; ++r2) {
        double v = A[r2][j];
#pragma unroll
        for (int q = 0; q < j; ++q) v -= Lc[r2][q] * Lc[j][q];
        Lc[r2][j] = v / rj;
      }
    }
    if (ok) {
      double y[P];
#pragma unroll
      for (int a = 0; a < P; ++a) {
        double v = s[G + a];
#pragma unroll
        for (int q = 0; q < a; ++q) v -= Lc[a][q] * y[q];
        y[a] = v / Lc[a][a];
      }
#pragma unroll
      for (int a = P - 1; a >= 0; --a) {
        double v = y[a];
#pragma unroll
        for (int q = a + 1; q < P; ++q) v -= Lc[q][a] * b[q];
        b[a] = v / Lc[a][a];
      }
    } else {
#pragma unroll
      for (int a = 0; a < P; ++a) b[a] = 0.0;
    }
  }
  // residual sums: theta = r - beta^T f over the observed days
  double st = s[G + P], st2 = s[G + P + 1];
  if (ok) {
    double bc = 0.0, bGb = 0.0, bf = 0.0;
    int g = 0;
#pragma unroll
    for (int a = 0; a < P; ++a) {
      bc = fma(b[a], s[G + a], bc);
      bf = fma(b[a], s[G + P + 3 + a], bf);
#pragma unroll
      for (int c2 = a; c2 < P; ++c2) { bGb += (a == c2 ? 1.0 : 2.0) * b[a] * b[c2] * s[g]; ++g; }
    }
    st -= bf;
    st2 = st2 - 2.0 * bc + bGb;
  }
  double d = 0.0;
  if (cnt >= 2.0) d = fmax((st2 - st * st / cnt) / (cnt - 1.0), 0.0);
#pragma unroll
  for (int a = 0; a < P; ++a) beta[(size_t)i * P + a] = b[a];
  D[i] = d;
  valid[i] = ok ? 1 : 0;
}

// Sigma_f = (Fr - mean)^T (Fr - mean) / (days - 1), one workgroup: each thread sums its
// days for all P means (pass 1) and all P(P+1)/2 centred products (pass 2); one
// fixed-order workgroup reduction per pass.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double x = v[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[w * NV + q] = x;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = red[q] + red[NV + q] + red[2 * NV + q] + red[3 * NV + q];
  __syncthreads();
}

template <int P>
__global__ __launch_bounds__(256) void k_rm_cov(int days, const double* __restrict__ Fr, double* __restrict__ Sf) {
  constexpr int G = P * (P + 1) / 2;
  __shared__ double red[4 * G];
  double mu[P];
#pragma unroll
  for (int a = 0; a < P; ++a) mu[a] = 0.0;
  for (int k = threadIdx.x; k < days; k += 256)
#pragma unroll
    for (int a = 0; a < P; ++a) mu[a] += Fr[(size_t)k * P + a];
  block_sum<P>(mu, red);
#pragma unroll
  for (int a = 0; a < P; ++a) mu[a] /= (double)days;
  double c[G];
#pragma unroll
  for (int g = 0; g < G; ++g) c[g] = 0.0;
  for (int k = threadIdx.x; k < days; k += 256) {
    double f[P];
#pragma unroll
    for (int a = 0; a < P; ++a) f[a] = Fr[(size_t)k * P + a] - mu[a];
    int g = 0;
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
      for (int b = a; b < P; ++b) { c[g] = fma(f[a], f[b], c[g]); ++g; }
  }
  block_sum<G>(c, red);
  if (threadIdx.x == 0) {
    int g = 0;
    for (int a = 0; a < P; ++a)
      for (int b = a; b < P; ++b) {
        const double v = c[g++] / (double)(days - 1);
        Sf[a * P + b] = v;
        Sf[b * P + a] = v;
      }
  }
}

template <int P>
int launch_rm(int days, int n, const double* R, const double* Fr, const uint8_t* mask, int min_obs, double* part,
              double* beta, double* Sf, double* D, int32_t* valid, hipStream_t st) {
  const int nchunk = (days + RM_CHUNK - 1) / RM_CHUNK;
  hipLaunchKernelGGL(k_rm_cov<P>, dim3(1), dim3(256), 0, st, days, Fr, Sf);
  hipLaunchKernelGGL(k_rm_partial<P>, dim3((n + 63) / 64, nchunk), dim3(256), 0, st, days, n, R, Fr, mask, part);
  hipLaunchKernelGGL(k_rm_solve<P>, dim3((n + 255) / 256), dim3(256), 0, st, n, nchunk, min_obs, part, beta, D, valid);
  return (int)hipGetLastError();
}

}  // namespace

size_t rm_workspace_bytes(int64_t days, int64_t n, int64_t p) {
  const int64_t nv = p * (p + 1) / 2 + 2 * p + 3;
  return (size_t)((days + RM_CHUNK - 1) / RM_CHUNK) * nv * n * sizeof(double);
}

int launch_risk_model(int days, int n, int p, const double* R, const double* Fr, const uint8_t* mask, int min_obs,
                      double* part, double* beta, double* Sf, double* D, int32_t* valid, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  switch (p) {
    case 1: return launch_rm<1>(days, n, R, Fr, mask, min_obs, part, beta, Sf, D, valid, st);
    case 2: return launch_rm<2>(days, n, R, Fr, mask, min_obs, part, beta, Sf, D, valid, st);
    case 3: return launch_rm<3>(days, n, R, Fr, mask, min_obs, part, beta, Sf, D, valid, st);
    case 4: return launch_rm<4>(days, n, R, Fr, mask, min_obs, part, beta, Sf, D, valid, st);
    case 5: return launch_rm<5>(days, n, R, Fr, mask, min_obs, part, beta, Sf, D, valid, st);
    case 6: return launch_rm<6>(days, n, R, Fr, mask, min_obs, part, beta, Sf, D, valid, st);
    case 7: return launch_rm<7>(days, n, R, Fr, mask, min_obs, part, beta, Sf, D, valid, st);
    case 8: return launch_rm<8>(days, n, R, Fr, mask, min_obs, part, beta, Sf, D, valid, st);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace ffo
