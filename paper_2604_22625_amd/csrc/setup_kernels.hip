// Setup kernels: assemble the scaled constraint rows and the elementwise data of the
// splitting (exposure rows A, factor rows G^T with G = F C, C C^T = Omega; trade rows).
//
// Scaling is diagonal (Pock & Chambolle 2011, alpha = 1): with row sums r_j and column
// sums c_i of |K| over the stacked operator (exposure, factor and trade rows),
// dr = 1/sqrt(r), dc = 1/sqrt(c) and K~ = diag(dr) K diag(dc).  Trade rows have unit
// entries, so their row sums are 1 (single-period, first and last multi-period trade)
// or 2, and every column gains 1 (single-period) or 2 (multi-period).
#include <algorithm>
#include <hip/hip_runtime.h>
#include "internal.h"

namespace ffo {

namespace {

constexpr int TB = 256;

// K[j][i] for j < m from A, for j = m + l from (F C)[i][l]; also the column sums.
__global__ __launch_bounds__(TB) void k_build(int n, int k, int m, int ldk, int tradecol,
                                              const double* __restrict__ F, const double* __restrict__ C,
                                              const double* __restrict__ A, double* __restrict__ K,
                                              double* __restrict__ dc) {
  extern __shared__ double sC[];  // k*k
  for (int e = threadIdx.x; e < k * k; e += TB) sC[e] = C[e];
  __syncthreads();
  const int i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  double cs = (double)tradecol;
  for (int j = 0; j < m; ++j) {
    const double a = A[(size_t)j * n + i];
    K[(size_t)j * ldk + i] = a;
    cs += fabs(a);
  }
  for (int l = 0; l < k; ++l) {
    double g = 0.0;
    for (int jj = 0; jj < k; ++jj) g = fma(F[(size_t)i * k + jj], sC[jj * k + l], g);
    K[(size_t)(m + l) * ldk + i] = g;
    cs += fabs(g);
  }
  dc[i] = 1.0 / sqrt(cs);
}

// One block per constraint row: row sum of |K| -> dr; factor rows also give bF = G^T c.
// Block nr computes crisk = g1 sum delta^2 c^2.
__global__ __launch_bounds__(TB) void k_rows(int n, int nr, int m, int ldk, const double* __restrict__ K,
                                             const double* __restrict__ cvec, const double* __restrict__ delta,
                                             double g1, double* __restrict__ dr, double* __restrict__ bF,
                                             double* __restrict__ crisk) {
  __shared__ double s1[TB], s2[TB];
  const int j = blockIdx.x;
  double a = 0.0, b = 0.0;
  if (j < nr) {
    for (int i = threadIdx.x; i < n; i += TB) {
      const double v = K[(size_t)j * ldk + i];
      a += fabs(v);
      b = fma(v, cvec[i], b);
    }
  } else {
    for (int i = threadIdx.x; i < n; i += TB) a = fma(delta[i] * delta[i], cvec[i] * cvec[i], a);
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (j < nr) {
      dr[j] = s1[0] > 0.0 ? 1.0 / sqrt(s1[0]) : 1.0;
      if (j >= m) bF[j - m] = s2[0];
    } else {
      crisk[0] = g1 * s1[0];
    }
  }
}

__global__ __launch_bounds__(TB) void k_scale(int n, int nr, int ldk, double* __restrict__ K,
                                              const double* __restrict__ dr, const double* __restrict__ dc) {
  const int i = blockIdx.x * TB + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= ldk || j >= nr) return;
  if (i < n) K[(size_t)j * ldk + i] *= (dr ? dr[j] : 1.0) * dc[i];
  else K[(size_t)j * ldk + i] = 0.0;
}

__global__ __launch_bounds__(TB) void k_elem(int n, int P, int Tp, int multi, const double* __restrict__ delta,
                                             const double* __restrict__ s, const double* __restrict__ q,
                                             const double* __restrict__ wT, double g1, double g2, double g3,
                                             double* __restrict__ drC, double* __restrict__ arisk,
                                             double* __restrict__ cvec, double* __restrict__ ca,
                                             double* __restrict__ cb) {
  const int i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  arisk[i] = 2.0 * g1 * delta[i] * delta[i];
  cvec[i] = multi ? wT[i] : 0.0;
  for (int t = 0; t < Tp; ++t) {
    const size_t e = (size_t)t * n + i;
    if (s) {
      ca[e] = g2 * s[e];
      cb[e] = g3 * q[e];
    }
    // trade row t touches w_{t-1} and w_t: two unit entries except at the ends
    drC[e] = (!multi || t == 0 || t == P) ? 1.0 : 0.70710678118654752440;
  }
}

// Batched form, per instance b: row scales over the instance's prefix of nb[b] columns,
// drs[b][j] = 1/sqrt(sum_{i < nb[b]} |K[j][i]|) (1 for an empty row).  One block per (j, b).
__global__ __launch_bounds__(TB) void k_rows_prefix(int nr, int ldk, const double* __restrict__ K,
                                                    const int64_t* __restrict__ nb, double* __restrict__ drs) {
  __shared__ double s1[TB];
  const int j = blockIdx.x, b = blockIdx.y;
  const int64_t n = nb[b];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += TB) a += fabs(K[(size_t)j * ldk + i]);
  s1[threadIdx.x] = a;
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s1[threadIdx.x] += s1[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) drs[(size_t)b * nr + j] = s1[0] > 0.0 ? 1.0 / sqrt(s1[0]) : 1.0;
}

// Batched form: per-asset cost coefficients of the packed instances.
__global__ __launch_bounds__(TB) void k_costs(int64_t N, const double* __restrict__ s, const double* __restrict__ q,
                                              double g2, double g3, double* __restrict__ ca, double* __restrict__ cb) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i >= N) return;
  ca[i] = g2 * s[i];
  cb[i] = g3 * q[i];
}

}  // namespace

int launch_setup_batch(int64_t B, const int64_t* nb_dev, int64_t n_max, int64_t k, int64_t m, int ldk,
                       const double* F, const double* Cfac, const double* A, const double* delta, int64_t N,
                       const double* s, const double* q, double g1, double g2, double g3, double* Kbuf,
                       double* drs, double* dc, double* drC, double* arisk, double* cvec, double* ca, double* cb,
                       void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const int nb = (int)((n_max + TB - 1) / TB);
  hipLaunchKernelGGL(k_elem, dim3(nb), dim3(TB), 0, st, (int)n_max, 1, 1, 0, delta, (const double*)nullptr,
                     (const double*)nullptr, (const double*)nullptr, g1, g2, g3, drC, arisk, cvec, (double*)nullptr,
                     (double*)nullptr);
  hipLaunchKernelGGL(k_costs, dim3((unsigned)((N + TB - 1) / TB)), dim3(TB), 0, st, N, s, q, g2, g3, ca, cb);
  hipLaunchKernelGGL(k_build, dim3(nb), dim3(TB), (size_t)(k * k) * sizeof(double), st, (int)n_max, (int)k, (int)m,
                     ldk, 1, F, Cfac, A, Kbuf, dc);
  const int nr = (int)(m + k);
  if (nr > 0) {
    hipLaunchKernelGGL(k_rows_prefix, dim3(nr, (unsigned)B), dim3(TB), 0, st, nr, ldk, Kbuf, nb_dev, drs);
    hipLaunchKernelGGL(k_scale, dim3((ldk + TB - 1) / TB, nr), dim3(TB), 0, st, (int)n_max, nr, ldk, Kbuf,
                       (const double*)nullptr, dc);
  }
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

__global__ __launch_bounds__(TB) void k_to_float(const double* __restrict__ K, float* __restrict__ Kf, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < count; i += (int64_t)gridDim.x * TB)
    Kf[i] = (float)K[i];
}

__global__ __launch_bounds__(TB) void k_to_bf16(double* __restrict__ K, uint16_t* __restrict__ Kb, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < count; i += (int64_t)gridDim.x * TB) {
    uint32_t u = __float_as_uint((float)K[i]);   // inputs are finite (validated)
    u += 0x7FFFu + ((u >> 16) & 1u);              // round to nearest, ties to even
    const uint16_t b = (uint16_t)(u >> 16);
    Kb[i] = b;
    K[i] = (double)__uint_as_float((uint32_t)b << 16);
  }
}

int launch_to_bf16(double* K, uint16_t* Kb, int64_t count, void* stream) {
  if (count <= 0) return 0;
  const int64_t nb = std::min<int64_t>((count + TB - 1) / TB, 4096);
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)nb), dim3(TB), 0, (hipStream_t)stream, K, Kb, count);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

int launch_to_float(const double* K, float* Kf, int64_t count, void* stream) {
  if (count <= 0) return 0;
  const int64_t nb = std::min<int64_t>((count + TB - 1) / TB, 4096);
  hipLaunchKernelGGL(k_to_float, dim3((unsigned)nb), dim3(TB), 0, (hipStream_t)stream, K, Kf, count);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

int launch_setup(int64_t n, int64_t k, int64_t m, int64_t P, int64_t Tp, int ldk, const double* F,
                 const double* Cfac, const double* A, const double* delta, const double* s,
                 const double* q, const double* wT, double g1, double g2, double g3, double* Kbuf,
                 double* dr, double* dc, double* drC, double* arisk, double* cvec, double* ca,
                 double* cb, double* bF, double* crisk_dev, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const int multi = Tp > 1 ? 1 : 0;
  const int nb = (int)((n + TB - 1) / TB);
  hipLaunchKernelGGL(k_elem, dim3(nb), dim3(TB), 0, st, (int)n, (int)P, (int)Tp, multi, delta, s, q, wT, g1,
                     g2, g3, drC, arisk, cvec, ca, cb);
  hipLaunchKernelGGL(k_build, dim3(nb), dim3(TB), (size_t)(k * k) * sizeof(double), st, (int)n, (int)k,
                     (int)m, ldk, multi ? 2 : 1, F, Cfac, A, Kbuf, dc);
  const int nr = (int)(m + k);
  hipLaunchKernelGGL(k_rows, dim3(nr + 1), dim3(TB), 0, st, (int)n, nr, (int)m, ldk, Kbuf, cvec, delta, g1,
                     dr, bF, crisk_dev);
  if (nr > 0)
    hipLaunchKernelGGL(k_scale, dim3((ldk + TB - 1) / TB, nr), dim3(TB), 0, st, (int)n, nr, ldk, Kbuf, dr, dc);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace ffo
