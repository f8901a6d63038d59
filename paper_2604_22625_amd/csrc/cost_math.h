// Cost-term maps of the splitting shared by the solver kernels (device code only).
//
// The trade cost of paper eq. 1 / eq. 4 for one asset is a|u| + b|u|^d (a = g2 s,
// b = g3 q, 1 < d <= 2).  prox_cost is its proximal map with step t', conj_cost its
// convex conjugate; the dual prox of the trade rows uses both through the Moreau
// identity.
#pragma once
#include <hip/hip_runtime.h>

namespace ffo {

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



}  // namespace ffo
