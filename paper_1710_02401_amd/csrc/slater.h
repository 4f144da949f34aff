// Slater-like antisymmetric Gaussian basis (Section 2, eq. (LSD)) for two
// electrons in one dimension each: item s's basis function m is
//   v_m(x1, x2) = (phi_l(x1) phi_p(x2) - phi_l(x2) phi_p(x1)) / sqrt(2),
// phi_l the l-th Gaussian of the item's first interval (dimension 0),
// phi_p the p-th of its second (dimension 1), l slowest; on a diagonal item
// (the same interval twice) only l < p.  Every v is a signed pair of tensor
// products of the extended list U = (first interval's n Gaussians, second
// interval's n), u < n from dimension 0 and u >= n from dimension 1:
//   v_m = (E_{l, n+p} - E_{n+p, l}) / sqrt(2),  E_{a,b} = U_a(x1) U_b(x2),
// which is how the matrices are assembled (slater.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace swr {

// (l, p) of basis function m of Slater item s.
__device__ inline void slater_pair(const Items& it, int s, int m, int* l, int* p) {
  const int n = it.nb[4 * s];
  if (it.idx[4 * s] == it.idx[4 * s + 1]) {
    int r = m, ll = 0;
    while (r >= n - 1 - ll) {
      r -= n - 1 - ll;
      ++ll;
    }
    *l = ll;
    *p = ll + 1 + r;
  } else {
    *l = m / n;
    *p = m - (m / n) * n;
  }
}

// Centre and exponent of U_u of item s.
__device__ inline void slater_gauss(const Items& it, int s, int u, double* a, double* d) {
  const int n = it.nb[4 * s];
  const int k = u < n ? 0 : 1;
  *a = it.alpha[it.aoff[4 * s + k] + (u - k * n)];
  *d = it.delta[4 * s + k];
}

// v_m(y) and, with grad, its partial derivatives along both coordinates.
__device__ inline double slater_value(const Items& it, int s, int m, const double* y,
                                      double* grad) {
  int l, p;
  slater_pair(it, s, m, &l, &p);
  const double a1 = it.alpha[it.aoff[4 * s] + l], d1 = it.delta[4 * s];
  const double a2 = it.alpha[it.aoff[4 * s + 1] + p], d2 = it.delta[4 * s + 1];
  const double g1x = exp(-d1 * (y[0] - a1) * (y[0] - a1)), g1y = exp(-d1 * (y[1] - a1) * (y[1] - a1));
  const double g2x = exp(-d2 * (y[0] - a2) * (y[0] - a2)), g2y = exp(-d2 * (y[1] - a2) * (y[1] - a2));
  const double r = 0.70710678118654752440;  // 1 / sqrt(2)
  if (grad) {
    const double d1x = -2.0 * d1 * (y[0] - a1) * g1x, d1y = -2.0 * d1 * (y[1] - a1) * g1y;
    const double d2x = -2.0 * d2 * (y[0] - a2) * g2x, d2y = -2.0 * d2 * (y[1] - a2) * g2y;
    grad[0] = r * (d1x * g2y - g1y * d2x);
    grad[1] = r * (g1x * d2y - d1y * g2x);
  }
  return r * (g1x * g2y - g1y * g2x);
}

// ---- launchers (slater.hip) ----
// A, Kin, Q (the field's coordinates), B, W of every item.
hipError_t launch_slater_assemble(const Items& it, double* A, double* Kin, double* Q, double* B,
                                  double* W, int K_max, hipStream_t st);
// Scratch (doubles) of the potential: per item (2n)^2 (q1 + 2) for the
// staged electron-electron term and the two electron-nucleus tables.
int64_t slater_pot_scratch(int n, int q1);
// V of every item; scratch at soff[s] per item.
hipError_t launch_slater_potential(const Items& it, const Potential& pot, const int64_t* soff,
                                   double* scratch, int n_max, int q_max, double* V, int K_max,
                                   hipStream_t st);
// Initial coefficients: the antisymmetrised Gaussian pair projected (A c = b).
hipError_t launch_slater_project(const Items& it, const double* A, double init_alpha,
                                 const double* center, double2* c0, int* flags, hipStream_t st);

}  // namespace swr
