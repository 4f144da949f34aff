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

// Functions per interval in the pairs: Gaussians, or local orbitals.
__device__ inline int slater_half(const Items& it, int s) {
  return it.lsd ? it.n_orb : it.nb[4 * s];
}

// (l, p) of basis function m of Slater item s.
__device__ inline void slater_pair(const Items& it, int s, int m, int* l, int* p) {
  const int n = slater_half(it, s);
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

// Local orbital l of the interval of item s's dimension t at x, and its
// derivative: sum_u C[u][l] g_u(x) over the interval's Gaussians.
__device__ inline double lsd_orbital(const Items& it, int s, int t, int l, double x, double* d) {
  const int n = it.nb[4 * s + t];
  const double* C = it.lo_C + (int64_t)it.idx[4 * s + t] * n * it.n_orb;
  const double* a = it.alpha + it.aoff[4 * s + t];
  const double dl = it.delta[4 * s + t];
  double v = 0.0, dv = 0.0;
  for (int u = 0; u < n; ++u) {
    const double g = exp(-dl * (x - a[u]) * (x - a[u]));
    v = fma(C[u * it.n_orb + l], g, v);
    dv = fma(C[u * it.n_orb + l], -2.0 * dl * (x - a[u]) * g, dv);
  }
  *d = dv;
  return v;
}

// Extended one-dimensional function u of item s at x (and its derivative):
// u < half from the first coordinate's interval, else from the second's;
// Gaussians, or local orbitals.
__device__ inline double slater_ext(const Items& it, int s, int u, double x, double* d) {
  const int half = slater_half(it, s);
  const int t = u < half ? 0 : 1;
  if (it.lsd) return lsd_orbital(it, s, t, u - t * half, x, d);
  const double a = it.alpha[it.aoff[4 * s + t] + (u - t * half)], dl = it.delta[4 * s + t];
  const double g = exp(-dl * (x - a) * (x - a));
  *d = -2.0 * dl * (x - a) * g;
  return g;
}

// v_m(y) and, with grad, its partial derivatives along both coordinates.
__device__ inline double slater_value(const Items& it, int s, int m, const double* y,
                                      double* grad) {
  int l, p;
  slater_pair(it, s, m, &l, &p);
  const int half = slater_half(it, s);
  double d1x, d1y, d2x, d2y;
  const double g1x = slater_ext(it, s, l, y[0], &d1x), g1y = slater_ext(it, s, l, y[1], &d1y);
  const double g2x = slater_ext(it, s, half + p, y[0], &d2x);
  const double g2y = slater_ext(it, s, half + p, y[1], &d2y);
  const double r = 0.70710678118654752440;  // 1 / sqrt(2)
  if (grad) {
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

// Local orbitals (Section 3), one block per interval i of n_iv: the
// orbital problem's S and H in the interval's Gaussians (those of item i's
// first dimension) by the interval's quadrature rule (x, w at qoff[i] ..
// qoff[i+1]), the nuclei inside the interval's box mollified with the
// rule (mx, mw) on [-1, 1] scaled to the mollifier's support, then the
// generalised eigenproblem (Cholesky, cyclic Jacobi): the n_eig lowest
// orbitals into columns 0 .. n_eig-1 of it.lo_C (n x it.n_orb per interval),
// S-normalised, signed so that sum_u (u+1) C[u][l] > 0; the remaining
// it.n_orb - n_eig columns (an even count g2 = 2g, Section 3.3) are unit
// vectors on Gaussians 0 .. g-1, then n-1 down to n-g.
struct LoParams {
  double barrier, width, v_inf, eps, sigma;
  int order, n_eig;
};
hipError_t launch_lo_orbitals(const Items& it, int n_iv, const Potential& pot, LoParams lp,
                              const double* qx, const double* qw, const int64_t* qoff,
                              const double* mx, const double* mw, int n_m, double* C_out,
                              int* flags, hipStream_t st);
// Per (item, dimension): the one-dimensional integrals of the item's
// extended orbitals into it.lo_tab (needs it.lo_C).
hipError_t launch_lo_tables(const Items& it, double* tab, hipStream_t st);

// Local orbitals of one electron in two dimensions (Section 3, d = 2), per
// item (box) s: the Gaussians at the orbital rule's nodes (x, w at
// qoff[2 s + k] .. qoff[2 s + k + 1] for dimension k) into gt, the
// one-dimensional integrals into tab, the nuclear term's first contraction
// into pp (64 per dimension-1 node), then the orbital problem (S, H over the
// box's n0 n1 <= 64 Gaussians) and its lp.n_eig lowest orbitals into C_out
// (n0 n1 x n_eig per item).  lp.sigma is the mollified Coulomb kernel's
// prefactor (slater.hip); ang: (sin, cos) of the angle rule's nodes on
// [0, pi/2], then (weight, 0).
hipError_t launch_lo2_orbitals(const Items& it, const Potential& pot, LoParams lp,
                               const double* qx, const double* qw, const int64_t* qoff,
                               const double2* ang, int n_m, int64_t n_q1_max, double* gt,
                               double* tab, double* pp, double* C_out, int* flags,
                               hipStream_t st);
// X = C^T XG C per item (XG over the box's Gaussians at offsets og).
hipError_t launch_lo2_transform(const Items& it, const int64_t* og, const double* XG, double* X,
                                hipStream_t st);

}  // namespace swr
