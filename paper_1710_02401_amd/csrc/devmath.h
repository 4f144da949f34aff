// Device helpers shared by the kernel files: complex arithmetic on
// interleaved (re, im) doubles, the closed-form one-dimensional Gaussian
// pair integrals, and index helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace swr {

constexpr int kFlagNaN = 1;
constexpr int kFlagPivot = 2;

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a*b + c
__device__ inline double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double2 crecip(double2 a) {
  // 1/a with scaling against overflow
  if (fabs(a.x) >= fabs(a.y)) {
    double r = a.y / a.x, d = a.x + a.y * r;
    return make_double2(1.0 / d, -r / d);
  }
  double r = a.x / a.y, d = a.y + a.x * r;
  return make_double2(r / d, -1.0 / d);
}
__device__ inline bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// index of the upper tile (I, J), I <= J, among T x T tiles stored row by row
__device__ inline int tile_index(int I, int J, int T) { return I * T - (I * (I - 1)) / 2 + (J - I); }

// erf(uh) - erf(ul), ul <= uh, with the complementary function in the tails
__device__ inline double erf_diff(double ul, double uh) {
  if (ul > 0.0) return erfc(ul) - erfc(uh);
  if (uh < 0.0) return erfc(-uh) - erfc(-ul);
  return erf(uh) - erf(ul);
}

// One-dimensional integrals of phi_a phi_b over [lo, hi] (Gaussian product
// rule): overlap S, position X, kinetic T = 1/2 int phi_a' phi_b'.
__device__ inline void pair_integrals(double aa, double da, double ab, double db, double lo,
                                      double hi, double* S, double* X, double* T) {
  const double p = da + db;
  const double P = (da * aa + db * ab) / p;
  const double E = exp(-da * db * (aa - ab) * (aa - ab) / p);
  const double sp = sqrt(p);
  const double ul = sp * (lo - P), uh = sp * (hi - P);
  const double I0 = 0.5 * sqrt(M_PI / p) * erf_diff(ul, uh);
  const double el = exp(-ul * ul), eh = exp(-uh * uh);
  const double I1 = (el - eh) / (2.0 * p);
  const double I2 = I0 / (2.0 * p) - ((hi - P) * eh - (lo - P) * el) / (2.0 * p);
  *S = E * I0;
  if (X) *X = E * (P * I0 + I1);
  if (T) *T = 2.0 * da * db * E * (I2 + (2.0 * P - aa - ab) * I1 + (P - aa) * (P - ab) * I0);
}

__device__ inline double pair_overlap(double aa, double da, double ab, double db, double lo,
                                      double hi) {
  double S;
  pair_integrals(aa, da, ab, db, lo, hi, &S, nullptr, nullptr);
  return S;
}

// split flat basis index (last dimension fastest) into per-dim indices
__device__ inline void split_index(int l, const int32_t* nb, int D, int* li) {
  for (int k = D - 1; k >= 0; --k) {
    li[k] = l % nb[k];
    l /= nb[k];
  }
}

// FP64 matrix-core product D = A B + C of 16 x 16 x 4 tiles.  Operand
// layouts: A entry (l % 16, l / 16) in lane l, B entry (l / 16, l % 16),
// and register r of D entry (4 r + l / 16, l % 16).
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// cross-lane moves inside rows of the wave (DPP, no LDS traffic); every
// lane's source is inside its row, so the value written is never the old one
template <int kCtrl>
__device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), kCtrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), kCtrl, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Block barrier for LDS traffic only: orders the block's LDS accesses as
// __syncthreads() does, without waiting for the wave's outstanding global
// stores (a workgroup fence over every address space waits for them).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// sum over each group of eight consecutive lanes, result in every lane:
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], then row_half_mirror (lane i
// of a half-row meets lane 7-i, i.e. the other quad)
__device__ inline double group8_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  return v;
}

// Compensated dot products (Ogita, Rump and Oishi's Dot2): exact products by
// fma, error-free additions, the rounding errors summed aside; as accurate as
// working in twice the precision.  No contraction: a product fused into these
// sums would break the exact error terms.
struct Dot2 {
  double s, c;  // running sum, accumulated rounding errors
};
__device__ inline void dot2_acc(Dot2& a, double x, double y) {  // a += x y
#pragma clang fp contract(off)
  const double p = x * y;
  const double e = fma(x, y, -p);
  const double t = a.s + p;
  const double z = t - a.s;
  a.c += ((a.s - (t - z)) + (p - z)) + e;
  a.s = t;
}

}  // namespace swr
