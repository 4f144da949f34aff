// HIP kernels (gfx950) of the SWR-Galerkin hot path.
//
// Layout conventions (all FP64, complex = double2 interleaved):
//   real matrices of item s: K_s x K_s row-major at off2[s];
//   histories / Robin data vectors: item s block of (n_steps+1) x K_s
//   entries, time-major, at (n_steps+1) * off1[s];
//   inverse Crank-Nicolson matrices (complex symmetric): item s, matrix n
//   at n_mats * offp[s] + n * P_s, P_s = 64 T (T+1) / 2 with T = ceil(K_s/8):
//   the upper 8x8 tiles (I <= J) row by row, each column-major (entry (a, b)
//   of tile (I, J) = M[8I+a][8J+b] at b * 8 + a), padding rows and columns
//   of the last tiles holding the identity.  Imaginary-time inverses (one per
//   item) are stored whole and transposed at off2[s].
#include <hip/hip_runtime.h>

#include <cmath>

#include "devmath.h"
#include "kernels.h"
#include "slater.h"

namespace swr {
namespace {

// ---------------------------------------------------------------------------
// Assembly of the separable matrices (Section 1.2 Galerkin form, Section 4.1
// eq. Q, Robin boundary mass, partition-of-unity mass).
__global__ void k_assemble(Items it, double* A, double* Kin, double* Q, double* Q2, double* B,
                           double* W, double* S1, const int64_t* s1off) {
  const int s = blockIdx.y;
  const int K = it.K[s];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * K) return;
  const int l = e / K, m = e % K;
  const int D = it.D;
  const int32_t* nb = it.nb + 4 * s;
  int li[4], mi[4];
  split_index(l, nb, D, li);
  split_index(m, nb, D, mi);
  double Sk[4], Xk[4], Tk[4], Bk[4], Wk[4];
  for (int k = 0; k < D; ++k) {
    const double lo = it.lo[4 * s + k], hi = it.hi[4 * s + k], d = it.delta[4 * s + k];
    const double* al = it.alpha + it.aoff[4 * s + k];
    const double aa = al[li[k]], ab = al[mi[k]];
    pair_integrals(aa, d, ab, d, lo, hi, &Sk[k], &Xk[k], &Tk[k]);
    const double fla = exp(-d * (lo - aa) * (lo - aa)), flb = exp(-d * (lo - ab) * (lo - ab));
    const double fha = exp(-d * (hi - aa) * (hi - aa)), fhb = exp(-d * (hi - ab) * (hi - ab));
    Bk[k] = fla * flb + fha * fhb;
    double w = Sk[k];
    const double eps = it.eps[k];
    if (it.idx[4 * s + k] > 0) w -= 0.5 * pair_overlap(aa, d, ab, d, lo, lo + eps);
    if (it.idx[4 * s + k] < it.L[k] - 1) w -= 0.5 * pair_overlap(aa, d, ab, d, hi - eps, hi);
    Wk[k] = w;
  }
  double a = 1.0, wprod = 1.0, kin = 0.0, bsum = 0.0, q = 0.0;
  for (int k = 0; k < D; ++k) {
    a *= Sk[k];
    wprod *= Wk[k];
    double tk = Tk[k], bk = Bk[k];
    for (int k2 = 0; k2 < D; ++k2)
      if (k2 != k) { tk *= Sk[k2]; bk *= Sk[k2]; }
    kin += tk;
    bsum += bk;
  }
  // dipole of the coordinates in a mask: sum over them of x_k with the
  // overlaps of the other dimensions
  double q2 = 0.0;
  for (int km = 0; km < D; ++km) {
    if (!((it.qmask0 | it.qmask1) >> km & 1)) continue;
    double x = Xk[km];
    for (int k2 = 0; k2 < D; ++k2)
      if (k2 != km) x *= Sk[k2];
    if (it.qmask0 >> km & 1) q += x;
    if (it.qmask1 >> km & 1) q2 += x;
  }
  const int64_t o = it.off2[s] + (int64_t)l * K + m;
  A[o] = a;
  Kin[o] = kin;
  Q[o] = q;
  if (Q2) Q2[o] = q2;
  B[o] = bsum;
  W[o] = wprod;
  // per-dimension overlap factors, written by the entry whose other indices are 0
  for (int k = 0; k < D; ++k) {
    bool base = true;
    for (int k2 = 0; k2 < D; ++k2)
      if (k2 != k && (li[k2] != 0 || mi[k2] != 0)) base = false;
    if (base) S1[s1off[4 * s + k] + (int64_t)li[k] * nb[k] + mi[k]] = Sk[k];
  }
}

// ---------------------------------------------------------------------------
// Soft-Coulomb potential matrix (eq. pseudo): electron-nucleus terms as
// one-dimensional Gauss-Legendre sums, the electron-electron term as the
// contraction chain sum_{q0} F0[a0 b0, q0] sum_{q1} F1[a1 b1, q1] U(q0, q1).
// One block per item; one space dimension per electron.
__global__ void k_potential(Items it, Potential pot, const double* S1, const int64_t* s1off,
                            double* V, double* scratch, const int64_t* scratch_off) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  const int D = it.D;
  const int N = it.n_elec;
  const int geom = s / it.n_sub;
  const int32_t* nb = it.nb + 4 * s;
  __shared__ double v1[2 * kSmallK * kSmallK];  // e-n tables, one per electron (D <= 2)
  int v1off[4];
  {
    int o = 0;
    for (int k = 0; k < D; ++k) { v1off[k] = o; o += nb[k] * nb[k]; }
  }
  // phase A: e-n one-dimensional tables
  for (int el = 0; el < N; ++el) {
    const int k = el;  // dim == 1
    const int n = nb[k];
    const double d = it.delta[4 * s + k];
    const double* al = it.alpha + it.aoff[4 * s + k];
    const double* qx = it.qx + it.qoff[4 * s + k];
    const double* qw = it.qw + it.qoff[4 * s + k];
    const int nq = it.qn[4 * s + k];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int a = e / n, b = e % n;
      double acc = 0.0;
      if (pot.n_nuc > 0) {
        for (int q = 0; q < nq; ++q) {
          const double x = qx[q];
          double u = 0.0;
          for (int A = 0; A < pot.n_nuc; ++A) {
            const double r = x - pot.pos[(geom * pot.n_nuc + A) * it.dim];
            u -= pot.charge[A] / sqrt(r * r + pot.eps_en * pot.eps_en);
          }
          acc += qw[q] * u * exp(-d * (x - al[a]) * (x - al[a])) * exp(-d * (x - al[b]) * (x - al[b]));
        }
      }
      v1[v1off[k] + e] = acc;
    }
  }
  // phase B: e-e contraction (two electrons in one dimension each)
  double* T1 = scratch + scratch_off[s];
  if (N == 2) {
    const int n0 = nb[0], n1 = nb[1];
    const double d0 = it.delta[4 * s + 0], d1 = it.delta[4 * s + 1];
    const double* al1 = it.alpha + it.aoff[4 * s + 1];
    const double* qx0 = it.qx + it.qoff[4 * s + 0];
    const double* qx1 = it.qx + it.qoff[4 * s + 1];
    const double* qw1 = it.qw + it.qoff[4 * s + 1];
    const int nq0 = it.qn[4 * s + 0], nq1 = it.qn[4 * s + 1];
    const double ee2 = pot.eps_ee * pot.eps_ee;
    for (int e = threadIdx.x; e < nq0 * n1 * n1; e += blockDim.x) {
      const int q0 = e / (n1 * n1), a1 = (e / n1) % n1, b1 = e % n1;
      const double x0 = qx0[q0];
      double acc = 0.0;
      for (int q1 = 0; q1 < nq1; ++q1) {
        const double x1 = qx1[q1];
        const double r = x0 - x1;
        acc += qw1[q1] * exp(-d1 * (x1 - al1[a1]) * (x1 - al1[a1])) *
               exp(-d1 * (x1 - al1[b1]) * (x1 - al1[b1])) / sqrt(r * r + ee2);
      }
      T1[e] = acc;
    }
    (void)d0;
    (void)n0;
  }
  __syncthreads();
  // phase C: combine into the full matrix
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int l = e / K, m = e % K;
    int li[4], mi[4];
    split_index(l, nb, D, li);
    split_index(m, nb, D, mi);
    double v = 0.0;
    for (int el = 0; el < N; ++el) {
      double t = v1[v1off[el] + li[el] * nb[el] + mi[el]];
      for (int k2 = 0; k2 < D; ++k2)
        if (k2 != el) t *= S1[s1off[4 * s + k2] + (int64_t)li[k2] * nb[k2] + mi[k2]];
      v += t;
    }
    if (N == 2) {
      const int n1 = nb[1];
      const double d0 = it.delta[4 * s + 0];
      const double* al0 = it.alpha + it.aoff[4 * s + 0];
      const double* qx0 = it.qx + it.qoff[4 * s + 0];
      const double* qw0 = it.qw + it.qoff[4 * s + 0];
      const int nq0 = it.qn[4 * s + 0];
      const int p1 = li[1] * n1 + mi[1];
      double acc = 0.0;
      for (int q0 = 0; q0 < nq0; ++q0) {
        const double x0 = qx0[q0];
        acc += qw0[q0] * exp(-d0 * (x0 - al0[li[0]]) * (x0 - al0[li[0]])) *
               exp(-d0 * (x0 - al0[mi[0]]) * (x0 - al0[mi[0]])) * T1[(int64_t)q0 * n1 * n1 + p1];
      }
      v += acc;
    }
    V[it.off2[s] + e] = v;
  }
}

// ---------------------------------------------------------------------------
// Soft-Coulomb potential with two space dimensions per electron (eq. pseudo,
// D = 2 N): every term is a sum over the tensor Gauss-Legendre grid of its
// dimensions, contracted one dimension at a time with the weighted product
// tables F_k (layout in pot2_layout).  Grid: (blocks, item); each kernel is
// one stage, grid-stride over the stage's outputs for its item.
__device__ inline void pot2_item(const Items& it, int s, int64_t* off, int* nq) {
  int32_t nb[4], qn[4];
  for (int k = 0; k < 4; ++k) {
    nb[k] = k < it.D ? it.nb[4 * s + k] : 1;
    qn[k] = k < it.D ? it.qn[4 * s + k] : 1;
    nq[k] = qn[k];
  }
  pot2_layout(nb, qn, it.n_elec, off);
}

__global__ void k_pot2_tables(Items it, double* scratch, const int64_t* scratch_off) {
  const int s = blockIdx.y;
  int64_t off[11];
  int nq[4];
  pot2_item(it, s, off, nq);
  double* base = scratch + scratch_off[s];
  for (int k = 0; k < it.D; ++k) {
    const int n = it.nb[4 * s + k];
    const double d = it.delta[4 * s + k];
    const double* al = it.alpha + it.aoff[4 * s + k];
    const double* qx = it.qx + it.qoff[4 * s + k];
    const double* qw = it.qw + it.qoff[4 * s + k];
    const int64_t tot = (int64_t)n * n * nq[k];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
      const int p = (int)(e / nq[k]), q = (int)(e - (int64_t)p * nq[k]);
      const int a = p / n, b = p - a * n;
      const double x = qx[q];
      base[off[k] + e] = qw[q] * exp(-d * (x - al[a]) * (x - al[a])) * exp(-d * (x - al[b]) * (x - al[b]));
    }
  }
}

// electron m's nucleus term: Ten[p0 P1 + p1] = sum_{q0, q1} F[p0][q0] F'[p1][q1] U(x_q0, y_q1)
__global__ void k_pot2_en(Items it, Potential pot, double* scratch, const int64_t* scratch_off) {
  const int s = blockIdx.y;
  int64_t off[11];
  int nq[4];
  pot2_item(it, s, off, nq);
  double* base = scratch + scratch_off[s];
  const int geom = s / it.n_sub;
  const double e2 = pot.eps_en * pot.eps_en;
  // written for every electron, zero without nuclei (the combine stage
  // reads every electron's table)
  for (int m = 0; m < it.n_elec; ++m) {
    const int k0 = 2 * m, k1 = 2 * m + 1;
    const int P0 = it.nb[4 * s + k0] * it.nb[4 * s + k0], P1 = it.nb[4 * s + k1] * it.nb[4 * s + k1];
    const double* x0 = it.qx + it.qoff[4 * s + k0];
    const double* x1 = it.qx + it.qoff[4 * s + k1];
    const double* F0 = base + off[k0];
    const double* F1 = base + off[k1];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)P0 * P1;
         e += (int64_t)gridDim.x * blockDim.x) {
      const int p0 = (int)(e / P1), p1 = (int)(e - (int64_t)p0 * P1);
      double acc = 0.0;
      for (int q0 = 0; q0 < nq[k0]; ++q0) {
        double inner = 0.0;
        for (int q1 = 0; q1 < nq[k1]; ++q1) {
          double u = 0.0;
          for (int A = 0; A < pot.n_nuc; ++A) {
            const double* R = pot.pos + (geom * pot.n_nuc + A) * 2;
            const double dx = x0[q0] - R[0], dy = x1[q1] - R[1];
            u -= pot.charge[A] / sqrt(dx * dx + dy * dy + e2);
          }
          inner = fma(F1[(int64_t)p1 * nq[k1] + q1], u, inner);
        }
        acc = fma(F0[(int64_t)p0 * nq[k0] + q0], inner, acc);
      }
      base[off[4 + m] + e] = acc;
    }
  }
}

// electron-electron term, stage 3 - st (st = 0..3): contract q3, then q2, q1, q0
__global__ void k_pot2_ee(Items it, Potential pot, int stage, double* scratch,
                          const int64_t* scratch_off) {
  const int s = blockIdx.y;
  int64_t off[11];
  int nq[4];
  pot2_item(it, s, off, nq);
  double* base = scratch + scratch_off[s];
  int64_t P[4];
  for (int k = 0; k < 4; ++k) P[k] = (int64_t)it.nb[4 * s + k] * it.nb[4 * s + k];
  const double e2 = pot.eps_ee * pot.eps_ee;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (stage == 0) {  // T3[(q0 nq1 + q1) nq2 + q2][p3] = sum_q3 F3[p3][q3] u
    const double* x0 = it.qx + it.qoff[4 * s + 0];
    const double* x1 = it.qx + it.qoff[4 * s + 1];
    const double* x2 = it.qx + it.qoff[4 * s + 2];
    const double* x3 = it.qx + it.qoff[4 * s + 3];
    const double* F3 = base + off[3];
    const int64_t tot = (int64_t)nq[0] * nq[1] * nq[2] * P[3];
    for (int64_t e = e0; e < tot; e += stride) {
      const int64_t g = e / P[3];
      const int p3 = (int)(e - g * P[3]);
      const int q2 = (int)(g % nq[2]);
      const int64_t g1 = g / nq[2];
      const int q1 = (int)(g1 % nq[1]), q0 = (int)(g1 / nq[1]);
      const double dx = x0[q0] - x2[q2];
      const double c = dx * dx + e2;
      double acc = 0.0;
      for (int q3 = 0; q3 < nq[3]; ++q3) {
        const double dy = x1[q1] - x3[q3];
        acc = fma(F3[(int64_t)p3 * nq[3] + q3], 1.0 / sqrt(fma(dy, dy, c)), acc);
      }
      base[off[6] + e] = acc;
    }
  } else if (stage == 1) {  // T2[(q0 nq1 + q1)][p2 P3 + p3] = sum_q2 F2[p2][q2] T3
    const double* F2 = base + off[2];
    const double* T3 = base + off[6];
    const int64_t tot = (int64_t)nq[0] * nq[1] * P[2] * P[3];
    for (int64_t e = e0; e < tot; e += stride) {
      const int64_t g = e / (P[2] * P[3]);
      const int64_t r = e - g * P[2] * P[3];
      const int p2 = (int)(r / P[3]), p3 = (int)(r - (int64_t)p2 * P[3]);
      double acc = 0.0;
      for (int q2 = 0; q2 < nq[2]; ++q2)
        acc = fma(F2[(int64_t)p2 * nq[2] + q2], T3[(g * nq[2] + q2) * P[3] + p3], acc);
      base[off[7] + e] = acc;
    }
  } else if (stage == 2) {  // T1[q0][p1 P2P3 + r] = sum_q1 F1[p1][q1] T2[q0 nq1 + q1][r]
    const double* F1 = base + off[1];
    const double* T2 = base + off[7];
    const int64_t R = P[2] * P[3];
    const int64_t tot = (int64_t)nq[0] * P[1] * R;
    for (int64_t e = e0; e < tot; e += stride) {
      const int64_t q0 = e / (P[1] * R);
      const int64_t t = e - q0 * P[1] * R;
      const int p1 = (int)(t / R);
      const int64_t r = t - (int64_t)p1 * R;
      double acc = 0.0;
      for (int q1 = 0; q1 < nq[1]; ++q1)
        acc = fma(F1[(int64_t)p1 * nq[1] + q1], T2[(q0 * nq[1] + q1) * R + r], acc);
      base[off[8] + e] = acc;
    }
  } else {  // Vee[p0 P1P2P3 + r] = sum_q0 F0[p0][q0] T1[q0][r]
    const double* F0 = base + off[0];
    const double* T1 = base + off[8];
    const int64_t R = P[1] * P[2] * P[3];
    for (int64_t e = e0; e < P[0] * R; e += stride) {
      const int p0 = (int)(e / R);
      const int64_t r = e - (int64_t)p0 * R;
      double acc = 0.0;
      for (int q0 = 0; q0 < nq[0]; ++q0)
        acc = fma(F0[(int64_t)p0 * nq[0] + q0], T1[(int64_t)q0 * R + r], acc);
      base[off[9] + e] = acc;
    }
  }
}

// V[l][m] = sum_m' Ten_m'[pairs of its dims] prod_{other dims} S1 + Vee[pairs]
__global__ void k_pot2_combine(Items it, const double* S1, const int64_t* s1off, double* V,
                               const double* scratch, const int64_t* scratch_off) {
  const int s = blockIdx.y;
  int64_t off[11];
  int nq[4];
  pot2_item(it, s, off, nq);
  const double* base = scratch + scratch_off[s];
  const int K = it.K[s];
  const int D = it.D;
  const int32_t* nb = it.nb + 4 * s;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)K * K;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e / K), m = (int)(e - (int64_t)l * K);
    int li[4], mi[4];
    split_index(l, nb, D, li);
    split_index(m, nb, D, mi);
    int64_t p[4];
    for (int k = 0; k < D; ++k) p[k] = (int64_t)li[k] * nb[k] + mi[k];
    double v = 0.0;
    for (int el = 0; el < it.n_elec; ++el) {
      const int k0 = 2 * el, k1 = 2 * el + 1;
      double t = base[off[4 + el] + p[k0] * ((int64_t)nb[k1] * nb[k1]) + p[k1]];
      for (int k2 = 0; k2 < D; ++k2)
        if (k2 != k0 && k2 != k1) t *= S1[s1off[4 * s + k2] + p[k2]];
      v += t;
    }
    if (it.n_elec == 2) {
      const int64_t P1 = (int64_t)nb[1] * nb[1], P2 = (int64_t)nb[2] * nb[2],
                    P3 = (int64_t)nb[3] * nb[3];
      v += base[off[9] + ((p[0] * P1 + p[1]) * P2 + p[2]) * P3 + p[3]];
    }
    V[it.off2[s] + e] = v;
  }
}

// ---------------------------------------------------------------------------
// Basis values at a point: v_l(y) = prod_k phi_{l_k}(y_k) (or the Slater
// pair of slater.h)
// Local orbital l of item s (one electron, two dimensions) at y, and its
// derivative along dimension kf when dv is given.
__device__ inline double lo2_value(const Items& it, int s, int l, const double* y, int kf,
                                   double* dv) {
  const int n0 = it.nb[4 * s], n1 = it.nb[4 * s + 1], M = it.n_orb;
  const double d0 = it.delta[4 * s], d1 = it.delta[4 * s + 1];
  const double* a0 = it.alpha + it.aoff[4 * s];
  const double* a1 = it.alpha + it.aoff[4 * s + 1];
  const double* C = it.lo_C + (int64_t)s * n0 * n1 * M + l;
  double g1[8], h1[8];  // at most 8 Gaussians per dimension
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const double t = u < n1 ? y[1] - a1[u] : 0.0;
    g1[u] = exp(-d1 * t * t);
    h1[u] = kf == 1 ? -2.0 * d1 * t * g1[u] : g1[u];
  }
  double v = 0.0, w = 0.0;
  for (int u0 = 0; u0 < n0; ++u0) {
    const double t = y[0] - a0[u0];
    const double g0 = exp(-d0 * t * t);
    const double h0 = kf == 0 ? -2.0 * d0 * t * g0 : g0;
#pragma unroll
    for (int u1 = 0; u1 < 8; ++u1)
      if (u1 < n1) {
        const double c = C[(int64_t)(u0 * n1 + u1) * M];
        v = fma(c * g0, g1[u1], v);
        w = fma(c * h0, h1[u1], w);
      }
  }
  if (dv) *dv = w;
  return v;
}

__device__ inline double basis_value(const Items& it, int s, int l, const double* y) {
  if (it.slater) return slater_value(it, s, l, y, nullptr);
  if (it.lo2) return lo2_value(it, s, l, y, 0, nullptr);
  const int32_t* nb = it.nb + 4 * s;
  int li[4];
  split_index(l, nb, it.D, li);
  double v = 1.0;
  for (int k = 0; k < it.D; ++k) {
    const double a = it.alpha[it.aoff[4 * s + k] + li[k]];
    const double d = it.delta[4 * s + k];
    v *= exp(-d * (y[k] - a) * (y[k] - a));
  }
  return v;
}

// v_m(y) of item j and its derivative along dimension kf.
__device__ inline double basis_value_deriv(const Items& it, int j, int m, const double* y, int kf,
                                           double* dv) {
  if (it.slater) {
    double gr[2];
    const double v = slater_value(it, j, m, y, gr);
    *dv = gr[kf];
    return v;
  }
  if (it.lo2) return lo2_value(it, j, m, y, kf, dv);
  int mi[4];
  split_index(m, it.nb + 4 * j, it.D, mi);
  double v = 1.0;
  for (int k = 0; k < it.D; ++k) {
    const double a = it.alpha[it.aoff[4 * j + k] + mi[k]];
    v *= exp(-it.delta[4 * j + k] * (y[k] - a) * (y[k] - a));
  }
  const double aj = it.alpha[it.aoff[4 * j + kf] + mi[kf]];
  *dv = -2.0 * it.delta[4 * j + kf] * (y[kf] - aj) * v;
  return v;
}

// Robin transfer operators (Section 4.1: averaged Robin data over O(y),
// eq. RTC with the outward normal of the receiving subdomain):
// T_ij[l][m] = sum_{y: j in O(y)} w_y / |O(y)| v_l^i(y) (n.grad + mu) v_m^j(y)
__global__ void k_transfer(Items it, Nodes nd, Pairs pr, double mu_re, double mu_im, double2* T) {
  const int p = blockIdx.y;
  const int i = pr.pi[p], j = pr.pj[p];
  const int Ki = it.K[i], Kj = it.K[j];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Ki * Kj) return;
  const int l = e / Kj, m = e % Kj;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t t = pr.noff[p]; t < pr.noff[p + 1]; ++t) {
    const int q = pr.node[t];
    const double* y = nd.x + 4 * (int64_t)q;
    const int face = nd.face[q];
    const int kf = face >> 1;
    const double sign = (face & 1) ? 1.0 : -1.0;
    const double vi = basis_value(it, i, l, y);
    double dj;
    const double vj = basis_value_deriv(it, j, m, y, kf, &dj);
    const double c = nd.w[q] / nd.count[q] * vi;
    acc.x += c * (sign * dj + mu_re * vj);
    acc.y += c * (mu_im * vj);
  }
  T[pr.toff[p] + e] = acc;
}

// Factored pieces of T_ij (D <= 2), one block per (pair, face) entry:
// beta[l_k] = phi^i_{l_k}(x_F), a[m_k] = (sign d/dx + mu) phi^j_{m_k}(x_F),
// X[l_t][m_t] = sum over the entry's nodes of w_y / |O(y)| phi^i_{l_t}(y_t)
// phi^j_{m_t}(y_t) (D = 1: X = sum of w_y / |O(y)| over the one node).
__global__ void k_transfer_tensor(Items it, Nodes nd, Pairs pr, TEnt te, double mu_re,
                                  double mu_im, double* beta, double2* a, double* X) {
  const int e = blockIdx.x;
  const int p = te.pair[e];
  const int i = pr.pi[p], j = pr.pj[p];
  const int face = te.face[e];
  const int kf = face >> 1;
  const double sign = (face & 1) ? 1.0 : -1.0;
  const double xF = nd.x[4 * (int64_t)pr.node[te.t0[e]] + kf];
  const int nbik = it.nb[4 * i + kf], nbjk = it.nb[4 * j + kf];
  for (int l = threadIdx.x; l < nbik; l += blockDim.x) {
    const double c = it.alpha[it.aoff[4 * i + kf] + l];
    beta[te.boff[e] + l] = exp(-it.delta[4 * i + kf] * (xF - c) * (xF - c));
  }
  for (int m = threadIdx.x; m < nbjk; m += blockDim.x) {
    const double c = it.alpha[it.aoff[4 * j + kf] + m];
    const double d = it.delta[4 * j + kf];
    const double v = exp(-d * (xF - c) * (xF - c));
    const double dv = -2.0 * d * (xF - c) * v;
    a[te.aoff[e] + m] = make_double2(sign * dv + mu_re * v, mu_im * v);
  }
  if (it.D == 1) {
    if (threadIdx.x == 0) {
      double acc = 0.0;
      for (int64_t t = te.t0[e]; t < te.t1[e]; ++t) {
        const int q = pr.node[t];
        acc += nd.w[q] / nd.count[q];
      }
      X[te.xoff[e]] = acc;
    }
    return;
  }
  const int tt = 1 - kf;
  const int nbit = it.nb[4 * i + tt], nbjt = it.nb[4 * j + tt];
  const double di = it.delta[4 * i + tt], dj = it.delta[4 * j + tt];
  for (int x = threadIdx.x; x < nbit * nbjt; x += blockDim.x) {
    const int lt = x / nbjt, mt = x % nbjt;
    const double ci = it.alpha[it.aoff[4 * i + tt] + lt];
    const double cj = it.alpha[it.aoff[4 * j + tt] + mt];
    double acc = 0.0;
    for (int64_t t = te.t0[e]; t < te.t1[e]; ++t) {
      const int q = pr.node[t];
      const double y = nd.x[4 * (int64_t)q + tt];
      acc += nd.w[q] / nd.count[q] * exp(-di * (y - ci) * (y - ci)) * exp(-dj * (y - cj) * (y - cj));
    }
    X[te.xoff[e] + x] = acc;
  }
}

// Factored face Gram pieces (D <= 2), one block per (item, face): face f
// = 2k + side of item j, normal dimension k, tangential t:
// b[l_k] = phi_{l_k}(x_F), W[l_t][m_t] = sum over the face's nodes of
// w_y phi_{l_t}(y_t) phi_{m_t}(y_t) (D = 1: W = sum of w_y), so that
// G_j = sum_F (b b^T) (x) W_F.
__global__ void k_gram_tensor(Items it, Nodes nd, TEnt te, double* gram) {
  const int j = blockIdx.x;
  const int f = blockIdx.y;
  const int D = it.D;
  if (f >= 2 * D) return;
  const int k = f >> 1;
  int64_t off = te.gram_off[j];
  for (int g = 0; g < f; ++g) {
    const int kg = g >> 1;
    const int nt = D == 2 ? it.nb[4 * j + (1 - kg)] : 1;
    off += it.nb[4 * j + kg] + nt * nt;
  }
  const int64_t t0 = te.fnode[(j * 8 + f) * 2], cnt = te.fnode[(j * 8 + f) * 2 + 1];
  const double xF = nd.x[4 * t0 + k];
  const int nbk = it.nb[4 * j + k];
  for (int l = threadIdx.x; l < nbk; l += blockDim.x) {
    const double c = it.alpha[it.aoff[4 * j + k] + l];
    gram[off + l] = exp(-it.delta[4 * j + k] * (xF - c) * (xF - c));
  }
  double* W = gram + off + nbk;
  if (D == 1) {
    if (threadIdx.x == 0) {
      double acc = 0.0;
      for (int64_t q = t0; q < t0 + cnt; ++q) acc += nd.w[q];
      W[0] = acc;
    }
    return;
  }
  const int t = 1 - k;
  const int nbt = it.nb[4 * j + t];
  const double dl = it.delta[4 * j + t];
  for (int x = threadIdx.x; x < nbt * nbt; x += blockDim.x) {
    const int a = x / nbt, b = x - a * nbt;
    const double ca = it.alpha[it.aoff[4 * j + t] + a], cb = it.alpha[it.aoff[4 * j + t] + b];
    double acc = 0.0;
    for (int64_t q = t0; q < t0 + cnt; ++q) {
      const double y = nd.x[4 * q + t];
      acc += nd.w[q] * exp(-dl * (y - ca) * (y - ca)) * exp(-dl * (y - cb) * (y - cb));
    }
    W[x] = acc;
  }
}

// Face Gram matrices G[l][m] = sum over every face node of w_y v_l v_m
// (residual of eq. residueRT in coefficient form).
__global__ void k_face_gram(Items it, Nodes nd, double* G) {
  const int s = blockIdx.y;
  const int K = it.K[s];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * K) return;
  const int l = e / K, m = e % K;
  double acc = 0.0;
  for (int64_t q = nd.off[s]; q < nd.off[s + 1]; ++q) {
    const double* y = nd.x + 4 * q;
    acc += nd.w[q] * basis_value(it, s, l, y) * basis_value(it, s, m, y);
  }
  G[it.off2[s] + e] = acc;
}

// ---------------------------------------------------------------------------
// Projection of the Gaussian Cauchy data (Section 4.4 step 1, Test 1.a):
// c~_l = <phi_0, v_l>_{Omega_i}, then A c = c~ by elimination in LDS (A is
// symmetric positive definite).
__global__ void k_project(Items it, const double* A, double init_alpha, const double* center,
                          double2* c0, int* flags) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  const int D = it.D;
  __shared__ double a[kSmallK * kSmallK];
  __shared__ double b[kSmallK];
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) a[e] = A[it.off2[s] + e];
  const double norm = pow(2.0 * init_alpha / M_PI, 0.25 * D);
  // local orbitals: the projections onto the box's Gaussians first, then
  // c~_l = sum_u C[u][l] c~_u
  __shared__ double bg[kSmallK];
  const int KG = it.lo2 ? it.nb[4 * s] * it.nb[4 * s + 1] : K;
  double* bt = it.lo2 ? bg : b;
  for (int l = threadIdx.x; l < KG; l += blockDim.x) {
    int li[4];
    split_index(l, it.nb + 4 * s, D, li);
    double v = norm;
    for (int k = 0; k < D; ++k) {
      const double al = it.alpha[it.aoff[4 * s + k] + li[k]];
      v *= pair_overlap(al, it.delta[4 * s + k], center[k], init_alpha, it.lo[4 * s + k],
                        it.hi[4 * s + k]);
    }
    bt[l] = v;
  }
  __syncthreads();
  if (it.lo2) {
    const double* C = it.lo_C + (int64_t)s * KG * K;
    for (int l = threadIdx.x; l < K; l += blockDim.x) {
      double v = 0.0;
      for (int u = 0; u < KG; ++u) v = fma(C[u * K + l], bg[u], v);
      b[l] = v;
    }
    __syncthreads();
  }
  // forward elimination without pivoting
  for (int p = 0; p < K; ++p) {
    const double piv = a[p * K + p];
    if (threadIdx.x == 0 && !(fabs(piv) > 0.0)) atomicOr(flags, kFlagPivot);
    for (int e = threadIdx.x; e < (K - p - 1) * (K - p); e += blockDim.x) {
      const int r = p + 1 + e / (K - p);
      const int c = p + e % (K - p);
      if (c == p) continue;
      a[r * K + c] -= a[r * K + p] / piv * a[p * K + c];
    }
    __syncthreads();
    for (int r = p + 1 + threadIdx.x; r < K; r += blockDim.x) {
      b[r] -= a[r * K + p] / piv * b[p];
      a[r * K + p] = 0.0;
    }
    __syncthreads();
  }
  // back substitution (single thread: K <= 64, once per geometry)
  if (threadIdx.x == 0) {
    for (int r = K - 1; r >= 0; --r) {
      double v = b[r];
      for (int c = r + 1; c < K; ++c) v -= a[r * K + c] * b[c];
      b[r] = v / a[r * K + r];
    }
  }
  __syncthreads();
  for (int l = threadIdx.x; l < K; l += blockDim.x) {
    c0[it.off1[s] + l] = make_double2(b[l], 0.0);
    if (!isfinite(b[l])) atomicOr(flags, kFlagNaN);
  }
}

// Real parts of the Crank-Nicolson pencil (or the implicit Euler matrix):
//   TDSE: Ar = A - (tau mu_im / 2) B, Ap = A + (tau mu_im / 2) B,
//         Hr = Kin + V + (mu_re / 2) B, so that
//         M^n = Ar + i tau (Hr + E_n Q), R^n = Ap - i tau (Hr + E_n Q);
//   TISE: Hr as above, Ar = A + dt Hr, Ap = A.
__global__ void k_cn_matrices(int64_t n, const double* A, const double* Kin, const double* V,
                              const double* B, double tau, double mu_re, double mu_im,
                              double* Ar, double* Ap, double* Hr, int tise, double dt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double h = Kin[e] + V[e] + 0.5 * mu_re * B[e];
  Hr[e] = h;
  if (tise) {
    Ar[e] = A[e] + dt * h;
    Ap[e] = A[e];
  } else {
    Ar[e] = A[e] - 0.5 * tau * mu_im * B[e];
    Ap[e] = A[e] + 0.5 * tau * mu_im * B[e];
  }
}

// ---------------------------------------------------------------------------
// Batched inversion on the matrix cores: blocked Gauss-Jordan with 16 x 16
// blocks, one wave per block row (NB = ceil(K/16) waves per matrix), complex
// block products as four real v_mfma_f64_16x16x4f64 per k-chunk.
// Block step k: the wave of block row k inverts its diagonal block D in
// registers (unblocked Gauss-Jordan, rows and columns broadcast through
// LDS), forms D A_kj for j != k and publishes the row; every other wave i
// forms A_ij - A_ik (D A_kj) and -A_ik D.  No pivoting (the Hermitian part
// of M is positive definite); padding rows and columns hold the identity.
// Tile layout ("D layout" of the instruction): lane l, register r holds
// entry (4r + l/16, l%16); register q of a tile is then exactly the B
// operand of k-chunk q, and the A operand (entry (l%16, 4q + l/16)) is
// read back from LDS.

// Modes: kInvSteps inverts M^{n+1} (field E_{n+1}) for n < n_mats into packed
// upper tiles; kInvReal inverts the real matrix Ar once per item (TISE) and
// writes it whole, transposed, at the item's K^2 offset; kInvAt inverts the
// matrix at field Eall[n] for n < n_mats and writes it whole, row-major, at
// n * out_stride + the item's K^2 offset.
constexpr int kInvSteps = 0, kInvReal = 1, kInvAt = 2;
template <int NB>
__global__ void __launch_bounds__(64 * NB) k_invert_mfma(Items it, int n_mats, const double* Ar,
                                                         const double* Hr, const double* Q,
                                                         const double* Eall, int64_t out_stride,
                                                         double tau, int mode, double2* Minv,
                                                         int* flags) {
  const int n = blockIdx.x;
  const int s = blockIdx.y;
  const int K = it.K[s];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lr = l >> 4, lc = l & 15;
  __shared__ double2 rowblk[NB][256];  // published block row, [position][r * 64 + lane]
  __shared__ double2 aop[NB][256];     // per wave: a tile row-major, read back as A operand
  __shared__ double2 prow[16], pcol[16];
  const int64_t o2 = it.off2[s];
  const bool tise = mode == kInvReal;
  const double E = mode == kInvAt ? Eall[n] : (tise ? 0.0 : Eall[n + 1]);
  // second component of a circular field (steps only: the series, which
  // uses the kInvAt mode, is never taken with one)
  const double* Q2 = mode == kInvSteps ? it.Q2 : nullptr;
  const double E2 = Q2 ? it.E2[n + 1] : 0.0;
  // the wave's block row; position t holds column block (k + t) mod NB at
  // block step k (rotated after every step), so the pivot block is always
  // position 0 and the step loop need not be unrolled
  double re[NB][4], im[NB][4];
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + 4 * r + lr, col = 16 * j + lc;
      if (row < K && col < K) {
        const int64_t e = o2 + (int64_t)row * K + col;
        re[j][r] = Ar[e];
        im[j][r] = tise ? 0.0 : tau * (Hr[e] + E * Q[e] + (Q2 ? E2 * Q2[e] : 0.0));
      } else {
        re[j][r] = row == col ? 1.0 : 0.0;
        im[j][r] = 0.0;
      }
    }
  bool bad = false;
#pragma unroll 1
  for (int k = 0; k < NB; ++k) {
    if (w == k) {
      // unblocked Gauss-Jordan on the diagonal tile, in place
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        if (lr == (p & 3)) prow[lc] = make_double2(re[0][p >> 2], im[0][p >> 2]);
        if (lc == p) {
#pragma unroll
          for (int r = 0; r < 4; ++r) pcol[4 * r + lr] = make_double2(re[0][r], im[0][r]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double2 piv = prow[p];
        bad |= !(piv.x != 0.0 || piv.y != 0.0);
        const double2 inv = crecip(piv);
        const double2 v = lc == p ? make_double2(1.0, 0.0) : prow[lc];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * r + lr;
          const double2 u = i == p ? make_double2(1.0 - inv.x, -inv.y) : cmul(pcol[i], inv);
          const double bx = lc == p ? (i == p ? 1.0 : 0.0) : re[0][r];
          const double by = lc == p ? 0.0 : im[0][r];
          re[0][r] = fma(-u.x, v.x, fma(u.y, v.y, bx));
          im[0][r] = fma(-u.x, v.y, fma(-u.y, v.x, by));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // A operand of D
#pragma unroll
      for (int r = 0; r < 4; ++r) aop[w][(4 * r + lr) * 16 + lc] = make_double2(re[0][r], im[0][r]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double ar[4], ai[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 t = aop[w][lc * 16 + 4 * q + lr];
        ar[q] = t.x;
        ai[q] = t.y;
      }
      // row update D A_kj at positions 1 ..
#pragma unroll
      for (int t = 1; t < NB; ++t) {
        v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          cr = mfma16(ar[q], re[t][q], cr);
          cr = mfma16(-ai[q], im[t][q], cr);
          ci = mfma16(ar[q], im[t][q], ci);
          ci = mfma16(ai[q], re[t][q], ci);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          re[t][r] = cr[r];
          im[t][r] = ci[r];
        }
      }
#pragma unroll
      for (int t = 0; t < NB; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) rowblk[t][r * 64 + l] = make_double2(re[t][r], im[t][r]);
    }
    __syncthreads();
    if (w != k) {
#pragma unroll
      for (int r = 0; r < 4; ++r) aop[w][(4 * r + lr) * 16 + lc] = make_double2(re[0][r], im[0][r]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double ar[4], ai[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 t = aop[w][lc * 16 + 4 * q + lr];
        ar[q] = t.x;
        ai[q] = t.y;
      }
      // A_ij - A_ik (D A_kj) at positions 1 ..
#pragma unroll
      for (int t = 1; t < NB; ++t) {
        v4d cr = {re[t][0], re[t][1], re[t][2], re[t][3]};
        v4d ci = {im[t][0], im[t][1], im[t][2], im[t][3]};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double2 b = rowblk[t][q * 64 + l];
          cr = mfma16(-ar[q], b.x, cr);
          cr = mfma16(ai[q], b.y, cr);
          ci = mfma16(-ar[q], b.y, ci);
          ci = mfma16(-ai[q], b.x, ci);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          re[t][r] = cr[r];
          im[t][r] = ci[r];
        }
      }
      // -A_ik D at position 0
      v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 b = rowblk[0][q * 64 + l];
        cr = mfma16(-ar[q], b.x, cr);
        cr = mfma16(ai[q], b.y, cr);
        ci = mfma16(-ar[q], b.y, ci);
        ci = mfma16(-ai[q], b.x, ci);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        re[0][r] = cr[r];
        im[0][r] = ci[r];
      }
    }
    // rotate: position t <- t + 1 (the next pivot block comes to position 0)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double x0 = re[0][r], y0 = im[0][r];
#pragma unroll
      for (int t = 0; t + 1 < NB; ++t) {
        re[t][r] = re[t + 1][r];
        im[t][r] = im[t + 1][r];
      }
      re[NB - 1][r] = x0;
      im[NB - 1][r] = y0;
    }
    __syncthreads();
  }
  if (bad) atomicOr(flags, kFlagPivot);
  bool nonfinite = false;
  if (mode != kInvSteps) {  // whole inverses
    double2* out = Minv + (int64_t)n * out_stride + o2;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * w + 4 * r + lr, col = 16 * j + lc;
        if (row < K && col < K) {
          out[tise ? (int64_t)col * K + row : (int64_t)row * K + col] =
              make_double2(re[j][r], im[j][r]);
          nonfinite |= !(isfinite(re[j][r]) && isfinite(im[j][r]));
        }
      }
  } else {  // packed upper 8x8 tiles (the inverse is complex symmetric)
    const int T8 = (K + 7) >> 3;
    double2* out = Minv + (int64_t)n_mats * it.offp[s] + (int64_t)n * 32 * T8 * (T8 + 1);
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * w + 4 * r + lr, col = 16 * j + lc;
        if (row < 8 * T8 && col < 8 * T8 && (row >> 3) <= (col >> 3)) {
          out[(int64_t)tile_index(row >> 3, col >> 3, T8) * 64 + (col & 7) * 8 + (row & 7)] =
              make_double2(re[j][r], im[j][r]);
          nonfinite |= !(isfinite(re[j][r]) && isfinite(im[j][r]));
        }
      }
  }
  if (nonfinite) atomicOr(flags, kFlagNaN);
}

// ---------------------------------------------------------------------------
// Inverses of the window's Crank-Nicolson matrices as series in the field.
// Chunk c of kSeriesChunk steps has its own anchor field E_c; for its steps
// M^n = M_c + d_n C with C = i tau Q, d_n = E_n - E_c, so
//   (M^n)^{-1} = sum_k (-d_n)^k P_k,  P_0 = M_c^{-1},  P_{k+1} = G P_k,
//   G = M_c^{-1} C = i tau P_0 Q.
// The P_k are complex symmetric (as M^n is).  Each chunk's matrices sit in a
// block of `cstride` complex entries: G, then P_0, P_1, ..., each whole and
// row-major at the item's K^2 offset, `stride` apart.

// out = scale * L R (+ add) for every item and chunk: L complex, R complex
// (Rc, chunk-strided like L) or real (Rr, shared by the chunks), add complex
// or null, all K x K row-major at the item's K^2 offset, K <= 64.  On the
// matrix cores: block (item, chunk) of four waves, wave w forms rows 16 w ..
// 16 w + 15 as four 16 x 16 tiles, each complex product four real
// v_mfma_f64_16x16x4f64 per k-chunk; L and R are staged in LDS (rows padded
// to 65 entries), zero past K.  A block reads only its own L and add, so out
// may be L (in place).
constexpr int kSerPad = kSmallK + 1;
template <bool kRealR>
__global__ void __launch_bounds__(kBlock) k_series_product(Items it, const double2* L,
                                                           const double2* Rc, const double* Rr,
                                                           double2 scale, const double2* add,
                                                           int64_t cstride, double2* out) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  const int64_t o2 = it.off2[s];
  const int64_t cz = (int64_t)blockIdx.y * cstride;
  __shared__ double2 sl[kSmallK * kSerPad];
  __shared__ double2 sr[kSmallK * kSerPad];
  for (int e = threadIdx.x; e < kSmallK * kSmallK; e += blockDim.x) {
    const int r = e >> 6, c = e & 63;
    const bool in = r < K && c < K;
    const int64_t g = o2 + (int64_t)r * K + c;
    sl[r * kSerPad + c] = in ? L[cz + g] : make_double2(0.0, 0.0);
    sr[r * kSerPad + c] = in ? (kRealR ? make_double2(Rr[g], 0.0) : Rc[cz + g])
                             : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lr = l >> 4, lc = l & 15;
  v4d cr[4], ci[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    cr[t] = v4d{0.0, 0.0, 0.0, 0.0};
    ci[t] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  for (int kk = 0; kk < kSmallK / 4; ++kk) {
    // A operand: entry (16 w + lc, 4 kk + lr); B operand: (4 kk + lr, 16 t + lc)
    const double2 a = sl[(16 * w + lc) * kSerPad + 4 * kk + lr];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double2 b = sr[(4 * kk + lr) * kSerPad + 16 * t + lc];
      cr[t] = mfma16(a.x, b.x, cr[t]);
      ci[t] = mfma16(a.y, b.x, ci[t]);
      if (!kRealR) {
        cr[t] = mfma16(-a.y, b.y, cr[t]);
        ci[t] = mfma16(a.x, b.y, ci[t]);
      }
    }
  }
  // D layout: register r of lane l is entry (4 r + l / 16, l % 16) of the tile
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + 4 * r + lr, col = 16 * t + lc;
      if (row < K && col < K) {
        const int64_t e = cz + o2 + (int64_t)row * K + col;
        const double2 v = cmul(scale, make_double2(cr[t][r], ci[t][r]));
        out[e] = add ? cadd(add[e], v) : v;
      }
    }
}

constexpr int kSerRows = 16;  // rows per block of the residual

// Residual of an anchor inverse, R = I - M_c X for every item and chunk c,
// M_c = Ar + i tau (Hr + E_c Q) formed entry by entry as the inversion forms
// it, X the chunk's P_0.  The sums are compensated dot products (Ogita, Rump
// and Oishi's Dot2: exact products by fma, error-free additions, errors
// summed aside), as accurate as working in twice the precision, so R is
// accurate although M_c X agrees with I to ~cond(M) eps; one step X + X R
// then brings X to the inverse of M_c rounded to working precision.  Layout
// and blocking as the product above.
__global__ void __launch_bounds__(kBlock) k_series_residual(Items it, const double* Ar,
                                                            const double* Hr, const double* Q,
                                                            const double* Eanchor, double tau,
                                                            const double2* X, int64_t cstride,
                                                            double2* R) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  const int r0 = blockIdx.y * kSerRows;
  if (r0 >= K) return;  // uniform over the block
  const int64_t o2 = it.off2[s];
  const int64_t cz = (int64_t)blockIdx.z * cstride;
  const double E = Eanchor[blockIdx.z];
  __shared__ double2 sm[kSerRows * kSmallK];
  __shared__ double2 sx[kSmallK * kSmallK];
  const int nr = K - r0 < kSerRows ? K - r0 : kSerRows;
  for (int e = threadIdx.x; e < nr * K; e += blockDim.x) {
    const int64_t g = o2 + (int64_t)r0 * K + e;
    sm[e] = make_double2(Ar[g], tau * (Hr[g] + E * Q[g]));
  }
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) sx[e] = X[cz + o2 + e];
  __syncthreads();
  const int col = threadIdx.x & 63, rq = 4 * (threadIdx.x >> 6);
  if (col >= K) return;
  // four rows at once: eight independent accumulation chains per thread
  // (rows past nr read row 0 of the block and are not stored)
  Dot2 re[4], im[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    re[q] = Dot2{r0 + rq + q == col ? 1.0 : 0.0, 0.0};
    im[q] = Dot2{0.0, 0.0};
  }
  for (int m = 0; m < K; ++m) {
    const double2 b = sx[m * K + col];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 a = sm[(rq + q < nr ? rq + q : 0) * K + m];
      dot2_acc(re[q], -a.x, b.x);
      dot2_acc(re[q], a.y, b.y);
      dot2_acc(im[q], -a.x, b.y);
      dot2_acc(im[q], -a.y, b.x);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (rq + q < nr)
      R[cz + o2 + (int64_t)(r0 + rq + q) * K + col] =
          make_double2(re[q].s + re[q].c, im[q].s + im[q].c);
}

// (M^{n+1})^{-1} = sum_{k < NT} (-d)^k P_k, d = E_{n+1} - E_c, into the packed
// upper tiles of every step n < n_mats (Horner in d).  Block (item, chunk c
// of kSeriesChunk steps); thread t keeps the NT coefficients of packed
// entries t, t + 256, ... in registers while it walks the chunk's steps.
// Entries outside K (padding of the last tile) hold the identity.
template <int NT>
__global__ void __launch_bounds__(kBlock) k_series_assemble(Items it, int n_mats,
                                                            const double2* P, int64_t stride,
                                                            int64_t cstride, const double* Eall,
                                                            const double* Eanchor,
                                                            double2* Minv) {
  const int s = blockIdx.x;
  const int c = blockIdx.y;
  const int K = it.K[s];
  const int T8 = (K + 7) >> 3;
  const int n_ent = 32 * T8 * (T8 + 1);
  const int n0 = c * kSeriesChunk;
  const int n1 = n0 + kSeriesChunk < n_mats ? n0 + kSeriesChunk : n_mats;
  const int64_t o2 = it.off2[s];
  const double2* Pc = P + (int64_t)c * cstride;
  const double Ec = Eanchor[c];
  double2* out = Minv + (int64_t)n_mats * it.offp[s];
  for (int e = threadIdx.x; e < n_ent; e += blockDim.x) {
    // tile (I, J), I <= J, of packed index e / 64; entry (a, b) at b 8 + a
    const int t = e >> 6;
    int I = 0;
    while (I + 1 < T8 && tile_index(I + 1, I + 1, T8) <= t) ++I;
    const int J = I + (t - tile_index(I, I, T8));
    const int row = 8 * I + (e & 7), col = 8 * J + ((e >> 3) & 7);
    const bool inside = row < K && col < K;
    double cx[NT], cy[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const double2 v = inside ? Pc[k * stride + o2 + (int64_t)row * K + col]
                               : make_double2(k == 0 && row == col ? 1.0 : 0.0, 0.0);
      cx[k] = v.x;
      cy[k] = v.y;
    }
    for (int n = n0; n < n1; ++n) {
      const double d = Ec - Eall[n + 1];  // -(E_{n+1} - E_c)
      double vx = cx[NT - 1], vy = cy[NT - 1];
#pragma unroll
      for (int k = NT - 2; k >= 0; --k) {
        vx = fma(d, vx, cx[k]);
        vy = fma(d, vy, cy[k]);
      }
      out[(int64_t)n * n_ent + e] = make_double2(vx, vy);
    }
  }
}

// ---------------------------------------------------------------------------
// Crank-Nicolson recurrence (Section 4.4 step 2), one block of 512 threads
// per (item, job); a job runs the steps n_lo .. n_lo+n_cnt-1 of one Schwarz
// iterate (the whole window, or one chunk of it).  With
// M^n = Ar + i tau (Hr + E_n Q) the matrix that was inverted and Ap the
// mass part of the explicit half step, the explicit matrix is
// Ap - i tau (Hr + E_n Q) = (Ar + Ap) - M^n, and M^n c^n is the right-hand
// side of the previous step.  So every step after the first costs one real
// product and the inverse:
//   rhs^n   = (Ar + Ap) c^n - rhs^{n-1} + (i tau / 2)(f^n + f^{n+1})
//   c^{n+1} = (M^{n+1})^{-1} rhs^n
// The map rhs^{n-1} -> rhs^n is the Cayley transform of the step, so
// rounding errors are carried, not amplified.  The first step of a job takes
// rhs^{n_lo-1} = M^{n_lo} c^{n_lo} from the carry the previous chunk of the
// iterate left, or forms it from the matrices at the start of the window.
// Thread (r, part) owns row r and the eight columns m = 8 j + part, one in
// each column block j: its entries of Ar + Ap stay in registers; the inverse matrix and the Robin
// data vector f^{n+1} of step n are prefetched PD steps ahead into a
// register buffer of their own (so no loaded register is ever moved before
// it is used: a move would wait for the load); the sums over the eight parts
// are DPP butterflies inside groups of eight lanes.
constexpr int kRecThreads = 512;
constexpr int kRecPrefetch = 3;  // steps between a load of the inverse and its use
// LDS vectors of the recurrence: entry m at (m / 8) * 9 + m % 8, so that the
// eight column groups read by a wave fall in different banks
constexpr int kVecPad = 9 * (kSmallK / 8);
__device__ inline int vpos(int m) { return (m >> 3) * 9 + (m & 7); }

struct RecState {
  double s2[8];         // Ar + Ap at this thread's columns of row r
  double2 cm[8];        // c^n at this thread's columns
  double2 fprev;        // f^n at row r
  double2 rprev;        // rhs^{n-1} = M^n c^n at row r
};

struct RecPipe {
  double2 m[8];         // inverse of M^{n+1}: row r, columns m (transposed storage)
  double2 f;            // f^{n+1} at row r
};


// Loads of everything step n consumes.  Unconditional, from clamped
// addresses: entries past K multiply the zero padding of the LDS vectors
// (columns) or are discarded (rows); steps past the job's end are never
// consumed.
// The inverse of step n is read from the packed upper tiles: entry
// (8 I + a, 8 j + part) is entry (a, part) of tile (I, j) when j >= I, else
// entry (part, a) of tile (j, I).  The 64 lanes of a wave share I (its eight
// rows are one tile row), so each load reads one whole tile: 1 KB
// contiguous.  Row and tile indices are clamped, so padding lanes read
// valid entries.
__device__ inline void prefetch(RecPipe& pp, const double2* Mb, const double2* F, int64_t hb,
                                int n, int n_end, int K, int r, int part) {
  const int rr = r < K ? r : K - 1;
  const int nn = n < n_end ? n : n_end - 1;
  pp.f = F[hb + (int64_t)(nn + 1) * K + rr];
  const int T8 = (K + 7) >> 3;
  const int I = rr >> 3, a = rr & 7;
  const double2* base = Mb + (int64_t)nn * 32 * T8 * (T8 + 1);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int J = j < T8 ? j : T8 - 1;
    pp.m[j] = J >= I ? base[tile_index(I, J, T8) * 64 + part * 8 + a]
                     : base[tile_index(J, I, T8) * 64 + a * 8 + part];
  }
}

template <int PD>
__device__ inline void cn_step(RecState& st, RecPipe& pp, int n, int n_end, int K, int r,
                               int part, double tau, const double2* Mb, const double2* F,
                               double2* hist, int64_t hb, double2* sc, double2* srhs, bool& bad) {
  double ax = 0.0, ay = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    ax = fma(st.s2[j], st.cm[j].x, ax);
    ay = fma(st.s2[j], st.cm[j].y, ay);
  }
  ax = group8_sum(ax);
  ay = group8_sum(ay);
  const double2 fs = cadd(st.fprev, pp.f);
  st.fprev = pp.f;
  const double2 rhs = make_double2(fma(-0.5 * tau, fs.y, ax - st.rprev.x),
                                   fma(0.5 * tau, fs.x, ay - st.rprev.y));
  st.rprev = rhs;
  if (r < K) srhs[vpos(r)] = rhs;
  __syncthreads();
  double ox = 0.0, oy = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double2 rm = srhs[j * 9 + part];  // zero padded past K
    ox = fma(pp.m[j].x, rm.x, fma(-pp.m[j].y, rm.y, ox));
    oy = fma(pp.m[j].x, rm.y, fma(pp.m[j].y, rm.x, oy));
  }
  ox = group8_sum(ox);
  oy = group8_sum(oy);
  prefetch(pp, Mb, F, hb, n + PD, n_end, K, r, part);
  const double2 v = make_double2(ox, oy);
  if (r < K) sc[vpos(r)] = v;
  // Every lane stores (no divergent branch around the store, which would
  // make the memory-counter waits conservative): the eight lanes of a row
  // hold the same value, and padding rows r >= K loaded row K-1's data, so
  // they write bit-identical copies of row K-1.
  hist[hb + (int64_t)(n + 1) * K + (r < K ? r : K - 1)] = v;
  bad |= !cfinite(v);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) st.cm[j] = sc[j * 9 + part];  // zero padded past K
}

// PD = prefetch distance in steps (register buffers in flight)
template <int PD>
__global__ void __launch_bounds__(kRecThreads) k_cn_recur(Items it, int n_steps, const double* Ar,
                                                          const double* Ap, const double* Hr,
                                                          const double* Q, const double* Eall,
                                                          double tau, const double2* Minv,
                                                          const double2* c0, RecJobs jobs,
                                                          int* flags) {
  const int s = blockIdx.x;
  const int job = blockIdx.y;
  const int K = it.K[s];
  const int n_lo = jobs.n_lo[job];
  const int n_end = n_lo + jobs.n_cnt[job];
  double2* hist = jobs.hist[job];
  const double2* F = jobs.F[job];
  double2* carry = jobs.carry[job];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int part = lane & 7;
  const int r = wave * 8 + (lane >> 3);
  __shared__ double2 sc[kVecPad];
  __shared__ double2 srhs[kVecPad];
  const int64_t o2 = it.off2[s];
  const int64_t hb = (int64_t)(n_steps + 1) * it.off1[s];
  const int rr = r < K ? r : K - 1;
  RecState st;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int m = 8 * j + part;
    const bool v = r < K && m < K;
    const int64_t e = o2 + (v ? (int64_t)m * K + r : 0);
    // symmetric matrices: entry (m, r) = entry (r, m)
    st.s2[j] = v ? Ar[e] + Ap[e] : 0.0;
  }
  st.fprev = F[hb + (int64_t)n_lo * K + rr];
  // The carried right-hand side goes through LDS, so that its load is waited
  // for here: a load still pending when the loop starts would make the
  // loop's memory waits drain every prefetch.
  const bool use_carry = n_lo > 0 && carry != nullptr;
  if (threadIdx.x < K) {
    double2 v;
    if (n_lo == 0) {
      v = c0[it.off1[s] + threadIdx.x];
      hist[hb + threadIdx.x] = v;
    } else {
      v = hist[hb + (int64_t)n_lo * K + threadIdx.x];
    }
    sc[vpos(threadIdx.x)] = v;
    if (use_carry) srhs[vpos(threadIdx.x)] = carry[it.off1[s] + threadIdx.x];
  } else if (threadIdx.x < kSmallK) {
    // padding past K stays zero for the whole job
    sc[vpos(threadIdx.x)] = make_double2(0.0, 0.0);
    srhs[vpos(threadIdx.x)] = make_double2(0.0, 0.0);
  }
  const double2* Mb = Minv + (int64_t)n_steps * it.offp[s];
  RecPipe pA, pB, pC;
  prefetch(pA, Mb, F, hb, n_lo, n_end, K, r, part);
  prefetch(pB, Mb, F, hb, n_lo + 1, n_end, K, r, part);
  if (PD == 3) prefetch(pC, Mb, F, hb, n_lo + 2, n_end, K, r, part);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) st.cm[j] = sc[j * 9 + part];
  if (use_carry) {
    // each wave reads only its own rows, which only it overwrites later
    st.rprev = r < K ? srhs[vpos(r)] : make_double2(0.0, 0.0);
  } else {
    // M^{n_lo} c^{n_lo} = Ar c + i tau (Hr + E Q + E2 Q2) c
    const double E = Eall[n_lo];
    const double E2 = it.Q2 ? it.E2[n_lo] : 0.0;
    double ax = 0.0, ay = 0.0, hx = 0.0, hy = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int m = 8 * j + part;
      const bool v = r < K && m < K;
      const int64_t e = o2 + (v ? (int64_t)m * K + r : 0);
      const double a = v ? Ar[e] : 0.0;
      const double h = v ? fma(E, Q[e], Hr[e]) + (it.Q2 ? E2 * it.Q2[e] : 0.0) : 0.0;
      ax = fma(a, st.cm[j].x, ax);
      ay = fma(a, st.cm[j].y, ay);
      hx = fma(h, st.cm[j].x, hx);
      hy = fma(h, st.cm[j].y, hy);
    }
    st.rprev = make_double2(group8_sum(fma(-tau, hy, ax)), group8_sum(fma(tau, hx, ay)));
  }
  bool bad = false;
  // unconditional PD-step body (a conditional tail inside the body would make
  // the loop-header wait state assume the first buffer was loaded last)
  int n = n_lo;
  for (; n + PD - 1 < n_end; n += PD) {
    cn_step<PD>(st, pA, n, n_end, K, r, part, tau, Mb, F, hist, hb, sc, srhs, bad);
    cn_step<PD>(st, pB, n + 1, n_end, K, r, part, tau, Mb, F, hist, hb, sc, srhs, bad);
    if (PD == 3) cn_step<PD>(st, pC, n + 2, n_end, K, r, part, tau, Mb, F, hist, hb, sc, srhs, bad);
  }
  if (n < n_end) cn_step<PD>(st, pA, n, n_end, K, r, part, tau, Mb, F, hist, hb, sc, srhs, bad);
  if (n + 1 < n_end) cn_step<PD>(st, pB, n + 1, n_end, K, r, part, tau, Mb, F, hist, hb, sc, srhs, bad);
  // rhs of the last step = M^{n_end} c^{n_end}, for the next chunk
  if (carry && part == 0 && r < K) carry[it.off1[s] + r] = st.rprev;
  if (bad) atomicOr(flags, kFlagNaN);
}

// ---------------------------------------------------------------------------
// The same recurrence with each step's inverse evaluated from the field
// series inside the step instead of read from HBM.  The chunk's terms
// P_0 .. P_{NT-1} at this thread's eight entries (row r, columns 8 j + part)
// stay in registers while the block walks the chunk's steps, and step n forms
// (M^{n+1})^{-1} entry by entry by Horner in d = E_c - E_{n+1}, as the packed
// assembly does: the same entries (a tile below the diagonal takes the
// transposed entry of the tile above it), the same operations in the same
// order, so the result is the one the stored inverses give.  HBM carries per
// step only the Robin data vector in and the coefficients out; the terms are
// read once per chunk of kSeriesChunk steps.  The Robin data and the
// offsets d (formed once per window, E_c - E_{n+1} rounded as the assembly
// rounds it) of kRecTile steps are staged in LDS one tile ahead; tiles are
// aligned to multiples of kRecTile, so every chunk starts on a tile.
constexpr int kRecTile = 16;
static_assert(kSeriesChunk % kRecTile == 0, "chunks start on tiles");

// Pi: the chunk's P_0 at the item (uniform); entries by 32-bit lane offsets
// (a 64-bit address per entry and term would be kept live across the loop)
template <int NT>
__device__ inline void load_terms(double2 (&p)[NT][8], const double2* Pi, int64_t stride, int K,
                                  int r, int part) {
  const int rr = r < K ? r : K - 1;
  const int I = rr >> 3;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int m = 8 * j + part;
    const int mm = m < K ? m : K - 1;
    const unsigned e = j >= I ? (unsigned)(rr * K + mm) : (unsigned)(mm * K + rr);
    // columns past K hold column K-1's (finite) entries: they meet the zero
    // padding of the LDS vector
#pragma unroll
    for (int k = 0; k < NT; ++k) p[k][j] = (Pi + k * stride)[e];
  }
}

// Staging registers of one tile: Robin data f^{n+1} of the tile's steps at
// two (step, row) entries of this thread, and d of step tid (tid < kRecTile).
// (Named fields, not an array: an array here is kept in scratch memory.)
struct RecTileRegs {
  double2 f0, f1;
  double d;
};
static_assert(kRecTile * kSmallK == 2 * kRecThreads, "two staged entries per thread");

__device__ inline double2 tile_entry(const double2* F, int64_t hb, int T, int e, int n_lo,
                                     int n_end, int K) {
  int n = T * kRecTile + (e >> 6);
  n = n < n_lo ? n_lo : (n < n_end ? n : n_end - 1);
  const int row = e & 63;
  return F[hb + (int64_t)(n + 1) * K + (row < K ? row : K - 1)];
}

__device__ inline void load_tile(RecTileRegs& tr, const double2* F, int64_t hb, int T, int n_lo,
                                 int n_end, int K, const double* D) {
  tr.f0 = tile_entry(F, hb, T, threadIdx.x, n_lo, n_end, K);
  tr.f1 = tile_entry(F, hb, T, threadIdx.x + kRecThreads, n_lo, n_end, K);
  int n = T * kRecTile + (threadIdx.x & (kRecTile - 1));
  n = n < n_lo ? n_lo : (n < n_end ? n : n_end - 1);
  tr.d = D[n];
}

__device__ inline void store_tile(const RecTileRegs& tr, double2 (*sf)[kSmallK], double* sd) {
  const int e0 = threadIdx.x, e1 = threadIdx.x + kRecThreads;
  sf[e0 >> 6][e0 & 63] = tr.f0;
  sf[e1 >> 6][e1 & 63] = tr.f1;
  // every thread holds d of step threadIdx.x % kRecTile: equal values, and
  // no branch (a store under a branch makes the memory waits conservative)
  sd[threadIdx.x & (kRecTile - 1)] = tr.d;
}

template <int NT>
__device__ inline void cn_step_series(RecState& st, const double2 (&p)[NT][8], double d,
                                      double2 fn, int K, int r, int part, double tau,
                                      double2* shrow, double2* sc, double2* srhs, bool& bad) {
  double ax = 0.0, ay = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    ax = fma(st.s2[j], st.cm[j].x, ax);
    ay = fma(st.s2[j], st.cm[j].y, ay);
  }
  ax = group8_sum(ax);
  ay = group8_sum(ay);
  const double2 fs = cadd(st.fprev, fn);
  st.fprev = fn;
  const double2 rhs = make_double2(fma(-0.5 * tau, fs.y, ax - st.rprev.x),
                                   fma(0.5 * tau, fs.x, ay - st.rprev.y));
  st.rprev = rhs;
  if (r < K) srhs[vpos(r)] = rhs;
  __syncthreads();
  double ox = 0.0, oy = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double mx = p[NT - 1][j].x, my = p[NT - 1][j].y;
#pragma unroll
    for (int k = NT - 2; k >= 0; --k) {
      mx = fma(d, mx, p[k][j].x);
      my = fma(d, my, p[k][j].y);
    }
    const double2 rm = srhs[j * 9 + part];  // zero padded past K
    ox = fma(mx, rm.x, fma(-my, rm.y, ox));
    oy = fma(mx, rm.y, fma(my, rm.x, oy));
  }
  ox = group8_sum(ox);
  oy = group8_sum(oy);
  const double2 v = make_double2(ox, oy);
  if (r < K) sc[vpos(r)] = v;
  // padding rows hold row K-1's entries: their value is row K-1's
  if (part == 0) *shrow = v;
  bad |= !cfinite(v);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) st.cm[j] = sc[j * 9 + part];
}

// The coefficients of tile T's steps (staged in LDS by the steps) to the
// history: two entries per thread, unconditional; entries outside the job's
// steps or past K take the nearest valid entry of the tile (the same value
// written twice).
__device__ inline void flush_tile(double2* hist, int64_t hb, const double2 (*sh)[kSmallK], int T,
                                  int n_lo, int n_end, int K) {
  const int lo = T * kRecTile > n_lo ? T * kRecTile : n_lo;
  const int hi = (T + 1) * kRecTile < n_end ? (T + 1) * kRecTile : n_end;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = threadIdx.x + h * kRecThreads;
    int n = T * kRecTile + (e >> 6);
    n = n < lo ? lo : (n < hi ? n : hi - 1);
    const int row = (e & 63) < K ? (e & 63) : K - 1;
    hist[hb + (int64_t)(n + 1) * K + row] = sh[n - T * kRecTile][row];
  }
}

template <int NT>
__global__ void __launch_bounds__(kRecThreads)
    k_cn_recur_series(Items it, int n_steps, const double* Ar, const double* Ap, const double* Hr,
                      const double* Q, const double* Eall, double tau, RecSeries se,
                      const double2* c0, RecJobs jobs, int* flags) {
  const int s = blockIdx.x;
  const int job = blockIdx.y;
  const int K = it.K[s];
  const int n_lo = jobs.n_lo[job];
  const int n_end = n_lo + jobs.n_cnt[job];
  double2* hist = jobs.hist[job];
  const double2* F = jobs.F[job];
  double2* carry = jobs.carry[job];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int part = lane & 7;
  const int r = wave * 8 + (lane >> 3);
  __shared__ double2 sc[kVecPad];
  __shared__ double2 srhs[kVecPad];
  __shared__ double2 sf[2][kRecTile][kSmallK];
  __shared__ double2 sh[2][kRecTile][kSmallK];
  __shared__ double sd[2][kRecTile];
  const int64_t o2 = it.off2[s];
  const int64_t hb = (int64_t)(n_steps + 1) * it.off1[s];
  const int rr = r < K ? r : K - 1;
  RecState st;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int m = 8 * j + part;
    const bool v = r < K && m < K;
    const int64_t e = o2 + (v ? (int64_t)m * K + r : 0);
    st.s2[j] = v ? Ar[e] + Ap[e] : 0.0;
  }
  st.fprev = F[hb + (int64_t)n_lo * K + rr];
  const bool use_carry = n_lo > 0 && carry != nullptr;
  if (threadIdx.x < K) {
    double2 v;
    if (n_lo == 0) {
      v = c0[it.off1[s] + threadIdx.x];
      hist[hb + threadIdx.x] = v;
    } else {
      v = hist[hb + (int64_t)n_lo * K + threadIdx.x];
    }
    sc[vpos(threadIdx.x)] = v;
    if (use_carry) srhs[vpos(threadIdx.x)] = carry[it.off1[s] + threadIdx.x];
  } else if (threadIdx.x < kSmallK) {
    sc[vpos(threadIdx.x)] = make_double2(0.0, 0.0);
    srhs[vpos(threadIdx.x)] = make_double2(0.0, 0.0);
  }
  int T = n_lo / kRecTile;
  RecTileRegs tr;
  load_tile(tr, F, hb, T, n_lo, n_end, K, se.D);
  double2 p[NT][8];
  load_terms<NT>(p, se.P + (int64_t)(n_lo / kSeriesChunk) * se.cstride + o2, se.stride, K, r,
                 part);
  store_tile(tr, sf[0], sd[0]);
  load_tile(tr, F, hb, T + 1, n_lo, n_end, K, se.D);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) st.cm[j] = sc[j * 9 + part];
  if (use_carry) {
    st.rprev = r < K ? srhs[vpos(r)] : make_double2(0.0, 0.0);
  } else {
    // M^{n_lo} c^{n_lo} = Ar c + i tau (Hr + E Q) c (the series path has one field)
    const double E = Eall[n_lo];
    double ax = 0.0, ay = 0.0, hx = 0.0, hy = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int m = 8 * j + part;
      const bool v = r < K && m < K;
      const int64_t e = o2 + (v ? (int64_t)m * K + r : 0);
      const double a = v ? Ar[e] : 0.0;
      const double h = v ? fma(E, Q[e], Hr[e]) : 0.0;
      ax = fma(a, st.cm[j].x, ax);
      ay = fma(a, st.cm[j].y, ay);
      hx = fma(h, st.cm[j].x, hx);
      hy = fma(h, st.cm[j].y, hy);
    }
    st.rprev = make_double2(group8_sum(fma(-tau, hy, ax)), group8_sum(fma(tau, hx, ay)));
  }
  bool bad = false;
  int buf = 0;
  int n = n_lo;
  // Global memory is touched only between tiles, in an order that keeps
  // every wait the compiler inserts on older operations: the staged tile
  // (loaded a tile ago) to LDS, the chunk's terms at a chunk start, the loads
  // of the tile after next, then the finished tile's coefficients out.  No
  // step waits on a load or a store.
  while (true) {
    const int te = (T + 1) * kRecTile < n_end ? (T + 1) * kRecTile : n_end;
    for (; n < te; ++n) {
      const int q = n - T * kRecTile;
      cn_step_series<NT>(st, p, sd[buf][q], sf[buf][q][r], K, r, part, tau, &sh[buf][q][r], sc,
                         srhs, bad);
    }
    if (n >= n_end) break;
    store_tile(tr, sf[buf ^ 1], sd[buf ^ 1]);
    if (n % kSeriesChunk == 0)
      load_terms<NT>(p, se.P + (int64_t)(n / kSeriesChunk) * se.cstride + o2, se.stride, K, r,
                     part);
    load_tile(tr, F, hb, T + 2, n_lo, n_end, K, se.D);
    flush_tile(hist, hb, sh[buf], T, n_lo, n_end, K);
    ++T;
    buf ^= 1;
    __syncthreads();
  }
  flush_tile(hist, hb, sh[buf], T, n_lo, n_end, K);
  if (carry && part == 0 && r < K) carry[it.off1[s] + r] = st.rprev;
  if (bad) atomicOr(flags, kFlagNaN);
}

// ---------------------------------------------------------------------------
// Transmission as a batched complex product: for receiving item i and a tile
// of time steps, F_i[n][l] = scale_n * sum_{pairs (i,j)} sum_m T_ij[l][m] C_j[n][m].
// Dense form (any D); one job per grid z.  The products run on the FP64
// matrix cores with A = C (steps x columns m) and B = T^T (columns m x
// receiver functions): per 16 x 16 output tile and four columns, four real
// v_mfma_f64_16x16x4f64 (re += Cr Tr - Ci Ti, im += Ci Tr + Cr Ti).
constexpr int kTN = 32;
constexpr int kTM = 16;
constexpr int kTRow = kSmallK + 1;
__global__ void __launch_bounds__(kBlock) k_transmit(Items it, Pairs pr, int n_steps,
                                                     const double2* T, TxJobs jobs) {
  const int i = blockIdx.y;
  const int job = blockIdx.z;
  const double* scale = jobs.scale[job];
  const int n0 = jobs.n_lo[job] + blockIdx.x * kTN;
  const int n_hi = jobs.n_hi[job];
  if (n0 > n_hi) return;  // uniform over the block
  const double2* hist = jobs.src[job];
  double2* F = jobs.dst[job];
  const int Ki = it.K[i];
  // T in slices of kTM columns (three blocks share a CU); rows of both
  // tiles padded to 65 entries, so that the operand reads (16 consecutive
  // rows or columns per quarter wave) spread over the banks
  __shared__ double2 Ts[kTM * kTRow];  // [m - m0][l]
  __shared__ double2 Cs[kTN * kTRow];  // [nn][m]
  // wave w: steps 16 (w & 1) .. + 15 of the tile, receiver tiles w >> 1 and
  // (w >> 1) + 2 (so that items with K <= 32 still keep every wave busy)
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane >> 4, lc = lane & 15;
  const int rt = w & 1, ct = w >> 1;
  const bool on0 = 16 * ct < Ki, on1 = 16 * (ct + 2) < Ki;  // uniform over the wave
  v4d re0 = {0.0, 0.0, 0.0, 0.0}, im0 = re0, re1 = re0, im1 = re0;
  // Stages (pair p, slice from column m0), each one's loads issued into
  // registers while the previous one computes.
  constexpr int kUT = kTM * kSmallK / kBlock, kUC = kTN * kSmallK / kBlock;
  double tx[kUT], ty[kUT], cx[kUC], cy[kUC];
  auto fetch = [&](int64_t p, int m0) {
    const int j = pr.pj[p];
    const int Kj = it.K[j];
    const int cnt = Kj - m0 < kTM ? Kj - m0 : kTM;
    const double2* Tp = T + pr.toff[p];
#pragma unroll
    for (int u = 0; u < kUT; ++u) {
      const int e = u * kBlock + (int)threadIdx.x;
      const int ll = e / cnt, mm = e - ll * cnt;
      const double2 v = e < Ki * cnt ? Tp[(int64_t)ll * Kj + m0 + mm] : make_double2(0.0, 0.0);
      tx[u] = v.x;
      ty[u] = v.y;
    }
    if (m0 == 0) {
      const int64_t hb = (int64_t)(n_steps + 1) * it.off1[j];
#pragma unroll
      for (int u = 0; u < kUC; ++u) {
        const int e = u * kBlock + (int)threadIdx.x;
        const int nn = e / Kj, mm = e - nn * Kj;
        const double2 v = (e < kTN * Kj && n0 + nn <= n_hi) ? hist[hb + (int64_t)(n0 + nn) * Kj + mm]
                                                             : make_double2(0.0, 0.0);
        cx[u] = v.x;
        cy[u] = v.y;
      }
    }
  };
  int64_t p = pr.poff[i];
  int m0 = 0;
  if (p < pr.poff[i + 1]) fetch(p, 0);
  while (p < pr.poff[i + 1]) {
    const int Kj = it.K[pr.pj[p]];
    const int cnt = Kj - m0 < kTM ? Kj - m0 : kTM;
    __syncthreads();  // the previous stage is read
#pragma unroll
    for (int u = 0; u < kUT; ++u) {
      const int e = u * kBlock + (int)threadIdx.x;
      const int ll = e / cnt, mm = e - ll * cnt;
      if (e < Ki * cnt) Ts[mm * kTRow + ll] = make_double2(tx[u], ty[u]);
    }
    if (m0 == 0)
#pragma unroll
      for (int u = 0; u < kUC; ++u) {
        const int e = u * kBlock + (int)threadIdx.x;
        const int nn = e / Kj, mm = e - nn * Kj;
        if (e < kTN * Kj) Cs[nn * kTRow + mm] = make_double2(cx[u], cy[u]);
      }
    // zeros in the columns that pad the slice to a multiple of four: T's
    // rows cnt .. (last slice of a pair), C's columns Kj .. (every row)
    if ((cnt & 3) && (int)threadIdx.x < 64 * (4 - (cnt & 3)))
      Ts[(cnt + (threadIdx.x >> 6)) * kTRow + (threadIdx.x & 63)] = make_double2(0.0, 0.0);
    if (m0 == 0 && (Kj & 3) && (int)threadIdx.x < kTN * (4 - (Kj & 3)))
      Cs[(threadIdx.x % kTN) * kTRow + Kj + threadIdx.x / kTN] = make_double2(0.0, 0.0);
    __syncthreads();
    const int cm0 = m0;
    m0 += kTM;
    if (m0 >= Kj) {
      m0 = 0;
      ++p;
    }
    if (p < pr.poff[i + 1]) fetch(p, m0);
    if (on0) {
      for (int kk = 0; kk < cnt; kk += 4) {
        const int mm = kk + lr;
        const double2 a = Cs[(16 * rt + lc) * kTRow + cm0 + mm];
        const double2 b0 = Ts[mm * kTRow + 16 * ct + lc];
        re0 = mfma16(a.x, b0.x, re0);
        re0 = mfma16(-a.y, b0.y, re0);
        im0 = mfma16(a.y, b0.x, im0);
        im0 = mfma16(a.x, b0.y, im0);
        if (on1) {
          const double2 b1 = Ts[mm * kTRow + 16 * (ct + 2) + lc];
          re1 = mfma16(a.x, b1.x, re1);
          re1 = mfma16(-a.y, b1.y, re1);
          im1 = mfma16(a.y, b1.x, im1);
          im1 = mfma16(a.x, b1.y, im1);
        }
      }
    }
  }
  // register r of a tile: step 16 rt + 4 r + lr, receiver function 16 ct + lc
  const int64_t fb = (int64_t)(n_steps + 1) * it.off1[i];
  const int l0 = 16 * ct + lc, l1 = l0 + 32;
  auto put = [&](int r, double a0, double b0, double a1, double b1) {
    const int n = n0 + 16 * rt + 4 * r + lr;
    if (n > n_hi) return;
    const double sc = scale ? scale[n] : 1.0;
    if (on0 && l0 < Ki) F[fb + (int64_t)n * Ki + l0] = make_double2(a0 * sc, b0 * sc);
    if (on1 && l1 < Ki) F[fb + (int64_t)n * Ki + l1] = make_double2(a1 * sc, b1 * sc);
  };
  put(0, re0.x, im0.x, re1.x, im1.x);
  put(1, re0.y, im0.y, re1.y, im1.y);
  put(2, re0.z, im0.z, re1.z, im1.z);
  put(3, re0.w, im0.w, re1.w, im1.w);
}

// Factored form (D <= 2), in two passes.  Per entry e (pair (i,j), face of
// i with normal dimension k and tangential dimension t) and step n:
//   u_e[m_t] = sum_{m_k} a_e[m_k] C_j[n][m_k, m_t]   (sender's Robin trace)
//   v_e[l_t] = sum_{m_t} X_e[l_t][m_t] u_e[m_t]      (tangential quadrature)
//   F_i[n][l_k, l_t] = sum_{e of i} beta_e[l_k] v_e[l_t]
// Flat basis indices put the last dimension fastest.  The sender pass reads
// every coefficient tile once (staged in LDS, rows padded to 65 entries
// against bank conflicts) and writes v for all entries the item sends; the
// receiver pass streams v and writes F.
constexpr int kCRow = kSmallK + 1;

// Copy n complex values to LDS rows: dst[(x / row) * dst_row + x % row] =
// src[x].  U loads per thread are issued before any store (a loop of
// load-then-store would pay one memory latency per iteration).
template <int U>
__device__ inline void gather_rows(double2* dst, int dst_row, const double2* src, int n, int row) {
  for (int base = 0; base < n; base += U * kBlock) {
    double tx[U], ty[U];  // scalar arrays: a vector-typed array would live in scratch
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = base + u * kBlock + (int)threadIdx.x;
      const double2 v = src[x < n ? x : 0];
      tx[u] = v.x;
      ty[u] = v.y;
    }
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the stores
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = base + u * kBlock + (int)threadIdx.x;
      if (x < n) {
        const int r = x / row;
        dst[r * dst_row + (x - r * row)] = make_double2(tx[u], ty[u]);
      }
    }
  }
}

template <int U>
__device__ inline void gather_ints(int* dst, const int* src, int n) {
  for (int base = 0; base < n; base += U * kBlock) {
    int t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = base + u * kBlock + (int)threadIdx.x;
      t[u] = src[x < n ? x : 0];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = base + u * kBlock + (int)threadIdx.x;
      if (x < n) dst[x] = t[u];
    }
  }
}

// Sizes of entry e's pieces: a (sender's normal basis, complex), X
// (receiver tangential x sender tangential, real).
__device__ inline void entry_dims(const Items& it, const Pairs& pr, const TEnt& te, int64_t e,
                                  int* na, int* nx) {
  const int p = te.pair[e];
  const int i = pr.pi[p], j = pr.pj[p];
  const int kf = te.face[e] >> 1;
  *na = it.nb[4 * j + kf];
  *nx = it.D == 2 ? it.nb[4 * i + (1 - kf)] * it.nb[4 * j + (1 - kf)] : 1;
}

// Packs, per sending item, the a and X pieces of its entries (in sender
// order, X padded to whole complex slots) into one blob, the LDS image the
// sender pass copies.  One block per item (assembly time).
__global__ void k_tx_pack(Items it, Pairs pr, TEnt te, double2* blob) {
  const int j = blockIdx.x;
  int64_t off = te.blob_off[j];
  for (int64_t q = te.soff[j]; q < te.soff[j + 1]; ++q) {
    const int e = te.sidx[q];
    int na, nx;
    entry_dims(it, pr, te, e, &na, &nx);
    for (int x = threadIdx.x; x < na; x += blockDim.x) blob[off + x] = te.a[te.aoff[e] + x];
    double* xs = reinterpret_cast<double*>(blob + off + na);
    for (int x = threadIdx.x; x < 2 * ((nx + 1) / 2); x += blockDim.x)
      xs[x] = x < nx ? te.X[te.xoff[e] + x] : 0.0;
    off += na + (nx + 1) / 2;
  }
}

// Sender pass: block = TT steps of sending item j.  Dynamic LDS:
// C [TT][65], U [2][TT][nbt] complex (u double buffered: one barrier per
// entry separates writing u from reading it), the item's blob, then the
// descriptors of its entries (kTxDesc ints each: entry, normal dimension,
// sender normal / tangential basis sizes, receiver tangential size, the two
// sender strides, offset of a in the blob).  Everything the entry loop
// reads is in LDS: per-entry reads of the global tables would be a chain of
// dependent memory round trips.
// NT > 0 (every tangential basis size <= NT): one thread per (entry, step)
// keeps u in registers and writes v directly, so the entry loop has no
// barriers; the residual likewise runs one thread per (face, step).  NT = 0:
// the general form above, u staged in LDS entry by entry.
template <int TT, int NT>
__global__ void __launch_bounds__(kBlock) k_tx_send(Items it, TEnt te, int n_steps, TxJobs jobs,
                                                    int nbt, int64_t pieces, int64_t gram_max) {
  const int j = blockIdx.y;
  const int job = blockIdx.z;
  const int n0 = jobs.n_lo[job] + blockIdx.x * TT;
  const int n_hi = jobs.n_hi[job];
  if (n0 > n_hi) return;  // uniform over the block
  const int Kj = it.K[j];
  // the sender's basis sizes per dimension, read before any store: a global
  // load after the trace stores would wait for them (one in-order counter)
  const int D = it.D;
  const int nbj0 = it.nb[4 * j], nbj1 = D == 2 ? it.nb[4 * j + 1] : 1;
  extern __shared__ double2 smem[];
  double2* Cs = smem;
  double2* Ub = Cs + TT * kCRow;  // general form only
  double2* piece = Ub + (NT > 0 ? 0 : 2 * TT * nbt);
  double* gpiece = reinterpret_cast<double*>(piece + pieces / 16);
  int* desc = reinterpret_cast<int*>(gpiece + gram_max);
  const int nrow = min(TT, n_hi - n0 + 1);
  const int64_t q0 = te.soff[j];
  const int ne = (int)(te.soff[j + 1] - q0);
  const int64_t hoff = (int64_t)(n_steps + 1) * it.off1[j] + (int64_t)n0 * Kj;
  // One memory round trip: the coefficient tile, the previous iterate's tile
  // (kept in registers until the residual), the sender's pieces, its face
  // Gram pieces and its descriptors are all requested before any is stored.
  double* part = jobs.part[job];
  constexpr int kU = TT * kSmallK / kBlock;
  constexpr int kUB = 4, kUG = 2, kUD = 2;  // per-thread batches of pieces, Gram, descriptors
  const int nC = nrow * Kj;
  const int nB = (int)(te.blob_off[j + 1] - te.blob_off[j]);
  const int nG = part ? (int)(te.gram_off[j + 1] - te.gram_off[j]) / 2 : 0;
  const int nD = ne * kTxDesc;
  const double2* csrc = jobs.src[job] + hoff;
  const double2* psrc = part ? jobs.prev[job] + hoff : csrc;
  const double2* bsrc = te.blob + te.blob_off[j];
  const double2* gsrc = reinterpret_cast<const double2*>(te.gram + te.gram_off[j]);
  const int* dsrc = te.sdesc + q0 * kTxDesc;
  double cx[kU], cy[kU], px[kU], py[kU], bx[kUB], by[kUB], gx[kUG], gy[kUG];
  int dv[kUD];
  const double2 z2 = make_double2(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int x = u * kBlock + (int)threadIdx.x;
    const double2 c = x < nC ? csrc[x] : z2;
    const double2 v = (part && x < nC) ? psrc[x] : z2;
    cx[u] = c.x;
    cy[u] = c.y;
    px[u] = v.x;
    py[u] = v.y;
  }
#pragma unroll
  for (int u = 0; u < kUB; ++u) {
    const int x = u * kBlock + (int)threadIdx.x;
    const double2 v = x < nB ? bsrc[x] : z2;
    bx[u] = v.x;
    by[u] = v.y;
  }
#pragma unroll
  for (int u = 0; u < kUG; ++u) {
    const int x = u * kBlock + (int)threadIdx.x;
    const double2 v = x < nG ? gsrc[x] : z2;
    gx[u] = v.x;
    gy[u] = v.y;
  }
#pragma unroll
  for (int u = 0; u < kUD; ++u) {
    const int x = u * kBlock + (int)threadIdx.x;
    dv[u] = x < nD ? dsrc[x] : 0;
  }
  __builtin_amdgcn_sched_barrier(0);  // every load above ahead of the stores below
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int x = u * kBlock + (int)threadIdx.x;
    if (x < nC) {
      const int r = x / Kj;
      Cs[r * kCRow + (x - r * Kj)] = make_double2(cx[u], cy[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < kUB; ++u) {
    const int x = u * kBlock + (int)threadIdx.x;
    if (x < nB) piece[x] = make_double2(bx[u], by[u]);
  }
#pragma unroll
  for (int u = 0; u < kUG; ++u) {
    const int x = u * kBlock + (int)threadIdx.x;
    if (x < nG) reinterpret_cast<double2*>(gpiece)[x] = make_double2(gx[u], gy[u]);
  }
#pragma unroll
  for (int u = 0; u < kUD; ++u) {
    const int x = u * kBlock + (int)threadIdx.x;
    if (x < nD) desc[x] = dv[u];
  }
  // senders larger than the batches: the rest element by element
  for (int x = kUB * kBlock + (int)threadIdx.x; x < nB; x += kBlock) piece[x] = bsrc[x];
  for (int x = kUG * kBlock + (int)threadIdx.x; x < nG; x += kBlock)
    reinterpret_cast<double2*>(gpiece)[x] = gsrc[x];
  for (int x = kUD * kBlock + (int)threadIdx.x; x < nD; x += kBlock) desc[x] = dsrc[x];
  __syncthreads();
  if (NT > 0) {
    for (int t = threadIdx.x; t < ne * nrow; t += blockDim.x) {
      const int q = t / nrow, nn = t - q * nrow;
      const int* d = desc + q * kTxDesc;
      const int e = d[0], nbjk = d[2], nbjt = d[3], nbit = d[4], sk = d[5], stt = d[6];
      const double2* a = piece + d[7];
      const double* X = reinterpret_cast<const double*>(a + nbjk);
      const double2* c = Cs + nn * kCRow;
      double ux[NT > 0 ? NT : 1], uy[NT > 0 ? NT : 1];
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) ux[mt] = uy[mt] = 0.0;
      for (int mk = 0; mk < nbjk; ++mk) {
        const double2 am = a[mk];
        const double2* cr = c + mk * sk;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
          if (mt < nbjt) {
            const double2 cv = cr[mt * stt];
            ux[mt] = fma(am.x, cv.x, fma(-am.y, cv.y, ux[mt]));
            uy[mt] = fma(am.x, cv.y, fma(am.y, cv.x, uy[mt]));
          }
      }
      double2* vout = te.v + ((int64_t)e * (n_steps + 1) + n0 + nn) * nbt;
      for (int lt = 0; lt < nbit; ++lt) {
        const double* xr = X + lt * nbjt;
        double vx = 0.0, vy = 0.0;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
          if (mt < nbjt) {
            vx = fma(xr[mt], ux[mt], vx);
            vy = fma(xr[mt], uy[mt], vy);
          }
        vout[lt] = make_double2(vx, vy);
      }
    }
  }
  for (int q = 0; NT == 0 && q < ne; ++q) {
    const int* d = desc + q * kTxDesc;
    const int e = d[0], nbjk = d[2], nbjt = d[3], nbit = d[4], sk = d[5], stt = d[6];
    const double2* a = piece + d[7];
    const double* X = reinterpret_cast<const double*>(a + nbjk);
    double2* U = Ub + (q & 1) * TT * nbt;
    for (int x = threadIdx.x; x < nrow * nbjt; x += blockDim.x) {
      const int nn = x / nbjt, mt = x - nn * nbjt;
      const double2* c = Cs + nn * kCRow + mt * stt;
      double2 u = make_double2(0.0, 0.0);
      for (int mk = 0; mk < nbjk; ++mk) u = cfma(a[mk], c[mk * sk], u);
      U[nn * nbt + mt] = u;
    }
    lds_barrier();
    double2* vout = te.v + ((int64_t)e * (n_steps + 1) + n0) * nbt;
    for (int x = threadIdx.x; x < nrow * nbit; x += blockDim.x) {
      const int nn = x / nbit, lt = x - nn * nbit;
      const double* xr = X + lt * nbjt;
      const double2* ur = U + nn * nbt;
      double2 v = make_double2(0.0, 0.0);
      for (int mt = 0; mt < nbjt; ++mt) {
        v.x = fma(xr[mt], ur[mt].x, v.x);
        v.y = fma(xr[mt], ur[mt].y, v.y);
      }
      vout[nn * nbt + lt] = v;
    }
  }
  if (!part) return;  // uniform over the block
  // Res^2 partial of this tile: sum_n w_n dc^H G_j dc with G_j factored per
  // face, dc = C - C_prev (formed in place of C, no longer read), and per
  // face w[m_t] = sum_{m_k} b[m_k] dc[m_k, m_t], term w^H W w.
  lds_barrier();
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int x = u * kBlock + (int)threadIdx.x;
    if (x < nrow * Kj) {
      const int r = x / Kj;
      double2& c = Cs[r * kCRow + (x - r * Kj)];
      c = make_double2(c.x - px[u], c.y - py[u]);
    }
  }
  lds_barrier();
  double acc = 0.0;
  if (NT > 0) {
    for (int t = threadIdx.x; t < 2 * D * nrow; t += blockDim.x) {
      const int f = t / nrow, nn = t - f * nrow;
      const int kf = f >> 1;
      const int nbk = kf == 0 ? nbj0 : nbj1;
      const int nbf = D == 2 ? (kf == 0 ? nbj1 : nbj0) : 1;
      const int sk = (D == 2 && kf == 0) ? nbj1 : 1;
      const int stt = (D == 2 && kf == 1) ? nbj1 : 1;
      int goff = 0;
      for (int f2 = 0; f2 < f; ++f2) {
        const int k2 = f2 >> 1;
        const int m = D == 2 ? (k2 == 0 ? nbj1 : nbj0) : 1;
        goff += (k2 == 0 ? nbj0 : nbj1) + m * m;
      }
      const double* b = gpiece + goff;
      const double* W = b + nbk;
      const double2* c = Cs + nn * kCRow;
      double wx[NT > 0 ? NT : 1], wy[NT > 0 ? NT : 1];
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) wx[mt] = wy[mt] = 0.0;
      for (int mk = 0; mk < nbk; ++mk) {
        const double bm = b[mk];
        const double2* cr = c + mk * sk;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
          if (mt < nbf) {
            const double2 cv = cr[mt * stt];
            wx[mt] = fma(bm, cv.x, wx[mt]);
            wy[mt] = fma(bm, cv.y, wy[mt]);
          }
      }
      double term = 0.0;
#pragma unroll
      for (int lt = 0; lt < NT; ++lt)
        if (lt < nbf) {
          double sx = 0.0, sy = 0.0;
#pragma unroll
          for (int mt = 0; mt < NT; ++mt)
            if (mt < nbf) {
              sx = fma(W[lt * nbf + mt], wx[mt], sx);
              sy = fma(W[lt * nbf + mt], wy[mt], sy);
            }
          term += wx[lt] * sx + wy[lt] * sy;
        }
      const int n = n0 + nn;
      acc += ((n == 0 || n == n_steps) ? 0.5 * jobs.dt : jobs.dt) * term;
    }
  }
  int goff = 0;
  for (int f = 0; NT == 0 && f < 2 * D; ++f) {
    const int kf = f >> 1;
    const int nbk = kf == 0 ? nbj0 : nbj1;
    const int nbf = D == 2 ? (kf == 0 ? nbj1 : nbj0) : 1;
    const int sk = (D == 2 && kf == 0) ? nbj1 : 1;
    const int stt = (D == 2 && kf == 1) ? nbj1 : 1;
    const double* b = gpiece + goff;
    const double* W = b + nbk;
    goff += nbk + nbf * nbf;
    for (int x = threadIdx.x; x < nrow * nbf; x += blockDim.x) {
      const int nn = x / nbf, mt = x - nn * nbf;
      const double2* c = Cs + nn * kCRow + mt * stt;
      double2 w = make_double2(0.0, 0.0);
      for (int mk = 0; mk < nbk; ++mk) {
        w.x = fma(b[mk], c[mk * sk].x, w.x);
        w.y = fma(b[mk], c[mk * sk].y, w.y);
      }
      Ub[nn * nbt + mt] = w;
    }
    lds_barrier();
    for (int x = threadIdx.x; x < nrow * nbf; x += blockDim.x) {
      const int nn = x / nbf, lt = x - nn * nbf;
      const double2* wr = Ub + nn * nbt;
      double sx = 0.0, sy = 0.0;
      for (int mt = 0; mt < nbf; ++mt) {
        sx = fma(W[lt * nbf + mt], wr[mt].x, sx);
        sy = fma(W[lt * nbf + mt], wr[mt].y, sy);
      }
      const int n = n0 + nn;
      const double wn = (n == 0 || n == n_steps) ? 0.5 * jobs.dt : jobs.dt;
      acc += wn * (wr[lt].x * sx + wr[lt].y * sy);
    }
    lds_barrier();
  }
  // block sum in a fixed order
  __shared__ double red[kBlock];
  red[threadIdx.x] = acc;
  lds_barrier();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    lds_barrier();
  }
  if (threadIdx.x == 0) part[(int64_t)j * jobs.part_stride + jobs.part_base[job] + blockIdx.x] = red[0];
}

// Receiver pass: block = TT steps of receiving item i, thread (l, step
// phase), no LDS and no barriers.  Entries go four at a time so that their
// loads are in flight together.
constexpr int kMaxRecvEntries = 64;
template <int TT>
__global__ void __launch_bounds__(kBlock) k_tx_recv(Items it, TEnt te, int n_steps, TxJobs jobs,
                                                    int nbt) {
  const int i = blockIdx.y;
  const int job = blockIdx.z;
  const double* scale = jobs.scale[job];
  const int n0 = jobs.n_lo[job] + blockIdx.x * TT;
  const int n_hi = jobs.n_hi[job];
  if (n0 > n_hi) return;
  const int Ki = it.K[i];
  const int l = threadIdx.x & 63;
  if (l >= Ki) return;
  const int nn0 = threadIdx.x >> 6;
  const int D = it.D;
  const int nbi1 = D == 2 ? it.nb[4 * i + 1] : 1;
  // l = l_k * nbi1 + l_t for faces normal to dimension 0, l_t * nbi1 + l_k otherwise
  const int l0 = D == 2 ? l / nbi1 : l, l1 = D == 2 ? l - (l / nbi1) * nbi1 : 0;
  const int rem = n_hi - n0 - nn0;
  const int nq = rem < 0 ? 0 : min(TT / 4, rem / 4 + 1);  // steps of this thread in range
  constexpr int kQ = TT / 4;
  double2 acc[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) acc[q] = make_double2(0.0, 0.0);
  const int64_t e0 = te.off[i], e1 = te.off[i + 1];
  const int64_t vstride = (int64_t)(n_steps + 1) * nbt;
  const double2* vbase = te.v + (int64_t)(n0 + nn0) * nbt;
  for (int64_t e = e0; e < e1; e += 4) {
    double b[4];
    double2 v[4][kQ];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t eu = e + u < e1 ? e + u : e1 - 1;  // clamped: weight 0 below
      const int kf = te.face[eu] >> 1;
      const int lk = kf == 0 ? l0 : l1, lt = kf == 0 ? l1 : l0;
      b[u] = e + u < e1 ? te.beta[te.boff[eu] + lk] : 0.0;
      const double2* vin = vbase + eu * vstride + (D == 2 ? lt : 0);
#pragma unroll
      for (int q = 0; q < kQ; ++q) v[u][q] = q < nq ? vin[(int64_t)4 * q * nbt] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        acc[q].x = fma(b[u], v[u][q].x, acc[q].x);
        acc[q].y = fma(b[u], v[u][q].y, acc[q].y);
      }
  }
  double2* F = jobs.dst[job] + (int64_t)(n_steps + 1) * it.off1[i];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int n = n0 + nn0 + 4 * q;
    if (q >= nq) break;
    const double sc = scale ? scale[n] : 1.0;
    F[(int64_t)n * Ki + l] = cscale(acc[q], sc);
  }
}

__global__ void k_fill_history(Items it, int n_steps, const double2* c0, double2* hist) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  const int64_t hb = (int64_t)(n_steps + 1) * it.off1[s];
  for (int64_t e = threadIdx.x; e < (int64_t)(n_steps + 1) * K; e += blockDim.x)
    hist[hb + e] = c0[it.off1[s] + e % K];
}

// Robin data given at the receiving face nodes (time-major [n_steps+1][n_nodes]):
// f_i^n[l] = sum_y w_y g(y, t_n) v_l^i(y).
__global__ void k_forcing_from_nodes(Items it, Nodes nd, int n_steps, const double2* g,
                                     double2* F) {
  const int s = blockIdx.y;
  const int K = it.K[s];
  const int n = blockIdx.x;
  const int64_t fb = (int64_t)(n_steps + 1) * it.off1[s];
  for (int l = threadIdx.x; l < K; l += blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t q = nd.off[s]; q < nd.off[s + 1]; ++q) {
      const double c = nd.w[q] * basis_value(it, s, l, nd.x + 4 * q);
      const double2 gv = g[(int64_t)n * nd.n + q];
      acc.x = fma(c, gv.x, acc.x);
      acc.y = fma(c, gv.y, acc.y);
    }
    F[fb + (int64_t)n * K + l] = acc;
  }
}

// ---------------------------------------------------------------------------
// Residual Res(k)^2 = sum_n w_n dt sum_i dc_i^H G_i dc_i (eq. residueRT,
// trapezoid in time, face Gauss-Legendre in space).  Deterministic two-pass
// reduction: per (item, time tile) partials, then one block sums them.
constexpr int kRN = 32;
__global__ void __launch_bounds__(kBlock) k_residual(Items it, int n_steps, double dt,
                                                     const double* G, const double2* cur,
                                                     const double2* prev, double* partial,
                                                     int n_tiles) {
  const int s = blockIdx.y;
  const int tile = blockIdx.x;
  const int K = it.K[s];
  __shared__ double g[kSmallK * kSmallK];
  __shared__ double2 d[kRN][kSmallK];
  __shared__ double red[kBlock];
  // loads first, stores after (one memory latency, not one per iteration)
  {
    constexpr int U = kSmallK * kSmallK / kBlock;
    double t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = u * kBlock + threadIdx.x;
      t[u] = G[it.off2[s] + (e < K * K ? e : 0)];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the stores
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = u * kBlock + threadIdx.x;
      if (e < K * K) g[e] = t[u];
    }
  }
  const int64_t hb = (int64_t)(n_steps + 1) * it.off1[s];
  {
    constexpr int U = kRN * kSmallK / kBlock;
    double ax[U], ay[U], bx[U], by[U];  // scalar arrays stay in registers
    const int nrow = min(kRN, n_steps + 1 - tile * kRN);
    const int64_t base = hb + (int64_t)tile * kRN * K;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = u * kBlock + threadIdx.x;
      const int ec = e < nrow * K ? e : 0;
      const double2 a = cur[base + ec], b = prev[base + ec];
      ax[u] = a.x;
      ay[u] = a.y;
      bx[u] = b.x;
      by[u] = b.y;
    }
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the stores
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = u * kBlock + threadIdx.x;
      const int nn = e / K, m = e - nn * K;
      if (e < nrow * K) d[nn][m] = make_double2(ax[u] - bx[u], ay[u] - by[u]);
      else if (e < kRN * K) d[nn][m] = make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  double acc = 0.0;
  for (int e = threadIdx.x; e < kRN * K; e += blockDim.x) {
    const int nn = e / K, r = e - nn * K;
    const int n = tile * kRN + nn;
    if (n > n_steps) continue;
    double2 y = make_double2(0.0, 0.0);
    for (int m = 0; m < K; ++m) {  // G symmetric: read column m (lanes r contiguous)
      y.x = fma(g[m * K + r], d[nn][m].x, y.x);
      y.y = fma(g[m * K + r], d[nn][m].y, y.y);
    }
    const double wn = (n == 0 || n == n_steps) ? 0.5 * dt : dt;
    acc += wn * (d[nn][r].x * y.x + d[nn][r].y * y.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)s * n_tiles + tile] = red[0];
}

__global__ void k_sum_sqrt(const double* partial, int64_t n, double* out) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) acc += partial[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

// ---------------------------------------------------------------------------
// Imaginary time (Section 4.2 eq. SIT, Section 4.4 step 2 / step 4).
// One launch per step n -> n+1, one block per item:
//   nu_n = sqrt(sum_i c~_i^T W_i c~_i) (every block sums the same partials in
//   the same order), c^n = c~^n / nu_n, then
//   c~^{n+1} = (A + dt H~)^{-1} (A c^n + (dt/2) f~^{n+1}) and its partial norm.
__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ inline double norm_from_partials(const double* partial, int n_items, double* red) {
  double acc = 0.0;
  for (int e = threadIdx.x; e < n_items; e += blockDim.x) acc += partial[e];
  return sqrt(block_sum(acc, red));
}

// normalize = 0: the flow without normalisation (nu = 1 at every step).
// Every product uses all four waves: lanes over rows r (contiguous reads of
// the symmetric A and W by column, and of the inverse, stored transposed),
// the columns m = w, w + 4, ... of wave w, partial sums added in LDS.  The
// three matrices' slices are loaded into registers first, so their latency
// overlaps the wait for the previous step's partial norms.
__global__ void __launch_bounds__(kBlock) k_ie_step(Items it, IeJobs jobs, int n_steps, double dt,
                                                    const double* A, const double* W,
                                                    const double2* Minv, int normalize,
                                                    int* flags) {
  constexpr int kWaves = kBlock / 64;
  constexpr int kCols = kSmallK / kWaves;
  const int s = blockIdx.x;
  const int job = blockIdx.y;
  const int n = jobs.step[job];
  double2* hist = jobs.hist[job];
  const double2* F = jobs.F[job];
  double* partial = jobs.partial[job];
  double* nus = jobs.nus[job];
  const int K = it.K[s];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ double c[kSmallK];
  __shared__ double rhs[kSmallK];
  __shared__ double ct[kSmallK];
  __shared__ double part[kWaves][kSmallK];
  __shared__ double red[kBlock];
  const int64_t hb = (int64_t)(n_steps + 1) * it.off1[s];
  const int64_t o2 = it.off2[s];
  const bool on = lane < K;
  double ra[kCols], rm[kCols], rw[kCols];
#pragma unroll
  for (int j = 0; j < kCols; ++j) {
    const int m = w + kWaves * j;
    const bool v = on && m < K;
    const int64_t e = o2 + (v ? (int64_t)m * K + lane : 0);
    ra[j] = v ? A[e] : 0.0;
    rm[j] = v ? Minv[e].x : 0.0;
    rw[j] = v ? W[e] : 0.0;
  }
  const double hn = threadIdx.x < K ? hist[hb + (int64_t)n * K + threadIdx.x].x : 0.0;
  const double fn = threadIdx.x < K ? F[hb + (int64_t)(n + 1) * K + threadIdx.x].x : 0.0;
  double nu = 1.0;
  if (n > 0 && normalize) nu = norm_from_partials(partial + (int64_t)n * it.n_items, it.n_items, red);
  if (s == 0 && threadIdx.x == 0) nus[n] = nu;
  if (threadIdx.x < K) {
    const double v = hn / nu;
    c[threadIdx.x] = v;
    hist[hb + (int64_t)n * K + threadIdx.x] = make_double2(v, 0.0);
  }
  __syncthreads();
  auto split = [&](const double* reg, const double* x) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kCols; ++j) {
      const int m = w + kWaves * j;
      if (m < K) v = fma(reg[j], x[m], v);
    }
    part[w][lane] = v;
    __syncthreads();
  };
  auto gather = [&]() {
    double v = part[0][threadIdx.x];
#pragma unroll
    for (int q = 1; q < kWaves; ++q) v += part[q][threadIdx.x];
    return v;
  };
  split(ra, c);
  if (threadIdx.x < K) rhs[threadIdx.x] = gather() + 0.5 * dt * fn;
  __syncthreads();
  split(rm, rhs);
  if (threadIdx.x < K) {
    const double v = gather();
    ct[threadIdx.x] = v;
    hist[hb + (int64_t)(n + 1) * K + threadIdx.x] = make_double2(v, 0.0);
    if (!isfinite(v)) atomicOr(flags, kFlagNaN);
  }
  __syncthreads();
  split(rw, ct);
  const double acc = threadIdx.x < K ? ct[threadIdx.x] * gather() : 0.0;
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)(n + 1) * it.n_items + s] = tot;
}

__global__ void k_ie_finish(Items it, int n_steps, double2* hist, const double* partial,
                            double* nus, int normalize) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  __shared__ double red[kBlock];
  const double nu =
      normalize ? norm_from_partials(partial + (int64_t)n_steps * it.n_items, it.n_items, red) : 1.0;
  if (s == 0 && threadIdx.x == 0) nus[n_steps] = nu;
  const int64_t hb = (int64_t)(n_steps + 1) * it.off1[s];
  for (int r = threadIdx.x; r < K; r += blockDim.x) {
    const double v = hist[hb + (int64_t)n_steps * K + r].x / nu;
    hist[hb + (int64_t)n_steps * K + r] = make_double2(v, 0.0);
  }
}

__global__ void k_norm_partials(Items it, const double* W, const double2* c0, double* partial) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int r = threadIdx.x; r < K; r += blockDim.x) {
    double v = 0.0;
    for (int m = 0; m < K; ++m) v = fma(W[it.off2[s] + (int64_t)r * K + m], c0[it.off1[s] + m].x, v);
    acc += c0[it.off1[s] + r].x * v;
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) partial[s] = tot;
}

__global__ void k_norm_apply(Items it, double2* c0, const double* partial) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  __shared__ double red[kBlock];
  const double nu = norm_from_partials(partial, it.n_items, red);
  for (int r = threadIdx.x; r < K; r += blockDim.x) {
    const double2 v = c0[it.off1[s] + r];
    c0[it.off1[s] + r] = make_double2(v.x / nu, v.y / nu);
  }
}

// ---------------------------------------------------------------------------
// Local generalized eigenproblems H~ x = lambda A x (Section 4.2), one block
// per item: Cholesky A = L L^T, C = L^{-1} H~ L^{-T}, cyclic Jacobi with a
// round-robin ordering of disjoint rotations, X = L^{-T} V, ascending sort,
// sign fixed by the largest-magnitude component.
__global__ void __launch_bounds__(kBlock) k_geneig(Items it, const double* A, const double* Hr,
                                                   double* lam, double* X, int* flags) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  __shared__ double L[kSmallK * kSmallK];
  __shared__ double C[kSmallK * kSmallK];
  __shared__ double Vv[kSmallK * kSmallK];
  __shared__ double cs[2 * (kSmallK / 2 + 1)];
  __shared__ int pp[2 * (kSmallK / 2 + 1)];
  __shared__ double red[kBlock];
  __shared__ double evals[kSmallK];
  const int64_t o2 = it.off2[s];
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    L[e] = A[o2 + e];
    C[e] = Hr[o2 + e];
    Vv[e] = (e / K == e % K) ? 1.0 : 0.0;
  }
  __syncthreads();
  // Cholesky (lower) in place
  for (int p = 0; p < K; ++p) {
    if (threadIdx.x == 0) {
      const double d = L[p * K + p];
      if (!(d > 0.0)) atomicOr(flags, kFlagPivot);
      L[p * K + p] = sqrt(d);
    }
    __syncthreads();
    const double dp = L[p * K + p];
    for (int r = p + 1 + threadIdx.x; r < K; r += blockDim.x) L[r * K + p] /= dp;
    __syncthreads();
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int r = e / K, c = e % K;
      if (r > p && c > p && c <= r) L[e] -= L[r * K + p] * L[c * K + p];
    }
    __syncthreads();
  }
  // Y = L^{-1} H (columns in parallel), then C = L^{-1} Y^T (symmetric)
  for (int pass = 0; pass < 2; ++pass) {
    for (int p = 0; p < K; ++p) {
      const double dp = L[p * K + p];
      for (int c = threadIdx.x; c < K; c += blockDim.x) C[p * K + c] /= dp;
      __syncthreads();
      for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
        const int r = e / K, c = e % K;
        if (r > p) C[e] -= L[r * K + p] * C[p * K + c];
      }
      __syncthreads();
    }
    // transpose C in place
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int r = e / K, c = e % K;
      if (r < c) {
        const double t = C[e];
        C[e] = C[c * K + r];
        C[c * K + r] = t;
      }
    }
    __syncthreads();
  }
  // symmetrise against rounding
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int r = e / K, c = e % K;
    if (r < c) {
      const double v = 0.5 * (C[e] + C[c * K + r]);
      C[e] = v;
      C[c * K + r] = v;
    }
  }
  __syncthreads();
  // cyclic Jacobi, round-robin pairing of Kp = K rounded up to even players
  const int Kp = K + (K & 1);
  const int npair = Kp / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int r = e / K, c = e % K;
      if (r != c) off += C[e] * C[e];
      else dia += C[e] * C[e];
    }
    off = block_sum(off, red);
    dia = block_sum(dia, red);
    if (off <= 1e-30 * dia) break;
    for (int round = 0; round < Kp - 1; ++round) {
      for (int q = threadIdx.x; q < npair; q += blockDim.x) {
        auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (Kp - 1)) + 1; };
        int a = player(q), b = player(Kp - 1 - q);
        if (a > b) { const int t = a; a = b; b = t; }
        double c = 1.0, sn = 0.0;
        if (b < K) {
          const double apq = C[a * K + b];
          if (apq != 0.0) {
            const double theta = (C[b * K + b] - C[a * K + a]) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
          }
        }
        pp[2 * q] = a;
        pp[2 * q + 1] = b;
        cs[2 * q] = c;
        cs[2 * q + 1] = sn;
      }
      __syncthreads();
      // columns of C and V
      for (int e = threadIdx.x; e < npair * K; e += blockDim.x) {
        const int q = e / K, r = e % K;
        const int a = pp[2 * q], b = pp[2 * q + 1];
        if (b >= K) continue;
        const double c = cs[2 * q], sn = cs[2 * q + 1];
        const double xa = C[r * K + a], xb = C[r * K + b];
        C[r * K + a] = c * xa - sn * xb;
        C[r * K + b] = sn * xa + c * xb;
        const double va = Vv[r * K + a], vb = Vv[r * K + b];
        Vv[r * K + a] = c * va - sn * vb;
        Vv[r * K + b] = sn * va + c * vb;
      }
      __syncthreads();
      // rows of C
      for (int e = threadIdx.x; e < npair * K; e += blockDim.x) {
        const int q = e / K, cc = e % K;
        const int a = pp[2 * q], b = pp[2 * q + 1];
        if (b >= K) continue;
        const double c = cs[2 * q], sn = cs[2 * q + 1];
        const double xa = C[a * K + cc], xb = C[b * K + cc];
        C[a * K + cc] = c * xa - sn * xb;
        C[b * K + cc] = sn * xa + c * xb;
      }
      __syncthreads();
    }
  }
  // keep the eigenvalues (diagonal of the rotated matrix), then
  // X = L^{-T} V by back substitution with the columns in parallel, into C
  for (int c = threadIdx.x; c < K; c += blockDim.x) evals[c] = C[c * K + c];
  __syncthreads();
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) C[e] = Vv[e];
  __syncthreads();
  for (int p = K - 1; p >= 0; --p) {
    const double dp = L[p * K + p];
    for (int c = threadIdx.x; c < K; c += blockDim.x) C[p * K + c] /= dp;
    __syncthreads();
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      const int r = e / K, c = e % K;
      if (r < p) C[e] -= L[p * K + r] * C[p * K + c];
    }
    __syncthreads();
  }
  // ascending order (ties by index) and sign of the largest component
  for (int c = threadIdx.x; c < K; c += blockDim.x) {
    int rk = 0;
    for (int c2 = 0; c2 < K; ++c2)
      if (evals[c2] < evals[c] || (evals[c2] == evals[c] && c2 < c)) ++rk;
    int arg = 0;
    double best = -1.0;
    for (int r = 0; r < K; ++r)
      if (fabs(C[r * K + c]) > best) { best = fabs(C[r * K + c]); arg = r; }
    const double sg = C[arg * K + c] < 0.0 ? -1.0 : 1.0;
    lam[it.off1[s] + rk] = evals[c];
    for (int r = 0; r < K; ++r) X[o2 + (int64_t)r * K + rk] = sg * C[r * K + c];
    if (!isfinite(evals[c])) atomicOr(flags, kFlagNaN);
  }
}

// ---------------------------------------------------------------------------
// Reconstruction (Section 4.3): mean of the covering local functions.
// antisym (two electrons, Appendix A): where electron 2's coordinates come
// after electron 1's (lexicographically), the value is minus the
// reconstruction at the point with the two electrons exchanged.
__global__ void k_reconstruct(Items it, int geom, int step, int n_steps, const double2* hist,
                              const double* pts, int64_t n_pts, int antisym, double2* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pts) return;
  const int D = it.D;
  double y[4];
  for (int k = 0; k < D; ++k) y[k] = pts[t * D + k];
  double sign = 1.0;
  if (antisym) {
    int a = 0;
    while (a < it.dim && y[it.dim + a] == y[a]) ++a;
    if (a < it.dim && y[it.dim + a] > y[a]) {
      for (int b = 0; b < it.dim; ++b) {
        const double u = y[b];
        y[b] = y[it.dim + b];
        y[it.dim + b] = u;
      }
      sign = -1.0;
    }
  }
  double2 acc = make_double2(0.0, 0.0);
  int cnt = 0;
  for (int i = 0; i < it.n_sub; ++i) {
    const int s = geom * it.n_sub + i;
    bool in = true;
    for (int k = 0; k < D; ++k)
      if (!(it.lo[4 * s + k] <= y[k] && y[k] <= it.hi[4 * s + k])) in = false;
    if (!in) continue;
    const int K = it.K[s];
    const double2* c = hist + (int64_t)(n_steps + 1) * it.off1[s] + (int64_t)step * K;
    double2 v = make_double2(0.0, 0.0);
    for (int l = 0; l < K; ++l) {
      const double b = basis_value(it, s, l, y);
      v.x = fma(b, c[l].x, v.x);
      v.y = fma(b, c[l].y, v.y);
    }
    acc = cadd(acc, v);
    ++cnt;
  }
  out[t] = cnt ? cscale(acc, sign / cnt) : make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------------------
// Learned warm start plumbing (Section 4.1: psi^(0) is a given function).
// Robin data at the receiving face nodes for selected steps of a history:
// g(y, t) = (1/|O(y)|) sum_{j in O(y)} (n.grad + mu) psi_j(y, t).
__global__ void k_face_data(Items it, Nodes nd, const int32_t* cover, StepList sl, int n_steps,
                            double mu_re, double mu_im, const double2* hist, double2* g) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sel = blockIdx.y;
  if (q >= nd.n) return;
  const int cnt = nd.count[q];
  double2 acc = make_double2(0.0, 0.0);
  if (cnt > 0) {
    const double* y = nd.x + 4 * q;
    const int face = nd.face[q];
    const int kf = face >> 1;
    const double sign = (face & 1) ? 1.0 : -1.0;
    for (int c = 0; c < cnt; ++c) {
      const int j = cover[q * 15 + c];
      const int Kj = it.K[j];
      const double2* cj = hist + (int64_t)(n_steps + 1) * it.off1[j] + (int64_t)sl.step[sel] * Kj;
      for (int m = 0; m < Kj; ++m) {
        double dv;
        const double v = basis_value_deriv(it, j, m, y, kf, &dv);
        const double2 b = make_double2(sign * dv + mu_re * v, mu_im * v);
        acc = cfma(b, cj[m], acc);
      }
    }
    acc = cscale(acc, 1.0 / cnt);
  }
  g[(int64_t)sel * nd.n + q] = acc;
}

// RMS of g0 over each item's receiving nodes (one block per item).
__global__ void k_learned_rms(Nodes nd, const double2* g0, double* rms) {
  const int s = blockIdx.x;
  __shared__ double red[kBlock];
  const int64_t a = nd.off[s];
  const int n = (int)(nd.off[s + 1] - a);
  double acc = 0.0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const double2 v = g0[a + q];
    acc += v.x * v.x + v.y * v.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) rms[s] = n > 0 ? sqrt(red[0] / n) : 0.0;
}

// Window scale: the largest item RMS, or 1 when g0 vanishes (one block).
__global__ void k_learned_max(int n_items, const double* rms, double* wmax) {
  __shared__ double red[kBlock];
  double m = 0.0;
  for (int s = threadIdx.x; s < n_items; s += blockDim.x) m = fmax(m, rms[s]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) wmax[0] = red[0] > 0.0 ? red[0] : 1.0;
}

// Network input per item: (Re, Im) of g0 / S at the item's nodes, zero
// padding, then M + 8 tail entries: field features, the item's box centre in
// global box coordinates, RMS_i / S, the window's start time, zeros.
// scale[s] holds RMS_i on entry
// and S on exit.
__global__ void k_learned_features(Items it, Nodes nd, const double2* g0, FieldFeat ff, int n_in,
                                   float* x, double* scale, const double* wmax) {
  const int s = blockIdx.x;
  const int64_t a = nd.off[s];
  const int n = (int)(nd.off[s + 1] - a);
  const double S = wmax[0];
  const double rms = scale[s];
  __syncthreads();  // every lane has read scale[s] before lane 0 overwrites it
  float* xs = x + (int64_t)s * n_in;
  const int tail = n_in - (ff.n + 8);
  for (int e = threadIdx.x; e < tail; e += blockDim.x) {
    const int q = e >> 1;
    float v = 0.0f;
    if (q < n) v = (float)(((e & 1) ? g0[a + q].y : g0[a + q].x) / S);
    xs[e] = v;
  }
  for (int m = threadIdx.x; m < ff.n + 8; m += blockDim.x) {
    double v = 0.0;
    const int m2 = m - ff.n;
    if (m2 < 0) {
      v = ff.v[m];
    } else if (m2 < 4) {
      if (m2 < it.D) v = (0.5 * (it.lo[4 * s + m2] + it.hi[4 * s + m2]) - ff.mid[m2]) / ff.half[m2];
    } else if (m2 == 4) {
      v = rms / S;
    } else if (m2 == 5) {
      v = ff.t0w;
    }
    xs[tail + m] = (float)v;
  }
  if (threadIdx.x == 0) scale[s] = S;
}

// Training targets: (g(t_m) - g0) / scale, [m][node][re, im] per item.
__global__ void k_learned_targets(Items it, Nodes nd, const double2* gm, int n_nodes_t,
                                  const double* scale, int n_out, float* y) {
  const int s = blockIdx.x;
  const int64_t a = nd.off[s];
  const int n = (int)(nd.off[s + 1] - a);
  float* ys = y + (int64_t)s * n_out;
  const int row = n > 0 ? 2 * n : 1;
  for (int e = threadIdx.x; e < n_out; e += blockDim.x) {
    const int m = e / row, r = e % row;
    float v = 0.0f;
    if (n > 0 && m < n_nodes_t) {
      const int q = r >> 1;
      const double2 d = csub(gm[(int64_t)m * nd.n + a + q], gm[a + q]);
      v = (float)(((r & 1) ? d.y : d.x) / scale[s]);
    }
    ys[e] = v;
  }
}

// Applied guess: g(t_n) = g0 + scale sum_m l_m(t_n) y_m at every node and step.
__global__ void k_learned_apply(Items it, Nodes nd, const float* y, const double* scale,
                                const double2* g0, const double* lag, int n_nodes_t, int n_out,
                                int n_steps, double2* g_all) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (q >= nd.n) return;
  const int s = nd.item[q];
  const int64_t a = nd.off[s];
  const int nn = (int)(nd.off[s + 1] - a);
  const int ql = (int)(q - a);
  const float* ys = y + (int64_t)s * n_out;
  double2 c = make_double2(0.0, 0.0);
  for (int m = 0; m < n_nodes_t; ++m) {
    const double l = lag[(int64_t)n * n_nodes_t + m];
    c.x = fma(l, (double)ys[m * 2 * nn + 2 * ql], c.x);
    c.y = fma(l, (double)ys[m * 2 * nn + 2 * ql + 1], c.y);
  }
  g_all[(int64_t)n * nd.n + q] = cadd(g0[q], cscale(c, scale[s]));
}

__global__ void k_last_step(Items it, int n_steps, const double2* hist, double2* c0) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  const int64_t hb = (int64_t)(n_steps + 1) * it.off1[s] + (int64_t)n_steps * K;
  for (int r = threadIdx.x; r < K; r += blockDim.x) c0[it.off1[s] + r] = hist[hb + r];
}

inline unsigned blocks_for(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ------------------------------- launchers ---------------------------------
hipError_t launch_assemble(const Items& it, double* A, double* Kin, double* Q, double* Q2,
                           double* B, double* W, double* S1, const int64_t* s1off, int K_max,
                           hipStream_t st) {
  dim3 grid(blocks_for((int64_t)K_max * K_max), it.n_items);
  hipLaunchKernelGGL(k_assemble, grid, dim3(kBlock), 0, st, it, A, Kin, Q, Q2, B, W, S1, s1off);
  return hipGetLastError();
}

hipError_t launch_potential(const Items& it, const Potential& pot, const double* S1,
                            const int64_t* s1off, double* V, double* scratch,
                            const int64_t* scratch_off, hipStream_t st) {
  if (it.dim == 1) {
    hipLaunchKernelGGL(k_potential, dim3(it.n_items), dim3(kBlock), 0, st, it, pot, S1, s1off, V,
                       scratch, scratch_off);
    return hipGetLastError();
  }
  if (it.dim != 2 || it.n_elec < 1 || it.n_elec > 2) return hipErrorInvalidValue;
  const dim3 grid(64, it.n_items);
  hipLaunchKernelGGL(k_pot2_tables, grid, dim3(kBlock), 0, st, it, scratch, scratch_off);
  hipLaunchKernelGGL(k_pot2_en, grid, dim3(kBlock), 0, st, it, pot, scratch, scratch_off);
  if (it.n_elec == 2)
    for (int stage = 0; stage < 4; ++stage)
      hipLaunchKernelGGL(k_pot2_ee, dim3(stage == 0 ? 1024 : 64, it.n_items), dim3(kBlock), 0, st,
                         it, pot, stage, scratch, scratch_off);
  hipLaunchKernelGGL(k_pot2_combine, grid, dim3(kBlock), 0, st, it, S1, s1off, V, scratch,
                     scratch_off);
  return hipGetLastError();
}

hipError_t launch_transfer(const Items& it, const Nodes& nd, const Pairs& pr, double mu_re,
                           double mu_im, double2* T, int K_max, hipStream_t st) {
  if (pr.n == 0) return hipSuccess;
  dim3 grid(blocks_for((int64_t)K_max * K_max), (unsigned)pr.n);
  hipLaunchKernelGGL(k_transfer, grid, dim3(kBlock), 0, st, it, nd, pr, mu_re, mu_im, T);
  return hipGetLastError();
}

hipError_t launch_face_gram(const Items& it, const Nodes& nd, double* G, int K_max,
                            hipStream_t st) {
  dim3 grid(blocks_for((int64_t)K_max * K_max), it.n_items);
  hipLaunchKernelGGL(k_face_gram, grid, dim3(kBlock), 0, st, it, nd, G);
  return hipGetLastError();
}

hipError_t launch_project(const Items& it, const double* A, double init_alpha,
                          const double* init_center, double2* c0, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_project, dim3(it.n_items), dim3(kBlock), 0, st, it, A, init_alpha,
                     init_center, c0, flags);
  return hipGetLastError();
}

hipError_t launch_cn_matrices(int64_t n, const double* A, const double* Kin, const double* V,
                              const double* B, double tau, double mu_re, double mu_im, double* Ar,
                              double* Ap, double* Hr, int tise, double dt, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cn_matrices, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, A, Kin, V, B,
                     tau, mu_re, mu_im, Ar, Ap, Hr, tise, dt);
  return hipGetLastError();
}

hipError_t launch_invert(const Items& it, int n_mats, const double* Ar, const double* Hr,
                         const double* Q, const double* Eall, int64_t out_stride, double tau,
                         int mode, double2* Minv, int* flags, hipStream_t st, int K_max) {
  dim3 grid(n_mats, it.n_items);
  const int NB = (K_max + 15) / 16;
  if (NB <= 1)
    hipLaunchKernelGGL(k_invert_mfma<1>, grid, dim3(64), 0, st, it, n_mats, Ar, Hr, Q, Eall,
                       out_stride, tau, mode, Minv, flags);
  else if (NB == 2)
    hipLaunchKernelGGL(k_invert_mfma<2>, grid, dim3(128), 0, st, it, n_mats, Ar, Hr, Q, Eall,
                       out_stride, tau, mode, Minv, flags);
  else if (NB == 3)
    hipLaunchKernelGGL(k_invert_mfma<3>, grid, dim3(192), 0, st, it, n_mats, Ar, Hr, Q, Eall,
                       out_stride, tau, mode, Minv, flags);
  else
    hipLaunchKernelGGL(k_invert_mfma<4>, grid, dim3(256), 0, st, it, n_mats, Ar, Hr, Q, Eall,
                       out_stride, tau, mode, Minv, flags);
  return hipGetLastError();
}

hipError_t launch_series_product(const Items& it, int n_chunks, const double2* L,
                                 const double2* Rc, const double* Rr, double2 scale,
                                 const double2* add, int64_t cstride, double2* out,
                                 hipStream_t st) {
  if (Rc)
    hipLaunchKernelGGL(k_series_product<false>, dim3(it.n_items, n_chunks), dim3(kBlock), 0, st,
                       it, L, Rc, Rr, scale, add, cstride, out);
  else
    hipLaunchKernelGGL(k_series_product<true>, dim3(it.n_items, n_chunks), dim3(kBlock), 0, st,
                       it, L, Rc, Rr, scale, add, cstride, out);
  return hipGetLastError();
}

hipError_t launch_series_residual(const Items& it, int n_chunks, const double* Ar,
                                  const double* Hr, const double* Q, const double* Eanchor,
                                  double tau, const double2* X, int64_t cstride, double2* R,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_series_residual, dim3(it.n_items, kSmallK / kSerRows, n_chunks),
                     dim3(kBlock), 0, st, it, Ar, Hr, Q, Eanchor, tau, X, cstride, R);
  return hipGetLastError();
}

hipError_t launch_series_assemble(const Items& it, int n_mats, int terms, const double2* P,
                                  int64_t stride, int64_t cstride, const double* Eall,
                                  const double* Eanchor, double2* Minv, hipStream_t st) {
  dim3 grid(it.n_items, (n_mats + kSeriesChunk - 1) / kSeriesChunk);
  switch (terms) {
#define SWR_SERIES_CASE(T)                                                                  \
  case T:                                                                                   \
    hipLaunchKernelGGL(k_series_assemble<T>, grid, dim3(kBlock), 0, st, it, n_mats, P,     \
                       stride, cstride, Eall, Eanchor, Minv);                               \
    break;
    SWR_SERIES_CASE(1) SWR_SERIES_CASE(2) SWR_SERIES_CASE(3) SWR_SERIES_CASE(4)
    SWR_SERIES_CASE(5) SWR_SERIES_CASE(6) SWR_SERIES_CASE(7) SWR_SERIES_CASE(8)
#undef SWR_SERIES_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cn_recur(const Items& it, int n_steps, const double* Ar, const double* Ap,
                           const double* Hr, const double* Q, const double* Eall, double tau,
                           const double2* Minv, const RecSeries* se, const double2* c0,
                           const RecJobs& jobs, int* flags, hipStream_t st) {
  if (jobs.n < 1 || jobs.n > kMaxJobs) return hipErrorInvalidValue;
  for (int q = 0; q < jobs.n; ++q)
    if (jobs.n_lo[q] < 0 || jobs.n_cnt[q] < 1 || jobs.n_lo[q] + jobs.n_cnt[q] > n_steps)
      return hipErrorInvalidValue;
  const dim3 grid(it.n_items, jobs.n);
  if (se) {
    if (!se->P || !se->D || it.Q2) return hipErrorInvalidValue;
    switch (se->terms) {
#define SWR_REC_SERIES_CASE(T)                                                                \
  case T:                                                                                     \
    hipLaunchKernelGGL(k_cn_recur_series<T>, grid, dim3(kRecThreads), 0, st, it, n_steps, Ar, \
                       Ap, Hr, Q, Eall, tau, *se, c0, jobs, flags);                           \
    break;
      SWR_REC_SERIES_CASE(1) SWR_REC_SERIES_CASE(2) SWR_REC_SERIES_CASE(3)
      SWR_REC_SERIES_CASE(4)
#undef SWR_REC_SERIES_CASE
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_cn_recur<kRecPrefetch>, grid, dim3(kRecThreads), 0, st, it, n_steps, Ar,
                     Ap, Hr, Q, Eall, tau, Minv, c0, jobs, flags);
  return hipGetLastError();
}

hipError_t launch_sum_sqrt(const double* partial, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(kBlock), 0, st, partial, n, out);
  return hipGetLastError();
}

hipError_t launch_transfer_tensor(const Items& it, const Nodes& nd, const Pairs& pr,
                                  const TEnt& te, double mu_re, double mu_im, double* beta,
                                  double2* a, double* X, hipStream_t st) {
  if (te.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transfer_tensor, dim3((unsigned)te.n), dim3(kBlock), 0, st, it, nd, pr, te,
                     mu_re, mu_im, beta, a, X);
  return hipGetLastError();
}

// dynamic LDS of the sender pass: C, two U buffers, pieces, Gram pieces,
// entry descriptors
size_t tx_send_lds(int tt, int nbt, int64_t pieces, int max_send, int64_t gram) {
  return (size_t)tt * (kCRow + 2 * nbt) * sizeof(double2) + (size_t)pieces + (size_t)gram +
         (size_t)max_send * kTxDesc * sizeof(int);
}

int transmit_tile_steps(int nbt, int64_t pieces, int max_send, int64_t gram) {
  if (nbt < 1 || nbt > kSmallK || pieces < 0 || pieces % 16 || gram < 0 || gram % 16 ||
      max_send < 1)
    return 0;
  // 2 KiB of static LDS (block sum) come on top
  if (tx_send_lds(32, nbt, pieces, max_send, gram) <= 63488) return 32;
  if (tx_send_lds(16, nbt, pieces, max_send, gram) <= 63488) return 16;
  return 0;
}

hipError_t launch_gram_tensor(const Items& it, const Nodes& nd, const TEnt& te, double* gram,
                              hipStream_t st) {
  // per item and face, whether or not any transfer entry exists (a lone
  // subdomain has only global faces, which the residual still covers)
  if (te.gram_off == nullptr || te.fnode == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gram_tensor, dim3(it.n_items, 2 * it.D), dim3(kBlock), 0, st, it, nd, te,
                     gram);
  return hipGetLastError();
}

__global__ void k_res_reduce(const double* part, int n_items, int part_stride, int n_steps, int S,
                             int n_chunks, int tt, double* out) {
  __shared__ double red[kBlock];
  const int tpc = (S + 1 + tt - 1) / tt;
  double acc = 0.0;
  for (int j = threadIdx.x; j < n_items; j += blockDim.x) {
    for (int c = 0; c < n_chunks; ++c) {
      const int len = c == 0 ? S + 1 : min(S, n_steps - c * S);
      const int tiles = (len + tt - 1) / tt;
      for (int b = 0; b < tiles; ++b) acc += part[(int64_t)j * part_stride + c * tpc + b];
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

hipError_t launch_res_reduce(const double* part, int n_items, int part_stride, int n_steps, int S,
                             int n_chunks, int tt, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_res_reduce, dim3(1), dim3(kBlock), 0, st, part, n_items, part_stride,
                     n_steps, S, n_chunks, tt, out);
  return hipGetLastError();
}

hipError_t launch_tx_pack(const Items& it, const Pairs& pr, const TEnt& te, double2* blob,
                          hipStream_t st) {
  if (te.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tx_pack, dim3(it.n_items), dim3(kBlock), 0, st, it, pr, te, blob);
  return hipGetLastError();
}

hipError_t launch_transmit(const Items& it, const Pairs& pr, const TEnt& te, int n_steps,
                           const double2* T, const TxJobs& jobs, int nbt,
                           int64_t pieces, int max_recv, int max_send, int64_t gram, int tile,
                           hipStream_t st) {
  if (jobs.n < 1 || jobs.n > kMaxJobs) return hipErrorInvalidValue;
  int span = 0;
  for (int q = 0; q < jobs.n; ++q) {
    if (jobs.n_lo[q] < 0 || jobs.n_hi[q] < jobs.n_lo[q] || jobs.n_hi[q] > n_steps)
      return hipErrorInvalidValue;
    span = jobs.n_hi[q] - jobs.n_lo[q] + 1 > span ? jobs.n_hi[q] - jobs.n_lo[q] + 1 : span;
  }
  if (te.n > 0) {
    if (nbt < 1 || nbt > kSmallK) return hipErrorInvalidValue;
    const int tt = tile;
    if ((tt != 16 && tt != 32) || tx_send_lds(tt, nbt, pieces, max_send, gram) > 63488 ||
        max_recv < 1 || max_recv > kMaxRecvEntries)
      return hipErrorInvalidValue;
    // register form when every tangential basis has at most 8 functions (it
    // needs no u buffer in LDS)
    const bool reg = nbt <= 8;
    const size_t lds = tx_send_lds(tt, reg ? 0 : nbt, pieces, max_send, gram);
    dim3 grid(blocks_for(span, tt), it.n_items, jobs.n);
    if (tt == 32) {
      if (reg)
        hipLaunchKernelGGL((k_tx_send<32, 8>), grid, dim3(kBlock), lds, st, it, te, n_steps, jobs,
                           nbt, pieces, gram / 8);
      else
        hipLaunchKernelGGL((k_tx_send<32, 0>), grid, dim3(kBlock), lds, st, it, te, n_steps, jobs,
                           nbt, pieces, gram / 8);
      hipLaunchKernelGGL(k_tx_recv<32>, grid, dim3(kBlock), 0, st, it, te, n_steps, jobs, nbt);
    } else {
      if (reg)
        hipLaunchKernelGGL((k_tx_send<16, 8>), grid, dim3(kBlock), lds, st, it, te, n_steps, jobs,
                           nbt, pieces, gram / 8);
      else
        hipLaunchKernelGGL((k_tx_send<16, 0>), grid, dim3(kBlock), lds, st, it, te, n_steps, jobs,
                           nbt, pieces, gram / 8);
      hipLaunchKernelGGL(k_tx_recv<16>, grid, dim3(kBlock), 0, st, it, te, n_steps, jobs, nbt);
    }
  } else {
    dim3 grid(blocks_for(span, kTN), it.n_items, jobs.n);
    hipLaunchKernelGGL(k_transmit, grid, dim3(kBlock), 0, st, it, pr, n_steps, T, jobs);
  }
  return hipGetLastError();
}

hipError_t launch_fill_history(const Items& it, int n_steps, const double2* c0, double2* hist,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_fill_history, dim3(it.n_items), dim3(kBlock), 0, st, it, n_steps, c0, hist);
  return hipGetLastError();
}

hipError_t launch_forcing_from_nodes(const Items& it, const Nodes& nd, int n_steps,
                                     const double2* g, double2* F, hipStream_t st) {
  dim3 grid(n_steps + 1, it.n_items);
  hipLaunchKernelGGL(k_forcing_from_nodes, grid, dim3(kBlock), 0, st, it, nd, n_steps, g, F);
  return hipGetLastError();
}

hipError_t launch_residual(const Items& it, int n_steps, double dt, const double* G,
                           const double2* cur, const double2* prev, double* partial,
                           double* out, hipStream_t st) {
  const int n_tiles = (n_steps + 1 + kRN - 1) / kRN;
  dim3 grid(n_tiles, it.n_items);
  hipLaunchKernelGGL(k_residual, grid, dim3(kBlock), 0, st, it, n_steps, dt, G, cur, prev,
                     partial, n_tiles);
  hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(kBlock), 0, st, partial,
                     (int64_t)n_tiles * it.n_items, out);
  return hipGetLastError();
}

hipError_t launch_ie_step(const Items& it, const IeJobs& jobs, int n_steps, double dt,
                          const double* A, const double* W, const double2* Minv, int normalize,
                          int* flags, hipStream_t st) {
  if (jobs.n < 1 || jobs.n > kMaxJobs) return hipErrorInvalidValue;
  for (int j = 0; j < jobs.n; ++j)
    if (jobs.step[j] < 0 || jobs.step[j] >= n_steps) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ie_step, dim3(it.n_items, jobs.n), dim3(kBlock), 0, st, it, jobs, n_steps,
                     dt, A, W, Minv, normalize, flags);
  return hipGetLastError();
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n)), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_ie_finish(const Items& it, int n_steps, double2* hist, const double* partial,
                            double* nus, int normalize, hipStream_t st) {
  hipLaunchKernelGGL(k_ie_finish, dim3(it.n_items), dim3(kBlock), 0, st, it, n_steps, hist,
                     partial, nus, normalize);
  return hipGetLastError();
}

hipError_t launch_global_normalise(const Items& it, const double* W, double2* c0,
                                   double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_norm_partials, dim3(it.n_items), dim3(kBlock), 0, st, it, W, c0, partial);
  hipLaunchKernelGGL(k_norm_apply, dim3(it.n_items), dim3(kBlock), 0, st, it, c0, partial);
  return hipGetLastError();
}

hipError_t launch_geneig(const Items& it, const double* A, const double* Hr, double* lam,
                         double* X, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_geneig, dim3(it.n_items), dim3(kBlock), 0, st, it, A, Hr, lam, X, flags);
  return hipGetLastError();
}

hipError_t launch_reconstruct(const Items& it, int geom, int step, int n_steps,
                              const double2* hist, const double* pts, int64_t n_pts, int antisym,
                              double2* out, hipStream_t st) {
  if (n_pts == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reconstruct, dim3(blocks_for(n_pts)), dim3(kBlock), 0, st, it, geom, step,
                     n_steps, hist, pts, n_pts, antisym, out);
  return hipGetLastError();
}

hipError_t launch_face_data(const Items& it, const Nodes& nd, const int32_t* cover,
                            const StepList& sl, int n_steps, double mu_re, double mu_im,
                            const double2* hist, double2* g, hipStream_t st) {
  if (nd.n == 0 || sl.n == 0) return hipSuccess;
  dim3 grid(blocks_for(nd.n), sl.n);
  hipLaunchKernelGGL(k_face_data, grid, dim3(kBlock), 0, st, it, nd, cover, sl, n_steps, mu_re,
                     mu_im, hist, g);
  return hipGetLastError();
}

hipError_t launch_learned_features(const Items& it, const Nodes& nd, const double2* g0,
                                   const FieldFeat& ff, int n_in, float* x, double* scale,
                                   double* wmax, hipStream_t st) {
  hipLaunchKernelGGL(k_learned_rms, dim3(it.n_items), dim3(kBlock), 0, st, nd, g0, scale);
  hipLaunchKernelGGL(k_learned_max, dim3(1), dim3(kBlock), 0, st, it.n_items, scale, wmax);
  hipLaunchKernelGGL(k_learned_features, dim3(it.n_items), dim3(kBlock), 0, st, it, nd, g0, ff,
                     n_in, x, scale, wmax);
  return hipGetLastError();
}

hipError_t launch_learned_targets(const Items& it, const Nodes& nd, const double2* gm,
                                  int n_nodes_t, const double* scale, int n_out, float* y,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_learned_targets, dim3(it.n_items), dim3(kBlock), 0, st, it, nd, gm,
                     n_nodes_t, scale, n_out, y);
  return hipGetLastError();
}

hipError_t launch_learned_apply(const Items& it, const Nodes& nd, const float* y,
                                const double* scale, const double2* g0, const double* lag,
                                int n_nodes_t, int n_out, int n_steps, double2* g_all,
                                hipStream_t st) {
  if (nd.n == 0) return hipSuccess;
  dim3 grid(blocks_for(nd.n), n_steps + 1);
  hipLaunchKernelGGL(k_learned_apply, grid, dim3(kBlock), 0, st, it, nd, y, scale, g0, lag,
                     n_nodes_t, n_out, n_steps, g_all);
  return hipGetLastError();
}

hipError_t launch_last_step(const Items& it, int n_steps, const double2* hist, double2* c0,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_last_step, dim3(it.n_items), dim3(kBlock), 0, st, it, n_steps, hist, c0);
  return hipGetLastError();
}

}  // namespace swr
