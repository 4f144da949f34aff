// Block path of the SWR hot path (gfx950): tensor Gaussian bases in two or
// four configuration dimensions with up to 2048 functions per subdomain, real
// time (Section 4.4 step 2 Crank-Nicolson; Section 4.1 Robin transmission
// averaged over multi-overlap zones; Section 5 eq. pseudo and eq. residueRT).
//
// Coordinates: y = (x_k L_k)^T c with S_k = L_k L_k^T per dimension (see
// block.h).  The Crank-Nicolson step of one iterate, with M'(E) =
// I + i tau (H' + E Q') and H' = Kin' + V' + mu/2 B',
//   y^{n+1} = M'(E_{n+1})^{-1} r - y^n,
//   r = 2 y^n + i tau (E_{n+1} - E_n) Q' y^n + (i tau / 2)(f'^n + f'^{n+1}),
// since (I - i tau (H' + E_n Q')) = 2 I - M'(E_{n+1}) + i tau (E_{n+1} - E_n) Q'.
// The inverse is the field series around the chunk's anchor E_c,
// M'(E)^{-1} = sum_k (-(E - E_c))^k P_k, P_k = (P_0 i tau Q')^k P_0,
// P_0 = M'(E_c)^{-1} (blocked Gauss-Jordan), kept in matrix-core fragment
// order.  All Schwarz iterates in flight advance together: per launch and
// item the step is one product of the stacked terms [P_0 .. P_t] with the
// right-hand sides of every iterate scaled by their (-d)^k, on the matrix
// cores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "block.h"
#include "devmath.h"

namespace swr {
namespace {

constexpr int kBT = 256;  // threads per block

inline unsigned nblk(int64_t n, int b = kBT) { return (unsigned)((n + b - 1) / b); }

// strides of the multi-index (last dimension fastest)
__device__ inline void blk_strides(const BlkDim* bd, int D, int* st) {
  int s = 1;
  for (int k = D - 1; k >= 0; --k) {
    st[k] = s;
    s *= bd[k].n;
  }
}

__device__ inline void blk_split(int l, const BlkDim* bd, int D, int* a) {
  for (int k = D - 1; k >= 0; --k) {
    a[k] = l % bd[k].n;
    l /= bd[k].n;
  }
}

// ---------------------------------------------------------------------------
// One-dimensional factors, their Cholesky transform and the transformed
// tables (one thread per item and dimension).
__global__ void k_blk_dims(Items it, BlkDim* bd, double mu_re, double mu_im, double ia,
                           const double* ic, int* flags) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= it.n_items * it.D) return;
  const int s = t / it.D, k = t % it.D;
  BlkDim& d = bd[4 * s + k];
  const int n = d.n;
  const double del = it.delta[4 * s + k];
  const double* al = it.alpha + it.aoff[4 * s + k];
  const double lo = d.lo, hi = d.hi;
  double L[kBlkN * kBlkN], Li[kBlkN * kBlkN];
  for (int a = 0; a < kBlkN * kBlkN; ++a) {
    L[a] = 0.0;
    Li[a] = 0.0;
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double S, X, T;
      pair_integrals(al[a], del, al[b], del, lo, hi, &S, &X, &T);
      d.S[a * kBlkN + b] = S;
      d.X[a * kBlkN + b] = X;
      d.Kin[a * kBlkN + b] = T;
      const double fla = exp(-del * (lo - al[a]) * (lo - al[a])), flb = exp(-del * (lo - al[b]) * (lo - al[b]));
      const double fha = exp(-del * (hi - al[a]) * (hi - al[a])), fhb = exp(-del * (hi - al[b]) * (hi - al[b]));
      d.B[a * kBlkN + b] = fla * flb + fha * fhb;
    }
  // Cholesky S = L L^T
  for (int j = 0; j < n; ++j) {
    double v = d.S[j * kBlkN + j];
    for (int q = 0; q < j; ++q) v -= L[j * kBlkN + q] * L[j * kBlkN + q];
    if (!(v > 0.0)) {
      atomicOr(flags, kFlagPivot);
      v = 1.0;
    }
    const double ljj = sqrt(v);
    L[j * kBlkN + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double u = d.S[i * kBlkN + j];
      for (int q = 0; q < j; ++q) u -= L[i * kBlkN + q] * L[j * kBlkN + q];
      L[i * kBlkN + j] = u / ljj;
    }
  }
  // L^{-1} (lower triangular)
  for (int j = 0; j < n; ++j) {
    Li[j * kBlkN + j] = 1.0 / L[j * kBlkN + j];
    for (int i = j + 1; i < n; ++i) {
      double u = 0.0;
      for (int q = j; q < i; ++q) u += L[i * kBlkN + q] * Li[q * kBlkN + j];
      Li[i * kBlkN + j] = -u / L[i * kBlkN + i];
    }
  }
  for (int a = 0; a < kBlkN * kBlkN; ++a) {
    d.Li[a] = Li[a];
    d.Lo[a] = L[a];
    d.Lt[a] = L[(a % kBlkN) * kBlkN + a / kBlkN];
    d.Lit[a] = Li[(a % kBlkN) * kBlkN + a / kBlkN];
  }
  // transformed matrices Li M Li^T
  const double* src[3] = {d.Kin, d.X, d.B};
  double* dst[3] = {d.Kp, d.Xp, d.Bp};
  for (int m = 0; m < 3; ++m)
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double acc = 0.0;
        for (int p = 0; p <= a; ++p)
          for (int q = 0; q <= b; ++q) acc += Li[a * kBlkN + p] * src[m][p * kBlkN + q] * Li[b * kBlkN + q];
        dst[m][a * kBlkN + b] = acc;
      }
  // transformed values, Robin vectors, tangential tables, projection
  const double eps = d.eps;
  const double xs[kBlkPos] = {lo, hi, hi - eps, lo + eps};
  const double sg[kBlkPos] = {-1.0, 1.0, -1.0, 1.0};
  double ph[kBlkN], dph[kBlkN];
  for (int side = 0; side < 2; ++side) {
    const double x = side ? hi : lo;
    for (int b = 0; b < n; ++b) ph[b] = exp(-del * (x - al[b]) * (x - al[b]));
    for (int a = 0; a < n; ++a) {
      double v = 0.0;
      for (int b = 0; b <= a; ++b) v += Li[a * kBlkN + b] * ph[b];
      d.val[side][a] = v;
    }
  }
  for (int p = 0; p < kBlkPos; ++p) {
    const double x = xs[p];
    for (int b = 0; b < n; ++b) {
      ph[b] = exp(-del * (x - al[b]) * (x - al[b]));
      dph[b] = -2.0 * del * (x - al[b]) * ph[b];
    }
    for (int a = 0; a < n; ++a) {
      double re = 0.0, im = 0.0;
      for (int b = 0; b <= a; ++b) {
        re += Li[a * kBlkN + b] * (sg[p] * dph[b] + mu_re * ph[b]);
        im += Li[a * kBlkN + b] * (mu_im * ph[b]);
      }
      d.rob[p][a] = make_double2(re, im);
    }
  }
  for (int tq = 0; tq < d.nt; ++tq) {
    const double x = d.tx[tq];
    for (int b = 0; b < n; ++b) ph[b] = exp(-del * (x - al[b]) * (x - al[b]));
    for (int a = 0; a < n; ++a) {
      double v = 0.0;
      for (int b = 0; b <= a; ++b) v += Li[a * kBlkN + b] * ph[b];
      d.phit[tq][a] = v;
    }
  }
  for (int b = 0; b < n; ++b) ph[b] = pair_overlap(al[b], del, ic[k], ia, lo, hi);
  for (int a = 0; a < n; ++a) {
    double v = 0.0;
    for (int b = 0; b <= a; ++b) v += Li[a * kBlkN + b] * ph[b];
    d.g0[a] = v;
  }
}

// ---------------------------------------------------------------------------
// Soft-Coulomb potential (Section 5, eq. pseudo) in the transformed basis:
// every term is the tensor Gauss-Legendre sum with the weighted product
// tables F'_k[a n + b][q] = w_q phi'_a(x_q) phi'_b(x_q), phi' = L^{-1} phi.
// Per-item scratch (doubles): the tables of the D dimensions, then the terms
// (electron 0's and 1's nucleus terms, the electron-electron term) and a
// stage buffer of the two-dimensional terms.
__host__ __device__ inline void blk_pot_layout(const int32_t* nb, const int32_t* qn, int D,
                                               int64_t* off) {
  int64_t o = 0;
  for (int k = 0; k < 4; ++k) {
    off[k] = o;
    if (k < D) o += (int64_t)nb[k] * nb[k] * qn[k];
  }
  const int64_t P0 = (int64_t)nb[0] * nb[0], P1 = D > 1 ? (int64_t)nb[1] * nb[1] : 1;
  const int64_t P2 = D > 2 ? (int64_t)nb[2] * nb[2] : 1, P3 = D > 3 ? (int64_t)nb[3] * nb[3] : 1;
  off[4] = o;  // electron 0's nucleus term
  o += D == 4 ? P0 * P1 : (D == 2 ? P0 * P1 : P0);
  off[5] = o;  // electron 1's nucleus term
  o += D == 4 ? P2 * P3 : P1;
  off[6] = o;  // electron-electron term
  o += D == 4 ? P0 * P1 * P2 * P3 : P0 * P1;
  off[7] = o;  // stage buffer of the two-dimensional terms
  int64_t g = 0;
  for (int k = 0; k + 1 < D; k += 1) {
    const int64_t v = (int64_t)qn[k] * nb[k + 1] * nb[k + 1];
    g = v > g ? v : g;
  }
  o += g;
  off[8] = o;
}

__global__ void k_blk_tables(BlkItems b, const int64_t* soff, double* scratch) {
  const Items& it = b.it;
  const int s = blockIdx.y;
  const BlkDim* bd = b.bd + 4 * s;
  int32_t nb[4], qn[4];
  for (int k = 0; k < 4; ++k) {
    nb[k] = k < it.D ? bd[k].n : 1;
    qn[k] = k < it.D ? it.qn[4 * s + k] : 1;
  }
  int64_t off[9];
  blk_pot_layout(nb, qn, it.D, off);
  double* base = scratch + soff[s];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 0; k < it.D; ++k) {
    if (q >= qn[k]) continue;
    const int n = nb[k];
    const double del = it.delta[4 * s + k];
    const double* al = it.alpha + it.aoff[4 * s + k];
    const double x = it.qx[it.qoff[4 * s + k] + q], w = it.qw[it.qoff[4 * s + k] + q];
    double ph[kBlkN], pt[kBlkN];
    for (int c = 0; c < n; ++c) ph[c] = exp(-del * (x - al[c]) * (x - al[c]));
    for (int a = 0; a < n; ++a) {
      double v = 0.0;
      for (int c = 0; c <= a; ++c) v += bd[k].Li[a * kBlkN + c] * ph[c];
      pt[a] = v;
    }
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c) base[off[k] + (int64_t)(a * n + c) * qn[k] + q] = w * pt[a] * pt[c];
  }
}

// nucleus term of electron m in one dimension: T[p] = sum_q F'_m[p][q] U(x_q)
__global__ void k_blk_pot1(BlkItems b, Potential pot, const int64_t* soff, double* scratch) {
  const Items& it = b.it;
  const int s = blockIdx.y;
  const int m = blockIdx.z;
  const BlkDim* bd = b.bd + 4 * s;
  int32_t nb[4], qn[4];
  for (int k = 0; k < 4; ++k) {
    nb[k] = k < it.D ? bd[k].n : 1;
    qn[k] = k < it.D ? it.qn[4 * s + k] : 1;
  }
  int64_t off[9];
  blk_pot_layout(nb, qn, it.D, off);
  double* base = scratch + soff[s];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = nb[m] * nb[m];
  if (p >= P) return;
  const int geom = s / it.n_sub;
  const double* F = base + off[m];
  const double* x = it.qx + it.qoff[4 * s + m];
  double acc = 0.0;
  for (int q = 0; q < qn[m]; ++q) {
    double u = 0.0;
    for (int A = 0; A < pot.n_nuc; ++A) {
      const double r = x[q] - pot.pos[(geom * pot.n_nuc + A) * it.dim];
      u -= pot.charge[A] / sqrt(r * r + pot.eps_en * pot.eps_en);
    }
    acc = fma(F[(int64_t)p * qn[m] + q], u, acc);
  }
  base[off[4 + m] + p] = acc;
}

// two-dimensional term over dimensions (k0, k1) = (2 m, 2 m + 1) (kind 0:
// electron m's nucleus term in two dimensions) or (0, 1) (kind 1: the
// electron-electron term of two electrons in one dimension each):
// G[q0][p1] = sum_q1 F'_k1[p1][q1] U(x_q0, y_q1), T[p0][p1] = sum_q0 F'_k0[p0][q0] G[q0][p1]
__global__ void __launch_bounds__(kBT) k_blk_pot2(BlkItems b, Potential pot, const int64_t* soff,
                                                  double* scratch, int kind, int m) {
  const Items& it = b.it;
  const int s = blockIdx.x;
  const BlkDim* bd = b.bd + 4 * s;
  int32_t nb[4], qn[4];
  for (int k = 0; k < 4; ++k) {
    nb[k] = k < it.D ? bd[k].n : 1;
    qn[k] = k < it.D ? it.qn[4 * s + k] : 1;
  }
  int64_t off[9];
  blk_pot_layout(nb, qn, it.D, off);
  double* base = scratch + soff[s];
  const int k0 = kind == 0 ? 2 * m : 0, k1 = k0 + 1;
  const int P0 = nb[k0] * nb[k0], P1 = nb[k1] * nb[k1];
  const int n0 = qn[k0], n1 = qn[k1];
  const double* F0 = base + off[k0];
  const double* F1 = base + off[k1];
  const double* x0 = it.qx + it.qoff[4 * s + k0];
  const double* x1 = it.qx + it.qoff[4 * s + k1];
  double* G = base + off[7];
  double* T = base + (kind == 0 ? off[4 + m] : off[6]);
  const int geom = s / it.n_sub;
  for (int e = threadIdx.x; e < n0 * P1; e += blockDim.x) {
    const int q0 = e / P1, p1 = e - q0 * P1;
    double acc = 0.0;
    for (int q1 = 0; q1 < n1; ++q1) {
      double u;
      if (kind == 0) {
        u = 0.0;
        for (int A = 0; A < pot.n_nuc; ++A) {
          const double* R = pot.pos + (geom * pot.n_nuc + A) * 2;
          const double dx = x0[q0] - R[0], dy = x1[q1] - R[1];
          u -= pot.charge[A] / sqrt(dx * dx + dy * dy + pot.eps_en * pot.eps_en);
        }
      } else {
        const double r = x0[q0] - x1[q1];
        u = 1.0 / sqrt(r * r + pot.eps_ee * pot.eps_ee);
      }
      acc = fma(F1[(int64_t)p1 * n1 + q1], u, acc);
    }
    G[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < P0 * P1; e += blockDim.x) {
    const int p0 = e / P1, p1 = e - p0 * P1;
    double acc = 0.0;
    for (int q0 = 0; q0 < n0; ++q0) acc = fma(F0[(int64_t)p0 * n0 + q0], G[(int64_t)q0 * P1 + p1], acc);
    T[e] = acc;
  }
}

// Electron-electron term of two electrons in two dimensions each (dims 0, 1
// for electron 1 and 2, 3 for electron 2; u = 1/sqrt((x0-x2)^2 + (x1-x3)^2
// + eps^2)), contracted in three stages through the batch stage buffer:
// A: W[q0 q2][p1 p3] = sum_{q1, q3} F'_1[p1][q1] F'_3[p3][q3] u
// B: Y[q0][p2][p1 p3] = sum_q2 F'_2[p2][q2] W[q0 q2][p1 p3]
// C: Vee[p0][p2][p1 p3] = sum_q0 F'_0[p0][q0] Y[q0][p2][p1 p3]
struct Ee4 {
  int nq[4], P[4];
  int64_t off[9];
};
__device__ inline Ee4 ee4_item(const BlkItems& b, int s) {
  Ee4 e;
  int32_t nb[4], qn[4];
  for (int k = 0; k < 4; ++k) {
    nb[k] = b.bd[4 * s + k].n;
    qn[k] = b.it.qn[4 * s + k];
    e.nq[k] = qn[k];
    e.P[k] = nb[k] * nb[k];
  }
  blk_pot_layout(nb, qn, 4, e.off);
  return e;
}

constexpr int kEeTile = 16;
__global__ void __launch_bounds__(kBT) k_blk_ee4_a(BlkItems b, Potential pot, const int64_t* soff,
                                                   const double* scratch, double* stage,
                                                   int64_t stage_item, int s0) {
  const Items& it = b.it;
  const int s = s0 + blockIdx.y;
  const Ee4 e = ee4_item(b, s);
  if ((int)blockIdx.x >= e.nq[0] * e.nq[2]) return;
  const int q0 = blockIdx.x / e.nq[2], q2 = blockIdx.x - q0 * e.nq[2];
  const double* x0 = it.qx + it.qoff[4 * s + 0];
  const double* x1 = it.qx + it.qoff[4 * s + 1];
  const double* x2 = it.qx + it.qoff[4 * s + 2];
  const double* x3 = it.qx + it.qoff[4 * s + 3];
  const double* base = scratch + soff[s];
  const double* F1 = base + e.off[1];
  const double* F3 = base + e.off[3];
  const int n1 = e.nq[1], n3 = e.nq[3], P1 = e.P[1], P3 = e.P[3];
  const double dx = x0[q0] - x2[q2];
  const double c = dx * dx + pot.eps_ee * pot.eps_ee;
  __shared__ double Z[kEeZ];                       // [n1][P3]
  __shared__ double U[kEeQ * (kEeTile + 1)];       // [n1][kEeTile + 1]
  __shared__ double Ft[kBlkN * kBlkN * (kEeTile + 1)];  // [P3][kEeTile + 1]
  for (int t = threadIdx.x; t < n1 * P3; t += blockDim.x) Z[t] = 0.0;
  for (int t0 = 0; t0 < n3; t0 += kEeTile) {
    const int w = min(kEeTile, n3 - t0);
    __syncthreads();
    for (int t = threadIdx.x; t < n1 * w; t += blockDim.x) {
      const int a = t / w, j = t - a * w;
      const double dy = x1[a] - x3[t0 + j];
      U[a * (kEeTile + 1) + j] = 1.0 / sqrt(fma(dy, dy, c));
    }
    for (int t = threadIdx.x; t < P3 * w; t += blockDim.x) {
      const int p = t / w, j = t - p * w;
      Ft[p * (kEeTile + 1) + j] = F3[(int64_t)p * n3 + t0 + j];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n1 * P3; t += blockDim.x) {
      const int a = t / P3, p = t - a * P3;
      double acc = Z[t];
      for (int j = 0; j < w; ++j) acc = fma(U[a * (kEeTile + 1) + j], Ft[p * (kEeTile + 1) + j], acc);
      Z[t] = acc;
    }
  }
  __syncthreads();
  double* W = stage + (int64_t)blockIdx.y * stage_item + (int64_t)blockIdx.x * P1 * P3;
  for (int t = threadIdx.x; t < P1 * P3; t += blockDim.x) {
    const int p1 = t / P3, p3 = t - p1 * P3;
    double acc = 0.0;
    for (int a = 0; a < n1; ++a) acc = fma(F1[(int64_t)p1 * n1 + a], Z[a * P3 + p3], acc);
    W[t] = acc;
  }
}

__global__ void k_blk_ee4_b(BlkItems b, const int64_t* soff, const double* scratch, double* stage,
                            int64_t stage_item, int s0) {
  const int s = s0 + blockIdx.y;
  const Ee4 e = ee4_item(b, s);
  const int64_t R = (int64_t)e.P[1] * e.P[3];
  const int64_t tot = (int64_t)e.nq[0] * e.P[2] * R;
  const double* F2 = scratch + soff[s] + e.off[2];
  const double* W = stage + (int64_t)blockIdx.y * stage_item;
  double* Y = stage + (int64_t)blockIdx.y * stage_item + (int64_t)e.nq[0] * e.nq[2] * R;
  const int n2 = e.nq[2];
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q0 = t / (e.P[2] * R);
    const int64_t rem = t - q0 * e.P[2] * R;
    const int p2 = (int)(rem / R);
    const int64_t r = rem - (int64_t)p2 * R;
    double acc = 0.0;
    for (int q2 = 0; q2 < n2; ++q2) acc = fma(F2[(int64_t)p2 * n2 + q2], W[(q0 * n2 + q2) * R + r], acc);
    Y[t] = acc;
  }
}

__global__ void k_blk_ee4_c(BlkItems b, const int64_t* soff, double* scratch, const double* stage,
                            int64_t stage_item, int s0) {
  const int s = s0 + blockIdx.y;
  const Ee4 e = ee4_item(b, s);
  const int64_t R = (int64_t)e.P[1] * e.P[3];
  const int64_t PR = (int64_t)e.P[2] * R;
  const int64_t tot = (int64_t)e.P[0] * PR;
  double* base = scratch + soff[s];
  const double* F0 = base + e.off[0];
  const double* Y = stage + (int64_t)blockIdx.y * stage_item + (int64_t)e.nq[0] * e.nq[2] * R;
  const int n0 = e.nq[0];
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int p0 = (int)(t / PR);
    const int64_t r = t - (int64_t)p0 * PR;
    double acc = 0.0;
    for (int q0 = 0; q0 < n0; ++q0) acc = fma(F0[(int64_t)p0 * n0 + q0], Y[(int64_t)q0 * PR + r], acc);
    base[e.off[6] + t] = acc;
  }
}

// V'[l][m]: every term with the Kronecker identity of the dimensions it does
// not involve (the transformed overlaps are the identity).
__global__ void k_blk_vfull(BlkItems b, const int64_t* soff, const double* scratch, double* Vp) {
  const Items& it = b.it;
  const int s = blockIdx.y;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s], D = it.D;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)K * K) return;
  const int l = (int)(e / K), mm = (int)(e - (int64_t)l * K);
  int32_t nb[4], qn[4];
  for (int k = 0; k < 4; ++k) {
    nb[k] = k < D ? bd[k].n : 1;
    qn[k] = k < D ? it.qn[4 * s + k] : 1;
  }
  int64_t off[9];
  blk_pot_layout(nb, qn, D, off);
  const double* base = scratch + soff[s];
  int a[4], c[4], p[4];
  blk_split(l, bd, D, a);
  blk_split(mm, bd, D, c);
  for (int k = 0; k < D; ++k) p[k] = a[k] * nb[k] + c[k];
  double v = 0.0;
  if (it.dim == 1) {  // D = 2: two electrons in one dimension
    if (a[1] == c[1]) v += base[off[4] + p[0]];
    if (a[0] == c[0]) v += base[off[5] + p[1]];
    v += base[off[6] + (int64_t)p[0] * nb[1] * nb[1] + p[1]];
  } else if (it.n_elec == 1) {  // D = 2: one electron in two dimensions
    v += base[off[4] + (int64_t)p[0] * nb[1] * nb[1] + p[1]];
  } else {  // D = 4
    const int64_t P1 = nb[1] * nb[1], P2 = nb[2] * nb[2], P3 = nb[3] * nb[3];
    if (a[2] == c[2] && a[3] == c[3]) v += base[off[4] + p[0] * P1 + p[1]];
    if (a[0] == c[0] && a[1] == c[1]) v += base[off[5] + p[2] * P3 + p[3]];
    v += base[off[6] + ((int64_t)p[0] * P2 + p[2]) * (P1 * P3) + p[1] * P3 + p[3]];
  }
  Vp[it.off2[s] + e] = v;
}

// ---------------------------------------------------------------------------
// Kronecker-sum entry of one-dimensional factors M_k over the dimensions in
// mask: sum_k M_k[a_k][c_k] prod_{k' != k} delta(a_k', c_k').
__device__ inline double kron_sum_entry(const BlkDim* bd, int D, const int* a, const int* c,
                                        int which, int mask) {
  int diff = 0, kd = -1;
  for (int k = 0; k < D; ++k)
    if (a[k] != c[k]) {
      ++diff;
      kd = k;
    }
  if (diff > 1) return 0.0;
  double v = 0.0;
  for (int k = 0; k < D; ++k) {
    if (!(mask >> k & 1)) continue;
    if (diff == 1 && k != kd) continue;
    const double* M = which == 0 ? bd[k].Kp : (which == 1 ? bd[k].Bp : bd[k].Xp);
    v += M[a[k] * kBlkN + c[k]];
  }
  return v;
}

__global__ void k_blk_anchor(BlkItems b, const double* Vp, const double* Ea, int64_t cstride,
                             double2* Z) {
  const Items& it = b.it;
  const int s = blockIdx.y, ch = blockIdx.z;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s], D = it.D;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)K * K) return;
  const int l = (int)(e / K), m = (int)(e - (int64_t)l * K);
  int a[4], c[4];
  blk_split(l, bd, D, a);
  blk_split(m, bd, D, c);
  const int all = (1 << D) - 1;
  const double kin = kron_sum_entry(bd, D, a, c, 0, all);
  const double bs = kron_sum_entry(bd, D, a, c, 1, all);
  const double q = kron_sum_entry(bd, D, a, c, 2, b.fmask);
  const double tau = b.tau;
  const double re = (l == m ? 1.0 : 0.0) - tau * 0.5 * b.mu_im * bs;
  const double im = tau * (kin + Vp[it.off2[s] + e] + 0.5 * b.mu_re * bs + Ea[ch] * q);
  Z[ch * cstride + it.off2[s] + e] = make_double2(re, im);
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion in place, panels of kBlkGJ columns, no
// pivoting (the Hermitian part of M' is I - tau Im(mu)/2 B', positive
// definite for Im mu <= 0).  Pivot step of panel J: D = Z[J][J];
// Z[J][J] <- D^{-1}, Z[J][c] <- D^{-1} Z[J][c]; the other rows take
// Z[i][:] -= Z_old[i][J] R[J][:] with R = the new row panel whose J block is
// I + D^{-1} (which leaves Z[i][J] = -Z_old[i][J] D^{-1}).
__global__ void __launch_bounds__(kBT) k_blk_gj_pivot(BlkItems b, int p, int64_t cstride,
                                                      double2* Z, double2* Cp, double2* Rp,
                                                      int64_t pstride, int* flags) {
  const Items& it = b.it;
  const int s = blockIdx.x, ch = blockIdx.y;
  const int K = it.K[s];
  const int J0 = p * kBlkGJ;
  if (J0 >= K) return;
  const int w = min(kBlkGJ, K - J0);
  double2* Zs = Z + ch * cstride + it.off2[s];
  double2* C = Cp + ch * pstride + (int64_t)kBlkGJ * it.off1[s];
  double2* R = Rp + ch * pstride + (int64_t)kBlkGJ * it.off1[s];
  __shared__ double2 Dm[kBlkGJ][kBlkGJ + 1];
  __shared__ double2 colf[kBlkGJ], rowf[kBlkGJ];
  __shared__ double2 pinv;
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int i = e / w, j = e - i * w;
    Dm[i][j] = Zs[(int64_t)(J0 + i) * K + J0 + j];
  }
  // old column panel of the other rows
  for (int64_t e = tid; e < (int64_t)K * kBlkGJ; e += blockDim.x) {
    const int i = (int)(e / kBlkGJ), j = (int)(e - (int64_t)i * kBlkGJ);
    double2 v = make_double2(0.0, 0.0);
    if (j < w && (i < J0 || i >= J0 + w)) v = Zs[(int64_t)i * K + J0 + j];
    C[e] = v;
  }
  __syncthreads();
  for (int r = 0; r < w; ++r) {
    if (tid == 0) {
      const double2 pv = Dm[r][r];
      if (!cfinite(pv) || (pv.x == 0.0 && pv.y == 0.0)) atomicOr(flags, kFlagPivot);
      pinv = crecip(pv);
    }
    if (tid < w) {
      colf[tid] = Dm[tid][r];
      rowf[tid] = Dm[r][tid];
    }
    __syncthreads();
    const double2 pi = pinv;
    for (int e = tid; e < w * w; e += blockDim.x) {
      const int i = e / w, c = e - i * w;
      double2 v;
      if (i == r && c == r) v = pi;
      else if (i == r) v = cmul(rowf[c], pi);
      else if (c == r) v = cmul(make_double2(-colf[i].x, -colf[i].y), pi);
      else v = csub(Dm[i][c], cmul(colf[i], cmul(rowf[c], pi)));
      Dm[i][c] = v;
    }
    __syncthreads();
  }
  // new row panel (thread per column)
  for (int c = tid; c < K; c += blockDim.x) {
    const bool inJ = c >= J0 && c < J0 + w;
    double2 old[kBlkGJ];
    if (!inJ)
      for (int i = 0; i < w; ++i) old[i] = Zs[(int64_t)(J0 + i) * K + c];
    for (int j = 0; j < kBlkGJ; ++j) {
      double2 rv = make_double2(0.0, 0.0), zv = make_double2(0.0, 0.0);
      if (j < w) {
        if (inJ) {
          zv = Dm[j][c - J0];
          rv = make_double2(zv.x + (j == c - J0 ? 1.0 : 0.0), zv.y);
        } else {
          double2 acc = make_double2(0.0, 0.0);
          for (int i = 0; i < w; ++i) acc = cfma(Dm[j][i], old[i], acc);
          zv = acc;
          rv = acc;
        }
        Zs[(int64_t)(J0 + j) * K + c] = zv;
      }
      R[(int64_t)j * K + c] = rv;
    }
  }
}

__device__ inline int item_of_tile_blk(const Items& it, const int64_t* toff, int64_t b) {
  int lo = 0, hi = it.n_items;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (toff[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Z[i][:] -= C[i][:] R for the rows i outside the panel; 64 x 64 output
// tiles, wave w the rows 16 w.. on the matrix cores.
__global__ void __launch_bounds__(kBT) k_blk_gj_update(BlkItems b, int p, const int64_t* toff,
                                                       int64_t cstride, double2* Z,
                                                       const double2* Cp, const double2* Rp,
                                                       int64_t pstride) {
  const Items& it = b.it;
  const int64_t bid = blockIdx.x;
  const int s = item_of_tile_blk(it, toff, bid);
  const int ch = blockIdx.y;
  const int K = it.K[s];
  const int J0 = p * kBlkGJ;
  if (J0 >= K) return;
  const int w = min(kBlkGJ, K - J0);
  const int T = (K + 63) / 64;
  const int tile = (int)(bid - toff[s]);
  const int r0 = (tile / T) * 64, c0 = (tile % T) * 64;
  // tiles entirely inside the panel rows have nothing to update
  if (r0 >= J0 && r0 + 64 <= J0 + w) return;
  double2* Zs = Z + ch * cstride + it.off2[s];
  const double2* C = Cp + ch * pstride + (int64_t)kBlkGJ * it.off1[s];
  const double2* R = Rp + ch * pstride + (int64_t)kBlkGJ * it.off1[s];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane >> 4, lc = lane & 15;
  const int row_a = r0 + 16 * wv + lc;
  v4d cr[4], ci[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    cr[t] = v4d{0.0, 0.0, 0.0, 0.0};
    ci[t] = v4d{0.0, 0.0, 0.0, 0.0};
  }
#pragma unroll
  for (int kk = 0; kk < kBlkGJ / 4; ++kk) {
    const int j = 4 * kk + lr;
    const double2 a = (row_a < K && j < w) ? C[(int64_t)row_a * kBlkGJ + j] : make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int col = c0 + 16 * t + lc;
      const double2 bv = (j < w && col < K) ? R[(int64_t)j * K + col] : make_double2(0.0, 0.0);
      cr[t] = mfma16(a.x, bv.x, cr[t]);
      cr[t] = mfma16(-a.y, bv.y, cr[t]);
      ci[t] = mfma16(a.x, bv.y, ci[t]);
      ci[t] = mfma16(a.y, bv.x, ci[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = r0 + 16 * wv + 4 * r + lr, gc = c0 + 16 * t + lc;
      if (gr < K && gc < K && (gr < J0 || gr >= J0 + w)) {
        const int64_t e = (int64_t)gr * K + gc;
        const double2 z = Zs[e];
        Zs[e] = make_double2(z.x - cr[t][r], z.y - ci[t][r]);
      }
    }
}

// out = i tau Q'(+) P (rows), per item and chunk
__global__ void k_blk_qapply(BlkItems b, int64_t cstride, const double2* P, double2* out) {
  const Items& it = b.it;
  const int s = blockIdx.y, ch = blockIdx.z;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s], D = it.D;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)K * K) return;
  const int l = (int)(e / K), m = (int)(e - (int64_t)l * K);
  int a[4], st[4];
  blk_split(l, bd, D, a);
  blk_strides(bd, D, st);
  const double2* Ps = P + ch * cstride + it.off2[s];
  double2 acc = make_double2(0.0, 0.0);
  for (int k = 0; k < D; ++k) {
    if (!(b.fmask >> k & 1)) continue;
    const int n = bd[k].n;
    const int base = l - a[k] * st[k];
    for (int c = 0; c < n; ++c) {
      const double x = bd[k].Xp[a[k] * kBlkN + c];
      const double2 v = Ps[(int64_t)(base + c * st[k]) * K + m];
      acc.x = fma(x, v.x, acc.x);
      acc.y = fma(x, v.y, acc.y);
    }
  }
  out[ch * cstride + it.off2[s] + e] = make_double2(-b.tau * acc.y, b.tau * acc.x);
}

// Fragment order of a K x K matrix: tile (rt, kt) of 16 rows x 4 columns,
// entry (16 rt + (lane & 15), 4 kt + (lane >> 4)) at ((rt KT) + kt) 64 + lane
// with KT = ceil(K / 4); zero outside the matrix.  One wave's load of a tile
// is one contiguous 1 KB read, and the tiles of a row strip follow each other.
__host__ __device__ inline int64_t blk_fsize(int K) {
  return (int64_t)((K + 15) / 16) * ((K + 3) / 4) * 64;
}

__global__ void k_blk_pack(BlkItems b, int64_t cstride, const double2* P, int k, int64_t fcstride,
                           double2* frag) {
  const Items& it = b.it;
  const int s = blockIdx.y, ch = blockIdx.z;
  const int K = it.K[s];
  const int64_t fs = blk_fsize(K);
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= fs) return;
  const int KT = (K + 3) / 4;
  const int64_t rt = e / ((int64_t)KT * 64);
  const int64_t rem = e - rt * KT * 64;
  const int kt = (int)(rem >> 6), lane = (int)(rem & 63);
  const int row = (int)(16 * rt + (lane & 15)), col = 4 * kt + (lane >> 4);
  double2 v = make_double2(0.0, 0.0);
  if (row < K && col < K) v = P[ch * cstride + it.off2[s] + (int64_t)row * K + col];
  frag[ch * fcstride + b.foff[s] + (int64_t)k * fs + e] = v;
}

// ---------------------------------------------------------------------------
// Step of the columns: right-hand sides (one block per item and column).
__device__ inline const double2* blk_forcing(const BlkState& S, const Items& it, int sel, int s) {
  if (sel == kBlkF1) return S.F1 + it.off1[s];
  if (sel == kBlkF0) return S.F0 + it.off1[s];
  return S.ring + (int64_t)sel * it.off1[it.n_items] + it.off1[s];
}

__global__ void __launch_bounds__(kBT) k_blk_rhs(BlkItems b, BlkState S, BlkCols cols, double2* Rb) {
  const Items& it = b.it;
  const int s = blockIdx.x, j = blockIdx.y;
  if (j >= cols.n) return;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s], D = it.D;
  const double2* y = S.hist + cols.slot[j] * S.hstride + (int64_t)(S.n_steps + 1) * it.off1[s] +
                     (int64_t)cols.step[j] * K;
  const double2* fa = blk_forcing(S, it, cols.fa[j], s);
  const double2* fb = blk_forcing(S, it, cols.fb[j], s);
  __shared__ double2 ys[kBlkK];
  for (int l = threadIdx.x; l < K; l += blockDim.x) ys[l] = y[l];
  __syncthreads();
  int st[4];
  blk_strides(bd, D, st);
  const double tau = b.tau, dE = cols.dE[j];
  for (int l = threadIdx.x; l < K; l += blockDim.x) {
    int a[4];
    blk_split(l, bd, D, a);
    double2 q = make_double2(0.0, 0.0);
    for (int k = 0; k < D; ++k) {
      if (!(b.fmask >> k & 1)) continue;
      const int base = l - a[k] * st[k];
      for (int c = 0; c < bd[k].n; ++c) {
        const double x = bd[k].Xp[a[k] * kBlkN + c];
        const double2 v = ys[base + c * st[k]];
        q.x = fma(x, v.x, q.x);
        q.y = fma(x, v.y, q.y);
      }
    }
    const double2 f = cadd(fa[l], fb[l]);
    double2 r;
    r.x = 2.0 * ys[l].x - tau * dE * q.y - 0.5 * tau * f.y;
    r.y = 2.0 * ys[l].y + tau * dE * q.x + 0.5 * tau * f.x;
    Rb[(it.off1[s] + l) * kBlkCols + j] = r;
  }
}

// Solve: Y = sum_k P_k (Rb diag(w_k)), y^{n+1} = Y - y^n.  Block of four
// waves = 64 rows of one item, all columns; k-slices of 32 rows of Rb staged
// in LDS.  Blocks of one item go to one XCD when the item count allows it.
constexpr int kSlice = 32;
__global__ void __launch_bounds__(kBT)
k_blk_solve(BlkItems b, BlkState S, BlkCols cols,
                                                   const double2* frag, const double2* Rb, int RB,
                                                   int xcd) {
  const Items& it = b.it;
  const int bid = blockIdx.x;
  int s, rg;
  if (xcd) {
    const int x = bid & 7, loc = bid >> 3;
    s = (loc / RB) * 8 + x;
    rg = loc % RB;
  } else {
    s = bid / RB;
    rg = bid % RB;
  }
  if (s >= it.n_items) return;
  const int K = it.K[s];
  if (rg * 64 >= K) return;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane >> 4, lc = lane & 15;
  const int rt = rg * 4 + wv;
  const bool active = rt * 16 < K;
  const int KT = (K + 3) / 4;
  const int64_t fs = blk_fsize(K);
  const int t_s = b.terms[s];
  // every load below is unconditional (no branch around a load, so the
  // compiler's wait counts stay exact and the prefetch overlaps): a wave
  // past the item's last row tile reads that tile and stores nothing, and
  // k-tiles past the end read the last one, which meets zero rows of Rb
  const int rt_ld = min(rt, (K + 15) / 16 - 1);
  const double2* fr = frag + b.foff[s] + (int64_t)rt_ld * KT * 64 + lane;
  __shared__ double2 Bs[kSlice][kBlkCols + 1];
  // complex products in three real ones: P1 = a c, P2 = b d, P3 = (a + b)(c + d)
  // for A = a + i b, Y = c + i d; AY = (P1 - P2) + i (P3 - P1 - P2)
  v4d p10 = {0.0, 0.0, 0.0, 0.0}, p20 = p10, p30 = p10, p11 = p10, p21 = p10, p31 = p10;
  double w0[kBlkTerms], w1[kBlkTerms];
#pragma unroll
  for (int k = 0; k < kBlkTerms; ++k) {
    w0[k] = cols.w[k][lc];
    w1[k] = cols.w[k][16 + lc];
  }
  const double2* rb = Rb + it.off1[s] * kBlkCols;
  // iterations (slice, term) in order; the next iteration's A fragments and
  // the next slice of right-hand sides are loaded while the matrix cores
  // work on the current one
  const int n_slices = (K + kSlice - 1) / kSlice;
  const int n_it = n_slices * t_s;
  double2 pb[kSlice * kBlkCols / kBT];
  int pk0 = 0;  // first row of the slice held in pb
  auto load_b = [&](int k0) {
    pk0 = k0;
#pragma unroll
    for (int q = 0; q < kSlice * kBlkCols / kBT; ++q) {
      const int e = threadIdx.x + q * kBT;
      const int r = e / kBlkCols, c = e % kBlkCols;
      pb[q] = rb[(int64_t)min(k0 + r, K - 1) * kBlkCols + c];
    }
  };
  auto load_a = [&](int itn, double2 (&a)[kSlice / 4]) {
    const int sl = itn / t_s, k = itn - sl * t_s;
    const int kt0 = sl * (kSlice / 4);
    const int ktl = KT - 1 - kt0;  // last k-tile of the matrix, relative
    const double2* ap = fr + (int64_t)k * fs + (int64_t)kt0 * 64;
#pragma unroll
    for (int q = 0; q < kSlice / 4; ++q) a[q] = ap[min(q, ktl) * 64];
  };
  // an odd count gets one padding iteration (the last one again, weight 0),
  // so the unrolled pair below runs without a branch around its second half
  const int n_pad = (n_it + 1) & ~1;
  auto body = [&](int itc, double2 (&ac)[kSlice / 4], double2 (&an)[kSlice / 4]) {
    const bool live = itc < n_it;
    const int itv = min(itc, n_it - 1);
    const int sl = itv / t_s, k = itv - sl * t_s;
    if (live && k == 0) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kSlice * kBlkCols / kBT; ++q) {
        const int e = threadIdx.x + q * kBT;
        const int r = e / kBlkCols;
        Bs[r][e % kBlkCols] = pk0 + r < K ? pb[q] : make_double2(0.0, 0.0);
      }
      __syncthreads();
      load_b(min(sl + 1, n_slices - 1) * kSlice);
    }
    load_a(min(itc + 1, n_it - 1), an);
    // keep the prefetch issued ahead of this iteration's products
    __builtin_amdgcn_sched_barrier(0);
    double sw0 = 0.0, sw1 = 0.0;
#pragma unroll
    for (int kk = 0; kk < kBlkTerms; ++kk)
      if (live && kk == k) {
        sw0 = w0[kk];
        sw1 = w1[kk];
      }
#pragma unroll
    for (int q = 0; q < kSlice / 4; ++q) {
      const double2 b0 = Bs[4 * q + lr][lc], b1 = Bs[4 * q + lr][16 + lc];
      const double b0x = b0.x * sw0, b0y = b0.y * sw0, b1x = b1.x * sw1, b1y = b1.y * sw1;
      const double as = ac[q].x + ac[q].y;
      p10 = mfma16(ac[q].x, b0x, p10);
      p20 = mfma16(ac[q].y, b0y, p20);
      p30 = mfma16(as, b0x + b0y, p30);
      p11 = mfma16(ac[q].x, b1x, p11);
      p21 = mfma16(ac[q].y, b1y, p21);
      p31 = mfma16(as, b1x + b1y, p31);
    }
  };
  double2 a0[kSlice / 4], a1[kSlice / 4];
  load_b(0);
  __builtin_amdgcn_sched_barrier(0);  // right-hand sides first, as in the loop
  load_a(0, a0);
#pragma unroll 1
  for (int itc = 0; itc < n_pad; itc += 2) {
    body(itc, a0, a1);
    body(itc + 1, a1, a0);
  }
  if (!active) return;
  const int64_t hoff = (int64_t)(S.n_steps + 1) * it.off1[s];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * rt + 4 * r + lr;
    if (row >= K) continue;
    const int c0 = lc, c1 = 16 + lc;
    if (c0 < cols.n) {
      double2* h = S.hist + cols.slot[c0] * S.hstride + hoff + (int64_t)cols.step[c0] * K + row;
      const double2 yo = h[0];
      h[K] = make_double2(p10[r] - p20[r] - yo.x, p30[r] - p10[r] - p20[r] - yo.y);
    }
    if (c1 < cols.n) {
      double2* h = S.hist + cols.slot[c1] * S.hstride + hoff + (int64_t)cols.step[c1] * K + row;
      const double2 yo = h[0];
      h[K] = make_double2(p11[r] - p21[r] - yo.x, p31[r] - p11[r] - p21[r] - yo.y);
    }
  }
}

// ---------------------------------------------------------------------------
// Face traces.  For the normal dimension k the tangential dimensions are the
// others in increasing order; a face tensor is indexed [t_0][t_1][t_2]
// (last fastest, absent dimensions of size 1).
struct Tang {
  int nd;        // tangential dimensions (D - 1)
  int dim[3];
  int n[3];      // basis sizes
  int nt[3];     // node counts
};
__device__ inline Tang tang_of(const BlkDim* bd, int D, int k) {
  Tang t;
  t.nd = 0;
  for (int c = 0; c < 3; ++c) {
    t.dim[c] = -1;
    t.n[c] = 1;
    t.nt[c] = 1;
  }
  for (int q = 0; q < D; ++q)
    if (q != k) {
      t.dim[t.nd] = q;
      t.n[t.nd] = bd[q].n;
      t.nt[t.nd] = bd[q].nt;
      ++t.nd;
    }
  return t;
}

// Threads of the transmission kernels: one block per (item, column) holds
// every face tensor of the item in LDS, so its latency is hidden by the
// block's own waves (16 per CU).  Both kernels take the dimension D as a
// template argument: every loop over dimensions unrolls and all per-
// dimension sizes stay in registers.
constexpr int kTxT = 1024;

// One contraction stage over dimension C of np stacked face tensors
// [d0][d1][d2] (last fastest; tensor p at in + p istr): dimension C becomes
// nout long, out[..o..] = sum_a M(o, a) in[..a..] with M(o, a) = M[o][a]
// (nodes from basis values), or M[a][o] when kT (basis from nodes); row
// stride kBlkN.
template <int C, bool kT>
__device__ inline void tx_stage(const double2* in, int istr, double2* out, int ostr, int np,
                                int d0, int d1, int d2, int nout, const double* M) {
  const int o0 = C == 0 ? nout : d0, o1 = C == 1 ? nout : d1, o2 = C == 2 ? nout : d2;
  const int tot = o0 * o1 * o2;
  const int nin = C == 0 ? d0 : C == 1 ? d1 : d2;
  const int sc = C == 0 ? d1 * d2 : C == 1 ? d2 : 1;
  for (int e = threadIdx.x; e < np * tot; e += blockDim.x) {
    const int p = e / tot, q = e - p * tot;
    const int i2 = q % o2, i1 = (q / o2) % o1, i0 = q / (o1 * o2);
    const int oc = C == 0 ? i0 : C == 1 ? i1 : i2;
    const int base = (C == 0 ? 0 : i0 * d1 * d2) + (C == 1 ? 0 : i1 * d2) + (C == 2 ? 0 : i2);
    const double2* src = in + p * istr + base;
    double2 acc = make_double2(0.0, 0.0);
    for (int a = 0; a < nin; ++a) {
      const double mv = kT ? M[a * kBlkN + oc] : M[oc * kBlkN + a];
      const double2 u = src[a * sc];
      acc.x = fma(mv, u.x, acc.x);
      acc.y = fma(mv, u.y, acc.y);
    }
    out[p * ostr + q] = acc;
  }
}

// The c-th tangential dimension of the normal dimension k (the others in
// increasing order).
__device__ constexpr int tdim(int k, int c) { return c < k ? c : c + 1; }

// Per-dimension basis sizes (1 beyond D) and multi-index strides (last
// dimension fastest; 0 beyond D).
template <int D>
__device__ inline void tx_sizes(const BlkDim* bd, int* nb, int* st) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    nb[m] = m < D ? bd[m].n : 1;
    st[m] = 0;
  }
  st[D - 1] = 1;
#pragma unroll
  for (int m = D - 2; m >= 0; --m) st[m] = st[m + 1] * nb[m + 1];
}

// Sender: per normal dimension k the six traces of the state (the four
// Robin positions of y, the values of y - y_prev at the two own faces for
// the residual) go through the contraction together, stacked, so that one
// barrier serves all six at every stage.
constexpr int kSendStack = kBlkPos + 2;
template <int D>
__global__ void __launch_bounds__(kTxT) k_blk_send(BlkItems b, BlkState S, BlkTx tx, double2* Tr,
                                                   int* flags) {
  constexpr int kF = D == 2 ? kBlkNt : kBlkFace;      // face tensor size bound
  constexpr int kKD = D == 2 ? kBlkN * kBlkN : kBlkK;  // basis size bound
  const Items& it = b.it;
  const int s = blockIdx.x, j = blockIdx.y;
  if (j >= tx.n) return;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s];
  __shared__ double2 y[kKD], dl[kKD];
  __shared__ double2 A[kSendStack * kF], B[kSendStack * kF];
  __shared__ double red[kTxT / 64];
  const int64_t hoff = (int64_t)(S.n_steps + 1) * it.off1[s];
  const double2* ysrc = tx.slot[j] >= 0
                            ? S.hist + tx.slot[j] * S.hstride + hoff + (int64_t)tx.step[j] * K
                            : S.y0 + it.off1[s];
  const bool resid = tx.prev[j] != -2;
  const double2* yp = nullptr;
  if (resid)
    yp = tx.prev[j] >= 0 ? S.hist + tx.prev[j] * S.hstride + hoff + (int64_t)tx.step[j] * K
                         : S.y0 + it.off1[s];
  for (int l = threadIdx.x; l < K; l += blockDim.x) {
    const double2 v = ysrc[l];
    y[l] = v;
    if (resid) dl[l] = csub(v, yp[l]);
  }
  __syncthreads();
  int nb[4], st[4];
  tx_sizes<D>(bd, nb, st);
  const int nt = bd[0].nt;  // face nodes per tangential dimension (all alike)
  const int nn = D == 2 ? nt : nt * nt * nt;
  double2* tr = Tr + ((int64_t)j * it.n_items + s) * D * kBlkPos * b.fstride;
  const int np = resid ? kSendStack : kBlkPos;
  double part = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int T0 = tdim(k, 0), T1 = tdim(k, 1), T2 = tdim(k, 2);
    const int n0 = nb[T0], n1 = D > 2 ? nb[T1] : 1, n2 = D > 3 ? nb[T2] : 1;
    const int s0 = st[T0], s1 = D > 2 ? st[T1] : 0, s2 = D > 3 ? st[T2] : 0;
    const int n_t = n0 * n1 * n2;
    const int sk = st[k], nk = nb[k];
    // dimension k against the six vectors
    for (int e = threadIdx.x; e < np * n_t; e += blockDim.x) {
      const int p = e / n_t, i = e - p * n_t;
      const int i2 = i % n2, i1 = (i / n2) % n1, i0 = i / (n1 * n2);
      const int base = i0 * s0 + i1 * s1 + i2 * s2;
      double2 acc = make_double2(0.0, 0.0);
      if (p < kBlkPos) {
        const double2* v = bd[k].rob[p];
        for (int a = 0; a < nk; ++a) acc = cfma(v[a], y[base + a * sk], acc);
      } else {
        const double* v = bd[k].val[p - kBlkPos];
        for (int a = 0; a < nk; ++a) {
          const double2 u = dl[base + a * sk];
          acc.x = fma(v[a], u.x, acc.x);
          acc.y = fma(v[a], u.y, acc.y);
        }
      }
      A[p * kF + i] = acc;
    }
    __syncthreads();
    // tangential dimensions: basis values -> face nodes (A -> B -> A -> B)
    tx_stage<0, false>(A, kF, B, kF, np, n0, n1, n2, nt, &bd[T0].phit[0][0]);
    __syncthreads();
    if (D > 2) {
      tx_stage<1, false>(B, kF, A, kF, np, nt, n1, n2, nt, &bd[T1].phit[0][0]);
      __syncthreads();
      tx_stage<2, false>(A, kF, B, kF, np, nt, nt, n2, nt, &bd[T2].phit[0][0]);
      __syncthreads();
    }
    for (int e = threadIdx.x; e < kBlkPos * nn; e += blockDim.x) {
      const int p = e / nn, q = e - p * nn;
      tr[(int64_t)(k * kBlkPos + p) * b.fstride + q] = B[p * kF + q];
    }
    if (resid) {
      const double* w0 = bd[T0].tw;
      const double* w1 = bd[D > 2 ? T1 : T0].tw;
      const double* w2 = bd[D > 3 ? T2 : T0].tw;
      for (int e = threadIdx.x; e < 2 * nn; e += blockDim.x) {
        const int p = e / nn, q = e - p * nn;
        double wgt;
        if (D == 2) {
          wgt = w0[q];
        } else {
          const int i2 = q % nt, i1 = (q / nt) % nt, i0 = q / (nt * nt);
          wgt = w0[i0] * w1[i1] * w2[i2];
        }
        const double2 f = B[(kBlkPos + p) * kF + q];
        part += wgt * (f.x * f.x + f.y * f.y);
      }
    }
    __syncthreads();
  }
  if (resid) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = 0.0;
      for (int q = 0; q < kTxT / 64; ++q) v += red[q];
      if (!isfinite(v)) atomicOr(flags, kFlagNaN);
      const int q = tx.slot[j] >= 0 ? tx.slot[j] : 0;
      S.part[q * S.pstride + (int64_t)s * (S.n_steps + 1) + tx.step[j]] = v;
    }
  }
}

// Receiving side: averaged Robin data g at every node of every face that is
// not on the global boundary, f'[l] = sum_F val'_F[l_k] sum_y w_y g(y)
// prod_c phi'_{l_c}(y_c).  The covering set of a node (Section 4.1
// multi-overlap zones, closed membership) is the subdomains at offsets o
// with o_k in {0, toward the face} and o_c in {0, -1 in the lower band,
// +1 in the upper band} (where the neighbour exists), o != 0.  The two faces
// of a normal dimension share their tables and go through each stage
// stacked; the dimensions follow one another inside one barrier interval.
template <int D>
__global__ void __launch_bounds__(kTxT) k_blk_recv(BlkItems b, BlkState S, BlkTx tx,
                                                   const double2* Tr) {
  constexpr int kF = D == 2 ? kBlkNt : kBlkFace;
  const Items& it = b.it;
  const int s = blockIdx.x, j = blockIdx.y;
  if (j >= tx.n) return;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s];
  __shared__ double2 A[2 * D * kF], B[2 * D * kF];
  const int geom = s / it.n_sub, lin = s - geom * it.n_sub;
  int idx[4], lstr[4], Lm[4];
  {
    int r = lin, sv = 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      Lm[m] = m < D ? it.L[m] : 1;
      idx[m] = r % Lm[m];
      r /= Lm[m];
      lstr[m] = sv;
      sv *= Lm[m];
    }
  }
  int nb[4], st[4];
  tx_sizes<D>(bd, nb, st);
  const double2* trj = Tr + (int64_t)j * it.n_items * D * kBlkPos * b.fstride;
  const int nt = bd[0].nt;
  const int nn = D == 2 ? nt : nt * nt * nt;
  // gather and average
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int T0 = tdim(k, 0), T1 = tdim(k, 1), T2 = tdim(k, 2);
    const BlkDim& b0 = bd[T0];
    const BlkDim& b1 = bd[D > 2 ? T1 : T0];
    const BlkDim& b2 = bd[D > 3 ? T2 : T0];
    const bool lo_open = idx[k] > 0, hi_open = idx[k] < Lm[k] - 1;
    for (int e = threadIdx.x; e < 2 * nn; e += blockDim.x) {
      const int side = e >= nn ? 1 : 0, q = e - side * nn;
      if (!(side ? hi_open : lo_open)) continue;
      int i0, i1 = 0, i2 = 0;
      if (D == 2) {
        i0 = q;
      } else {
        i2 = q % nt;
        i1 = (q / nt) % nt;
        i0 = q / (nt * nt);
      }
      // per tangential dimension the one possible nonzero offset (0: none)
      auto sgn = [&](const BlkDim& dc, int ic, int m) {
        if (ic < dc.band && idx[m] > 0) return -1;
        if (ic >= dc.band + dc.mid && idx[m] < Lm[m] - 1) return 1;
        return 0;
      };
      const int g0 = sgn(b0, i0, T0);
      const int g1 = D > 2 ? sgn(b1, i1, T1) : 0;
      const int g2 = D > 3 ? sgn(b2, i2, T2) : 0;
      const int p0 = b0.band + b0.mid, p1 = b1.band + b1.mid, p2 = b2.band + b2.mid;
      double wgt = b0.tw[i0];
      if (D > 2) wgt *= b1.tw[i1] * b2.tw[i2];
      const int ok = side ? 1 : -1;
      const int nt1 = D > 2 ? nt : 1, nt2 = D > 3 ? nt : 1;
      double2 sum = make_double2(0.0, 0.0);
      int cnt = 0;
      for (int on = 0; on < 2; ++on)
        for (int m = 0; m < 8; ++m) {
          if (on == 0 && m == 0) continue;
          if (((m & 1) && !g0) || ((m & 2) && !g1) || ((m & 4) && !g2)) continue;
          const int o0 = (m & 1) ? g0 : 0, o1 = (m & 2) ? g1 : 0, o2 = (m & 4) ? g2 : 0;
          const int sl = lin + (on ? ok * lstr[k] : 0) + o0 * lstr[T0] +
                         (D > 2 ? o1 * lstr[T1] : 0) + (D > 3 ? o2 * lstr[T2] : 0);
          const int node = ((i0 - o0 * p0) * nt1 + (i1 - o1 * p1)) * nt2 + (i2 - o2 * p2);
          const int pos = on ? (side == 0 ? 2 : 3) : side;
          const int sj = geom * it.n_sub + sl;
          sum = cadd(sum, trj[((int64_t)sj * D + k) * kBlkPos * b.fstride +
                              (int64_t)pos * b.fstride + node]);
          ++cnt;
        }
      A[(2 * k + side) * kF + q] = cscale(sum, wgt / cnt);
    }
  }
  __syncthreads();
  // nodes -> tangential basis indices (A -> B -> A -> B); closed faces go
  // through the stages too and are never read
#pragma unroll
  for (int k = 0; k < D; ++k)
    tx_stage<0, true>(A + 2 * k * kF, kF, B + 2 * k * kF, kF, 2, nt, D > 2 ? nt : 1,
                      D > 3 ? nt : 1, nb[tdim(k, 0)], &bd[tdim(k, 0)].phit[0][0]);
  __syncthreads();
  if (D > 2) {
#pragma unroll
    for (int k = 0; k < D; ++k)
      tx_stage<1, true>(B + 2 * k * kF, kF, A + 2 * k * kF, kF, 2, nb[tdim(k, 0)], nt, nt,
                        nb[tdim(k, 1)], &bd[tdim(k, 1)].phit[0][0]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < D; ++k)
      tx_stage<2, true>(A + 2 * k * kF, kF, B + 2 * k * kF, kF, 2, nb[tdim(k, 0)],
                        nb[tdim(k, 1)], nt, nb[tdim(k, 2)], &bd[tdim(k, 2)].phit[0][0]);
    __syncthreads();
  }
  // f'[l] = sum over open faces of val'[side][l_k] tang_F[l without digit k]
  double2* dst = tx.dst[j] == kBlkF1   ? S.F1 + it.off1[s]
                 : tx.dst[j] == kBlkF0 ? S.F0 + it.off1[s]
                                       : S.ring + (int64_t)tx.dst[j] * it.off1[it.n_items] + it.off1[s];
  for (int l = threadIdx.x; l < K; l += blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int ak = (l / st[k]) % nb[k];
      const int ti = (l / (st[k] * nb[k])) * st[k] + l % st[k];
      if (idx[k] > 0) acc = cadd(acc, cscale(B[2 * k * kF + ti], bd[k].val[0][ak]));
      if (idx[k] < Lm[k] - 1) acc = cadd(acc, cscale(B[(2 * k + 1) * kF + ti], bd[k].val[1][ak]));
    }
    dst[l] = acc;
  }
}

__global__ void k_blk_res_reduce(const double* part, int n_items, int n_steps, double dt,
                                 double* out) {
  __shared__ double red[kBT];
  double acc = 0.0;
  const int64_t tot = (int64_t)n_items * (n_steps + 1);
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int n = (int)(e % (n_steps + 1));
    const double w = (n == 0 || n == n_steps) ? 0.5 * dt : dt;
    acc += w * part[e];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

// out = (x_k M_k) in per (item, vector): vector v of item s read at
// in + imult off1[s] + (ivec0 + v) K_s and written at out + omult off1[s] +
// v K_s; M_k = L^T (which 0), L^{-T} (1), L^{-1} (2), the identity (3).
__global__ void __launch_bounds__(kBT) k_blk_kron(BlkItems b, int which, const double2* in,
                                                  int64_t imult, int ivec0, double2* out,
                                                  int64_t omult) {
  const Items& it = b.it;
  const int s = blockIdx.x, v = blockIdx.y;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s], D = it.D;
  __shared__ double2 x0[kBlkK], x1[kBlkK];
  const int64_t io = imult * it.off1[s] + (int64_t)(ivec0 + v) * K;
  const int64_t oo = omult * it.off1[s] + (int64_t)v * K;
  for (int l = threadIdx.x; l < K; l += blockDim.x) x0[l] = in[io + l];
  __syncthreads();
  int st[4];
  blk_strides(bd, D, st);
  double2* cur = x0;
  double2* nxt = x1;
  for (int k = 0; k < D && which != 3; ++k) {
    const double* M = which == 0 ? bd[k].Lt : (which == 1 ? bd[k].Lit : bd[k].Li);
    const int n = bd[k].n;
    for (int l = threadIdx.x; l < K; l += blockDim.x) {
      int a[4];
      blk_split(l, bd, D, a);
      const int base = l - a[k] * st[k];
      double2 acc = make_double2(0.0, 0.0);
      for (int c = 0; c < n; ++c) {
        const double m = M[a[k] * kBlkN + c];
        const double2 u = cur[base + c * st[k]];
        acc.x = fma(m, u.x, acc.x);
        acc.y = fma(m, u.y, acc.y);
      }
      nxt[l] = acc;
    }
    __syncthreads();
    double2* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  for (int l = threadIdx.x; l < K; l += blockDim.x) out[oo + l] = cur[l];
}

__global__ void k_blk_project(BlkItems b, double norm, double2* y0) {
  const Items& it = b.it;
  const int s = blockIdx.y;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s];
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= K) return;
  int a[4];
  blk_split(l, bd, it.D, a);
  double v = norm;
  for (int k = 0; k < it.D; ++k) v *= bd[k].g0[a[k]];
  y0[it.off1[s] + l] = make_double2(v, 0.0);
}

// dense original-basis matrices (Kronecker forms)
__global__ void k_blk_dense(BlkItems b, int which, double* out) {
  const Items& it = b.it;
  const int s = blockIdx.y;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s], D = it.D;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)K * K) return;
  const int l = (int)(e / K), m = (int)(e - (int64_t)l * K);
  int a[4], c[4];
  blk_split(l, bd, D, a);
  blk_split(m, bd, D, c);
  double v = 0.0;
  if (which == 0) {
    v = 1.0;
    for (int k = 0; k < D; ++k) v *= bd[k].S[a[k] * kBlkN + c[k]];
  } else {
    for (int k = 0; k < D; ++k) {
      if (which == 3 && !(b.fmask >> k & 1)) continue;
      const double* M = which == 1 ? bd[k].Kin : (which == 3 ? bd[k].X : bd[k].B);
      double t = M[a[k] * kBlkN + c[k]];
      for (int k2 = 0; k2 < D; ++k2)
        if (k2 != k) t *= bd[k2].S[a[k2] * kBlkN + c[k2]];
      v += t;
    }
  }
  out[it.off2[s] + e] = v;
}

// one Kronecker pass over the rows (cols = 0) or columns (cols = 1) of a
// real K x K matrix: out = (x_k L_k) applied to each row / column vector
__global__ void __launch_bounds__(kBT) k_blk_kron_mat(BlkItems b, int cols, const double* in,
                                                      double* out) {
  const Items& it = b.it;
  const int s = blockIdx.x, v = blockIdx.y;
  const BlkDim* bd = b.bd + 4 * s;
  const int K = it.K[s], D = it.D;
  if (v >= K) return;
  __shared__ double x0[kBlkK], x1[kBlkK];
  const int64_t base0 = it.off2[s] + (cols ? (int64_t)v : (int64_t)v * K);
  const int64_t es = cols ? K : 1;
  for (int l = threadIdx.x; l < K; l += blockDim.x) x0[l] = in[base0 + l * es];
  __syncthreads();
  int st[4];
  blk_strides(bd, D, st);
  double* cur = x0;
  double* nxt = x1;
  for (int k = 0; k < D; ++k) {
    for (int l = threadIdx.x; l < K; l += blockDim.x) {
      int a[4];
      blk_split(l, bd, D, a);
      const int base = l - a[k] * st[k];
      double acc = 0.0;
      for (int c = 0; c < bd[k].n; ++c) acc = fma(bd[k].Lo[a[k] * kBlkN + c], cur[base + c * st[k]], acc);
      nxt[l] = acc;
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  for (int l = threadIdx.x; l < K; l += blockDim.x) out[base0 + l * es] = cur[l];
}

}  // namespace

// ------------------------------- launchers ---------------------------------

hipError_t launch_blk_dims(const Items& it, BlkDim* bd, double mu_re, double mu_im,
                           double init_alpha, const double* init_center, int* flags,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_blk_dims, dim3(nblk((int64_t)it.n_items * it.D, 64)), dim3(64), 0, st, it,
                     bd, mu_re, mu_im, init_alpha, init_center, flags);
  return hipGetLastError();
}

int64_t blk_pot_item_doubles(const int32_t* nb, const int32_t* qn, int D) {
  int64_t off[9];
  blk_pot_layout(nb, qn, D, off);
  return off[8];
}

int64_t blk_pot_stage_doubles(const int32_t* nb, const int32_t* qn, int D, int n_elec) {
  if (D != 4 || n_elec != 2) return 0;
  const int64_t R = (int64_t)nb[1] * nb[1] * nb[3] * nb[3];
  return (int64_t)qn[0] * qn[2] * R + (int64_t)qn[0] * nb[2] * nb[2] * R;
}

hipError_t launch_blk_potential(const BlkItems& b, const Potential& pot, const int64_t* soff,
                                double* scratch, double* stage, int64_t stage_item, int batch,
                                int q_max, int qq_max, int K_max, double* Vp, hipStream_t st) {
  const Items& it = b.it;
  const int n_items = it.n_items;
  hipLaunchKernelGGL(k_blk_tables, dim3(nblk(q_max), n_items), dim3(kBT), 0, st, b, soff, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (it.dim == 1) {
    // both electrons' nucleus terms (zero without nuclei), then the
    // electron-electron term
    hipLaunchKernelGGL(k_blk_pot1, dim3(1, n_items, 2), dim3(kBT), 0, st, b, pot, soff, scratch);
    hipLaunchKernelGGL(k_blk_pot2, dim3(n_items), dim3(kBT), 0, st, b, pot, soff, scratch, 1, 0);
  } else {
    for (int m = 0; m < it.n_elec; ++m)
      hipLaunchKernelGGL(k_blk_pot2, dim3(n_items), dim3(kBT), 0, st, b, pot, soff, scratch, 0, m);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (it.D == 4 && it.n_elec == 2) {
    for (int s0 = 0; s0 < n_items; s0 += batch) {
      const int nb_ = std::min(batch, n_items - s0);
      hipLaunchKernelGGL(k_blk_ee4_a, dim3(qq_max, nb_), dim3(kBT), 0, st, b, pot, soff, scratch,
                         stage, stage_item, s0);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_blk_ee4_b, dim3(2048, nb_), dim3(kBT), 0, st, b, soff, scratch, stage,
                         stage_item, s0);
      hipLaunchKernelGGL(k_blk_ee4_c, dim3(2048, nb_), dim3(kBT), 0, st, b, soff, scratch, stage,
                         stage_item, s0);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_blk_vfull, dim3(nblk((int64_t)K_max * K_max), n_items), dim3(kBT), 0, st, b,
                     soff, scratch, Vp);
  return hipGetLastError();
}

hipError_t launch_blk_anchor(const BlkItems& b, const double* Vp, const double* Ea, int n_chunks,
                             int64_t cstride, double2* Z, int K_max, hipStream_t st) {
  hipLaunchKernelGGL(k_blk_anchor, dim3(nblk((int64_t)K_max * K_max), b.it.n_items, n_chunks),
                     dim3(kBT), 0, st, b, Vp, Ea, cstride, Z);
  return hipGetLastError();
}

hipError_t launch_blk_invert(const BlkItems& b, int n_chunks, int64_t cstride, double2* Z,
                             double2* Cp, double2* Rp, int64_t pstride, const int64_t* toff,
                             int64_t n_tiles, int K_max, int* flags, hipStream_t st) {
  const int n_panels = (K_max + kBlkGJ - 1) / kBlkGJ;
  for (int p = 0; p < n_panels; ++p) {
    hipLaunchKernelGGL(k_blk_gj_pivot, dim3(b.it.n_items, n_chunks), dim3(kBT), 0, st, b, p,
                       cstride, Z, Cp, Rp, pstride, flags);
    hipLaunchKernelGGL(k_blk_gj_update, dim3((unsigned)n_tiles, n_chunks), dim3(kBT), 0, st, b, p,
                       toff, cstride, Z, Cp, Rp, pstride);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_blk_qapply(const BlkItems& b, int n_chunks, int64_t cstride, const double2* P,
                             double2* out, int K_max, hipStream_t st) {
  hipLaunchKernelGGL(k_blk_qapply, dim3(nblk((int64_t)K_max * K_max), b.it.n_items, n_chunks),
                     dim3(kBT), 0, st, b, cstride, P, out);
  return hipGetLastError();
}

hipError_t launch_blk_pack(const BlkItems& b, int n_chunks, int64_t cstride, const double2* P,
                           int k, int64_t fcstride, double2* frag, int K_max, hipStream_t st) {
  hipLaunchKernelGGL(k_blk_pack, dim3(nblk(blk_fsize(K_max)), b.it.n_items, n_chunks), dim3(kBT),
                     0, st, b, cstride, P, k, fcstride, frag);
  return hipGetLastError();
}

hipError_t launch_blk_step(const BlkItems& b, const BlkState& S, const BlkCols& cols,
                           const double2* frag, double2* Rb, int K_max, hipStream_t st) {
  if (cols.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_blk_rhs, dim3(b.it.n_items, cols.n), dim3(kBT), 0, st, b, S, cols, Rb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int RB = (K_max + 63) / 64;
  const int xcd = (b.it.n_items % 8) == 0 ? 1 : 0;
  hipLaunchKernelGGL(k_blk_solve, dim3((unsigned)(b.it.n_items * RB)), dim3(kBT), 0, st, b, S, cols,
                     frag, Rb, RB, xcd);
  return hipGetLastError();
}

hipError_t launch_blk_transmit(const BlkItems& b, const BlkState& S, const BlkTx& tx, double2* Tr,
                               int K_max, int* flags, hipStream_t st) {
  if (tx.n <= 0) return hipSuccess;
  (void)K_max;
  const dim3 grid(b.it.n_items, tx.n);
  if (b.it.D == 2)
    hipLaunchKernelGGL(k_blk_send<2>, grid, dim3(kTxT), 0, st, b, S, tx, Tr, flags);
  else
    hipLaunchKernelGGL(k_blk_send<4>, grid, dim3(kTxT), 0, st, b, S, tx, Tr, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (b.it.D == 2)
    hipLaunchKernelGGL(k_blk_recv<2>, grid, dim3(kTxT), 0, st, b, S, tx, Tr);
  else
    hipLaunchKernelGGL(k_blk_recv<4>, grid, dim3(kTxT), 0, st, b, S, tx, Tr);
  return hipGetLastError();
}

hipError_t launch_blk_res_reduce(const double* part, int n_items, int n_steps, double dt,
                                 double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_blk_res_reduce, dim3(1), dim3(kBT), 0, st, part, n_items, n_steps, dt, out);
  return hipGetLastError();
}

hipError_t launch_blk_kron(const BlkItems& b, int which, const double2* in, int64_t imult,
                           int ivec0, double2* out, int64_t omult, int n_vec, hipStream_t st) {
  hipLaunchKernelGGL(k_blk_kron, dim3(b.it.n_items, n_vec), dim3(kBT), 0, st, b, which, in, imult,
                     ivec0, out, omult);
  return hipGetLastError();
}

hipError_t launch_blk_project(const BlkItems& b, double norm, int K_max, double2* y0,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_blk_project, dim3(nblk(K_max), b.it.n_items), dim3(kBT), 0, st, b, norm, y0);
  return hipGetLastError();
}

hipError_t launch_blk_dense(const BlkItems& b, int which, const double* Vp, double* out,
                            int K_max, hipStream_t st) {
  if (which == 2) {
    // rows out of place, then columns in place (each block owns one column)
    hipLaunchKernelGGL(k_blk_kron_mat, dim3(b.it.n_items, K_max), dim3(kBT), 0, st, b, 0, Vp, out);
    hipLaunchKernelGGL(k_blk_kron_mat, dim3(b.it.n_items, K_max), dim3(kBT), 0, st, b, 1, out, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_blk_dense, dim3(nblk((int64_t)K_max * K_max), b.it.n_items), dim3(kBT), 0,
                     st, b, which, out);
  return hipGetLastError();
}

}  // namespace swr
