// Slater-like antisymmetric Gaussian basis (Section 2, eq. (LSD)): assembly
// of the local matrices, the soft-Coulomb potential (Section 5 eq. (pseudo))
// and the projection of the antisymmetrised initial state (Section 4.4 step
// 1).  Every entry is the signed combination of the four extended-basis
// tensor entries its two pairs span (slater.h):
//   M[m][m'] = 1/2 sum_{t,t'} s_t s_t' M_E[(a_t, b_t), (a'_t', b'_t')],
// with (a_0, b_0) = (l, n + p), (a_1, b_1) = (n + p, l), s = (+1, -1), and
// M_E a product (or sum of products) of one-dimensional integrals of the
// extended Gaussians over the item's two intervals.
#include <hip/hip_runtime.h>

#include "devmath.h"
#include "kernels.h"
#include "slater.h"

namespace swr {
namespace {

constexpr int kST = 256;

struct OneD {
  double S, X, T, B, W;
};

// One-dimensional integrals of U_u and U_v over the item's interval of
// dimension k: overlap, position, kinetic (1/2 int u' v'), boundary values,
// partition-of-unity overlap (the shared bands halved).
__device__ inline OneD slater_1d(const Items& it, int s, int k, int u, int v) {
  double a, d, b, e;
  slater_gauss(it, s, u, &a, &d);
  slater_gauss(it, s, v, &b, &e);
  const double lo = it.lo[4 * s + k], hi = it.hi[4 * s + k];
  OneD r;
  pair_integrals(a, d, b, e, lo, hi, &r.S, &r.X, &r.T);
  r.B = exp(-d * (lo - a) * (lo - a)) * exp(-e * (lo - b) * (lo - b)) +
        exp(-d * (hi - a) * (hi - a)) * exp(-e * (hi - b) * (hi - b));
  const double eps = it.eps[k];
  r.W = r.S;
  if (it.idx[4 * s + k] > 0) r.W -= 0.5 * pair_overlap(a, d, b, e, lo, lo + eps);
  if (it.idx[4 * s + k] < it.L[k] - 1) r.W -= 0.5 * pair_overlap(a, d, b, e, hi - eps, hi);
  return r;
}

__global__ void k_slater_assemble(Items it, double* A, double* Kin, double* Q, double* B,
                                  double* W) {
  const int s = blockIdx.y;
  const int K = it.K[s];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * K) return;
  const int m = e / K, m2 = e - m * K;
  const int n = it.nb[4 * s];
  int l, p, l2, p2;
  slater_pair(it, s, m, &l, &p);
  slater_pair(it, s, m2, &l2, &p2);
  const int ua[2] = {l, n + p}, ub[2] = {n + p, l};
  const int va[2] = {l2, n + p2}, vb[2] = {n + p2, l2};
  double sa = 0.0, sk = 0.0, sq = 0.0, sb = 0.0, sw = 0.0;
  for (int t = 0; t < 2; ++t)
    for (int t2 = 0; t2 < 2; ++t2) {
      const double sg = t == t2 ? 1.0 : -1.0;
      const OneD x = slater_1d(it, s, 0, ua[t], va[t2]);
      const OneD y = slater_1d(it, s, 1, ub[t], vb[t2]);
      sa += sg * x.S * y.S;
      sk += sg * (x.T * y.S + x.S * y.T);
      sq += sg * (((it.qmask0 & 1) ? x.X * y.S : 0.0) + ((it.qmask0 & 2) ? x.S * y.X : 0.0));
      sb += sg * (x.B * y.S + x.S * y.B);
      sw += sg * x.W * y.W;
    }
  const int64_t o = it.off2[s] + e;
  A[o] = 0.5 * sa;
  Kin[o] = 0.5 * sk;
  Q[o] = 0.5 * sq;
  B[o] = 0.5 * sb;
  W[o] = 0.5 * sw;
}

__device__ inline double u_nuclei(const Potential& pot, double x) {
  double u = 0.0;
  for (int A = 0; A < pot.n_nuc; ++A) {
    const double r = x - pot.pos[A];
    u -= pot.charge[A] / sqrt(r * r + pot.eps_en * pot.eps_en);
  }
  return u;
}

// Potential, stage 1: one block per (item, pair (u, v) of extended
// Gaussians).  With the quadrature rules (x_q, w_q) of the first and (y_r,
// w'_r) of the second interval:
//   G[u v][r] = sum_q w_q U_u(x_q) U_v(x_q) / sqrt((x_q - y_r)^2 + eps_ee^2),
//   N0[u v] = sum_q w_q U_u U_v u_nuc(x_q),  N1[u v] = sum_r w'_r U_u U_v u_nuc(y_r).
__global__ void __launch_bounds__(kST) k_slater_pot_stage(Items it, Potential pot,
                                                          const int64_t* soff, double* scratch) {
  const int s = blockIdx.x;
  const int n2 = 2 * it.nb[4 * s];
  const int pr = blockIdx.y;
  if (pr >= n2 * n2) return;
  const int u = pr / n2, v = pr - u * n2;
  double au, du, av, dv;
  slater_gauss(it, s, u, &au, &du);
  slater_gauss(it, s, v, &av, &dv);
  const int q0n = it.qn[4 * s], q1n = it.qn[4 * s + 1];
  const double* x = it.qx + it.qoff[4 * s];
  const double* wx = it.qw + it.qoff[4 * s];
  const double* y = it.qx + it.qoff[4 * s + 1];
  const double* wy = it.qw + it.qoff[4 * s + 1];
  double* G = scratch + soff[s] + (int64_t)pr * q1n;
  double* N0 = scratch + soff[s] + (int64_t)n2 * n2 * q1n;
  double* N1 = N0 + n2 * n2;
  __shared__ double red0[kST], red1[kST];
  const double ee2 = pot.eps_ee * pot.eps_ee;
  for (int r = threadIdx.x; r < q1n; r += blockDim.x) {
    double acc = 0.0;
    for (int q = 0; q < q0n; ++q) {
      const double f = wx[q] * exp(-du * (x[q] - au) * (x[q] - au)) * exp(-dv * (x[q] - av) * (x[q] - av));
      const double dxy = x[q] - y[r];
      acc += f / sqrt(dxy * dxy + ee2);
    }
    G[r] = acc;
  }
  double a0 = 0.0, a1 = 0.0;
  for (int q = threadIdx.x; q < q0n; q += blockDim.x)
    a0 += wx[q] * exp(-du * (x[q] - au) * (x[q] - au)) * exp(-dv * (x[q] - av) * (x[q] - av)) *
          u_nuclei(pot, x[q]);
  for (int r = threadIdx.x; r < q1n; r += blockDim.x)
    a1 += wy[r] * exp(-du * (y[r] - au) * (y[r] - au)) * exp(-dv * (y[r] - av) * (y[r] - av)) *
          u_nuclei(pot, y[r]);
  red0[threadIdx.x] = a0;
  red1[threadIdx.x] = a1;
  __syncthreads();
  for (int w = kST / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red0[threadIdx.x] += red0[threadIdx.x + w];
      red1[threadIdx.x] += red1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    N0[pr] = red0[0];
    N1[pr] = red1[0];
  }
}

// Potential, stage 2: one thread per entry, the four signed extended
// entries V_E[(a, b), (a', b')] = N0[a a'] S1[b b'] + S0[a a'] N1[b b'] +
// sum_r G[a a'][r] w'_r U_b(y_r) U_b'(y_r).
__global__ void k_slater_pot_combine(Items it, const int64_t* soff, const double* scratch,
                                     double* V) {
  const int s = blockIdx.y;
  const int K = it.K[s];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * K) return;
  const int m = e / K, m2 = e - m * K;
  const int n = it.nb[4 * s], n2 = 2 * n;
  int l, p, l2, p2;
  slater_pair(it, s, m, &l, &p);
  slater_pair(it, s, m2, &l2, &p2);
  const int ua[2] = {l, n + p}, ub[2] = {n + p, l};
  const int va[2] = {l2, n + p2}, vb[2] = {n + p2, l2};
  const int q1n = it.qn[4 * s + 1];
  const double* y = it.qx + it.qoff[4 * s + 1];
  const double* wy = it.qw + it.qoff[4 * s + 1];
  const double* N0 = scratch + soff[s] + (int64_t)n2 * n2 * q1n;
  const double* N1 = N0 + n2 * n2;
  double acc = 0.0;
  for (int t = 0; t < 2; ++t)
    for (int t2 = 0; t2 < 2; ++t2) {
      const double sg = t == t2 ? 1.0 : -1.0;
      const int a = ua[t], a2 = va[t2], b = ub[t], b2 = vb[t2];
      double ab, db, ab2, db2;
      slater_gauss(it, s, b, &ab, &db);
      slater_gauss(it, s, b2, &ab2, &db2);
      const double* G = scratch + soff[s] + (int64_t)(a * n2 + a2) * q1n;
      double ee = 0.0;
      for (int r = 0; r < q1n; ++r)
        ee += G[r] * wy[r] * exp(-db * (y[r] - ab) * (y[r] - ab)) * exp(-db2 * (y[r] - ab2) * (y[r] - ab2));
      const double s0 = slater_1d(it, s, 0, a, a2).S, s1 = slater_1d(it, s, 1, b, b2).S;
      acc += sg * (N0[a * n2 + a2] * s1 + s0 * N1[b * n2 + b2] + ee);
    }
  V[it.off2[s] + e] = 0.5 * acc;
}

// Initial coefficients: b_m = <phi_0, v_m> with phi_0 the normalised
// antisymmetrised Gaussian pair, then A c = b by elimination without
// pivoting (A symmetric positive definite).
__global__ void k_slater_project(Items it, const double* A, double init_alpha, const double* center,
                                 double2* c0, int* flags) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  const int n = it.nb[4 * s];
  __shared__ double a[kSmallK * kSmallK];
  __shared__ double b[kSmallK];
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) a[e] = A[it.off2[s] + e];
  const double c1 = center[0], c2 = center[1];
  const double g2 = M_PI / (2.0 * init_alpha);
  const double N = 1.0 / sqrt(2.0 * g2 * (1.0 - exp(-init_alpha * (c1 - c2) * (c1 - c2))));
  auto proj = [&](int k, int u, double c) {
    double au, du;
    slater_gauss(it, s, u, &au, &du);
    return pair_overlap(au, du, c, init_alpha, it.lo[4 * s + k], it.hi[4 * s + k]);
  };
  for (int m = threadIdx.x; m < K; m += blockDim.x) {
    int l, p;
    slater_pair(it, s, m, &l, &p);
    const int ua[2] = {l, n + p}, ub[2] = {n + p, l};
    double v = 0.0;
    for (int t = 0; t < 2; ++t) {
      const double e = proj(0, ua[t], c1) * proj(1, ub[t], c2) - proj(0, ua[t], c2) * proj(1, ub[t], c1);
      v += (t == 0 ? 1.0 : -1.0) * e;
    }
    b[m] = 0.70710678118654752440 * N * v;
  }
  __syncthreads();
  for (int q = 0; q < K; ++q) {
    const double piv = a[q * K + q];
    if (threadIdx.x == 0 && !(fabs(piv) > 0.0)) atomicOr(flags, kFlagPivot);
    for (int e = threadIdx.x; e < (K - q - 1) * (K - q); e += blockDim.x) {
      const int r = q + 1 + e / (K - q);
      const int c = q + e % (K - q);
      if (c == q) continue;
      a[r * K + c] -= a[r * K + q] / piv * a[q * K + c];
    }
    __syncthreads();
    for (int r = q + 1 + threadIdx.x; r < K; r += blockDim.x) {
      b[r] -= a[r * K + q] / piv * b[q];
      a[r * K + q] = 0.0;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int r = K - 1; r >= 0; --r) {
      double v = b[r];
      for (int c = r + 1; c < K; ++c) v -= a[r * K + c] * b[c];
      b[r] = v / a[r * K + r];
    }
  }
  __syncthreads();
  for (int m = threadIdx.x; m < K; m += blockDim.x) {
    c0[it.off1[s] + m] = make_double2(b[m], 0.0);
    if (!isfinite(b[m])) atomicOr(flags, kFlagNaN);
  }
}

}  // namespace

hipError_t launch_slater_assemble(const Items& it, double* A, double* Kin, double* Q, double* B,
                                  double* W, int K_max, hipStream_t st) {
  const unsigned bx = (unsigned)(((int64_t)K_max * K_max + kST - 1) / kST);
  hipLaunchKernelGGL(k_slater_assemble, dim3(bx, it.n_items), dim3(kST), 0, st, it, A, Kin, Q, B, W);
  return hipGetLastError();
}

int64_t slater_pot_scratch(int n, int q1) { return (int64_t)(2 * n) * (2 * n) * (q1 + 2); }

hipError_t launch_slater_potential(const Items& it, const Potential& pot, const int64_t* soff,
                                   double* scratch, int n_max, int q_max, double* V, int K_max,
                                   hipStream_t st) {
  (void)q_max;
  hipLaunchKernelGGL(k_slater_pot_stage, dim3(it.n_items, 4 * n_max * n_max), dim3(kST), 0, st, it,
                     pot, soff, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned bx = (unsigned)(((int64_t)K_max * K_max + kST - 1) / kST);
  hipLaunchKernelGGL(k_slater_pot_combine, dim3(bx, it.n_items), dim3(kST), 0, st, it, soff,
                     scratch, V);
  return hipGetLastError();
}

hipError_t launch_slater_project(const Items& it, const double* A, double init_alpha,
                                 const double* center, double2* c0, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_slater_project, dim3(it.n_items), dim3(kST), 0, st, it, A, init_alpha,
                     center, c0, flags);
  return hipGetLastError();
}

}  // namespace swr
