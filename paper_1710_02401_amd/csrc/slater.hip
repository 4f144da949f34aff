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

// The same integrals for the extended functions of either basis: local
// orbitals read them from the item's table (k_lo_tables).
__device__ inline OneD ext_1d(const Items& it, int s, int k, int a, int b) {
  if (!it.lsd) return slater_1d(it, s, k, a, b);
  const int m2 = 2 * it.n_orb, sz = m2 * m2;
  const double* t = it.lo_tab + ((int64_t)s * 2 + k) * 5 * sz + a * m2 + b;
  OneD r;
  r.S = t[0];
  r.X = t[sz];
  r.T = t[2 * sz];
  r.B = t[3 * sz];
  r.W = t[4 * sz];
  return r;
}

__global__ void k_slater_assemble(Items it, double* A, double* Kin, double* Q, double* B,
                                  double* W) {
  const int s = blockIdx.y;
  const int K = it.K[s];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * K) return;
  const int m = e / K, m2 = e - m * K;
  const int n = slater_half(it, s);
  int l, p, l2, p2;
  slater_pair(it, s, m, &l, &p);
  slater_pair(it, s, m2, &l2, &p2);
  const int ua[2] = {l, n + p}, ub[2] = {n + p, l};
  const int va[2] = {l2, n + p2}, vb[2] = {n + p2, l2};
  double sa = 0.0, sk = 0.0, sq = 0.0, sb = 0.0, sw = 0.0;
  for (int t = 0; t < 2; ++t)
    for (int t2 = 0; t2 < 2; ++t2) {
      const double sg = t == t2 ? 1.0 : -1.0;
      const OneD x = ext_1d(it, s, 0, ua[t], va[t2]);
      const OneD y = ext_1d(it, s, 1, ub[t], vb[t2]);
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
// functions).  With the quadrature rules (x_q, w_q) of the first and (y_r,
// w'_r) of the second interval:
//   G[u v][r] = sum_q w_q U_u(x_q) U_v(x_q) / sqrt((x_q - y_r)^2 + eps_ee^2),
//   N0[u v] = sum_q w_q U_u U_v u_nuc(x_q),  N1[u v] = sum_r w'_r U_u U_v u_nuc(y_r).
// w_q U_u(x_q) U_v(x_q) is formed once per node (in LDS up to kSlaterQ
// nodes, else per use: the same values).
constexpr int kSlaterQ = 2048;
__global__ void __launch_bounds__(kST) k_slater_pot_stage(Items it, Potential pot,
                                                          const int64_t* soff, double* scratch) {
  const int s = blockIdx.x;
  const int n2 = 2 * slater_half(it, s);
  const int pr = blockIdx.y;
  if (pr >= n2 * n2) return;
  const int u = pr / n2, v = pr - u * n2;
  const int q0n = it.qn[4 * s], q1n = it.qn[4 * s + 1];
  const double* x = it.qx + it.qoff[4 * s];
  const double* wx = it.qw + it.qoff[4 * s];
  const double* y = it.qx + it.qoff[4 * s + 1];
  const double* wy = it.qw + it.qoff[4 * s + 1];
  double* G = scratch + soff[s] + (int64_t)pr * q1n;
  double* N0 = scratch + soff[s] + (int64_t)n2 * n2 * q1n;
  double* N1 = N0 + n2 * n2;
  __shared__ double red0[kST], red1[kST];
  __shared__ double fq[kSlaterQ];
  auto f = [&](int q) {
    double d;
    return wx[q] * slater_ext(it, s, u, x[q], &d) * slater_ext(it, s, v, x[q], &d);
  };
  const bool staged = q0n <= kSlaterQ;  // uniform over the block
  if (staged)
    for (int q = threadIdx.x; q < q0n; q += blockDim.x) fq[q] = f(q);
  __syncthreads();
  const double ee2 = pot.eps_ee * pot.eps_ee;
  for (int r = threadIdx.x; r < q1n; r += blockDim.x) {
    double acc = 0.0;
    for (int q = 0; q < q0n; ++q) {
      const double fv = staged ? fq[q] : f(q);
      const double dxy = x[q] - y[r];
      acc += fv / sqrt(dxy * dxy + ee2);
    }
    G[r] = acc;
  }
  double a0 = 0.0, a1 = 0.0;
  for (int q = threadIdx.x; q < q0n; q += blockDim.x)
    a0 += (staged ? fq[q] : f(q)) * u_nuclei(pot, x[q]);
  for (int r = threadIdx.x; r < q1n; r += blockDim.x) {
    double d;
    a1 += wy[r] * slater_ext(it, s, u, y[r], &d) * slater_ext(it, s, v, y[r], &d) *
          u_nuclei(pot, y[r]);
  }
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
  const int n = slater_half(it, s), n2 = 2 * n;
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
      const double* G = scratch + soff[s] + (int64_t)(a * n2 + a2) * q1n;
      double ee = 0.0;
      for (int r = 0; r < q1n; ++r) {
        double d;
        ee += G[r] * wy[r] * slater_ext(it, s, b, y[r], &d) * slater_ext(it, s, b2, y[r], &d);
      }
      const double s0 = ext_1d(it, s, 0, a, a2).S, s1 = ext_1d(it, s, 1, b, b2).S;
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
  const int n = slater_half(it, s);
  __shared__ double a[kSmallK * kSmallK];
  __shared__ double b[kSmallK];
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) a[e] = A[it.off2[s] + e];
  const double c1 = center[0], c2 = center[1];
  const double g2 = M_PI / (2.0 * init_alpha);
  const double N = 1.0 / sqrt(2.0 * g2 * (1.0 - exp(-init_alpha * (c1 - c2) * (c1 - c2))));
  auto proj = [&](int k, int u, double c) {
    const double lo = it.lo[4 * s + k], hi = it.hi[4 * s + k];
    if (it.lsd) {
      // orbital u: sum over its interval's Gaussians
      const int t = u < n ? 0 : 1, l = u - t * n, ng = it.nb[4 * s + t];
      const double* C = it.lo_C + (int64_t)it.idx[4 * s + t] * ng * it.n_orb;
      const double* al = it.alpha + it.aoff[4 * s + t];
      double acc = 0.0;
      for (int w = 0; w < ng; ++w)
        acc = fma(C[w * it.n_orb + l], pair_overlap(al[w], it.delta[4 * s + t], c, init_alpha, lo, hi),
                  acc);
      return acc;
    }
    double au, du;
    slater_gauss(it, s, u, &au, &du);
    return pair_overlap(au, du, c, init_alpha, lo, hi);
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

// ---------------------------------------------------------------------------
// Local orbitals (Section 3): the orbital problem of interval i in its
// Gaussians, and its generalised eigenproblem.

constexpr int kLoN = 16;  // Gaussians per interval at most

__device__ inline double lo_step(double t, double width) {
  double u = t / width + 0.5;
  u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
  return u * u * u * (10.0 - 15.0 * u + 6.0 * u * u);
}

// (V * B)(x) for V(r) = -Z / sqrt(r^2 + eta^2) and the order-`order`
// mollifier of half-width eps: sum_k w_k sigma (1 - t_k^2)^order V(x - eps t_k)
// over the rule (t_k, w_k) on [-1, 1].
__device__ inline double lo_mollified(double x, double Z, double eta, const LoParams& lp,
                                      const double* mx, const double* mw, int n_m) {
  double acc = 0.0;
  for (int k = 0; k < n_m; ++k) {
    const double t = mx[k];
    double b = 1.0;
    for (int j = 0; j < lp.order; ++j) b *= 1.0 - t * t;
    const double r = x - lp.eps * t;
    acc += mw[k] * lp.sigma * b * (-Z / sqrt(r * r + eta * eta));
  }
  return acc;
}

// Generalised symmetric eigenproblem H c = lambda S c (n <= NMAX) by one
// thread: Cholesky S = L L^T, A = L^{-1} H L^{-T}, cyclic Jacobi on A, the
// M lowest eigenvectors back-transformed, C[u * ld + l].
template <int NMAX>
__device__ void lo_eigen(int n, int M, int ld, double* S, double* H, double* V, double* C,
                         int* flags) {
  for (int j = 0; j < n; ++j) {
    double d = S[j * n + j];
    for (int k = 0; k < j; ++k) d -= S[j * n + k] * S[j * n + k];
    if (!(d > 0.0)) {
      atomicOr(flags, kFlagPivot);
      return;
    }
    d = sqrt(d);
    S[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = S[i * n + j];
      for (int k = 0; k < j; ++k) v -= S[i * n + k] * S[j * n + k];
      S[i * n + j] = v / d;
    }
  }
  // Y = L^{-1} H (columns), then A = L^{-1} Y^T (H symmetric)
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = 0; c < n; ++c)
      for (int i = 0; i < n; ++i) {
        double v = H[i * n + c];
        for (int k = 0; k < i; ++k) v -= S[i * n + k] * H[k * n + c];
        H[i * n + c] = v / S[i * n + i];
      }
    for (int i = 0; i < n; ++i)
      for (int c = i + 1; c < n; ++c) {
        const double t = H[i * n + c];
        H[i * n + c] = H[c * n + i];
        H[c * n + i] = t;
      }
  }
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < n; ++c) V[i * n + c] = i == c ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < n; ++i) {
      dia += H[i * n + i] * H[i * n + i];
      for (int c = i + 1; c < n; ++c) off += H[i * n + c] * H[i * n + c];
    }
    if (off <= 1e-34 * dia) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = H[p * n + q];
        if (apq == 0.0) continue;
        const double th = (H[q * n + q] - H[p * n + p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = H[k * n + p], akq = H[k * n + q];
          H[k * n + p] = c * akp - sn * akq;
          H[k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = H[p * n + k], aqk = H[q * n + k];
          H[p * n + k] = c * apk - sn * aqk;
          H[q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - sn * vkq;
          V[k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
  bool used[NMAX] = {};
  for (int l = 0; l < M; ++l) {
    int best = -1;
    for (int i = 0; i < n; ++i)
      if (!used[i] && (best < 0 || H[i * n + i] < H[best * n + best])) best = i;
    used[best] = true;
    // c = L^{-T} v (back substitution)
    double c[NMAX];
    for (int i = n - 1; i >= 0; --i) {
      double v = V[i * n + best];
      for (int k = i + 1; k < n; ++k) v -= S[k * n + i] * c[k];
      c[i] = v / S[i * n + i];
    }
    double sg = 0.0;
    for (int u = 0; u < n; ++u) sg += (u + 1) * c[u];
    const double f = sg < 0.0 ? -1.0 : 1.0;
    for (int u = 0; u < n; ++u) {
      C[u * ld + l] = f * c[u];
      if (!isfinite(c[u])) atomicOr(flags, kFlagNaN);
    }
  }
}

__global__ void __launch_bounds__(kST) k_lo_orbitals(Items it, Potential pot, LoParams lp,
                                                     const double* qx, const double* qw,
                                                     const int64_t* qoff, const double* mx,
                                                     const double* mw, int n_m, double* C_out,
                                                     int* flags) {
  const int i = blockIdx.x;  // interval i: item i carries its Gaussians in dimension 0
  const int n = it.nb[4 * i];
  const int M = it.n_orb;
  const double* al = it.alpha + it.aoff[4 * i];
  const double dl = it.delta[4 * i];
  const double lo = it.lo[4 * i], hi = it.hi[4 * i];
  const double xc = 0.5 * (lo + hi);
  __shared__ double sx[kST], sw[kST], sa[kST], sv[kST];
  __shared__ double Sm[kLoN * kLoN], Hm[kLoN * kLoN], Vm[kLoN * kLoN];
  const bool mine = (int)threadIdx.x < n * n;
  const int u = mine ? threadIdx.x / n : 0, w = mine ? threadIdx.x % n : 0;
  double accS = 0.0, accH = 0.0;
  for (int64_t q0 = qoff[i]; q0 < qoff[i + 1]; q0 += kST) {
    const int64_t q = q0 + threadIdx.x;
    if (q < qoff[i + 1]) {
      const double x = qx[q];
      const double st = lo_step(fabs(x - xc) - lp.barrier, lp.width);
      double v = lp.v_inf * st;
      for (int A = 0; A < pot.n_nuc; ++A) {
        const double R = pot.pos[A], Z = pot.charge[A];
        if (lo <= R && R <= hi)
          v += lo_mollified(x - R, Z, pot.eps_en, lp, mx, mw, n_m);
        else
          v += -Z / sqrt((x - R) * (x - R) + pot.eps_en * pot.eps_en);
      }
      sx[threadIdx.x] = x;
      sw[threadIdx.x] = qw[q];
      sa[threadIdx.x] = 1.0 - st;
      sv[threadIdx.x] = v;
    }
    __syncthreads();
    const int cnt = qoff[i + 1] - q0 < kST ? (int)(qoff[i + 1] - q0) : kST;
    if (mine)
      for (int k = 0; k < cnt; ++k) {
        const double x = sx[k];
        const double gu = exp(-dl * (x - al[u]) * (x - al[u]));
        const double gw = exp(-dl * (x - al[w]) * (x - al[w]));
        const double du = -2.0 * dl * (x - al[u]) * gu, dw = -2.0 * dl * (x - al[w]) * gw;
        accS += sw[k] * gu * gw;
        accH += sw[k] * (0.5 * sa[k] * du * dw + sv[k] * gu * gw);
      }
    __syncthreads();
  }
  if (mine) {
    Sm[u * n + w] = accS;
    Hm[u * n + w] = accH;
  }
  __syncthreads();
  double* C = C_out + (int64_t)i * n * M;
  if (threadIdx.x == 0) lo_eigen<kLoN>(n, lp.n_eig, M, Sm, Hm, Vm, C, flags);
  // Section 3.3: the Gaussians added at the interval's ends, unit columns
  const int g = (M - lp.n_eig) / 2;
  for (int e = threadIdx.x; e < n * 2 * g; e += blockDim.x) {
    const int uu = e / (2 * g), c = e % (2 * g);
    const int at = c < g ? c : n - 1 - (c - g);
    C[uu * M + lp.n_eig + c] = uu == at ? 1.0 : 0.0;
  }
}

// Per (item s, dimension k): T[q][a][b] = sum_{u,w} Ce[u][a] Ce[w][b] G[q][u][w]
// for the extended Gaussians' one-dimensional integrals G (slater_1d: S, X,
// T, B, W over the item's box of dimension k) and Ce the block-diagonal
// coefficients of the item's two intervals (orbitals a < M from the first
// coordinate's interval, a >= M from the second's).
__global__ void __launch_bounds__(kST) k_lo_tables(Items it, double* tab) {
  const int s = blockIdx.x, k = blockIdx.y;
  const int n = it.nb[4 * s], M = it.n_orb;
  const int n2 = 2 * n, m2 = 2 * M;
  __shared__ double G[5][4 * kLoN * kLoN];
  __shared__ double Y[5][2 * kLoN * 2 * 8];
  const double* C0 = it.lo_C + (int64_t)it.idx[4 * s] * n * M;
  const double* C1 = it.lo_C + (int64_t)it.idx[4 * s + 1] * n * M;
  auto ce = [&](int uu, int a) {  // Ce[uu][a]
    if (uu < n) return a < M ? C0[uu * M + a] : 0.0;
    return a >= M ? C1[(uu - n) * M + (a - M)] : 0.0;
  };
  for (int e = threadIdx.x; e < n2 * n2; e += blockDim.x) {
    const OneD o = slater_1d(it, s, k, e / n2, e % n2);
    G[0][e] = o.S;
    G[1][e] = o.X;
    G[2][e] = o.T;
    G[3][e] = o.B;
    G[4][e] = o.W;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n2 * m2; e += blockDim.x) {
    const int uu = e / m2, b = e % m2;
    const int w0 = b < M ? 0 : n;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int w = w0; w < w0 + n; ++w) {
      const double c = ce(w, b);
#pragma unroll
      for (int q = 0; q < 5; ++q) acc[q] = fma(G[q][uu * n2 + w], c, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) Y[q][e] = acc[q];
  }
  __syncthreads();
  double* out = tab + ((int64_t)s * 2 + k) * 5 * m2 * m2;
  for (int e = threadIdx.x; e < m2 * m2; e += blockDim.x) {
    const int a = e / m2, b = e % m2;
    const int u0 = a < M ? 0 : n;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int uu = u0; uu < u0 + n; ++uu) {
      const double c = ce(uu, a);
#pragma unroll
      for (int q = 0; q < 5; ++q) acc[q] = fma(c, Y[q][uu * m2 + b], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) out[(int64_t)q * m2 * m2 + e] = acc[q];
  }
}


// ---- local orbitals of one electron in two dimensions (Section 3, d = 2) ----

// (1/|.| * B)(rho), B(y) = sigma / eps^2 (1 - |y|^2 / eps^2)^M on |y| <= eps.
// About the evaluation point, the two rays of directions theta and
// theta + pi together cross the support along one chord of length 2 sqrt(D),
// D = eps^2 - rho^2 sin^2 theta, on which B integrates in closed form,
// int ((r - r1)(r2 - r))^M dr = (r2 - r1)^(2M+1) (M!)^2 / (2M+1)!; so
//   G = pref int_0^{pi/2} D^(M+1/2) dtheta                                   (rho <= eps),
//   G = pref int_0^{pi/2} (eps cos p)^(2M+1) (eps/rho) cos p / sqrt(1 - (eps sin p / rho)^2) dp
//                                         (rho > eps, sin theta = (eps / rho) sin p),
// pref = 2 sigma 2^(2M+1) (M!)^2 / ((2M+1)! eps^(2M+2)) (lp.sigma), both by
// a Gauss-Legendre rule on [0, pi/2]: ang[j] = (sin, cos) of its nodes,
// ang[n_m + j] = (weight, 0).
__device__ double lo2_coulomb(double rho, const LoParams& lp, const double2* ang, int n_m) {
  const double e = lp.eps;
  double acc = 0.0;
  if (rho <= e) {
    for (int j = 0; j < n_m; ++j) {
      const double sn = ang[j].x * rho;
      const double D = e * e - sn * sn;
      double p = sqrt(D);
      for (int k = 0; k < lp.order; ++k) p *= D;
      acc = fma(ang[n_m + j].x, p, acc);
    }
  } else {
    const double r = e / rho;
    for (int j = 0; j < n_m; ++j) {
      const double c = ang[j].y, sn = ang[j].x * r;
      const double pe = e * c;
      double p = pe;
      for (int k = 0; k < lp.order; ++k) p *= pe * pe;
      acc = fma(ang[n_m + j].x, p * r * c / sqrt(1.0 - sn * sn), acc);
    }
  }
  return lp.sigma * acc;
}

// The generalised problem of lo_eigen solved by the whole block (n <= 64):
// Cholesky one column at a time, L^{-1} H L^{-T} by triangular solves, one
// column per thread, then cyclic Jacobi in the round-robin ordering (each
// round n/2 disjoint rotations, computed from the round's matrix and applied
// together: disjoint rotations commute), the M lowest eigenvectors
// back-transformed (one per thread) and signed as lo_eigen's.  Every barrier
// is reached by every thread (loop bounds are block-uniform).
__device__ void lo_eigen_block(int n, int M, int ld, double* S, double* H, double* V, double* C,
                               int* flags) {
  __shared__ double rc[32], rs[32], red[kST];
  __shared__ int rp[32], rq[32], order[kSmallK];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (t == 0) {
      double d = S[j * n + j];
      for (int k = 0; k < j; ++k) d -= S[j * n + k] * S[j * n + k];
      if (!(d > 0.0)) bad = 1;
      S[j * n + j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    for (int i = j + 1 + t; i < n; i += blockDim.x) {
      double v = S[i * n + j];
      for (int k = 0; k < j; ++k) v -= S[i * n + k] * S[j * n + k];
      S[i * n + j] = v / S[j * n + j];
    }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) atomicOr(flags, kFlagPivot);
    return;  // uniform: bad is read after a barrier
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = t; c < n; c += blockDim.x)
      for (int i = 0; i < n; ++i) {
        double v = H[i * n + c];
        for (int k = 0; k < i; ++k) v -= S[i * n + k] * H[k * n + c];
        H[i * n + c] = v / S[i * n + i];
      }
    __syncthreads();
    for (int e = t; e < n * n; e += blockDim.x) {
      const int i = e / n, c = e % n;
      if (c > i) {
        const double x = H[i * n + c];
        H[i * n + c] = H[c * n + i];
        H[c * n + i] = x;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += blockDim.x) V[e] = (e / n == e % n) ? 1.0 : 0.0;
  const int m = n + (n & 1);  // players of the round-robin (one idle if n is odd)
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = t; e < n * n; e += blockDim.x) {
      const int i = e / n, c = e % n;
      const double x = H[e] * H[e];
      if (i == c) dia += x;
      else if (c > i) off += x;
    }
    red[t] = off;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    const double off_all = red[0];
    __syncthreads();
    red[t] = dia;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    const double dia_all = red[0];
    __syncthreads();
    if (off_all <= 1e-34 * dia_all) break;  // uniform
    for (int r = 0; r < m - 1; ++r) {
      if (t < m / 2) {
        int a, b;
        if (t == 0) {
          a = r;
          b = m - 1;
        } else {
          a = (r + t) % (m - 1);
          b = (r - t + m - 1) % (m - 1);
        }
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, sn = 0.0;
        if (q < n) {
          const double apq = H[p * n + q];
          if (apq != 0.0) {
            const double th = (H[q * n + q] - H[p * n + p]) / (2.0 * apq);
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            sn = tt * c;
          }
        }
        rp[t] = p;
        rq[t] = q < n ? q : p;
        rc[t] = c;
        rs[t] = sn;
      }
      __syncthreads();
      // columns of H and V
      for (int e = t; e < (m / 2) * n; e += blockDim.x) {
        const int g = e / n, k = e % n;
        const int p = rp[g], q = rq[g];
        if (p == q) continue;
        const double c = rc[g], sn = rs[g];
        const double hp = H[k * n + p], hq = H[k * n + q];
        H[k * n + p] = c * hp - sn * hq;
        H[k * n + q] = sn * hp + c * hq;
        const double vp = V[k * n + p], vq = V[k * n + q];
        V[k * n + p] = c * vp - sn * vq;
        V[k * n + q] = sn * vp + c * vq;
      }
      __syncthreads();
      // rows of H
      for (int e = t; e < (m / 2) * n; e += blockDim.x) {
        const int g = e / n, k = e % n;
        const int p = rp[g], q = rq[g];
        if (p == q) continue;
        const double c = rc[g], sn = rs[g];
        const double hp = H[p * n + k], hq = H[q * n + k];
        H[p * n + k] = c * hp - sn * hq;
        H[q * n + k] = sn * hp + c * hq;
      }
      __syncthreads();
    }
  }
  if (t == 0) {
    // the M lowest eigenvalues, ascending (ties to the lower index)
    for (int l = 0; l < M; ++l) {
      int best = -1;
      for (int i = 0; i < n; ++i) {
        bool taken = false;
        for (int k = 0; k < l; ++k) taken |= order[k] == i;
        if (!taken && (best < 0 || H[i * n + i] < H[best * n + best])) best = i;
      }
      order[l] = best;
    }
  }
  __syncthreads();
  for (int l = t; l < M; l += blockDim.x) {
    const int b = order[l];
    // c = L^{-T} v in place in column b of V (back substitution)
    for (int i = n - 1; i >= 0; --i) {
      double v = V[i * n + b];
      for (int k = i + 1; k < n; ++k) v -= S[k * n + i] * V[k * n + b];
      V[i * n + b] = v / S[i * n + i];
    }
    double sg = 0.0;
    for (int u = 0; u < n; ++u) sg += (u + 1) * V[u * n + b];
    const double f = sg < 0.0 ? -1.0 : 1.0;
    for (int u = 0; u < n; ++u) {
      const double x = f * V[u * n + b];
      C[u * ld + l] = x;
      if (!isfinite(x)) atomicOr(flags, kFlagNaN);
    }
  }
}

// Per (item s, dimension k): the Gaussians at the orbital rule's nodes,
// gt[q * 8 + u] (q the rule's global node index), and the one-dimensional
// integrals tab[((s * 2 + k) * 4 + kind) * 64 + u * 8 + w] of kind
// S = int g g, A = int a g g, Ad = int a g' g', Bs = int s g g over the rule.
__global__ void __launch_bounds__(kST) k_lo2_tables(Items it, LoParams lp, const double* qx,
                                                    const double* qw, const int64_t* qoff,
                                                    double* gt, double* tab) {
  const int s = blockIdx.x, k = blockIdx.y;
  const int n = it.nb[4 * s + k];
  const double* al = it.alpha + it.aoff[4 * s + k];
  const double dl = it.delta[4 * s + k];
  const double xc = 0.5 * (it.lo[4 * s + k] + it.hi[4 * s + k]);
  const int64_t q0 = qoff[2 * s + k], q1 = qoff[2 * s + k + 1];
  for (int64_t e = threadIdx.x; e < (q1 - q0) * 8; e += blockDim.x) {
    const int64_t q = q0 + e / 8;
    const int u = (int)(e % 8);
    gt[q * 8 + u] = u < n ? exp(-dl * (qx[q] - al[u]) * (qx[q] - al[u])) : 0.0;
  }
  const int kind = threadIdx.x >> 6, u = (threadIdx.x >> 3) & 7, w = threadIdx.x & 7;
  if (u >= n || w >= n) return;
  double acc = 0.0;
  for (int64_t q = q0; q < q1; ++q) {
    const double x = qx[q];
    const double gu = exp(-dl * (x - al[u]) * (x - al[u]));
    const double gw = exp(-dl * (x - al[w]) * (x - al[w]));
    const double st = lo_step(fabs(x - xc) - lp.barrier, lp.width);
    double f;
    if (kind == 0) f = gu * gw;
    else if (kind == 1) f = (1.0 - st) * gu * gw;
    else if (kind == 2) f = (1.0 - st) * (-2.0 * dl * (x - al[u]) * gu) * (-2.0 * dl * (x - al[w]) * gw);
    else f = st * gu * gw;
    acc = fma(qw[q], f, acc);
  }
  tab[((s * 2 + k) * 4 + kind) * 64 + u * 8 + w] = acc;
}

// First contraction of the nuclear term: for the item's dimension-1 nodes
// q1 of this block (64 of them) and pairs p = (u0, w0),
//   P[q1][p] = sum_{q0} w0 w1 V_n(x0, x1) g0[q0][u0] g0[q0][w0],
// V_n = sum_A -Z_A G(|x - R_A|), P at pp[q1 * 64 + p] (q1 global).
constexpr int kLo2Q = 64;
__global__ void __launch_bounds__(kST) k_lo2_nuclear(Items it, Potential pot, LoParams lp,
                                                     const double* qx, const double* qw,
                                                     const int64_t* qoff, const double2* ang,
                                                     int n_m, const double* gt, double* pp) {
  const int s = blockIdx.x;
  const int64_t b0 = qoff[2 * s], b1 = qoff[2 * s + 1], c0 = qoff[2 * s + 1], c1 = qoff[2 * s + 2];
  const int64_t q1a = c0 + (int64_t)blockIdx.y * kLo2Q;
  if (q1a >= c1) return;  // uniform over the block
  const int n0 = it.nb[4 * s];
  __shared__ double sv[kLo2Q][kLo2Q + 1];  // [q0 - chunk][q1 - q1a]
  __shared__ double sg[kLo2Q][8];
  const int ql = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t q1 = q1a + ql;
  double acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0;
  for (int64_t ch = b0; ch < b1; ch += kLo2Q) {
    __syncthreads();
    for (int e = threadIdx.x; e < kLo2Q * kLo2Q; e += blockDim.x) {
      const int a = e / kLo2Q, bq = e % kLo2Q;
      const int64_t qa = ch + a, qb = q1a + bq;
      double v = 0.0;
      if (qa < b1 && qb < c1) {
        const double x0 = qx[qa], x1 = qx[qb];
        for (int A = 0; A < pot.n_nuc; ++A) {
          const double r0 = x0 - pot.pos[2 * A], r1 = x1 - pot.pos[2 * A + 1];
          v -= pot.charge[A] * lo2_coulomb(sqrt(r0 * r0 + r1 * r1), lp, ang, n_m);
        }
        v *= qw[qa] * qw[qb];
      }
      sv[a][bq] = v;
    }
    for (int e = threadIdx.x; e < kLo2Q * 8; e += blockDim.x) {
      const int64_t qa = ch + e / 8;
      sg[e / 8][e % 8] = qa < b1 ? gt[qa * 8 + e % 8] : 0.0;
    }
    __syncthreads();
    const int lim = b1 - ch < kLo2Q ? (int)(b1 - ch) : kLo2Q;
    for (int a = 0; a < lim; ++a) {
      const double v = sv[a][ql];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int p = grp * 16 + j;  // (u0, w0) = (p / 8, p % 8)
        acc[j] = fma(v * sg[a][p >> 3], sg[a][p & 7], acc[j]);
      }
    }
  }
  if (q1 < c1)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int p = grp * 16 + j;
      if ((p >> 3) < n0 && (p & 7) < n0) pp[q1 * 64 + p] = acc[j];
    }
}

// The orbital problem of item s: N[(u0,w0),(u1,w1)] = sum_{q1} P[q1][(u0,w0)]
// g1[q1][u1] g1[q1][w1], then S = S0 x S1 and
// H = 1/2 (Ad0 x A1 + A0 x Ad1) + V_inf (Bs0 x S1 + S0 x Bs1) + N over
// u = u0 n1 + u1, and the n_eig lowest orbitals into C_out + s n0 n1 n_eig.
__global__ void __launch_bounds__(kST) k_lo2_orbitals(Items it, LoParams lp, const int64_t* qoff,
                                                      const double* gt, const double* pp,
                                                      const double* tab, double* C_out,
                                                      int* flags) {
  const int s = blockIdx.x;
  const int n0 = it.nb[4 * s], n1 = it.nb[4 * s + 1], KG = n0 * n1;
  __shared__ double Sm[kSmallK * kSmallK], Hm[kSmallK * kSmallK], Vm[kSmallK * kSmallK];
  const double* t0 = tab + (size_t)(s * 2) * 4 * 64;
  const double* t1 = tab + (size_t)(s * 2 + 1) * 4 * 64;
  const int64_t c0 = qoff[2 * s + 1], c1 = qoff[2 * s + 2];
  for (int e = threadIdx.x; e < KG * KG; e += blockDim.x) {
    const int ua = e / KG, wa = e % KG;
    const int u0 = ua / n1, u1 = ua % n1, w0 = wa / n1, w1 = wa % n1;
    const int p0 = u0 * 8 + w0, p1 = u1 * 8 + w1;
    double nuc = 0.0;
    for (int64_t q = c0; q < c1; ++q) nuc = fma(pp[q * 64 + p0], gt[q * 8 + u1] * gt[q * 8 + w1], nuc);
    const double S0 = t0[p0], A0 = t0[64 + p0], Ad0 = t0[128 + p0], B0 = t0[192 + p0];
    const double S1 = t1[p1], A1 = t1[64 + p1], Ad1 = t1[128 + p1], B1 = t1[192 + p1];
    Sm[e] = S0 * S1;
    Hm[e] = 0.5 * (Ad0 * A1 + A0 * Ad1) + lp.v_inf * (B0 * S1 + S0 * B1) + nuc;
  }
  __syncthreads();
  lo_eigen_block(KG, lp.n_eig, lp.n_eig, Sm, Hm, Vm, C_out + (int64_t)s * KG * lp.n_eig, flags);
}

// Every matrix of the basis: X[l][m] = sum_{u,w} C[u][l] XG[u][w] C[w][m],
// XG over the item's Gaussians (offsets og), X over its orbitals (it.off2).
__global__ void __launch_bounds__(kST) k_lo2_transform(Items it, const int64_t* og,
                                                       const double* XG, double* X) {
  const int s = blockIdx.x;
  const int KG = it.nb[4 * s] * it.nb[4 * s + 1], M = it.n_orb;
  const double* C = it.lo_C + (int64_t)s * KG * M;
  __shared__ double Y[kSmallK * kSmallK];  // [u][m] = sum_w XG[u][w] C[w][m]
  for (int e = threadIdx.x; e < KG * M; e += blockDim.x) {
    const int u = e / M, m = e % M;
    double v = 0.0;
    for (int w = 0; w < KG; ++w) v = fma(XG[og[s] + (int64_t)u * KG + w], C[w * M + m], v);
    Y[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
    const int l = e / M, m = e % M;
    double v = 0.0;
    for (int u = 0; u < KG; ++u) v = fma(C[u * M + l], Y[u * M + m], v);
    X[it.off2[s] + e] = v;
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

hipError_t launch_lo_orbitals(const Items& it, int n_iv, const Potential& pot, LoParams lp,
                              const double* qx, const double* qw, const int64_t* qoff,
                              const double* mx, const double* mw, int n_m, double* C_out,
                              int* flags, hipStream_t st) {
  if (n_iv < 1) return hipSuccess;
  hipLaunchKernelGGL(k_lo_orbitals, dim3(n_iv), dim3(kST), 0, st, it, pot, lp, qx, qw, qoff, mx,
                     mw, n_m, C_out, flags);
  return hipGetLastError();
}

hipError_t launch_lo_tables(const Items& it, double* tab, hipStream_t st) {
  hipLaunchKernelGGL(k_lo_tables, dim3(it.n_items, 2), dim3(kST), 0, st, it, tab);
  return hipGetLastError();
}

hipError_t launch_lo2_orbitals(const Items& it, const Potential& pot, LoParams lp,
                               const double* qx, const double* qw, const int64_t* qoff,
                               const double2* ang, int n_m, int64_t n_q1_max, double* gt,
                               double* tab, double* pp, double* C_out, int* flags,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_lo2_tables, dim3(it.n_items, 2), dim3(kST), 0, st, it, lp, qx, qw, qoff,
                     gt, tab);
  const int chunks = (int)((n_q1_max + kLo2Q - 1) / kLo2Q);
  hipLaunchKernelGGL(k_lo2_nuclear, dim3(it.n_items, chunks), dim3(kST), 0, st, it, pot, lp, qx,
                     qw, qoff, ang, n_m, gt, pp);
  hipLaunchKernelGGL(k_lo2_orbitals, dim3(it.n_items), dim3(kST), 0, st, it, lp, qoff, gt, pp,
                     tab, C_out, flags);
  return hipGetLastError();
}

hipError_t launch_lo2_transform(const Items& it, const int64_t* og, const double* XG, double* X,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_lo2_transform, dim3(it.n_items), dim3(kST), 0, st, it, og, XG, X);
  return hipGetLastError();
}

}  // namespace swr
