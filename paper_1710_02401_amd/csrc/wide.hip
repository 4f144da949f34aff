// Wide-basis path of the SWR hot path (gfx950): one space dimension, up to
// kWideK Gaussians per subdomain, uneven sizes, many geometries in one batch.
//
// The window's per-step inverses do not fit in memory at these sizes (a
// 256-Gaussian subdomain's inverse is 1 MB per step), so the Crank-Nicolson
// recurrence applies the field series of the inverse inside each step.  With
// M^{n+1} = M_c + i tau (E_{n+1} - E_c) Q around the anchor field E_c of the
// step's chunk and P_0 = M_c^{-1},
//   (M^{n+1})^{-1} = sum_k (E_c - E_{n+1})^k P_k,   P_k = (i tau P_0 Q)^k P_0,
// and the P_k of every chunk are formed once per window: the anchor inverse
// by blocked Gauss-Jordan (k_invert_wide), refined once with a compensated
// residual (k_residual_wide), the terms by batched complex products
// (k_gemm_wide), inversion and products on the matrix cores, then packed into
// symmetric tiles for the recurrence (k_pack_wide).  Matrices are K x K
// row-major at the item's K^2 offset unless said to be packed.
#include <hip/hip_runtime.h>

#include <cmath>

#include "devmath.h"
#include "kernels.h"

namespace swr {
namespace {

constexpr int kWideThreads = 256;  // threads per block of the wide kernels

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Soft-Coulomb potential of one electron in one dimension (eq. pseudo):
// V[a][b] = sum_q w_q u(x_q) phi_a(x_q) phi_b(x_q) with
// u(x) = -sum_A Z_A / sqrt((x - X_A)^2 + eps^2) over the item's composite
// Gauss-Legendre nodes.  phi_a phi_b = exp(-delta ((x-a)^2 + (x-b)^2)); nodes
// where that exponent exceeds 746 contribute an exact zero and are skipped.
// One thread per entry, grid (entry blocks, item).
__global__ void k_potential_wide(Items it, Potential pot, double* V) {
  const int s = blockIdx.y;
  const int K = it.K[s];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * K) return;
  const int a = e / K, b = e - a * K;
  const int geom = s / it.n_sub;
  const double d = it.delta[4 * s];
  const double* al = it.alpha + it.aoff[4 * s];
  const double* qx = it.qx + it.qoff[4 * s];
  const double* qw = it.qw + it.qoff[4 * s];
  const int nq = it.qn[4 * s];
  const double ca = al[a], cb = al[b];
  const double e2 = pot.eps_en * pot.eps_en;
  double acc = 0.0;
  for (int q = 0; q < nq; ++q) {
    const double x = qx[q];
    const double z = d * ((x - ca) * (x - ca) + (x - cb) * (x - cb));
    if (z > 746.0) continue;
    double u = 0.0;
    for (int A = 0; A < pot.n_nuc; ++A) {
      const double r = x - pot.pos[(geom * pot.n_nuc + A) * it.dim];
      u -= pot.charge[A] / sqrt(r * r + e2);
    }
    acc += qw[q] * u * exp(-z);
  }
  V[it.off2[s] + e] = acc;
}

// S2 = Ar + Ap (the real matrix of the explicit half step's identity).
__global__ void k_add_wide(int64_t n, const double* Ar, const double* Ap, double* S2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) S2[e] = Ar[e] + Ap[e];
}

// ---------------------------------------------------------------------------
// Projection of the Gaussian Cauchy data (Section 4.4 step 1): c~_l =
// <phi_0, v_l>_{Omega_i}, then A c = c~ by elimination without pivoting (A is
// symmetric positive definite) on a copy of A in scr (the item's K^2 block),
// then back substitution by columns.  One block per item.
__global__ void __launch_bounds__(kWideThreads) k_project_wide(Items it, const double* A,
                                                               double init_alpha,
                                                               const double* center, double* scr,
                                                               double2* c0, int* flags) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  __shared__ double b[kWideK];
  double* a = scr + it.off2[s];
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) a[e] = A[it.off2[s] + e];
  const double norm = pow(2.0 * init_alpha / M_PI, 0.25);
  for (int l = threadIdx.x; l < K; l += blockDim.x) {
    const double al = it.alpha[it.aoff[4 * s] + l];
    b[l] = norm * pair_overlap(al, it.delta[4 * s], center[0], init_alpha, it.lo[4 * s],
                               it.hi[4 * s]);
  }
  __syncthreads();
  for (int p = 0; p < K; ++p) {
    const double piv = a[p * K + p];
    if (threadIdx.x == 0 && !(fabs(piv) > 0.0)) atomicOr(flags, kFlagPivot);
    const int w = K - p - 1;
    // rows below the pivot: neither row p nor column p is written here
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
      const int r = p + 1 + e / w, c = p + 1 + e % w;
      a[r * K + c] -= a[r * K + p] / piv * a[p * K + c];
    }
    for (int r = p + 1 + threadIdx.x; r < K; r += blockDim.x) b[r] -= a[r * K + p] / piv * b[p];
    __syncthreads();
  }
  for (int p = K - 1; p >= 0; --p) {
    const double x = b[p] / a[p * K + p];
    __syncthreads();  // every thread has read b[p]
    for (int r = threadIdx.x; r < p; r += blockDim.x) b[r] -= a[r * K + p] * x;
    if (threadIdx.x == 0) b[p] = x;
    __syncthreads();
  }
  for (int l = threadIdx.x; l < K; l += blockDim.x) {
    c0[it.off1[s] + l] = make_double2(b[l], 0.0);
    if (!isfinite(b[l])) atomicOr(flags, kFlagNaN);
  }
}

// ---------------------------------------------------------------------------
// Anchor inverses of the field series: X = M_c^{-1}, M_c = Ar + i tau (Hr +
// E_c Q), by Gauss-Jordan in place without pivoting (the Hermitian part of
// M_c, Ar, is positive definite for Im mu <= 0), blocked in panels of 16
// columns.  One block per (item, chunk); the matrix lives at X + c cstride +
// the item's K^2 offset.  Panel P (columns and rows p0 .. p0+15): with C =
// X[:, P], D = X[P, P] and R = D^{-1} X[P, :], every entry becomes
//   X[i][j] - C[i] R[:, j]  (i, j outside P),   -C[i] D^{-1}  (column P),
//   R[:, j]  (row P),   D^{-1}  (the pivot block),
// i.e. Z - A B with Z the matrix with row and column panel zeroed, A = C
// whose panel rows are -I, and B = R whose panel columns are D^{-1}.  A and B
// are staged in LDS, D is inverted there (16 unblocked pivots), and the
// update runs as 16 x 16 blocks on the matrix cores (wave w takes blocks w,
// w + 4, ...), so the matrix is streamed once per panel instead of once per
// pivot.  Padding rows and columns past K are zero in A and B, identity in D.
constexpr int kGJ = 16;
__global__ void __launch_bounds__(kWideThreads) k_invert_wide(Items it, const double* Ar,
                                                              const double* Hr, const double* Q,
                                                              const double* Eanchor, double tau,
                                                              double2* X, int64_t cstride,
                                                              int* flags) {
  const int s = blockIdx.x, c = blockIdx.y;
  const int K = it.K[s];
  const int T = (K + kGJ - 1) / kGJ;
  const int KP = T * kGJ;
  const int64_t o2 = it.off2[s];
  double2* x = X + (int64_t)c * cstride + o2;
  const double E = Eanchor[c];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lr = lane >> 4, lc = lane & 15;
  const double2 z2 = make_double2(0.0, 0.0);
  __shared__ double2 As[kWideK][kGJ + 1];   // A = column panel, rows past K zero
  __shared__ double2 Bs[kGJ][kWideK + 1];   // B = row panel, columns past K zero
  __shared__ double2 Ds[kGJ][kGJ + 1];      // pivot block, inverted in place
  for (int e = t; e < K * K; e += blockDim.x)
    x[e] = make_double2(Ar[o2 + e], tau * fma(E, Q[o2 + e], Hr[o2 + e]));
  bool bad = false;
  __syncthreads();
  for (int p = 0; p < T; ++p) {
    const int p0 = p * kGJ;
    for (int e = t; e < kGJ * KP; e += blockDim.x) {
      const int i = e >> 4, q = e & 15;  // column panel entry (i, p0 + q)
      As[i][q] = (i < K && p0 + q < K) ? x[(int64_t)i * K + p0 + q] : z2;
      const int r = e / KP, j = e - r * KP;  // row panel entry (p0 + r, j)
      Bs[r][j] = (p0 + r < K && j < K) ? x[(int64_t)(p0 + r) * K + j] : z2;
    }
    __syncthreads();
    const int a = t >> 4, b = t & 15;
    Ds[a][b] = (p0 + a < K && p0 + b < K) ? As[p0 + a][b] : make_double2(a == b ? 1.0 : 0.0, 0.0);
    __syncthreads();
    for (int q = 0; q < kGJ; ++q) {
      const double2 pv = Ds[q][q], ca = Ds[a][q], rb = Ds[q][b], v0 = Ds[a][b];
      __syncthreads();
      if (t == 0 && !(fabs(pv.x) > 0.0 || fabs(pv.y) > 0.0)) bad = true;
      const double2 ip = crecip(pv);
      double2 v;
      if (a == q)
        v = b == q ? ip : cmul(rb, ip);
      else if (b == q)
        v = cmul(make_double2(-ca.x, -ca.y), ip);
      else
        v = csub(v0, cmul(ca, cmul(rb, ip)));
      Ds[a][b] = v;
      __syncthreads();
    }
    // B = D^{-1} (row panel), column by column; the panel's own columns take
    // D^{-1}; A's panel rows become -I
    for (int j = t; j < KP; j += blockDim.x) {
      if (j >= p0 && j < p0 + kGJ) {
        for (int k = 0; k < kGJ; ++k) Bs[k][j] = Ds[k][j - p0];
      } else {
        double2 col[kGJ];
#pragma unroll
        for (int m = 0; m < kGJ; ++m) col[m] = Bs[m][j];
#pragma unroll
        for (int k = 0; k < kGJ; ++k) {
          double2 acc = z2;
#pragma unroll
          for (int m = 0; m < kGJ; ++m) acc = cfma(Ds[k][m], col[m], acc);
          Bs[k][j] = acc;
        }
      }
    }
    As[p0 + a][b] = make_double2(a == b ? -1.0 : 0.0, 0.0);
    __syncthreads();
    for (int blk = w; blk < T * T; blk += 4) {
      const int ib = blk / T, jb = blk - ib * T;
      const bool keep = ib != p && jb != p;
      v4d cr, ci;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ib * kGJ + 4 * r + lr, col = jb * kGJ + lc;
        const double2 v = (keep && row < K && col < K) ? x[(int64_t)row * K + col] : z2;
        cr[r] = v.x;
        ci[r] = v.y;
      }
#pragma unroll
      for (int kk = 0; kk < kGJ / 4; ++kk) {
        const double2 av = As[ib * kGJ + lc][4 * kk + lr];
        const double2 bv = Bs[4 * kk + lr][jb * kGJ + lc];
        cr = mfma16(-av.x, bv.x, cr);
        cr = mfma16(av.y, bv.y, cr);
        ci = mfma16(-av.x, bv.y, ci);
        ci = mfma16(-av.y, bv.x, ci);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ib * kGJ + 4 * r + lr, col = jb * kGJ + lc;
        if (row < K && col < K) x[(int64_t)row * K + col] = make_double2(cr[r], ci[r]);
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(flags, kFlagPivot);
  for (int e = t; e < K * K; e += blockDim.x)
    if (!cfinite(x[e])) {
      atomicOr(flags, kFlagNaN);
      break;
    }
}

// ---------------------------------------------------------------------------
// Batched complex products of the series terms: out = scale L R (+ add) per
// item and chunk (chunk c of L, Rc, add and out at c cstride); R is Rc
// (complex) when not null, else Rr (real, the same for every chunk).  64 x 64
// output tiles, k-slices of 16 staged in LDS; wave w computes rows 16 w ..
// 16 w + 15 of the tile on the matrix cores (four real products per complex
// 16 x 16 x 4 step, two for real R).  Grid (tiles over all items, chunks);
// toff holds the prefix sums of ceil(K/64)^2, so a block finds its item by
// bisection.
constexpr int kGT = 64, kGK = 16;
__device__ inline int item_of_tile(const Items& it, const int64_t* toff, int64_t b) {
  int lo = 0, hi = it.n_items;  // toff[lo] <= b < toff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (toff[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <bool kRealR>
__global__ void __launch_bounds__(kWideThreads) k_gemm_wide(Items it, const int64_t* toff,
                                                            const double2* L, const double2* Rc,
                                                            const double* Rr, double2 scale,
                                                            const double2* add, int64_t cstride,
                                                            double2* out) {
  const int64_t b = blockIdx.x;
  const int s = item_of_tile(it, toff, b);
  const int K = it.K[s];
  const int T = (K + kGT - 1) / kGT;
  const int tile = (int)(b - toff[s]);
  const int r0 = (tile / T) * kGT, q0 = (tile % T) * kGT;
  const int64_t co = (int64_t)blockIdx.y * cstride + it.off2[s];
  const double2* l = L + co;
  const double2* rc = kRealR ? nullptr : Rc + co;
  const double* rr = kRealR ? Rr + it.off2[s] : nullptr;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane >> 4, lc = lane & 15;
  __shared__ double2 Ls[kGT][kGK + 1];
  __shared__ double2 Rs[kGK][kGT + 1];
  v4d cr[4], ci[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    cr[t] = v4d{0.0, 0.0, 0.0, 0.0};
    ci[t] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  // the next k-slice is loaded into registers while the current one is
  // multiplied (L slice: 64 rows x 16 columns; R slice: 16 rows x 64 columns)
  double2 pl[4], pr[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * kWideThreads;
      const int lrw = e >> 4, lk = e & 15;
      const int gr = r0 + lrw, gk = k0 + lk;
      pl[q] = (gr < K && gk < K) ? l[(int64_t)gr * K + gk] : make_double2(0.0, 0.0);
      const int rk = e >> 6, rq = e & 63;
      const int gk2 = k0 + rk, gq = q0 + rq;
      const bool in = gk2 < K && gq < K;
      if (kRealR)
        pr[q] = make_double2(in ? rr[(int64_t)gk2 * K + gq] : 0.0, 0.0);
      else
        pr[q] = in ? rc[(int64_t)gk2 * K + gq] : make_double2(0.0, 0.0);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += kGK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * kWideThreads;
      Ls[e >> 4][e & 15] = pl[q];
      Rs[e >> 6][e & 63] = pr[q];
    }
    __syncthreads();
    if (k0 + kGK < K) fetch(k0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK / 4; ++kk) {
      const double2 a = Ls[16 * w + lc][4 * kk + lr];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 bv = Rs[4 * kk + lr][16 * t + lc];
        cr[t] = mfma16(a.x, bv.x, cr[t]);
        ci[t] = mfma16(a.y, bv.x, ci[t]);
        if (!kRealR) {
          cr[t] = mfma16(-a.y, bv.y, cr[t]);
          ci[t] = mfma16(a.x, bv.y, ci[t]);
        }
      }
    }
    __syncthreads();
  }
  double2* o = out + co;
  const double2* ad = add ? add + co : nullptr;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = r0 + 16 * w + 4 * r + lr, gq = q0 + 16 * t + lc;
      if (gr < K && gq < K) {
        const int64_t e = (int64_t)gr * K + gq;
        const double2 y = cmul(scale, make_double2(cr[t][r], ci[t][r]));
        o[e] = ad ? cadd(y, ad[e]) : y;
      }
    }
}

// ---------------------------------------------------------------------------
// Residual of the anchor inverses, R = I - M_c X per item and chunk (M_c as
// in k_invert_wide, X and R chunk-strided as there), with every product
// exact (two-product by fma) and the sums in double-double (Ogita, Rump and
// Oishi's Dot2): R is then accurate to a few units of its own size, so one
// correction X + X R removes the inversion's error to first order.  64 x 64
// output tiles of 256 threads (4 x 4 outputs each: rows ty + 16 u, columns
// tx + 16 v), k-slices of 16 staged in LDS.
__global__ void __launch_bounds__(kWideThreads) k_residual_wide(Items it, const int64_t* toff,
                                                                const double* Ar, const double* Hr,
                                                                const double* Q,
                                                                const double* Eanchor, double tau,
                                                                const double2* X, int64_t cstride,
                                                                double2* R) {
  const int64_t b = blockIdx.x;
  const int s = item_of_tile(it, toff, b);
  const int K = it.K[s];
  const int T = (K + kGT - 1) / kGT;
  const int tile = (int)(b - toff[s]);
  const int r0 = (tile / T) * kGT, q0 = (tile % T) * kGT;
  const int64_t o2 = it.off2[s];
  const int64_t co = (int64_t)blockIdx.y * cstride + o2;
  const double E = Eanchor[blockIdx.y];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ double2 Ms[kGT][kGK + 1];
  __shared__ double2 Xs[kGK][kGT];
  Dot2 re[4][4], im[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      re[u][v] = Dot2{(r0 + ty + 16 * u == q0 + tx + 16 * v) ? 1.0 : 0.0, 0.0};
      im[u][v] = Dot2{0.0, 0.0};
    }
  for (int k0 = 0; k0 < K; k0 += kGK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * kWideThreads;
      const int lr = e >> 4, lk = e & 15;
      const int gr = r0 + lr, gk = k0 + lk;
      if (gr < K && gk < K) {
        const int64_t m = o2 + (int64_t)gr * K + gk;
        Ms[lr][lk] = make_double2(Ar[m], tau * fma(E, Q[m], Hr[m]));
      } else {
        Ms[lr][lk] = make_double2(0.0, 0.0);
      }
      const int rk = e >> 6, rq = e & 63;
      const int gk2 = k0 + rk, gq = q0 + rq;
      Xs[rk][rq] = (gk2 < K && gq < K) ? X[co + (int64_t)gk2 * K + gq] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int kk = 0; kk < kGK; ++kk) {
      double2 mv[4], xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) mv[u] = Ms[ty + 16 * u][kk];
#pragma unroll
      for (int v = 0; v < 4; ++v) xv[v] = Xs[kk][tx + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // subtract (m.x + i m.y)(x.x + i x.y)
          dot2_acc(re[u][v], -mv[u].x, xv[v].x);
          dot2_acc(re[u][v], mv[u].y, xv[v].y);
          dot2_acc(im[u][v], -mv[u].x, xv[v].y);
          dot2_acc(im[u][v], -mv[u].y, xv[v].x);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gr = r0 + ty + 16 * u, gq = q0 + tx + 16 * v;
      if (gr < K && gq < K)
        R[co + (int64_t)gr * K + gq] =
            make_double2(re[u][v].s + re[u][v].c, im[u][v].s + im[u][v].c);
    }
}

// ---------------------------------------------------------------------------
// Packed symmetric storage for the recurrence: the upper 8 x 8 tiles (I <= J)
// row by row, each column-major (entry (a, b) of tile (I, J) = M[8I+a][8J+b]
// at b * 8 + a), padding entries zero; item s at offp[s].  Full matrix
// (c, j) of item s at src + c sc + j sj + off2[s] goes to dst + c dc + j dj +
// offp[s]; grid (item, chunk, term).
__device__ inline double zero_of(double) { return 0.0; }
__device__ inline double2 zero_of(double2) { return make_double2(0.0, 0.0); }

template <class T>
__global__ void __launch_bounds__(kWideThreads) k_pack_wide(Items it, const T* src, int64_t sc,
                                                            int64_t sj, T* dst, int64_t dc,
                                                            int64_t dj) {
  const int s = blockIdx.x;
  const int K = it.K[s];
  const int Tn = (K + 7) >> 3;
  const int64_t n = 32 * (int64_t)Tn * (Tn + 1);
  const T* a = src + blockIdx.y * sc + blockIdx.z * sj + it.off2[s];
  T* o = dst + blockIdx.y * dc + blockIdx.z * dj + it.offp[s];
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    int t = (int)(e >> 6);
    const int l = (int)(e & 63);
    int I = 0;
    while (t >= Tn - I) {
      t -= Tn - I;
      ++I;
    }
    const int row = 8 * I + (l & 7), col = 8 * (I + t) + (l >> 3);
    o[e] = (row < K && col < K) ? a[(int64_t)row * K + col] : zero_of(T());
  }
}

// ---------------------------------------------------------------------------
// Crank-Nicolson recurrence of the wide path (Section 4.4 step 2), the whole
// window of one Schwarz iterate, one block per item (items in the order
// given, largest first).  As in the narrow path, M^n c^n is the previous
// step's right-hand side, so
//   rhs^n   = S2 c^n - rhs^{n-1} + (i tau / 2)(f^n + f^{n+1}),  S2 = Ar + Ap,
//   c^{n+1} = (sum_k d^k P_k) rhs^n,  d = E_c - E_{n+1},
// with rhs^{-1} = M^0 c^0 formed from the full matrices.  Both products read
// the packed symmetric tiles once: wave w walks strips of upper tiles (I,
// I..T-1) (strips I = w and 7 - w of every group of eight, which balances
// the strip lengths); lane (a, b) = (lane % 8, lane / 8) holds entry (a, b)
// of the tile (one coalesced 1 KB load per term), keeps row I's sums over
// the strip in registers (reduced over b at the strip's end) and adds the
// transposed contribution to rows 8J + b (reduced over a by DPP) to the
// wave's own vector in LDS; the four wave vectors are summed by row.
template <bool kCplx>
__device__ inline void strip_pass(int T, int w, int lane, const double2* x, double2* yw,
                                  const double* Sp, const double2* Pp, int terms,
                                  int64_t tstride, double d) {
  const int a = lane & 7, b = lane >> 3;
  for (int i = lane; i < 8 * T; i += 64) yw[i] = make_double2(0.0, 0.0);
  for (int I0 = 0; I0 < T; I0 += 8)
    for (int h = 0; h < 2; ++h) {
      const int I = I0 + (h == 0 ? w : 7 - w);
      if (I >= T) continue;
      const double2 xa = x[8 * I + a];
      double dx = 0.0, dy = 0.0;
      const int t0 = tile_index(I, I, T);
#pragma unroll 2
      for (int J = I; J < T; ++J) {
        const int64_t e = (int64_t)(t0 + J - I) * 64 + lane;
        double2 m;
        if (kCplx) {
          double2 v[kWideTerms];
#pragma unroll
          for (int j = 0; j < kWideTerms; ++j)
            v[j] = j < terms ? Pp[e + j * tstride] : make_double2(0.0, 0.0);
          m = v[kWideTerms - 1];
#pragma unroll
          for (int j = kWideTerms - 2; j >= 0; --j)
            m = make_double2(fma(d, m.x, v[j].x), fma(d, m.y, v[j].y));
        } else {
          m = make_double2(Sp[e], 0.0);
        }
        const double2 xb = x[8 * J + b];
        double tx, ty;
        if (kCplx) {
          dx = fma(m.x, xb.x, fma(-m.y, xb.y, dx));
          dy = fma(m.x, xb.y, fma(m.y, xb.x, dy));
          tx = fma(m.x, xa.x, -m.y * xa.y);
          ty = fma(m.x, xa.y, m.y * xa.x);
        } else {
          dx = fma(m.x, xb.x, dx);
          dy = fma(m.x, xb.y, dy);
          tx = m.x * xa.x;
          ty = m.x * xa.y;
        }
        if (J > I) {
          tx = group8_sum(tx);
          ty = group8_sum(ty);
          if (a == 0) {
            const double2 y = yw[8 * J + b];
            yw[8 * J + b] = make_double2(y.x + tx, y.y + ty);
          }
        }
      }
#pragma unroll
      for (int o = 8; o < 64; o <<= 1) {
        dx += __shfl_xor(dx, o, 64);
        dy += __shfl_xor(dy, o, 64);
      }
      if (b == 0) {
        const double2 y = yw[8 * I + a];
        yw[8 * I + a] = make_double2(y.x + dx, y.y + dy);
      }
    }
}

__global__ void __launch_bounds__(kWideThreads) k_cn_recur_wide(
    Items it, const int32_t* order, int n_steps, const double* S2p, const double* Ar,
    const double* Hr, const double* Q, const double* Eall, const double* Eanchor, double tau,
    const double2* Pp, const int32_t* terms_item, int64_t tstride, int64_t cstride,
    const double2* c0, double2* hist, const double2* F, int* flags) {
  const int s = order[blockIdx.x];
  const int K = it.K[s];
  const int T = (K + 7) >> 3;
  const int terms = terms_item[s];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t o2 = it.off2[s], op = it.offp[s];
  const int64_t hb = (int64_t)(n_steps + 1) * it.off1[s];
  __shared__ double2 sv[kWideK];        // c^n, zero past K
  __shared__ double2 sr[kWideK];        // rhs^n, zero past K
  __shared__ double2 yw[4][kWideK];     // the waves' partial products
  for (int i = t; i < 8 * T; i += kWideThreads) {
    const double2 v = i < K ? c0[it.off1[s] + i] : make_double2(0.0, 0.0);
    sv[i] = v;
    sr[i] = make_double2(0.0, 0.0);
    if (i < K) hist[hb + i] = v;
  }
  __syncthreads();
  double2 rprev = make_double2(0.0, 0.0), fprev = make_double2(0.0, 0.0);
  if (t < K) {
    const double E = Eall[0];
    double ax = 0.0, ay = 0.0, hx = 0.0, hy = 0.0;
    for (int m = 0; m < K; ++m) {
      const int64_t e = o2 + (int64_t)m * K + t;
      const double av = Ar[e], h = fma(E, Q[e], Hr[e]);
      const double2 cm = sv[m];
      ax = fma(av, cm.x, ax);
      ay = fma(av, cm.y, ay);
      hx = fma(h, cm.x, hx);
      hy = fma(h, cm.y, hy);
    }
    rprev = make_double2(fma(-tau, hy, ax), fma(tau, hx, ay));
    fprev = F[hb + t];
  }
  bool bad = false;
  for (int n = 0; n < n_steps; ++n) {
    strip_pass<false>(T, w, lane, sv, yw[w], S2p + op, nullptr, 0, 0, 0.0);
    __syncthreads();
    if (t < K) {
      const double2 u = cadd(cadd(yw[0][t], yw[1][t]), cadd(yw[2][t], yw[3][t]));
      const double2 f1 = F[hb + (int64_t)(n + 1) * K + t];
      const double2 fs = cadd(fprev, f1);
      fprev = f1;
      const double2 rhs = make_double2(fma(-0.5 * tau, fs.y, u.x - rprev.x),
                                       fma(0.5 * tau, fs.x, u.y - rprev.y));
      rprev = rhs;
      sr[t] = rhs;
    }
    __syncthreads();
    const int c = n / kSeriesChunk;
    strip_pass<true>(T, w, lane, sr, yw[w], nullptr, Pp + (int64_t)c * cstride + op, terms,
                     tstride, Eanchor[c] - Eall[n + 1]);
    __syncthreads();
    if (t < K) {
      const double2 v = cadd(cadd(yw[0][t], yw[1][t]), cadd(yw[2][t], yw[3][t]));
      sv[t] = v;
      hist[hb + (int64_t)(n + 1) * K + t] = v;
      bad |= !cfinite(v);
    }
    __syncthreads();
  }
  if (bad) atomicOr(flags, kFlagNaN);
}

// ---------------------------------------------------------------------------
// Transmission and residual of the wide path (Section 4.1 eqs. (S1), (RTC),
// multi-overlap average; Section 5 eq. (residueRT)).  In one dimension every
// face is a single node, and the factored pieces give, for receiving item i
// and step n,
//   f_i^n[l] = sum over entries e of i of X_e beta_e[l] (a_e . c_{j(e)}^n)
// (X_e = w_y / |O(y)|, beta_e = phi^i(x_F), a_e = (n.d/dx + mu) phi^j(x_F));
// with prev, the residual partial sum_n w_n sum_F W_F |b_F . (c_i^n -
// prev_i^n)|^2 of the block's steps (trapezoid weights w_n, face Gram pieces
// b_F = phi^i(x_F), W_F = sum of the face's node weights) goes to
// part[i * gridDim.y + blockIdx.y].  Grid (item, tiles of TS steps; TS
// chosen by the autotuner); wave w takes the steps n0 + w, n0 + w + 4, ...
template <int TS>
__global__ void __launch_bounds__(kWideThreads) k_tx_wide(Items it, Pairs pr, TEnt te, int n_steps,
                                                          const double2* src, double2* dst,
                                                          const double2* prev, double* part,
                                                          double dt) {
  const int i = blockIdx.x;
  const int Ki = it.K[i];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n0 = blockIdx.y * TS;
  const int64_t hbi = (int64_t)(n_steps + 1) * it.off1[i];
  __shared__ double red[kWideThreads / 64];
  double racc = 0.0;
  for (int q = w; q < TS; q += 4) {
    const int n = n0 + q;
    if (n > n_steps) break;
    double2 fl[kWideK / 64];
#pragma unroll
    for (int u = 0; u < kWideK / 64; ++u) fl[u] = make_double2(0.0, 0.0);
    for (int64_t e = te.off[i]; e < te.off[i + 1]; ++e) {
      const int j = pr.pj[te.pair[e]];
      const int Kj = it.K[j];
      const double2* a = te.a + te.aoff[e];
      const double2* cj = src + (int64_t)(n_steps + 1) * it.off1[j] + (int64_t)n * Kj;
      double dx = 0.0, dy = 0.0;
      for (int m = lane; m < Kj; m += 64) {
        const double2 am = a[m], cm = cj[m];
        dx = fma(am.x, cm.x, fma(-am.y, cm.y, dx));
        dy = fma(am.x, cm.y, fma(am.y, cm.x, dy));
      }
      const double X = te.X[te.xoff[e]];
      const double gx = X * wave_sum(dx), gy = X * wave_sum(dy);
      const double* beta = te.beta + te.boff[e];
#pragma unroll
      for (int u = 0; u < kWideK / 64; ++u) {
        const int l = lane + 64 * u;
        if (l < Ki) {
          const double bl = beta[l];
          fl[u].x = fma(bl, gx, fl[u].x);
          fl[u].y = fma(bl, gy, fl[u].y);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kWideK / 64; ++u) {
      const int l = lane + 64 * u;
      if (l < Ki) dst[hbi + (int64_t)n * Ki + l] = fl[u];
    }
    if (prev) {
      double rs = 0.0;
      for (int f = 0; f < 2; ++f) {
        if (te.fnode[((int64_t)i * 8 + f) * 2 + 1] == 0) continue;
        const double* bF = te.gram + te.gram_off[i] + (int64_t)f * (Ki + 1);
        double dx = 0.0, dy = 0.0;
        for (int l = lane; l < Ki; l += 64) {
          const double2 cv = src[hbi + (int64_t)n * Ki + l], pv = prev[hbi + (int64_t)n * Ki + l];
          dx = fma(bF[l], cv.x - pv.x, dx);
          dy = fma(bF[l], cv.y - pv.y, dy);
        }
        dx = wave_sum(dx);
        dy = wave_sum(dy);
        rs = fma(bF[Ki], dx * dx + dy * dy, rs);
      }
      racc = fma((n == 0 || n == n_steps) ? 0.5 * dt : dt, rs, racc);
    }
  }
  if (part) {
    if (lane == 0) red[w] = racc;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)i * gridDim.y + blockIdx.y] = red[0] + red[1] + red[2] + red[3];
  }
}

}  // namespace

// ---- launchers ----
hipError_t launch_potential_wide(const Items& it, const Potential& pot, double* V, int K_max,
                                 hipStream_t st) {
  const unsigned bx = (unsigned)(((int64_t)K_max * K_max + kWideThreads - 1) / kWideThreads);
  hipLaunchKernelGGL(k_potential_wide, dim3(bx, it.n_items), dim3(kWideThreads), 0, st, it, pot, V);
  return hipGetLastError();
}

hipError_t launch_add_wide(int64_t n, const double* Ar, const double* Ap, double* S2,
                           hipStream_t st) {
  const unsigned bx = (unsigned)((n + kWideThreads - 1) / kWideThreads);
  hipLaunchKernelGGL(k_add_wide, dim3(bx), dim3(kWideThreads), 0, st, n, Ar, Ap, S2);
  return hipGetLastError();
}

hipError_t launch_project_wide(const Items& it, const double* A, double init_alpha,
                               const double* center, double* scr, double2* c0, int* flags,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_project_wide, dim3(it.n_items), dim3(kWideThreads), 0, st, it, A,
                     init_alpha, center, scr, c0, flags);
  return hipGetLastError();
}

hipError_t launch_invert_wide(const Items& it, int n_chunks, const double* Ar, const double* Hr,
                              const double* Q, const double* Eanchor, double tau, double2* X,
                              int64_t cstride, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_invert_wide, dim3(it.n_items, n_chunks), dim3(kWideThreads), 0, st, it, Ar,
                     Hr, Q, Eanchor, tau, X, cstride, flags);
  return hipGetLastError();
}

hipError_t launch_gemm_wide(const Items& it, const int64_t* toff, int64_t n_tiles, int n_chunks,
                            const double2* L, const double2* Rc, const double* Rr,
                            double2 scale, const double2* add, int64_t cstride, double2* out,
                            hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (out == L || (Rc && out == Rc)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_tiles, n_chunks);
  if (Rc)
    hipLaunchKernelGGL(k_gemm_wide<false>, grid, dim3(kWideThreads), 0, st, it, toff, L, Rc, Rr,
                       scale, add, cstride, out);
  else
    hipLaunchKernelGGL(k_gemm_wide<true>, grid, dim3(kWideThreads), 0, st, it, toff, L, Rc, Rr,
                       scale, add, cstride, out);
  return hipGetLastError();
}

hipError_t launch_residual_wide(const Items& it, const int64_t* toff, int64_t n_tiles,
                                int n_chunks, const double* Ar, const double* Hr, const double* Q,
                                const double* Eanchor, double tau, const double2* X,
                                int64_t cstride, double2* R, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (R == X) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_residual_wide, dim3((unsigned)n_tiles, n_chunks), dim3(kWideThreads), 0, st,
                     it, toff, Ar, Hr, Q, Eanchor, tau, X, cstride, R);
  return hipGetLastError();
}

hipError_t launch_pack_wide(const Items& it, const double* src, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_wide<double>, dim3(it.n_items, 1, 1), dim3(kWideThreads), 0, st, it,
                     src, (int64_t)0, (int64_t)0, dst, (int64_t)0, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_pack_wide(const Items& it, int n_chunks, int terms, const double2* src,
                            int64_t sc, int64_t sj, double2* dst, int64_t dc, int64_t dj,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_pack_wide<double2>, dim3(it.n_items, n_chunks, terms), dim3(kWideThreads),
                     0, st, it, src, sc, sj, dst, dc, dj);
  return hipGetLastError();
}

hipError_t launch_cn_recur_wide(const Items& it, const int32_t* order, int n_steps,
                                const double* S2p, const double* Ar, const double* Hr,
                                const double* Q, const double* Efield, const double* Eanchor,
                                double tau, const double2* Pp, const int32_t* terms_item,
                                int64_t tstride, int64_t cstride, const double2* c0,
                                double2* hist, const double2* F, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_cn_recur_wide, dim3(it.n_items), dim3(kWideThreads), 0, st, it, order,
                     n_steps, S2p, Ar, Hr, Q, Efield, Eanchor, tau, Pp, terms_item, tstride,
                     cstride, c0, hist, F, flags);
  return hipGetLastError();
}

int tx_wide_tiles(int n_steps, int tile) { return (n_steps + 1 + tile - 1) / tile; }

hipError_t launch_tx_wide(const Items& it, const Pairs& pr, const TEnt& te, int n_steps,
                          const double2* src, double2* dst, const double2* prev, double* part,
                          double dt, int tile, hipStream_t st) {
  const dim3 grid(it.n_items, tx_wide_tiles(n_steps, tile));
  if (tile == 8)
    hipLaunchKernelGGL(k_tx_wide<8>, grid, dim3(kWideThreads), 0, st, it, pr, te, n_steps, src,
                       dst, prev, part, dt);
  else if (tile == 32)
    hipLaunchKernelGGL(k_tx_wide<32>, grid, dim3(kWideThreads), 0, st, it, pr, te, n_steps, src,
                       dst, prev, part, dt);
  else
    hipLaunchKernelGGL(k_tx_wide<16>, grid, dim3(kWideThreads), 0, st, it, pr, te, n_steps, src,
                       dst, prev, part, dt);
  return hipGetLastError();
}

}  // namespace swr
