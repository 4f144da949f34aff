// Block path of the SWR hot path (block.hip): tensor Gaussian bases in two or
// four configuration dimensions up to K = 1536 per subdomain (the
// two-electron, two-dimension workload's 6^4 = 1296), in real time.
//
// Every local problem is solved in the basis orthonormalised per dimension:
// with the one-dimensional Gram matrices S_k = L_k L_k^T (Cholesky), the
// coefficients are y = (L_1 x .. x L_D)^T c, so the Gram matrix becomes the
// identity, the Crank-Nicolson matrix I + i tau (H' + E Q') is well
// conditioned whatever the condition of A, and every Kronecker-structured
// operator (kinetic, boundary mass, dipole, traces at faces) keeps its
// structure with transformed one-dimensional factors L_k^{-1} M L_k^{-T}.
// The computed function is the same Galerkin solution; only the coordinates
// of the linear algebra change.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace swr {

constexpr int kBlkN = 8;        // Gaussians per dimension at most
constexpr int kBlkNt = 32;      // face nodes per tangential dimension at most
constexpr int kBlkFace = 512;   // face nodes per face at most (nt^(D-1))
constexpr int kBlkK = 1536;     // basis size per subdomain at most
constexpr int kBlkCols = 32;    // Schwarz iterates advanced by one solve launch at most
constexpr int kBlkTerms = 6;    // field-series terms at most
constexpr int kBlkPos = 4;      // Robin trace positions per dimension
constexpr int kBlkGJ = 32;      // Gauss-Jordan panel width

// Per (item, dimension) one-dimensional data.  The host fills n .. tw; the
// device (launch_blk_dims) the rest.  Matrices are row-major n x n.
struct BlkDim {
  int32_t n, nt, band, mid;  // basis size; tangential face nodes = 2 band + mid
  double lo, hi, eps;        // subdomain interval; overlap width
  double tx[kBlkNt], tw[kBlkNt];  // tangential face rule (composite Gauss-Legendre)
  double S[kBlkN * kBlkN], Kin[kBlkN * kBlkN], X[kBlkN * kBlkN], B[kBlkN * kBlkN];  // original
  double Li[kBlkN * kBlkN];   // L^{-1}
  double Lt[kBlkN * kBlkN];   // L^T  (c -> y)
  double Lit[kBlkN * kBlkN];  // L^{-T} (y -> c)
  double Lo[kBlkN * kBlkN];   // L
  double Kp[kBlkN * kBlkN], Xp[kBlkN * kBlkN], Bp[kBlkN * kBlkN];  // transformed
  double val[2][kBlkN];       // transformed values at lo (0) and hi (1)
  double2 rob[kBlkPos][kBlkN];  // transformed Robin vectors at the positions
                                // 0: lo (-d + mu), 1: hi (+d + mu),
                                // 2: hi - eps (-d + mu), 3: lo + eps (+d + mu)
  double phit[kBlkNt][kBlkN];   // transformed values at the tangential nodes
  double g0[kBlkN];             // transformed projection of phi_0's factor
};

// Device state of the block path's iteration (pointers into the workspace).
// Histories: slot q holds one iterate's states, item s at step n at
// hist + q hstride + (n_T + 1) off1[s] + n K_s.  Robin data vectors of the
// next steps: ring + (2 q + (n & 1)) sum_K + off1[s].  F1: the first
// iterate's (warm-start) data, constant in time; F0: the data of the initial
// state (every later iterate's step 0); y0: the initial state.
struct BlkState {
  double2* hist;
  int64_t hstride;
  double2* ring;
  double2* F1;
  double2* F0;
  const double2* y0;
  double* part;          // residual partials: slot q, item s, step n at
  int64_t pstride;       // part + q pstride + s (n_T + 1) + n
  int n_steps;
};

// Forcing selectors of a column: a ring entry (>= 0: 2 q + parity) or
constexpr int kBlkF1 = -1;    // the warm-start data F1
constexpr int kBlkF0 = -2;    // the initial state's data F0

// One solve launch: the iterates (columns) it advances by one step each,
// column j from step[j] to step[j] + 1 in history slot slot[j], with Robin
// data fa (step) and fb (step + 1).
struct BlkCols {
  int n;                       // active columns (<= kBlkCols)
  int step[kBlkCols];
  int slot[kBlkCols];
  int fa[kBlkCols];
  int fb[kBlkCols];
  double dE[kBlkCols];         // E_{n+1} - E_n
  double w[kBlkTerms][kBlkCols];  // (-d)^k with d = E_{n+1} - E_anchor
};

// Transmission of one launch: column j sends the state of slot[j] at
// step[j] (slot -1: the initial state y0), with the residual against the
// state of prev[j] at the same step (-1: y0; -2: no residual), and writes
// the Robin data vectors of the next iterate to ring entry dst[j] (>= 0) or
// to F0 / F1 (kBlkF0, kBlkF1).
struct BlkTx {
  int n;
  int slot[kBlkCols];
  int step[kBlkCols];
  int prev[kBlkCols];
  int dst[kBlkCols];
};

struct BlkItems {
  Items it;
  const BlkDim* bd;        // [n_items][4]
  const int32_t* terms;    // [n_items] series terms applied
  const int64_t* foff;     // [n_items + 1] offsets of the packed terms (complex)
  int fmask;               // configuration coordinates the field couples to
  int fstride;             // face nodes per face stride of the trace scratch
  double tau, mu_re, mu_im;
};

hipError_t launch_blk_dims(const Items& it, BlkDim* bd, double mu_re, double mu_im,
                           double init_alpha, const double* init_center, int* flags,
                           hipStream_t st);
// Potential in the transformed basis, written as a dense real K x K matrix
// per item at off2[s] of Vp.  scratch: per item sizes from blk_pot_scratch;
// items are processed in batches of `batch` through the staged scratch.
int64_t blk_pot_item_doubles(const int32_t* nb, const int32_t* qn, int D);
int64_t blk_pot_stage_doubles(const int32_t* nb, const int32_t* qn, int D, int n_elec);
// qq_max: the largest nq_0 nq_2 over items (four dimensions); q_max the
// largest node count of any dimension.
hipError_t launch_blk_potential(const BlkItems& b, const Potential& pot, const int64_t* soff,
                                double* scratch, double* stage, int64_t stage_item,
                                int batch, int q_max, int qq_max, int K_max, double* Vp,
                                hipStream_t st);
// Largest sizes the four-dimensional electron-electron stage handles.
constexpr int kEeQ = 256;       // nodes of dimension 1
constexpr int kEeZ = 12288;     // nodes of dimension 1 x pairs of dimension 3
// Anchor matrices M' = I + i tau (H' + E_c Q') of chunk c at Z + c cstride.
hipError_t launch_blk_anchor(const BlkItems& b, const double* Vp, const double* Ea, int n_chunks,
                             int64_t cstride, double2* Z, int K_max, hipStream_t st);
// In-place Gauss-Jordan inversion of every item's matrix (chunk-strided);
// Cp, Rp: per item and chunk K x kBlkGJ scratch each (at kBlkGJ off1[s] +
// c pstride).
hipError_t launch_blk_invert(const BlkItems& b, int n_chunks, int64_t cstride, double2* Z,
                             double2* Cp, double2* Rp, int64_t pstride, const int64_t* toff,
                             int64_t n_tiles, int K_max, int* flags, hipStream_t st);
// out = i tau Q'(+) P per item and chunk (Kronecker sum over the field's
// coordinates acting on the row index).
hipError_t launch_blk_qapply(const BlkItems& b, int n_chunks, int64_t cstride, const double2* P,
                             double2* out, int K_max, hipStream_t st);
// Fragment-ordered copy of term k of chunk c: at frag + c fcstride +
// foff[s] + k fsize(s) ... (see block.hip).
hipError_t launch_blk_pack(const BlkItems& b, int n_chunks, int64_t cstride, const double2* P,
                           int k, int64_t fcstride, double2* frag, int K_max, hipStream_t st);
// One step of every column of a launch (all in one chunk: its terms at
// frag + chunk offset): right-hand sides into Rb, then the solve.
hipError_t launch_blk_step(const BlkItems& b, const BlkState& S, const BlkCols& cols,
                           const double2* frag, double2* Rb, int K_max, hipStream_t st);
// Traces (Robin data at the four positions of every dimension) of every
// column's state and its residual partial, then the Robin data vectors of
// the next iterate.  Tr: scratch [kBlkCols][n_items][D][4][fstride].
hipError_t launch_blk_transmit(const BlkItems& b, const BlkState& S, const BlkTx& tx,
                               double2* Tr, int K_max, int* flags, hipStream_t st);
// Residual reduction of complete iterates: out[q] = sqrt(sum_n w_n sum_s
// part[q][s][n]) with the trapezoid weights of the step dt.
hipError_t launch_blk_res_reduce(const double* part, int n_items, int n_steps, double dt,
                                 double* out, hipStream_t st);
// out = (x_k M_k) in for n_vec vectors per item: vector v of item s read at
// in + imult off1[s] + (ivec0 + v) K_s, written at out + omult off1[s] +
// v K_s; M_k = which 0: L^T, 1: L^{-T}, 2: L^{-1}, 3: the identity.
hipError_t launch_blk_kron(const BlkItems& b, int which, const double2* in, int64_t imult,
                           int ivec0, double2* out, int64_t omult, int n_vec, hipStream_t st);
// Initial state y0 = (x_k L_k^{-1} g_k) (2a/pi)^(D/4).
hipError_t launch_blk_project(const BlkItems& b, double norm, int K_max, double2* y0,
                              hipStream_t st);
// Dense real matrices of the original basis: which 0 A, 1 Kin, 3 Q, 4 B
// (Kronecker forms), 2 V = L V' L^T (from Vp).
hipError_t launch_blk_dense(const BlkItems& b, int which, const double* Vp, double* out,
                            int K_max, hipStream_t st);

}  // namespace swr
