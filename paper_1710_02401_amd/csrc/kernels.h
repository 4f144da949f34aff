// Device-side data views and kernel launchers of the SWR library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace swr {

constexpr int kSmallK = 64;      // in-LDS kernels handle K <= kSmallK
constexpr int kWideK = 256;      // wide-basis path (one dimension): K <= kWideK
constexpr int kWideTerms = 6;    // series terms the wide recurrence applies at most
constexpr int kBlock = 256;      // threads per block of the batched kernels

// Per-item tables (device pointers), passed by value to kernels.
struct Items {
  int n_items, n_sub, D, n_elec, dim;
  // 1: the Slater-like antisymmetric basis (slater.h), 0: tensor Gaussians
  int slater;
  // with slater: 1 for local Slater determinants of local orbitals (Section
  // 3).  n_orb orbitals per interval; interval i's coefficients at lo_C +
  // i * nb * n_orb, entry u * n_orb + l (Gaussian u of the interval, orbital
  // l); lo_tab: per (item, dimension) the one-dimensional integrals of the
  // item's extended orbitals (slater.hip)
  int lsd, n_orb;
  const double* lo_C;
  const double* lo_tab;
  // 1: local orbitals of one electron in two dimensions (Section 3, d = 2):
  // item s's function l is sum_u C[u][l] g_u over its tensor Gaussians g_u
  // (u = u0 nb1 + u1), C at lo_C + s nb0 nb1 n_orb, entry u * n_orb + l
  int lo2;
  // configuration coordinates (bit el * dim + a) the field couples to: the
  // first (or only) component and the second of a circular field (0: none)
  int qmask0, qmask1;
  // second field component (circular field only, else null): its dipole
  // matrix [sum K^2] and its value at the time nodes [n_T + 1]; every M^n
  // then carries E(t_n) Q + E2(t_n) Q2
  const double* Q2;
  const double* E2;
  const int32_t* K;      // [n_items]
  const int64_t* off1;   // [n_items+1] prefix sums of K
  const int64_t* off2;   // [n_items+1] prefix sums of K^2
  const int64_t* offp;   // [n_items+1] prefix sums of the packed symmetric size
                         // 64 T (T+1) / 2, T = ceil(K / 8) (upper 8x8 tiles)
  const int32_t* idx;    // [n_items][4] multi-index
  const int32_t* nb;     // [n_items][4] basis size per dimension
  const int32_t* L;      // [4]
  const double* lo;      // [n_items][4]
  const double* hi;      // [n_items][4]
  const double* eps;     // [4]
  const double* delta;   // [n_items][4]
  const int64_t* aoff;   // [n_items][4] offsets into alpha
  const double* alpha;   // centres
  const int64_t* qoff;   // [n_items][4] offsets into qx/qw
  const int32_t* qn;     // [n_items][4]
  const double* qx;
  const double* qw;
};

// Receiving face nodes (struct-of-arrays).
struct Nodes {
  int64_t n;
  const int32_t* item;   // [n]
  const int32_t* face;   // [n] 2*k + side
  const int32_t* count;  // [n] |O(y)|, 0 on global faces
  const double* x;       // [n][4]
  const double* w;       // [n]
  const int64_t* off;    // [n_items+1]
};

struct Pairs {
  int64_t n;
  const int32_t* pi;     // [n] receiving item
  const int32_t* pj;     // [n] sending item
  const int64_t* poff;   // [n_items+1] pairs of item i
  const int64_t* toff;   // [n+1] offsets of T_ij entries (complex)
  const int32_t* node;   // node lists
  const int64_t* noff;   // [n+1]
};

// Factored transfer operators (D <= 2), one entry per (pair, face):
// T_ij = sum over entries of (beta a^T) (x) X, beta/a on the face's normal
// dimension, X on the tangential one (a 1 x 1 weight when D = 1).
constexpr int kTxDesc = 8;  // ints per sender-side entry descriptor
struct TEnt {
  int64_t n;
  const int32_t* pair;   // [n] pair index
  const int32_t* face;   // [n] 2*k + side of the receiving item
  const int64_t* t0;     // [n] run of the pair's node list
  const int64_t* t1;
  const int64_t* off;    // [n_items+1] entries of item i
  const int64_t* boff;   // [n] offsets of beta (real)
  const int64_t* aoff;   // [n] offsets of a (complex)
  const int64_t* xoff;   // [n] offsets of X (real, receiver rows x sender columns)
  const int64_t* soff;   // [n_items+1] entries whose sender is item j
  const int32_t* sidx;   // entry indices grouped by sender
  const int64_t* blob_off;  // [n_items+1] per-sender packed a/X pieces (complex units)
  const double2* blob;
  const int32_t* sdesc;  // [n][kTxDesc] per-entry descriptors in sender order
  // factored face Gram matrices G_j = sum_F (b b^T) (x) W_F of every item:
  // per face b (normal basis at the face) then W (tangential Gram, weights
  // w_y); item j's faces at gram[gram_off[j] ..), face node runs in fnode
  const int64_t* gram_off;  // [n_items+1] (doubles, even)
  const double* gram;
  const int64_t* fnode;     // [n_items][8][2] first node, node count
  const double* beta;
  const double2* a;
  const double* X;
  double2* v;            // scratch [n][n_steps+1][nbt]: tangential traces
};

// Work lists of the chunked sweep, passed by value: job q covers the steps
// [n_lo, n_hi] (transmit) or the Crank-Nicolson steps n_lo .. n_lo+n_cnt-1
// (recurrence) of one Schwarz iterate.
constexpr int kMaxJobs = 16;
struct TxJobs {
  int n;
  const double2* src[kMaxJobs];  // sending histories
  double2* dst[kMaxJobs];        // Robin data vectors
  int n_lo[kMaxJobs], n_hi[kMaxJobs];
  // Optional residual of the sending history against prev over the job's
  // steps (factored transmission only): one partial per block at
  // part[item * part_stride + part_base + block]; null part: none.
  const double2* prev[kMaxJobs];
  double* part[kMaxJobs];
  int part_base[kMaxJobs];
  int part_stride;
  double dt;
  // Optional per-step factor of the job's Robin data (imaginary time: the
  // sending iterate's normalisation factors); null: 1.
  const double* scale[kMaxJobs];
};
struct RecJobs {
  int n;
  double2* hist[kMaxJobs];       // history written (reads step n_lo unless n_lo == 0)
  const double2* F[kMaxJobs];    // Robin data vectors of the iterate
  // Right-hand side of the job's last step, M^{n_end} c^{n_end} ([sum K],
  // item offsets off1): written at the end, read at the start when n_lo > 0
  // (the previous chunk of the same iterate wrote it).  Null: not written,
  // and recomputed from the matrices at the start.
  double2* carry[kMaxJobs];
  int n_lo[kMaxJobs], n_cnt[kMaxJobs];
};

struct StepList {   // up to 64 selected time steps, passed by value
  int n;
  int step[64];
};

struct FieldFeat {  // tail features of the learned warm start, by value
  int n;              // time nodes M (field values in v)
  double v[64];       // 10 E(t0 + t_m)
  double mid[4];      // centre of the global box per dimension
  double half[4];     // half width of the global box per dimension
  double t0w;         // t0 / (8 T), T the window length
};

struct Potential {
  int n_nuc;
  const double* pos;     // [n_geom][n_nuc][dim]
  const double* charge;  // [n_nuc]
  double eps_en, eps_ee;
};

// Scratch layout of the potential for two space dimensions per electron
// (doubles, from the item's scratch offset): off[k] the weighted product
// table F_k[a n_k + b][q] = w_q phi_a(x_q) phi_b(x_q) of dimension k < D;
// off[4 + m] electron m's nucleus table over the pair indices of its two
// dimensions; off[6..9] the stages of the electron-electron contraction
// T3[q0 q1 q2][p3], T2[q0 q1][p2 p3], T1[q0][p1 p2 p3], Vee[p0 p1 p2 p3];
// off[10] the total.  nb, qn: basis and quadrature sizes per dimension.
__host__ __device__ inline void pot2_layout(const int32_t* nb, const int32_t* qn, int n_elec,
                                            int64_t* off) {
  const int D = 2 * n_elec;
  int64_t o = 0;
  int64_t P[4] = {1, 1, 1, 1};
  for (int k = 0; k < 4; ++k) {
    off[k] = o;
    if (k < D) {
      P[k] = (int64_t)nb[k] * nb[k];
      o += P[k] * qn[k];
    }
  }
  for (int m = 0; m < 2; ++m) {
    off[4 + m] = o;
    if (m < n_elec) o += P[2 * m] * P[2 * m + 1];
  }
  const bool ee = n_elec == 2;
  off[6] = o;
  if (ee) o += (int64_t)qn[0] * qn[1] * qn[2] * P[3];
  off[7] = o;
  if (ee) o += (int64_t)qn[0] * qn[1] * P[2] * P[3];
  off[8] = o;
  if (ee) o += (int64_t)qn[0] * P[1] * P[2] * P[3];
  off[9] = o;
  if (ee) o += P[0] * P[1] * P[2] * P[3];
  off[10] = o;
}

// ---- launchers (return hipError_t of the launch) ----
// Q2: the second component's dipole matrix (it.qmask1), or null.
hipError_t launch_assemble(const Items& it, double* A, double* Kin, double* Q, double* Q2,
                           double* B, double* W, double* S1, const int64_t* s1off, int K_max,
                           hipStream_t st);
hipError_t launch_potential(const Items& it, const Potential& pot, const double* S1,
                            const int64_t* s1off, double* V, double* scratch,
                            const int64_t* scratch_off, hipStream_t st);
hipError_t launch_transfer(const Items& it, const Nodes& nd, const Pairs& pr, double mu_re,
                           double mu_im, double2* T, int K_max, hipStream_t st);
hipError_t launch_face_gram(const Items& it, const Nodes& nd, double* G, int K_max,
                            hipStream_t st);
hipError_t launch_project(const Items& it, const double* A, double init_alpha,
                          const double* init_center, double2* c0, int* flags,
                          hipStream_t st);
hipError_t launch_cn_matrices(int64_t n, const double* A, const double* Kin, const double* V,
                              const double* B, double tau, double mu_re, double mu_im, double* Ar,
                              double* Ap, double* Hr, int tise, double dt, hipStream_t st);
// mode: 0 every step's M^{n+1}, packed upper tiles (TDSE); 1 the real Ar once
// per item, whole and transposed at the item's K^2 offset (TISE); 2 the
// matrix at field Efield[n], n < n_mats, whole and row-major at
// n * out_stride + the item's K^2 offset.
hipError_t launch_invert(const Items& it, int n_mats, const double* Ar, const double* Hr,
                         const double* Q, const double* Efield, int64_t out_stride, double tau,
                         int mode, double2* Minv, int* flags, hipStream_t st, int K_max);
// Series inverses: the steps of chunk c (kSeriesChunk of them) expand around
// an anchor field of their own.
constexpr int kSeriesChunk = 128;
// out = scale * L R + add per item and chunk (K x K row-major at the item's
// K^2 offset, chunk c at c * cstride); R is Rc (complex, chunk-strided) when
// not null, else Rr (real, one for every chunk); add may be null; out may be L.
hipError_t launch_series_product(const Items& it, int n_chunks, const double2* L,
                                 const double2* Rc, const double* Rr, double2 scale,
                                 const double2* add, int64_t cstride, double2* out,
                                 hipStream_t st);
// R = I - M_c X per item and chunk, M_c = Ar + i tau (Hr + Eanchor[c] Q), with
// exact products and double-double sums (layout as above).
hipError_t launch_series_residual(const Items& it, int n_chunks, const double* Ar,
                                  const double* Hr, const double* Q, const double* Eanchor,
                                  double tau, const double2* X, int64_t cstride, double2* R,
                                  hipStream_t st);
// Packed inverses of every step n < n_mats: sum_{k < terms} (Eanchor[c] -
// E_{n+1})^k P_k with c = n / kSeriesChunk, P_k = P + c cstride + k stride
// (1 <= terms <= 8).
hipError_t launch_series_assemble(const Items& it, int n_mats, int terms, const double2* P,
                                  int64_t stride, int64_t cstride, const double* Efield,
                                  const double* Eanchor, double2* Minv, hipStream_t st);
// The field series of a window as the recurrence reads it: chunk c's P_k at
// P + c cstride + k stride + the item's K^2 offset (K x K row-major); D[n] =
// E_c - E_{n+1} for step n of chunk c (the anchor field minus the step's).
struct RecSeries {
  const double2* P;
  int64_t stride, cstride;
  const double* D;
  int terms;
};
// Most series terms the recurrence evaluates in the step (registers); with
// more, the inverses are assembled and read.
constexpr int kRecSeriesMax = 4;
// Crank-Nicolson recurrence of the jobs: with se, each step's inverse is
// evaluated from the series (1 <= se->terms <= kRecSeriesMax, one field
// component); else read from Minv (packed, every step).
hipError_t launch_cn_recur(const Items& it, int n_steps, const double* Ar, const double* Ap,
                           const double* Hr, const double* Q, const double* Efield, double tau,
                           const double2* Minv, const RecSeries* se, const double2* c0,
                           const RecJobs& jobs, int* flags, hipStream_t st);
hipError_t launch_sum_sqrt(const double* partial, int64_t n, double* out, hipStream_t st);
hipError_t launch_transfer_tensor(const Items& it, const Nodes& nd, const Pairs& pr,
                                  const TEnt& te, double mu_re, double mu_im, double* beta,
                                  double2* a, double* X, hipStream_t st);
// Factored face Gram pieces of every item and face (assembly), also when no
// transfer entry exists.
hipError_t launch_gram_tensor(const Items& it, const Nodes& nd, const TEnt& te, double* gram,
                              hipStream_t st);
// Steps per block of the factored transmission for these LDS needs (32 or
// 16), or 0 if they do not fit.
int transmit_tile_steps(int nbt, int64_t pieces, int max_send, int64_t gram);
// Res = sqrt(sum of the valid block partials) of a window transmitted in
// n_chunks jobs: chunk 0 holds steps [0, S], chunk c > 0 steps
// (cS, min((c+1)S, n_T)], tiles of tt steps, item stride part_stride.
hipError_t launch_res_reduce(const double* part, int n_items, int part_stride, int n_steps, int S,
                             int n_chunks, int tt, double* out, hipStream_t st);
// Pack the a and X pieces of every sending item into te.blob (assembly).
hipError_t launch_tx_pack(const Items& it, const Pairs& pr, const TEnt& te, double2* blob,
                          hipStream_t st);
// Robin data vectors of every job; the factored operators when te.n > 0,
// else the dense T.  jobs.scale (per job and step, may be null) multiplies
// the result; nbt = largest tangential basis size over items (1 when D = 1); pieces =
// largest LDS bytes of the a and X pieces an item sends; max_recv / max_send
// = largest number of entries an item receives / sends; tile = steps per
// block of the factored form (16 or 32, and its LDS must fit).
hipError_t launch_transmit(const Items& it, const Pairs& pr, const TEnt& te, int n_steps,
                           const double2* T, const TxJobs& jobs, int nbt,
                           int64_t pieces, int max_recv, int max_send, int64_t gram, int tile,
                           hipStream_t st);
hipError_t launch_fill_history(const Items& it, int n_steps, const double2* c0, double2* hist,
                               hipStream_t st);
hipError_t launch_forcing_from_nodes(const Items& it, const Nodes& nd, int n_steps,
                                     const double2* g, double2* F, hipStream_t st);
hipError_t launch_residual(const Items& it, int n_steps, double dt, const double* G,
                           const double2* cur, const double2* prev, double* partial,
                           double* out, hipStream_t st);
// normalize = 0: imaginary-time steps without the global normalisation
// One imaginary-time step of each job (a Schwarz iterate: its history, Robin
// data, partial norms [n_T + 1][n_items] and normalisation factors
// [n_T + 1], at its own step n), every item; one launch for all jobs.
struct IeJobs {
  int n;
  double2* hist[kMaxJobs];
  const double2* F[kMaxJobs];
  double* partial[kMaxJobs];
  double* nus[kMaxJobs];
  int step[kMaxJobs];
};
hipError_t launch_ie_step(const Items& it, const IeJobs& jobs, int n_steps, double dt,
                          const double* A, const double* W, const double2* Minv, int normalize,
                          int* flags, hipStream_t st);
hipError_t launch_ie_finish(const Items& it, int n_steps, double2* hist, const double* partial,
                            double* nus, int normalize, hipStream_t st);
// p[0..n) = v
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_global_normalise(const Items& it, const double* W, double2* c0,
                                   double* partial, hipStream_t st);
hipError_t launch_geneig(const Items& it, const double* A, const double* Hr, double* lam,
                         double* X, int* flags, hipStream_t st);
// antisym: two electrons, the exchanged half from the mirrored point with
// the sign reversed (points where electron 2 comes after electron 1).
hipError_t launch_reconstruct(const Items& it, int geom, int step, int n_steps,
                              const double2* hist, const double* pts, int64_t n_pts, int antisym,
                              double2* out, hipStream_t st);

hipError_t launch_face_data(const Items& it, const Nodes& nd, const int32_t* cover,
                            const StepList& sl, int n_steps, double mu_re, double mu_im,
                            const double2* hist, double2* g, hipStream_t st);
hipError_t launch_learned_features(const Items& it, const Nodes& nd, const double2* g0,
                                   const FieldFeat& ff, int n_in, float* x, double* scale,
                                   double* wmax, hipStream_t st);
hipError_t launch_learned_targets(const Items& it, const Nodes& nd, const double2* gm,
                                  int n_nodes_t, const double* scale, int n_out, float* y,
                                  hipStream_t st);
hipError_t launch_learned_apply(const Items& it, const Nodes& nd, const float* y,
                                const double* scale, const double2* g0, const double* lag,
                                int n_nodes_t, int n_out, int n_steps, double2* g_all,
                                hipStream_t st);
// ---- wide-basis path (D = 1, K <= kWideK; wide.hip) ----
// One-electron soft-Coulomb matrix of every item, written whole.
hipError_t launch_potential_wide(const Items& it, const Potential& pot, double* V, int K_max,
                                 hipStream_t st);
// S2 = Ar + Ap over n entries.
hipError_t launch_add_wide(int64_t n, const double* Ar, const double* Ap, double* S2,
                           hipStream_t st);
// Projection of the Cauchy data; scr: scratch of sum K^2 doubles.
hipError_t launch_project_wide(const Items& it, const double* A, double init_alpha,
                               const double* center, double* scr, double2* c0, int* flags,
                               hipStream_t st);
// Anchor inverses (M_c at field Eanchor[c])^{-1} of every item and chunk,
// K x K row-major at X + c cstride + the item's K^2 offset.
hipError_t launch_invert_wide(const Items& it, int n_chunks, const double* Ar, const double* Hr,
                              const double* Q, const double* Eanchor, double tau, double2* X,
                              int64_t cstride, int* flags, hipStream_t st);
// out = scale L R + add per item and chunk (layout as above; R = Rc complex
// and chunk-strided when not null, else Rr real; add may be null or L); out
// must not alias L or R.  toff: prefix sums of ceil(K/64)^2 over items,
// n_tiles its last entry.
hipError_t launch_gemm_wide(const Items& it, const int64_t* toff, int64_t n_tiles, int n_chunks,
                            const double2* L, const double2* Rc, const double* Rr,
                            double2 scale, const double2* add, int64_t cstride, double2* out,
                            hipStream_t st);
// R = I - M_c X per item and chunk (M_c at field Eanchor[c]; layout as
// above), exact products and double-double sums; R must not alias X.
hipError_t launch_residual_wide(const Items& it, const int64_t* toff, int64_t n_tiles,
                                int n_chunks, const double* Ar, const double* Hr, const double* Q,
                                const double* Eanchor, double tau, const double2* X,
                                int64_t cstride, double2* R, hipStream_t st);
// Packed upper 8 x 8 tiles (the inverses' layout, zero padding) of full
// symmetric matrices: the real S2 of every item (src at off2, dst at offp),
// and the complex series terms (c, j) < (n_chunks, terms) at src + c sc +
// j sj (+ off2) to dst + c dc + j dj (+ offp).
hipError_t launch_pack_wide(const Items& it, const double* src, double* dst, hipStream_t st);
hipError_t launch_pack_wide(const Items& it, int n_chunks, int terms, const double2* src,
                            int64_t sc, int64_t sj, double2* dst, int64_t dc, int64_t dj,
                            hipStream_t st);
// Whole-window recurrence of one iterate with the series applied per step,
// from packed matrices: S2p (real), the term P_k of chunk c at Pp + c cstride
// + k tstride, item s using terms_item[s] terms (device, each in
// 1..kWideTerms and at most the terms packed); order: the items by
// decreasing K (the launch order of the blocks).
hipError_t launch_cn_recur_wide(const Items& it, const int32_t* order, int n_steps,
                                const double* S2p, const double* Ar, const double* Hr,
                                const double* Q, const double* Efield, const double* Eanchor,
                                double tau, const double2* Pp, const int32_t* terms_item,
                                int64_t tstride, int64_t cstride, const double2* c0,
                                double2* hist, const double2* F, int* flags, hipStream_t st);
// Robin data of the whole window from src into dst; with prev, one residual
// partial per (item, step tile) at part[item * tx_wide_tiles(n_steps, tile) +
// tile index].  tile: steps per block, 8, 16 or 32.
int tx_wide_tiles(int n_steps, int tile);
hipError_t launch_tx_wide(const Items& it, const Pairs& pr, const TEnt& te, int n_steps,
                          const double2* src, double2* dst, const double2* prev, double* part,
                          double dt, int tile, hipStream_t st);

hipError_t launch_last_step(const Items& it, int n_steps, const double2* hist, double2* c0,
                            hipStream_t st);

}  // namespace swr
