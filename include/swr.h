/*
 * swr.h -- C ABI of the MI355X Schwarz Waveform Relaxation (SWR) Galerkin
 * library for the N-body Schrodinger equation (Lorin, arXiv 1710.02401).
 *
 * Conventions (every entry point):
 *   - Returns int32_t: SWR_OK (0) or a negative SWR_E_* code.  Nothing throws
 *     across the ABI.  Out-parameters are written only on SWR_OK.  After an
 *     error, swr_last_error(handle) returns a static-lifetime description.
 *   - "dev" pointers are device (HBM) addresses on the handle's GPU; "host"
 *     pointers are ordinary process memory.  The caller owns every buffer it
 *     passes; the library owns the opaque handle and its host-side tables.
 *   - Device memory: the library never allocates it.  The caller queries
 *     swr_workspace_bytes, allocates one buffer (any allocator) and binds it
 *     with swr_bind_workspace; every device array of the handle lives there.
 *   - Streams: every device operation is enqueued on the hipStream_t passed
 *     as `stream` (typed void* so this header needs no HIP include; NULL is
 *     the default stream).  Calls that return host values (residuals,
 *     energies, run statistics) synchronise that stream before returning.
 *   - Complex numbers are interleaved (re, im) FP64 pairs.  Every floating
 *     point quantity is FP64 except the warm-start network (FP32).  Integers
 *     are int32 unless stated.
 *   - Items: with n_geom geometries of n_sub = prod(L) subdomains each, item
 *     s = g * n_sub + i (i = linear subdomain index, first dimension
 *     fastest, Section 3.4 / Section 5 indexing Omega_{i+Lj}).
 *   - One handle per host thread; calls on one handle are not thread safe.
 */
#ifndef SWR_H
#define SWR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SWR_OK = 0,
  SWR_E_ARG = -1,      /* invalid argument (null pointer, out-of-range value) */
  SWR_E_SIZE = -2,     /* buffer too small / size beyond a kernel's limit      */
  SWR_E_DEVICE = -3,   /* HIP runtime error (launch, copy, no device)          */
  SWR_E_STATE = -4,    /* call out of order (e.g. sweep before assemble)       */
  SWR_E_SINGULAR = -5, /* a matrix singular to working precision: a Gram
                          matrix at swr_create, or a zero pivot met in a
                          device factorisation                               */
  SWR_E_NAN = -6,      /* non-finite value produced on the device              */
  SWR_E_NOCONV = -7,   /* iteration cap reached above the residual target      */
  SWR_E_COND = -8      /* a local Gram matrix is too ill-conditioned for the
                          accuracy of the path (see swr_create and, for
                          local orbital bases, swr_assemble)                 */
};

enum { SWR_TDSE = 0, SWR_TISE = 1 };

/* Schwarz initial guess psi^(0) of a window (Section 4.1: "psi^(k=0) is a
 * given function").  PLAIN: the window's initial state held constant in
 * time; ZERO: no transmission data; GIVEN: Robin data supplied by the caller
 * at the receiving face nodes (used by the learned warm start). */
enum { SWR_WARM_PLAIN = 0, SWR_WARM_ZERO = 1, SWR_WARM_GIVEN = 2 };

/* Problem description, copied by swr_create.  Lengths in atomic units.
 * Geometry (Section 5, opening paragraph): per configuration dimension k the
 * stated box [box_lo, box_hi] is the outer box [a - eps/2, b + eps/2], split
 * into L[k] cores of width (b - a)/L[k]; subdomain i spans
 * [a + i h - eps/2, a + (i+1) h + eps/2].
 * Basis (Section 2, eq. gauss1d; Test 1.a): per dimension n equispaced
 * centres over the subdomain (basis_extend spacings past each end), Gaussian
 * exp(-delta (x - alpha)^2) with delta = 1/(2 sigma^2), sigma = width if
 * width > 0 else width_ratio * spacing. */
typedef struct swr_desc {
  int32_t mode;              /* SWR_TDSE or SWR_TISE                          */
  int32_t n_elec, dim;       /* N electrons in d dimensions; D = N*d <= 4     */
  int32_t n_geom;            /* independent geometries batched together (>=1;
                                imaginary time: 1)                           */
  int32_t L[4];              /* subdomains per configuration dimension        */
  double box_lo[4], box_hi[4], overlap[4];
  const int32_t* nbasis;     /* host: [D], or [n_sub][D] if per_subdomain     */
  int32_t per_subdomain_basis;
  int32_t basis_extend;
  double width, width_ratio;
  int32_t n_nuc;
  const double* nuc_pos;     /* host: [n_geom][n_nuc][dim]                    */
  const double* nuc_charge;  /* host: [n_nuc]                                 */
  double eps_en, eps_ee;     /* soft-Coulomb regularisation (eq. pseudo)      */
  double dt;
  int32_t n_steps;           /* time steps per window                         */
  double mu_re, mu_im;       /* Robin coefficient mu (eq. RTC)                */
  double E0, omega, phase;   /* E(t) = E0 sin(omega t + phase)                */
  int32_t axis;              /* spatial axis of the field, 0 <= axis < dim    */
  double init_alpha;         /* phi_0 = (2a/pi)^(D/4) exp(-a |x - x0|^2)      */
  double init_center[4];
  int32_t face_nodes_band, face_nodes_mid; /* GL nodes per tangential panel   */
  int32_t quad_nodes;        /* GL nodes per potential quadrature panel       */
  int32_t learned_nodes;     /* time nodes M of the learned warm start, 2..64; 0 = 8 */
  int32_t factor_mode;       /* SWR_FACTOR_AUTO, _DIRECT or _WIDE (swr_factor) */
  int32_t unnormalized;      /* TISE only: 1 = imaginary-time steps without the
                                global normalisation, i.e. the heat-type flow
                                d_t phi = -H~ phi (swr_run reports no energy) */
  /* Field shape (SWR_FIELD_SINE: the single component above along `axis` of
   * every electron).  SWR_FIELD_CIRCULAR, the circular pulse of Section 5
   * Test 3: two components
   *   E_1(t) = E0 cos(omega t + phase) exp(-pulse_nu (t - pulse_center)^2),
   *   E_2(t) = E0 sin(omega t + phase) exp(-pulse_nu (t - pulse_center)^2),
   * component c coupling to the sum of the configuration coordinates whose
   * bits (el * dim + a) are set in field_mask[c] (non-empty, disjoint masks
   * within the D coordinates; real time only).  Every M^n then carries
   * E_1(t_n) Q_1 + E_2(t_n) Q_2, so swr_factor inverts every step (the
   * series in one scalar E does not apply) and `axis` is not used. */
  int32_t field_shape;
  double pulse_nu, pulse_center;
  int32_t field_mask[2];
  /* Local basis (SWR_BASIS_GAUSSIAN: tensor products of one-dimensional
   * Gaussians, Section 2).  SWR_BASIS_SLATER, the Slater-like antisymmetric
   * Gaussian basis of Section 2 eq. (LSD), for two electrons in one
   * dimension each on a decomposition symmetric under the exchange of the
   * two coordinates (equal L, box, overlap and Gaussians per interval):
   * with phi_l the Gaussians of the first coordinate's interval and phi_p
   * those of the second's,
   *   v_{l,p}(x1, x2) = (phi_l(x1) phi_p(x2) - phi_l(x2) phi_p(x1)) / sqrt(2),
   * l slowest; n^2 functions off the diagonal of the decomposition, the
   * n(n-1)/2 with l < p on it (the same interval twice).  The initial state
   * is then the antisymmetrised product of two Gaussians,
   *   phi_0 = N (g_c1(x1) g_c2(x2) - g_c2(x1) g_c1(x2)),
   *   g_c(x) = exp(-init_alpha (x - c)^2), c1, c2 = init_center[0], [1],
   * N normalising phi_0 on the whole plane.  Narrow path only (K <= 64;
   * the transmission is formed densely), the sine field.
   * SWR_BASIS_LSD, local Slater determinants of local orbitals (Section 3):
   * the same construction with phi_l, phi_p the interval's local orbitals
   * instead of its Gaussians, lsd_orbitals (M) per interval: M^2 functions
   * off the diagonal, M(M-1)/2 on it.  The orbitals of interval D_i are the
   * M lowest eigenfunctions of
   *   -1/2 d/dx (a(x) d/dx) + V_n(x) + V_inf s(|x - x_c| - x_b),
   *   a(x) = 1 - s(|x - x_c| - x_b),
   * in the interval's Gaussians over the real line (x_c the centre of the
   * interval's box, x_b = lsd_barrier, s the C^2 quintic step from 0 to 1
   * across [-lsd_barrier_width/2, lsd_barrier_width/2], V_inf = lsd_v_inf),
   * S-normalised and signed so that sum_u (u + 1) C[u][l] > 0.  V_n sums the
   * nuclei: a nucleus inside the interval's box contributes its
   * soft-Coulomb term (eps_en) convolved with the mollifier of eq. (Beps),
   *   B(x) = sigma_M / eps (1 - (x/eps)^2)^M on |x| <= eps,
   * eps = lsd_moll_eps, M = lsd_moll_order, sigma_M normalising B; the
   * others their soft-Coulomb term.  Augmented local bases (Section 3.3):
   * lsd_augment = g > 0 adds the interval's g Gaussians nearest each end of
   * its box (the first g, then the last g from the end inwards; g = 1 adds
   * the two centred on the box's ends) to the orbitals as further
   * one-electron functions, so the pairs run over M + 2g functions.
   * SWR_BASIS_LO, local orbitals of one electron in two dimensions
   * (Section 3 with d = 2): the basis of each subdomain (a box with centre
   * x_c and n_0 x n_1 <= 64 tensor Gaussians, at most 8 per dimension) is
   * its lsd_orbitals (M) lowest eigenfunctions of
   *   -1/2 div(a grad) + V_n + V_inf sum_k s(|x_k - x_ck| - x_b),
   *   a = prod_k (1 - s(|x_k - x_ck| - x_b)),
   * in the box's Gaussians over the plane (s, x_b, V_inf as above), with
   * V_n = sum_A -Z_A G(|x - R_A|) for every nucleus, G the bare Coulomb
   * kernel 1/|x| convolved with B(y) = (M' + 1) / (pi eps^2)
   * (1 - |y|^2 / eps^2)^M' on |y| <= eps (eps = lsd_moll_eps, M' =
   * lsd_moll_order in 2..8), S-normalised and signed so that
   * sum_u (u + 1) C[u][l] > 0; every matrix is C^T (Gaussian matrix) C.
   * One geometry, the sine field, the narrow path (dense transmission);
   * lsd_augment must be 0.  The SWR Hamiltonian keeps its soft-Coulomb
   * terms (eps_en). */
  int32_t basis_kind;
  /* Local orbitals (SWR_BASIS_LSD only; 2 <= M <= Gaussians per interval,
   * M <= 8; 0 <= lsd_augment and M + 2 lsd_augment at most 8 and at most
   * the Gaussians per interval). */
  int32_t lsd_orbitals;
  double lsd_barrier, lsd_barrier_width, lsd_v_inf, lsd_moll_eps;
  int32_t lsd_moll_order;
  int32_t lsd_augment;
} swr_desc;

enum { SWR_FIELD_SINE = 0, SWR_FIELD_CIRCULAR = 1 };
enum { SWR_BASIS_GAUSSIAN = 0, SWR_BASIS_SLATER = 1, SWR_BASIS_LSD = 2, SWR_BASIS_LO = 3 };

typedef struct swr_handle_s* swr_handle;

/* Sizes of a created handle (host struct, filled by swr_query). */
typedef struct swr_info {
  int32_t D, n_sub, n_items, K_max;
  int64_t sum_K, sum_K2;     /* total coefficients / matrix entries           */
  int64_t n_face_nodes;      /* receiving face nodes over all items           */
  int64_t n_pairs;           /* (item, neighbour) transfer pairs              */
  int64_t sum_KK_pairs;      /* entries of all transfer operators             */
  int32_t n_steps;
  int32_t depth;             /* Schwarz iterates swr_run keeps in flight      */
  uint64_t workspace_bytes;
  int32_t learned_nodes;     /* M, time nodes of the learned warm start       */
  int32_t factor_terms;      /* series terms of the last swr_factor minus one;
                                -1: direct inversion per step (or none yet)  */
  int32_t tx_tile;           /* steps per block of the transmission in use:
                                16 or 32 (narrow, factored), 8, 16 or 32
                                (wide); 0: dense transmission / block path   */
  int32_t depth_run;         /* depth swr_run uses for opts.depth = 0
                                (swr_info.depth until swr_autotune)          */
  int32_t wide;              /* 1: the wide-basis path (see swr_factor)       */
  int32_t block;             /* 1: the block path (see swr_factor)            */
  int32_t wide_order;        /* wide path: the recurrence's item order, 0
                                largest K first, 1 item order                */
  int32_t tuned;             /* 1: the schedule was taken from the tuning
                                table at swr_assemble (see swr_autotune)     */
  int32_t rec_series;        /* 1: the last swr_factor's series is evaluated
                                in each recurrence step (no per-step inverses
                                are formed; see swr_factor)                  */
} swr_info;

/* ---- lifetime ------------------------------------------------------------*/

/* Build the decomposition, bases, face quadrature nodes, covering sets O(y)
 * and neighbour lists on the host (Section 4.1 SWR setting; Section 5
 * decomposition).  Validates the description: SWR_E_ARG for inconsistent
 * fields, SWR_E_SIZE if a basis exceeds the kernels' limits: K <= 64 per
 * subdomain, or K <= 256 for one electron in one dimension in real time
 * (the wide-basis path, see swr_factor), or the block path's limits
 * (tensor bases in two or four dimensions up to K = 1536).  SWR_E_SINGULAR
 * if some subdomain's Gram matrix A is singular to working precision (its
 * Cholesky factorisation fails, or its condition exceeds 1e14: e.g. two
 * coinciding or nearly constant Gaussians), on every path.  SWR_E_COND if
 * it has a condition number above 1e6 on the narrow and wide paths: their
 * recurrence (swr_sweep) reuses the previous right-hand side as M^n c^n,
 * which feeds the stored inverses' residual (about cond(M) eps) into every
 * later step, and such bases would end measurably away from the LU-solved
 * answer while reporting success (the block path solves in orthonormalised
 * coordinates and is not limited this way).  *out receives a new handle. */
int32_t swr_create(const swr_desc* desc, swr_handle* out);
void swr_destroy(swr_handle h);
const char* swr_last_error(swr_handle h);
int32_t swr_query(swr_handle h, swr_info* info);

/* Bytes of device workspace the handle needs (256-byte aligned start). */
int32_t swr_workspace_bytes(swr_handle h, uint64_t* bytes);
/* Bind caller-owned device memory of at least swr_workspace_bytes bytes.
 * SWR_E_SIZE if too small, SWR_E_ARG if null or misaligned. */
int32_t swr_bind_workspace(swr_handle h, void* dev, uint64_t bytes);

/* ---- assembly (Section 4.1 local ODE systems, eq. Q; once per geometry) --*/

/* Upload the host tables and assemble, for every item, the Gram matrix A,
 * kinetic matrix Kin = 1/2 <grad v, grad v>, soft-Coulomb matrix V
 * (Gauss-Legendre quadrature), dipole matrix Q = sum_m <x_m v, v>, boundary
 * mass B, partition-of-unity mass W, the Robin transfer operators and the
 * face Gram matrices used by the residual.  Requires a bound workspace.
 * Synchronises the stream.  In the local Slater determinant and local
 * orbital bases (not tensor bases, their orbitals computed here) the
 * condition limits of swr_create apply to the assembled Gram matrices instead:
 * SWR_E_COND above 1e6, SWR_E_SINGULAR above 1e14 or when one is not
 * positive definite; the handle then stays unassembled. */
int32_t swr_assemble(swr_handle h, void* stream);

/* Local Cauchy data (Section 4.4 step 1; Test 1.a): c0_dev == NULL projects
 * the Gaussian phi_0 of the description (solves A c = <phi_0, v>), else
 * copies sum_K complex coefficients from c0_dev.  In TISE mode the result is
 * divided by its global partition-of-unity norm. */
int32_t swr_set_initial(swr_handle h, const void* c0_dev, void* stream);

/* Schwarz initial guess of the current window (see SWR_WARM_*).  For GIVEN,
 * g_dev holds complex Robin data g(y, t_n) on every receiving face node:
 * layout [n_steps+1][n_face_nodes] (time-major).  Resets the iteration count
 * and the residual reference to the window's initial state. */
int32_t swr_warm_start(swr_handle h, int32_t mode, const void* g_dev, void* stream);

/* ---- the SWR iteration (Section 4.1 eq. S1; Section 4.4) ------------------*/

/* Factor every Crank-Nicolson matrix of the window,
 * M^n = A + i dt/2 (Kin + V + mu/2 B + E(t_n) Q), n = 1..n_steps
 * (independent of the Schwarz iterate), starting at time t0: the library
 * keeps the inverses (complex symmetric, packed upper 8 x 8 tiles).  TISE:
 * the implicit Euler matrix A + dt (Kin + V + mu/2 B) once per item.
 * The matrices differ only in the scalar E(t_n): on each chunk of 128
 * consecutive steps, M^n = M_a + d_n C with C = i dt/2 Q, M_a the matrix at
 * the midpoint E_a of the chunk's field range and d_n = E(t_n) - E_a.
 * SWR_FACTOR_AUTO inverts one M_a per chunk and sums
 * (M^n)^{-1} = sum_k (-d_n)^k (M_a^{-1} C)^k M_a^{-1}, k = 0..K: when
 * Im mu <= 0 the Hermitian part of A^{-1/2} M_a A^{-1/2} is at least the
 * identity, so in the A-norm |d_n M_a^{-1} C| <= rho = dt/2 max|d_n| X with
 * X = max over items of sum_m max |x_m| along the field axis on the item's
 * box, and the tail after K is at most rho^{K+1}/(1-rho); K is the least
 * with that bound <= 2^-53 (reported in swr_info.factor_terms).  With
 * K <= 3 the inverses are not formed: the recurrence keeps each chunk's
 * terms (M_a^{-1} C)^k M_a^{-1} and evaluates the sum in every step, entry
 * by entry in the same order of operations as the formed inverses, so the
 * result is the same (swr_info.rec_series); with K = 4..7 the inverses of
 * every step are formed from the sum.  With Im mu > 0, K > 7, or
 * SWR_FACTOR_DIRECT, every M^n is inverted.
 * Wide-basis path (one electron in one dimension, real time; taken when some
 * K > 64, or asked for with SWR_FACTOR_WIDE): the inverses of the steps are
 * never formed.  Per chunk the library keeps M_a^{-1} (Gauss-Jordan, then
 * one correction X + X (I - M_a X) with the residual in compensated
 * arithmetic) and the terms (M_a^{-1} C)^k M_a^{-1}, packed symmetric, and
 * swr_sweep applies the sum to each step's right-hand side, each item with
 * the terms its own box needs (the bound above with the item's X); the
 * bound must hold with K <= 5, else SWR_E_SIZE (as for Im mu > 0 or
 * SWR_FACTOR_DIRECT, which the wide path refuses at creation).
 * A circular field (SWR_FIELD_CIRCULAR) has two scalars per step: every M^n
 * is inverted. */
enum { SWR_FACTOR_AUTO = 0, SWR_FACTOR_DIRECT = 1, SWR_FACTOR_WIDE = 2, SWR_FACTOR_BLOCK = 3 };
int32_t swr_factor(swr_handle h, double t0, void* stream);

/* One Schwarz iteration of local solves for every item (Section 4.4 step 2):
 * TDSE Crank-Nicolson
 *   M^{n+1} c^{n+1} = (A - i dt/2 (H~ + E_n Q)) c^n + (i dt/4)(f^n + f^{n+1}),
 * TISE implicit Euler with global normalisation (eq. SIT),
 * using the current Robin data f.  Requires swr_factor for the window.
 * Accuracy: M^n c^n is taken from the previous step's right-hand side, so
 * the stored inverses' residual (about cond(M) eps) enters every later step:
 * the error per step is about cond(M)^2 eps.  Bases whose Gram matrices are
 * nearly singular (condition above 1e6) are refused by swr_create. */
int32_t swr_sweep(swr_handle h, void* stream);

/* Transmission (Section 4.1, averaged Robin TC in multi-overlap zones, eq.
 * RTC) from the iterate just computed, and the residual Res(k) of eq.
 * (residueRT) between it and the previous iterate.  Writes Res(k) to
 * *residual_host (synchronises the stream). */
int32_t swr_transmit(swr_handle h, double* residual_host, void* stream);

/* Whole window: factor, then sweep + transmit until Res(k) <= tol with
 * k >= 2, or k == k_max.  iters/res receive up to 64 entries.  tol <= 0
 * runs exactly k_max iterations; with tol > 0, reaching k_max above tol
 * returns SWR_E_NOCONV, with *stats filled as on success (the state is the
 * last iterate's, as after a success).
 * Growth guard (GIVEN warm start only, whose Robin data came from outside
 * the method, e.g. the learned predictor): growth_guard consecutive
 * increases of Res(k) stop the run, and the window is run again from the
 * PLAIN warm start, with the same options; stats then describe that run and
 * fallback = 1.  The pipelined and one-at-a-time runs check as the
 * residuals arrive; a graph-replayed window (residuals read after it) is
 * checked afterwards.
 * TDSE with depth P > 1: the window is cut into P chunks of steps and
 * iterate k works on chunk c while iterate k+1 works on chunk c-1 (each
 * chunk of iterate k+1 needs only chunk c of iterate k and its own chunk
 * c-1), so P iterates of every item run at once.  Every iterate is computed
 * with the same arithmetic as at depth 1 (identical results); up to P-1
 * iterates past the stopping one are started and discarded.  depth 0 takes
 * swr_info.depth (sized at creation so that P x n_items fills the GPU,
 * P <= 16); 1 runs one iterate at a time; larger values are capped at
 * swr_info.depth.  TISE pipelines the same way, with one launch per step
 * (its global normalisation couples every item at every step) advancing
 * every iterate in flight; each iterate keeps its own normalisation
 * factors, and its residual is taken once it is complete.  Results agree
 * with depth 1 to rounding (the residual is summed in another order).
 * The HIP graph (opts.graph) is for TDSE only. */
typedef struct swr_run_opts {
  int32_t k_max;
  double tol;
  double t0;
  int32_t warm;              /* SWR_WARM_*                                    */
  const void* g_dev;         /* Robin data for SWR_WARM_GIVEN                 */
  int32_t depth;             /* 0: swr_info.depth; 1: one iterate at a time   */
  int32_t timing;            /* 1: time every kernel launch with HIP events    */
  int32_t graph;             /* 1: with tol < 0 (exactly k_max iterations),
                                depth > 1 and no timing, the window's launches
                                are captured once into a HIP graph (per k_max
                                and depth) and replayed, in real and in
                                imaginary time; the residuals are read after
                                the window                                   */
  int32_t growth_guard;      /* GIVEN warm start: consecutive increases of
                                Res(k) that trigger the PLAIN fallback
                                (0: 2; negative: never)                      */
} swr_run_opts;
/* With timing, ms_* hold the summed durations (HIP events recorded on the
 * run's stream around each launch) and n_* the launch counts of the
 * factorisation, Robin data (transmission), recurrence and residual kernels;
 * otherwise they are zero. */
typedef struct swr_run_stats {
  int32_t iters;
  int32_t converged;
  double res[64];
  double energy;             /* TISE: (1/nu - 1)/dt at the last step          */
  double ms_factor, ms_transmit, ms_recur, ms_residual;
  int32_t n_factor, n_transmit, n_recur, n_residual;
  int32_t fallback;          /* 1: the GIVEN warm start was abandoned for the
                                PLAIN one by the growth guard                */
} swr_run_stats;
int32_t swr_run(swr_handle h, const swr_run_opts* opts, swr_run_stats* stats, void* stream);

/* ---- schedule autotuning ---------------------------------------------------*/

/* Measures, on this problem and GPU, every schedule: on the narrow path
 * every pipeline depth 1..swr_info.depth (TDSE; 1 for TISE) and every
 * transmission tile that fits (16 or 32 steps per block); on the wide path
 * every transmission tile (8, 16 or 32 steps per block) and both
 * recurrence orders (largest K first, item order).  Each is timed as a
 * whole window of k_iters Schwarz iterations (swr_run with tol < 0 from the
 * current initial coefficients, field origin t0, plain warm start; one
 * untimed window first) with HIP events on the stream, and the fastest is
 * kept: later swr_run calls with depth 0 use its depth, and every
 * transmission and sweep its tile and order.  The choice only reorders the
 * same arithmetic (results are unchanged; residuals to rounding).  The
 * choice is also entered in the library's tuning table under (GPU
 * architecture, path, dimensions, items, steps, counts of items per 64-wide
 * band of basis sizes); swr_assemble of a later handle with the same key
 * takes the schedule from the table without measuring (swr_info.tuned).
 * With the environment variable SWR_TUNING_FILE naming a file, the table is
 * read from it on first use and written back after each swr_autotune (one
 * line per key: depth, tile, order, ms, a tab, the key).  The iteration
 * state is left as after the last trial window.  Synchronises the stream. */
typedef struct swr_tuning {
  int32_t depth;             /* iterates in flight chosen                     */
  int32_t tx_tile;           /* transmission tile chosen (0: dense)           */
  double ms_per_window;      /* measured for the choice                       */
  int32_t candidates;        /* schedules measured                            */
  int32_t order;             /* wide path: recurrence order chosen            */
} swr_tuning;
int32_t swr_autotune(swr_handle h, int32_t k_iters, double t0, swr_tuning* out, void* stream);

/* Sets the schedule swr_autotune would choose, without measuring: depth in
 * 1..swr_info.depth (1 for TISE), the transmission tile (narrow factored
 * path: 16, or 32 where its LDS fits; wide path: 8, 16 or 32; otherwise
 * the tile in use) and the recurrence order (wide path: 0
 * largest K first, 1 item order; otherwise 0).  SWR_E_ARG for any other
 * value, SWR_E_STATE before swr_assemble.  Like swr_autotune it only
 * reorders the same arithmetic; the tuning table is not changed. */
int32_t swr_set_schedule(swr_handle h, int32_t depth, int32_t tx_tile, int32_t order, void* stream);

/* ---- outputs and inspection ------------------------------------------------*/

/* Coefficient history of the current iterate: complex [item blocks], item s
 * occupying (n_steps+1) * K_s entries time-major, items in order. */
int32_t swr_get_history(swr_handle h, void* dst_dev, uint64_t bytes, void* stream);
/* Robin data vectors f for the next sweep: same layout as the history. */
int32_t swr_get_forcing(swr_handle h, void* dst_dev, uint64_t bytes, void* stream);
/* Initial coefficients (complex, sum_K). */
int32_t swr_get_initial(swr_handle h, void* dst_dev, uint64_t bytes, void* stream);
/* Assembled real matrices, which = 0 A, 1 Kin, 2 V, 3 Q, 4 B, 5 W, 6 face
 * Gram G, 7 Q2 (the second component's dipole, circular field only, else
 * SWR_E_ARG); item s occupies K_s*K_s row-major entries, items in order. */
int32_t swr_get_matrix(swr_handle h, int32_t which, void* dst_dev, uint64_t bytes, void* stream);
/* Per-item sizes: host int32 [n_items][2 + 2*4]: K, n_face_nodes, then the
 * multi-index and the per-dimension basis sizes (padded with 0). */
int32_t swr_get_items(swr_handle h, int32_t* dst_host, uint64_t n);
/* Series terms each item applies per step after the last swr_factor (host
 * int32 [n_items]): swr_info.factor_terms + 1 for every item on the narrow
 * path (0 when every step was inverted), the item's own count on the
 * wide-basis path.  SWR_E_STATE before the first swr_factor. */
int32_t swr_get_terms(swr_handle h, int32_t* dst_host, uint64_t n);
/* Subdomain boxes, host double [n_items][4][2] (lo, hi per dimension,
 * computed with the formula order of the geometry, no contraction). */
int32_t swr_get_boxes(swr_handle h, double* dst_host, uint64_t n);
/* Covering-set index map: host int32 [n_face_nodes][16]; per receiving node
 * (item, face k=0..D-1 side 0/1, node) record [count, j_0..j_14] with the
 * subdomain linear indices (within the geometry) of O(y) in increasing
 * order, -1 padded; count = -1 on faces lying on the global boundary. */
int32_t swr_get_index_maps(swr_handle h, int32_t* dst_host, uint64_t n);
/* Receiving face nodes: host double [n_face_nodes][4] coordinates and
 * [n_face_nodes] tangential quadrature weights. */
int32_t swr_get_face_nodes(swr_handle h, double* coords_host, double* weights_host, uint64_t n);

/* Reconstruction (Section 4.3): psi(x) = mean over the subdomains whose
 * closure holds x of psi_i(x), at time step `step` of the current history,
 * for n_pts points (device double [n_pts][D]) of geometry `geom`; writes
 * complex [n_pts] to out_dev (0 where no subdomain covers x). */
int32_t swr_reconstruct(swr_handle h, int32_t geom, int32_t step, const void* pts_dev,
                        int64_t n_pts, void* out_dev, void* stream);
/* Antisymmetric reconstruction of two electrons (Appendix A, mirrored
 * subdomains; Section 5, a posteriori antisymmetrisation): where electron
 * 2's coordinates come after electron 1's (lexicographic over the space
 * dimensions), the value is minus swr_reconstruct at the point with the two
 * electrons exchanged; elsewhere it is swr_reconstruct's.  The result is
 * antisymmetric under exchange; for an exchange-symmetric state it is the
 * sign change of Section 5.  Same arguments as swr_reconstruct; SWR_E_ARG
 * unless there are two electrons. */
int32_t swr_reconstruct_antisym(swr_handle h, int32_t geom, int32_t step, const void* pts_dev,
                                int64_t n_pts, void* out_dev, void* stream);

/* TISE local generalized eigenproblems H~_i x = lambda A_i x (Section 4.2):
 * eigenvalues ascending, device double [sum_K], and A-orthonormal
 * eigenvectors (columns, largest-magnitude component positive), device
 * double [sum_K2] row-major per item.  Requires a real Robin coefficient. */
int32_t swr_local_eigen(swr_handle h, void* lambda_dev, void* vectors_dev, void* stream);

/* Last TISE normaliser nu of every step of the current iterate, device
 * double [n_steps+1] (nu_0 = 1). */
int32_t swr_get_norms(swr_handle h, void* dst_dev, uint64_t bytes, void* stream);

/* ---- learned warm start (Section 4.1: psi^(0) of a window is free) ------
 * The plain guess holds the window's initial Robin data g0 constant; the
 * learned guess adds a correction predicted at M time nodes (steps
 * n_m = round(n_T (1 - cos(pi m/(M-1)))/2), M = swr_info.learned_nodes) and
 * interpolated to every step with the barycentric Lagrange form.  RMS_i = sqrt(mean |g0|^2) over item i's
 * receiving nodes; the window scale S = max_i RMS_i (1 if g0 vanishes).
 * Network input of item i (n_in entries): (Re, Im) of g0/S node by node,
 * zero padding to n_in - (M + 8), then M + 8 tail entries: 10 E(t0 + t_m)
 * for the M nodes; the item's box centre as (c_k - mid_k)/half_k of the global
 * box for k < D, zero padded to four; RMS_i / S; t0 / (8 T) with T the
 * window length; two zeros.
 * Network output (n_out entries) = (g(t_m) - g0)/S as [m][node][re, im].
 * Items' receiving nodes are contiguous in the canonical node order.
 * The rounded nodes must be distinct (n_steps >= 11 for M = 8, >= 46 for
 * M = 16, >= 195 for M = 32): on shorter windows swr_time_nodes and the
 * three swr_learned_* calls return SWR_E_ARG. */

/* Change E0, omega and phase of the field (either shape; the pulse envelope
 * and the masks are kept) used by later swr_factor. */
int32_t swr_set_field(swr_handle h, double E0, double omega, double phase);
/* Start the next window: initial coefficients := last step of the current
 * iterate, then the plain warm start (as swr_set_initial). */
int32_t swr_advance_window(swr_handle h, void* stream);
/* The M time-node steps (host int32 [M]). */
int32_t swr_time_nodes(swr_handle h, int32_t* steps_host);
/* Robin data g(y, t_n) at every receiving node for n_sel <= 64 steps of the
 * current iterate (device complex [n_sel][n_face_nodes]); 0 on global faces. */
int32_t swr_face_data(swr_handle h, int32_t n_sel, const int32_t* steps_host, void* g_dev,
                      void* stream);
/* Network input (device float [n_items][n_in]) and scale (device double
 * [n_items], every entry S) from g0 (device complex [n_face_nodes]) for the
 * window starting at t0.  SWR_E_SIZE if n_in < 2 * max nodes per item + M + 8. */
int32_t swr_learned_features(swr_handle h, const void* g0_dev, double t0, int32_t n_in,
                             float* x_dev, double* scale_dev, void* stream);
/* Training targets (device float [n_items][n_out]) from the Robin data at
 * the M time nodes (device complex [M][n_face_nodes], node 0 = g0). */
int32_t swr_learned_targets(swr_handle h, const void* g_nodes_dev, const double* scale_dev,
                            int32_t n_out, float* y_dev, void* stream);
/* Robin data of the learned guess at every step (device complex
 * [n_steps+1][n_face_nodes]) from network outputs (device float
 * [n_items][n_out]); feed it to swr_warm_start(SWR_WARM_GIVEN). */
int32_t swr_learned_apply(swr_handle h, const float* y_dev, const double* scale_dev,
                          const void* g0_dev, int32_t n_out, void* g_all_dev, void* stream);

/* Network of the learned warm start: n_layers hidden layers of width
 * n_hidden with exact-erf GELU, linear output; FP32.  Parameters are one
 * flat vector, layer by layer: weight (out x in, row-major), then bias.
 * These calls need no SWR handle; device buffers are caller-owned and the
 * workspace size comes from swr_mlp_workspace_bytes.  Errors: SWR_E_ARG for
 * null pointers or invalid sizes, SWR_E_SIZE for a small workspace. */
typedef struct swr_mlp_desc {
  int32_t n_in, n_hidden, n_layers, n_out;
} swr_mlp_desc;
int32_t swr_mlp_param_count(const swr_mlp_desc* d, int64_t* count);
int32_t swr_mlp_workspace_bytes(const swr_mlp_desc* d, int32_t batch, uint64_t* bytes);
/* y = network(x) for a batch (device float [batch][n_in] -> [batch][n_out]). */
int32_t swr_mlp_forward(const swr_mlp_desc* d, const float* params, const float* x, int32_t batch,
                        float* y, void* ws_dev, uint64_t ws_bytes, void* stream);
/* The same forward pass for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument and no allocation; the activations
 * live in a 64 MiB array of the library, one per GPU, kept until the
 * process ends.  SWR_E_SIZE when the batch's activations need more than
 * that (2 x batch x (n_layers x n_hidden + n_out) floats, each layer's
 * buffers aligned to 256 bytes, plus 4 KiB); the output equals
 * swr_mlp_forward's.  Calls on one GPU share the array: calls that overlap
 * in time on one GPU (several host threads or streams) race and must be
 * serialised by the caller. */
int32_t swr_mlp_forward_noalloc(const swr_mlp_desc* d, const float* params, const float* x,
                                int32_t batch, float* y, void* stream);
/* Mean-squared-error loss against t (written to loss_dev[0]) and its
 * gradient with respect to every parameter (device float [n_params]). */
int32_t swr_mlp_loss_grad(const swr_mlp_desc* d, const float* params, const float* x,
                          const float* t, int32_t batch, float* loss_dev, float* grad,
                          void* ws_dev, uint64_t ws_bytes, void* stream);
/* One Adam step (step >= 1 for the bias corrections) over n parameters. */
int32_t swr_mlp_adam(int64_t n, float* params, const float* grad, float* m, float* v,
                     int32_t step, float lr, float b1, float b2, float eps, void* stream);

/* Pending device error flags (NaN / zero pivot) since the last call:
 * synchronises the stream, returns SWR_E_NAN / SWR_E_SINGULAR or SWR_OK,
 * and clears them. */
int32_t swr_status_sync(swr_handle h, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SWR_H */
