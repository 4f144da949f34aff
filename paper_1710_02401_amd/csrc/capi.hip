// C ABI of the SWR library: handle lifetime, caller-owned workspace, and the
// stream-ordered sequence assemble -> set_initial -> warm_start -> factor ->
// (sweep -> transmit)*.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/swr.h"
#include "geometry.h"
#include "block.h"
#include "slater.h"
#include "kernels.h"

using swr::Geometry;

namespace {

thread_local std::string g_create_error;

constexpr double kFieldScale = 10.0;  // field feature = 10 E(t)

// time nodes of the learned warm start: M Chebyshev-Lobatto positions
// rounded to the time grid
std::vector<int> time_nodes(int n_T, int M) {
  std::vector<int> n(M);
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < M; ++m)
    n[m] = (int)std::lround(n_T * (1.0 - std::cos(pi * m / (M - 1))) / 2.0);
  return n;
}

// the interpolation needs distinct nodes (n_T >= 11 for M = 8)
bool distinct_time_nodes(int n_T, int M) {
  const std::vector<int> n = time_nodes(n_T, M);
  for (int m = 1; m < M; ++m)
    if (n[m] <= n[m - 1]) return false;
  return true;
}

constexpr int kMaxDepth = 16;   // iterates in flight at most (one job each per launch)
constexpr int kMaxSlots = kMaxDepth + 2;  // + the previous iterate, + one for the residual lag
static_assert(kMaxDepth <= swr::kMaxJobs, "one job per iterate in flight");
constexpr int kResEvents = 8;   // residual read-backs in flight
constexpr int kGpuCUs = 256;    // MI355X compute units
// recurrence blocks per compute unit the depth aims at (its 512-thread block
// needs more than 128 registers per lane, so a second one is not resident)
constexpr int kRecPerCU = 1;
// imaginary-time step blocks resident per CU (256 threads, < 128 registers)
constexpr int kIePerCU = 4;
// series inverses of the window (swr_factor): at most this many terms
constexpr int kSeriesMaxTerms = 8;
// K^2 slots per chunk of the wide path's series: G (or the refinement
// residual), the unrefined anchor inverse, then the terms P_0, P_1, ...
constexpr int kWideSlots = swr::kWideTerms + 2;

// Largest condition number of a subdomain's Gram matrix A that the stored-
// inverse recurrence serves: it takes M^n c^n from the previous step's
// right-hand side, so the explicit inverses' residual (about cond eps)
// enters every later step.  Validated to agree with the oracle to 1e-10 up
// to 2e5 (the paper's Test 2.b boxes); the Test 3 boxes with delta = 0.5
// (condition 1.6e8) end 3 % away.
constexpr double kCondLimit = 1e6;
// Above this a Gram matrix is taken as singular to working precision.
constexpr double kSingularLimit = 1e14;

// Condition number (2-norm) of a symmetric positive definite n x n matrix
// S (row-major): Cholesky, then power iteration for the largest eigenvalue
// and inverse iteration for the smallest (an estimate within a small
// factor, enough for a limit check); infinity when S is not numerically
// positive definite.
double spd_condition(const double* S, int n) {
  if (n <= 1) return 1.0;
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double v = S[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) v -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(v > 0.0)) return INFINITY;
    const double ljj = std::sqrt(v);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double u = S[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) u -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = u / ljj;
    }
  }
  auto normalise = [n](std::vector<double>& x) {
    double s = 0.0;
    for (double v : x) s += v * v;
    s = std::sqrt(s);
    for (double& v : x) v /= s;
    return s;
  };
  std::vector<double> x(n), y(n);
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.25 * (i % 3);
  normalise(x);
  double lmax = 0.0;
  for (int it = 0; it < 30; ++it) {
    for (int i = 0; i < n; ++i) {
      double v = 0.0;
      for (int j = 0; j < n; ++j) v += S[(size_t)i * n + j] * x[j];
      y[i] = v;
    }
    lmax = normalise(y);
    x.swap(y);
  }
  for (int i = 0; i < n; ++i) x[i] = 1.0 - 0.5 * (i % 2);
  normalise(x);
  double inv = 0.0;
  for (int it = 0; it < 30; ++it) {
    for (int i = 0; i < n; ++i) {  // L z = x
      double v = x[i];
      for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * y[k];
      y[i] = v / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {  // L^T w = z
      double v = y[i];
      for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * y[k];
      y[i] = v / L[(size_t)i * n + i];
    }
    inv = normalise(y);
    x.swap(y);
  }
  return lmax * inv;
}

// The same for the one-dimensional Gram matrix
// S_ab = int_lo^hi exp(-d (x - a_a)^2) exp(-d (x - a_b)^2) dx.
double gram_condition_1d(const double* al, int n, double d, double lo, double hi) {
  if (n <= 1) return 1.0;
  std::vector<double> S((size_t)n * n);
  const double pi = 3.14159265358979323846;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const double p = 2.0 * d, P = 0.5 * (al[a] + al[b]);
      const double E = std::exp(-0.5 * d * (al[a] - al[b]) * (al[a] - al[b]));
      const double r = std::sqrt(p);
      S[(size_t)a * n + b] = E * 0.5 * std::sqrt(pi / p) * (std::erf(r * (hi - P)) - std::erf(r * (lo - P)));
    }
  return spd_condition(S.data(), n);
}

// Largest Gram condition over the subdomains of one geometry (the boxes and
// bases are shared by every geometry): the product of the per-dimension
// conditions, exact for tensor bases; *worst_1d receives the largest
// one-dimensional factor's.
double max_gram_condition(const Geometry& g, double* worst_1d) {
  double worst = 1.0, w1 = 1.0;
  for (int s = 0; s < g.n_sub; ++s) {
    double c = 1.0;
    for (int k = 0; k < g.D; ++k) {
      const size_t q = (size_t)s * 4 + k;
      const double c1 = gram_condition_1d(&g.alpha[g.aoff[q]], g.nb[q], g.delta[q], g.lo[q], g.hi[q]);
      c *= c1;
      w1 = std::isnan(c1) ? c1 : std::max(w1, c1);
    }
    worst = std::max(worst, c);
  }
  *worst_1d = w1;
  return worst;
}

const char* const kShortWindow =
    "the learned warm start's time nodes are not distinct: the window has too few steps";

struct Buf {
  size_t off = 0, bytes = 0;
};

struct Layout {
  size_t total = 0;
  Buf add(size_t bytes) {
    Buf b;
    total = (total + 255) & ~size_t(255);
    b.off = total;
    b.bytes = bytes;
    total += bytes;
    return b;
  }
};

}  // namespace

// Growth guard of a GIVEN warm start: counts consecutive increases of the
// residuals as they arrive; hit once `limit` of them are seen (limit 0: off).
struct Growth {
  int limit = 0;
  int run = 0;
  double last = -1.0;
  bool hit = false;
  bool step(double r) {
    run = (last >= 0.0 && r > last) ? run + 1 : 0;
    last = r;
    hit = hit || (limit > 0 && run >= limit);
    return hit;
  }
};

struct swr_handle_s {
  Geometry g;
  std::string err;
  Growth growth;  // the current swr_run's growth guard
  int wide_tile = 16;     // wide path: steps per transmission block (8, 16, 32)
  int wide_order = 0;     // wide path: recurrence order, 0 largest K first, 1 item order
  bool tuned_cached = false;  // a schedule came from the tuning table
  int n_mats = 0;
  int64_t sum_K = 0, sum_K2 = 0, n_T = 0, s1_total = 0, scratch_total = 0;
  int n_res_tiles = 0;
  std::vector<int64_t> s1off, scratch_off;
  std::vector<double> E_host;   // field table, kept alive for the async upload
  std::vector<double> E2_host;  // the second component's (circular field)
  std::vector<double> lag_host; // Lagrange rows of the learned warm start

  // workspace
  char* ws = nullptr;
  uint64_t ws_bytes = 0;
  Layout lay;
  Buf bOffP;
  std::vector<int64_t> offp;  // prefix sums of the packed symmetric sizes
  Buf bK, bOff1, bOff2, bIdx, bNb, bL, bLo, bHi, bEps, bDelta, bAoff, bAlpha, bQoff, bQn, bQx, bQw;
  // local orbitals (SWR_BASIS_LSD): coefficients per interval, the items'
  // one-dimensional orbital integrals, the orbital problem's rules
  Buf bLoC, bLoTab, bLoQx, bLoQw, bLoQoff, bLoMx, bLoMw;
  // local orbitals in two dimensions: the Gaussian matrices (offsets
  // lo_off2g, sizes lo_kg), the angle rule, node Gaussians, 1-D integrals
  // and the nuclear term's first contraction
  Buf bKG, bOff2G, bAG, bKinG, bVG, bQG, bBG, bWG, bLoAng, bLoGt, bLoPP;
  std::vector<int32_t> lo_kg;
  std::vector<int64_t> lo_off2g;
  std::vector<double> lo_ang;
  Buf bNItem, bNFace, bNCount, bNCover, bNX, bNW, bNOff, bLag, bLMax;
  Buf bPI, bPJ, bPOff, bTOff, bPNode, bPNOff;
  Buf bPos, bCharge, bS1Off, bS1, bScrOff, bScr, bCenter;
  Buf bA, bKin, bV, bQ, bB, bW, bG, bAr, bAp, bHr;
  Buf bQ2, bE2;  // second component of a circular field (else unallocated)
  // imaginary time, per history slot: partial norms [n_T + 1][n_items] and
  // normalisation factors [n_T + 1] of the iterate in the slot
  Buf bIePart[kMaxSlots], bNus[kMaxSlots];
  Buf bTePair, bTeFace, bTeT0, bTeT1, bTeOff, bTeBoff, bTeAoff, bTeXoff, bTeBeta, bTeA, bTeX;
  Buf bTeSoff, bTeSidx, bTeV, bTeBlobOff, bTeBlob, bTeSdesc, bTeGramOff, bTeGram, bTeFnode;
  Buf bParts;                        // residual partials of the factored transmission
  std::vector<int64_t> te_gram_off;  // per-item face Gram pieces (doubles, even)
  std::vector<int64_t> te_fnode;     // [n_items][8][2] first node and count per face
  std::vector<int64_t> te_blob_off;  // per-sender blob offsets (complex units)
  // TDSE series inverses, per chunk of kSeriesChunk steps: G then P_0 ..
  // P_{kSeriesMaxTerms-1}, each sum_K2 complex; the chunks' anchor fields
  Buf bSeries, bEanchor, bDser;
  std::vector<double> Ea_host;
  std::vector<double> D_host;  // E_c - E_{n+1} per step n of chunk c (series recurrence)
  // wide-basis path (D = 1, K <= kWideK): S2 = Ar + Ap packed, the series
  // terms packed (per chunk kWideTerms slots of the packed size), a K^2
  // scratch (projection, S2 before packing), the items by decreasing K,
  // prefix sums of the 64 x 64 tiles of the products
  bool wide = false;
  Buf bS2P, bSeriesP, bScrW, bOrder, bTileOff;
  std::vector<int32_t> order;          // wide path: items by decreasing K
  std::vector<int32_t> order_natural;  // wide path: items in their own order
  std::vector<int64_t> tile_off;
  Buf bT, bC0, bH[kMaxSlots], bF[kMaxSlots], bRc[kMaxSlots], bMinv, bE, bResPart, bResOut, bResv,
      bFlags;

  // state
  bool bound = false, assembled = false, initial = false, warm = false, factored = false;
  int cur = 0;      // history slot holding the latest iterate
  int k = 0;        // Schwarz iterations done in this window
  double t0 = 0.0;
  int depth = 1;    // iterates swr_run keeps in flight (TDSE)
  int n_nodes_t = 8;  // time nodes M of the learned warm start
  double dipole_max = 0.0;  // max over items of sum_m max |x_m| along the field axis
  std::vector<double> dipole;        // the same per item
  std::vector<int32_t> terms_item;   // wide path: series terms each item needs
  Buf bTermsW;
  int factor_terms = -1;    // series terms - 1 of the last swr_factor; -1: direct
  // the recurrence evaluates the series in the step (terms <= kRecSeriesMax,
  // narrow path): the per-step inverses are not assembled
  bool rec_series = false;
  swr::RecSeries rec_se() {
    const int64_t cstride = (int64_t)(kSeriesMaxTerms + 1) * sum_K2;
    return swr::RecSeries{ptr<double2>(bSeries) + sum_K2, sum_K2, cstride, ptr<double>(bDser),
                          factor_terms + 1};
  }
  int nbt = 1;      // largest tangential basis size (factored transmission)
  int64_t te_pieces = 0;  // largest LDS bytes of the pieces one item sends
  int te_max_recv = 0;    // largest number of entries one item receives
  int te_max_send = 0;    // largest number of entries one item sends
  int64_t te_gram_max = 0;  // largest LDS bytes of one item's face Gram pieces
  int tx_tt = 0;            // steps per block of the factored transmission (in use)
  int tx_tt_max = 0;        // the largest whose LDS fits (16 or 32)
  int depth_run = 1;        // depth swr_run uses when asked for depth 0 (autotuned)
  int part_stride = 0;      // residual partials per item and iterate slot
  std::vector<int32_t> te_sdesc;  // sender-side entry descriptors
  int n_slots = 2;  // history / Robin data slots: iterate k uses slot k % n_slots

  // block path (tensor bases in two or four dimensions up to K = 1536,
  // orthonormalised per dimension; block.hip)
  bool block = false;
  std::vector<swr::BlkDim> bdim;       // [n_items][4] (host part)
  std::vector<int64_t> pot_off;        // [n_items + 1] potential scratch (doubles)
  std::vector<int64_t> blk_foff;       // [n_items + 1] packed-term offsets (complex)
  std::vector<int32_t> blk_terms;      // [n_items] series terms of the last factor
  std::vector<int64_t> blk_toff;       // [n_items + 1] 64 x 64 tiles
  std::vector<double> blk_Ea;          // anchor field per chunk
  Buf bBd, bBlkPotOff, bBlkVp, bBlkY0, bBlkF0, bBlkF1, bBlkRing, bBlkPart, bBlkRb, bBlkTr,
      bBlkFrag, bBlkTerms, bBlkFoff, bBlkTileOff, bBlkEa, bBlkCp, bBlkRp, bBlkCvec, bBlkRegion;
  int blk_depth = 1;       // iterates in flight at most
  int blk_slots = 2;       // history slots (depth + 1)
  int blk_chunks = 1;      // anchors per window
  int blk_chunk_len = 1;   // steps per anchor
  int blk_pot_batch = 1;   // items per batch of the four-dimensional potential stage
  int64_t blk_stage_item = 0;  // doubles of one item's potential stage
  int blk_qmax = 1, blk_qqmax = 1;
  int blk_fstride = 1;     // face nodes per face (trace scratch stride)
  int64_t blk_pot_total = 0;   // doubles of the potential scratch
  int blk_k = 0;           // Schwarz iterations done in the window
  int blk_cur = 0;         // history slot of iterate blk_k
  int blk_warm = SWR_WARM_PLAIN;
  double blk_last_res = 0.0;

  // host side of the pipelined run's residual read-back
  double* res_pinned = nullptr;
  hipEvent_t ev[kResEvents] = {};
  bool ev_ready = false;

  // optional per-launch timing of swr_run: event pairs around each launch
  bool timing = false;
  std::vector<hipEvent_t> tev;        // pool, grown on demand, reused
  std::vector<int> tkind;             // kind of pair q (events 2q, 2q+1)
  size_t tused = 0;

  // a pipelined window captured as a HIP graph (fixed iteration count), for
  // its iteration count and depth
  hipGraphExec_t gexec = nullptr;
  int g_kmax = 0, g_P = 0;
  hipStream_t cap_stream = nullptr;  // capture only (the caller's may be the null stream)

  ~swr_handle_s() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (res_pinned) (void)hipHostFree(res_pinned);
    if (ev_ready)
      for (auto& e : ev) (void)hipEventDestroy(e);
    for (auto& e : tev) (void)hipEventDestroy(e);
  }

  template <class T>
  T* ptr(const Buf& b) const { return reinterpret_cast<T*>(ws + b.off); }

  swr::Items items() const {
    swr::Items it{};
    it.n_items = g.n_items;
    it.n_sub = g.n_sub;
    it.D = g.D;
    it.n_elec = g.desc.n_elec;
    it.dim = g.desc.dim;
    it.slater =
        g.desc.basis_kind == SWR_BASIS_SLATER || g.desc.basis_kind == SWR_BASIS_LSD ? 1 : 0;
    if (g.desc.basis_kind == SWR_BASIS_LSD) {
      it.lsd = 1;
      it.n_orb = swr::lsd_functions(g.desc);
      it.lo_C = ptr<double>(bLoC);
      it.lo_tab = ptr<double>(bLoTab);
    }
    if (g.desc.basis_kind == SWR_BASIS_LO) {
      it.lo2 = 1;
      it.n_orb = g.desc.lsd_orbitals;
      it.lo_C = ptr<double>(bLoC);
    }
    if (g.desc.field_shape == SWR_FIELD_CIRCULAR) {
      it.qmask0 = g.desc.field_mask[0];
      it.qmask1 = g.desc.field_mask[1];
      it.Q2 = ptr<double>(bQ2);
      it.E2 = ptr<double>(bE2);
    } else {
      for (int el = 0; el < g.desc.n_elec; ++el) it.qmask0 |= 1 << (el * g.desc.dim + g.desc.axis);
    }
    it.K = ptr<int32_t>(bK);
    it.off1 = ptr<int64_t>(bOff1);
    it.off2 = ptr<int64_t>(bOff2);
    it.offp = ptr<int64_t>(bOffP);
    it.idx = ptr<int32_t>(bIdx);
    it.nb = ptr<int32_t>(bNb);
    it.L = ptr<int32_t>(bL);
    it.lo = ptr<double>(bLo);
    it.hi = ptr<double>(bHi);
    it.eps = ptr<double>(bEps);
    it.delta = ptr<double>(bDelta);
    it.aoff = ptr<int64_t>(bAoff);
    it.alpha = ptr<double>(bAlpha);
    it.qoff = ptr<int64_t>(bQoff);
    it.qn = ptr<int32_t>(bQn);
    it.qx = ptr<double>(bQx);
    it.qw = ptr<double>(bQw);
    return it;
  }
  // local orbitals: the same items over their tensor Gaussians (the
  // assembly of the matrices the orbitals transform)
  swr::Items items_gaussian() const {
    swr::Items it = items();
    it.lo2 = 0;
    it.K = ptr<int32_t>(bKG);
    it.off2 = ptr<int64_t>(bOff2G);
    return it;
  }

  swr::Nodes nodes() const {
    swr::Nodes nd{};
    nd.n = (int64_t)g.nodes.size();
    nd.item = ptr<int32_t>(bNItem);
    nd.face = ptr<int32_t>(bNFace);
    nd.count = ptr<int32_t>(bNCount);
    nd.x = ptr<double>(bNX);
    nd.w = ptr<double>(bNW);
    nd.off = ptr<int64_t>(bNOff);
    return nd;
  }
  swr::Pairs pairs() const {
    swr::Pairs pr{};
    pr.n = (int64_t)g.pair_i.size();
    pr.pi = ptr<int32_t>(bPI);
    pr.pj = ptr<int32_t>(bPJ);
    pr.poff = ptr<int64_t>(bPOff);
    pr.toff = ptr<int64_t>(bTOff);
    pr.node = ptr<int32_t>(bPNode);
    pr.noff = ptr<int64_t>(bPNOff);
    return pr;
  }
  double2* hist(int which) const { return ptr<double2>(bH[which]); }
  double2* hist_of(int k) const { return ptr<double2>(bH[k % n_slots]); }
  double2* F_of(int k) const { return ptr<double2>(bF[k % n_slots]); }
  double* nus_of(int k) const { return ptr<double>(bNus[k % n_slots]); }
  double* iepart_of(int k) const { return ptr<double>(bIePart[k % n_slots]); }
  // right-hand side a chunk of iterate k leaves for the next chunk
  double2* carry_of(int k) const { return ptr<double2>(bRc[k % n_slots]); }
  double* parts_of(int k) const {
    return ptr<double>(bParts) + (size_t)(k % n_slots) * g.n_items * part_stride;
  }
  bool fused_residual() const { return g.te_ok; }
  swr::BlkItems blk_items() const {
    swr::BlkItems b{};
    b.it = items();
    b.bd = ptr<swr::BlkDim>(bBd);
    b.terms = ptr<int32_t>(bBlkTerms);
    b.foff = ptr<int64_t>(bBlkFoff);
    b.fmask = b.it.qmask0;
    b.fstride = blk_fstride;
    b.tau = 0.5 * g.desc.dt;
    b.mu_re = g.desc.mu_re;
    b.mu_im = g.desc.mu_im;
    return b;
  }
  swr::BlkState blk_state() const {
    swr::BlkState S{};
    S.hist = ptr<double2>(bBlkRegion);
    S.hstride = (n_T + 1) * sum_K;
    S.ring = ptr<double2>(bBlkRing);
    S.F1 = ptr<double2>(bBlkF1);
    S.F0 = ptr<double2>(bBlkF0);
    S.y0 = ptr<double2>(bBlkY0);
    S.part = ptr<double>(bBlkPart);
    S.pstride = (int64_t)g.n_items * (n_T + 1);
    S.n_steps = (int)n_T;
    return S;
  }
  swr::TEnt te() const {
    swr::TEnt t{};
    t.n = g.te_ok ? (int64_t)g.te_pair.size() : 0;
    t.pair = ptr<int32_t>(bTePair);
    t.face = ptr<int32_t>(bTeFace);
    t.t0 = ptr<int64_t>(bTeT0);
    t.t1 = ptr<int64_t>(bTeT1);
    t.off = ptr<int64_t>(bTeOff);
    t.boff = ptr<int64_t>(bTeBoff);
    t.aoff = ptr<int64_t>(bTeAoff);
    t.xoff = ptr<int64_t>(bTeXoff);
    t.soff = ptr<int64_t>(bTeSoff);
    t.sidx = ptr<int32_t>(bTeSidx);
    t.v = ptr<double2>(bTeV);
    t.blob_off = ptr<int64_t>(bTeBlobOff);
    t.blob = ptr<double2>(bTeBlob);
    t.sdesc = ptr<int32_t>(bTeSdesc);
    t.gram_off = ptr<int64_t>(bTeGramOff);
    t.gram = ptr<double>(bTeGram);
    t.fnode = ptr<int64_t>(bTeFnode);
    t.beta = ptr<double>(bTeBeta);
    t.a = ptr<double2>(bTeA);
    t.X = ptr<double>(bTeX);
    return t;
  }
};

namespace {

// Residual partials per item for a run of depth at most P: the window
// whole, or in p <= P chunks of ceil(n_T / p) steps (chunk 0 one step more).
int parts_needed(swr_handle h, int P, int tt) {
  const int nT = (int)h->n_T;
  int need = (nT + 1 + tt - 1) / tt;
  for (int p = 2; p <= P; ++p) {
    const int S = (nT + p - 1) / p;
    const int n_chunks = (nT + S - 1) / S;
    need = std::max(need, n_chunks * ((S + 1 + tt - 1) / tt));
  }
  return need;
}


int fail(swr_handle h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

#define HIPCHECK(h, expr)                                                        \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(h, SWR_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
hipError_t upload(swr_handle h, const Buf& b, const std::vector<T>& v, hipStream_t st) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(h->ws + b.off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

void plan_layout(swr_handle h) {
  const Geometry& g = h->g;
  const size_t NI = g.n_items;
  const size_t nn = g.nodes.size();
  const size_t np = g.pair_i.size();
  Layout& L = h->lay;
  L = Layout();
  h->bK = L.add(NI * 4);
  h->bOff1 = L.add((NI + 1) * 8);
  h->bOff2 = L.add((NI + 1) * 8);
  h->bIdx = L.add(NI * 16);
  h->bNb = L.add(NI * 16);
  h->bL = L.add(16);
  h->bLo = L.add(NI * 32);
  h->bHi = L.add(NI * 32);
  h->bEps = L.add(32);
  h->bDelta = L.add(NI * 32);
  h->bAoff = L.add(NI * 32);
  h->bAlpha = L.add(g.alpha.size() * 8);
  h->bQoff = L.add(NI * 32);
  h->bQn = L.add(NI * 16);
  h->bQx = L.add(g.qx.size() * 8);
  h->bQw = L.add(g.qw.size() * 8);
  h->bNItem = L.add(nn * 4);
  h->bNFace = L.add(nn * 4);
  h->bNCount = L.add(nn * 4);
  h->bNCover = L.add(nn * 15 * 4);
  h->bNX = L.add(nn * 32);
  h->bNW = L.add(nn * 8);
  h->bNOff = L.add((NI + 1) * 8);
  h->bPI = L.add(np * 4);
  h->bPJ = L.add(np * 4);
  h->bPOff = L.add((NI + 1) * 8);
  h->bTOff = L.add((np + 1) * 8);
  h->bPNode = L.add(g.pnode.size() * 4);
  h->bPNOff = L.add((np + 1) * 8);
  h->bPos = L.add(std::max<size_t>(1, g.nuc_pos.size()) * 8);
  h->bCharge = L.add(std::max<size_t>(1, g.nuc_charge.size()) * 8);
  h->bS1Off = L.add(NI * 32);
  h->bS1 = L.add(h->s1_total * 8);
  h->bScrOff = L.add(NI * 8);
  h->bScr = L.add(std::max<int64_t>(1, h->scratch_total) * 8);
  h->bCenter = L.add(32);
  if (g.desc.basis_kind == SWR_BASIS_LSD) {
    const int M = swr::lsd_functions(g.desc);
    h->bLoC = L.add((size_t)g.L[0] * g.nb[0] * M * 8);
    h->bLoTab = L.add(NI * 2 * 5 * (size_t)(4 * M * M) * 8);
    h->bLoQx = L.add(g.lo_qx.size() * 8);
    h->bLoQw = L.add(g.lo_qw.size() * 8);
    h->bLoQoff = L.add(g.lo_qoff.size() * 8);
    h->bLoMx = L.add(g.lo_mx.size() * 8);
    h->bLoMw = L.add(g.lo_mw.size() * 8);
  }
  if (g.desc.basis_kind == SWR_BASIS_LO) {
    const int M = g.desc.lsd_orbitals;
    h->lo_kg.assign(NI, 0);
    h->lo_off2g.assign(NI + 1, 0);
    for (size_t s = 0; s < NI; ++s) {
      h->lo_kg[s] = g.nb[s * 4] * g.nb[s * 4 + 1];
      h->lo_off2g[s + 1] = h->lo_off2g[s] + (int64_t)h->lo_kg[s] * h->lo_kg[s];
    }
    const size_t g2 = (size_t)h->lo_off2g[NI] * 8;
    h->bKG = L.add(NI * 4);
    h->bOff2G = L.add((NI + 1) * 8);
    h->bAG = L.add(g2);
    h->bKinG = L.add(g2);
    h->bVG = L.add(g2);
    h->bQG = L.add(g2);
    h->bBG = L.add(g2);
    h->bWG = L.add(g2);
    h->bLoC = L.add(NI * (size_t)swr::kSmallK * M * 8);
    h->bLoQx = L.add(g.lo_qx.size() * 8);
    h->bLoQw = L.add(g.lo_qw.size() * 8);
    h->bLoQoff = L.add(g.lo_qoff.size() * 8);
    h->bLoAng = L.add(2 * g.lo_mx.size() * 16);
    h->bLoGt = L.add(g.lo_qx.size() * 8 * 8);
    h->bLoTab = L.add(NI * 2 * 4 * 64 * 8);
    h->bLoPP = L.add(g.lo_qx.size() * 64 * 8);
    // the angle rule on [0, pi/2]: (sin, cos) of the nodes, then (weight, 0)
    const double qa = 0.25 * 3.14159265358979323846;
    const size_t nm = g.lo_mx.size();
    h->lo_ang.assign(4 * nm, 0.0);
    for (size_t j = 0; j < nm; ++j) {
      const double a = qa * (g.lo_mx[j] + 1.0);
      h->lo_ang[2 * j] = std::sin(a);
      h->lo_ang[2 * j + 1] = std::cos(a);
      h->lo_ang[2 * (nm + j)] = qa * g.lo_mw[j];
    }
  }
  const size_t m2 = h->sum_K2 * 8;
  h->bA = L.add(m2);
  h->bKin = L.add(m2);
  h->bV = L.add(m2);
  h->bQ = L.add(m2);
  if (g.desc.field_shape == SWR_FIELD_CIRCULAR) {
    h->bQ2 = L.add(m2);
    h->bE2 = L.add((h->n_T + 1) * 8);
  }
  h->bB = L.add(m2);
  h->bW = L.add(m2);
  h->bG = L.add(m2);
  h->bAr = L.add(m2);
  h->bAp = L.add(m2);
  h->bHr = L.add(m2);
  // dense transfer operators only where the factored form does not apply
  h->bT = L.add(g.te_ok ? 16 : g.pair_toff.back() * 16);
  const size_t ne = g.te_pair.size();
  h->bTePair = L.add(ne * 4);
  h->bTeFace = L.add(ne * 4);
  h->bTeT0 = L.add(ne * 8);
  h->bTeT1 = L.add(ne * 8);
  h->bTeOff = L.add((NI + 1) * 8);
  h->bTeBoff = L.add(ne * 8);
  h->bTeAoff = L.add(ne * 8);
  h->bTeXoff = L.add(ne * 8);
  h->bTeBeta = L.add(g.te_nb * 8);
  h->bTeA = L.add(g.te_na * 16);
  h->bTeX = L.add(g.te_nx * 8);
  h->bTeSoff = L.add((NI + 1) * 8);
  h->bTeSidx = L.add(ne * 4);
  // tangential traces of every entry at every step (one buffer serves every
  // job of a launch: their step ranges are disjoint)
  h->bTeV = L.add(ne * (size_t)(h->n_T + 1) * h->nbt * 16);
  h->bTeBlobOff = L.add((NI + 1) * 8);
  h->bTeBlob = L.add((h->te_blob_off.empty() ? 1 : h->te_blob_off.back()) * 16);
  h->bTeSdesc = L.add(h->te_sdesc.size() * 4);
  h->bTeGramOff = L.add((NI + 1) * 8);
  h->bTeGram = L.add((h->te_gram_off.empty() ? 1 : h->te_gram_off.back()) * 8);
  h->bTeFnode = L.add(NI * 16 * 8);
  h->bParts = L.add((size_t)h->n_slots * NI * std::max(1, h->part_stride) * 8);
  h->bC0 = L.add(h->sum_K * 16);
  const size_t hist = (size_t)(h->n_T + 1) * h->sum_K * 16;
  for (int q = 0; q < h->n_slots; ++q) {
    h->bH[q] = L.add(hist);
    h->bF[q] = L.add(hist);
    h->bRc[q] = L.add(h->sum_K * 16);
  }
  h->bOffP = L.add((NI + 1) * 8);
  const int n_chunks = (int)((h->n_mats + swr::kSeriesChunk - 1) / swr::kSeriesChunk);
  if (h->wide) {
    // no per-step inverses: per chunk G (or the refinement residual), the
    // anchor inverse before refinement, then P_0 .. P_{kWideTerms-1}
    h->bMinv = L.add(16);
    h->bSeries = L.add((size_t)n_chunks * kWideSlots * h->sum_K2 * 16);
    h->bSeriesP = L.add((size_t)n_chunks * swr::kWideTerms * h->offp.back() * 16);
    h->bS2P = L.add(h->offp.back() * 8);
    h->bScrW = L.add(m2);
    h->bOrder = L.add(NI * 4);
    h->bTileOff = L.add((NI + 1) * 8);
    h->bTermsW = L.add(NI * 4);
  } else {
    h->bMinv = L.add((size_t)h->n_mats * std::max<int64_t>(h->sum_K2, h->offp.back()) * 16);
    if (g.desc.mode == SWR_TDSE)
      h->bSeries = L.add((size_t)n_chunks * (kSeriesMaxTerms + 1) * h->sum_K2 * 16);
  }
  if (g.desc.mode == SWR_TDSE) {
    h->bEanchor = L.add((size_t)n_chunks * 8);
    h->bDser = L.add((size_t)h->n_mats * 8);
  }
  h->bE = L.add((h->n_T + 1) * 8);
  h->bResPart = L.add((size_t)h->n_res_tiles * NI * 8);
  h->bResOut = L.add(8);
  h->bResv = L.add(64 * 8);
  for (int q = 0; q < h->n_slots; ++q) {
    h->bIePart[q] = L.add((size_t)(h->n_T + 1) * NI * 8);
    h->bNus[q] = L.add((h->n_T + 1) * 8);
  }
  h->bFlags = L.add(8);
  h->bLag = L.add((h->n_T + 1) * h->n_nodes_t * 8);
  h->bLMax = L.add(8);
}

// ---------------------------------------------------------------------------
// Tuning table: the schedule swr_autotune chose, per (GPU architecture, path,
// dimensions, electrons, items, steps, items per 64-wide band of basis
// sizes).  Later handles with the same key start from it (swr_assemble).
// SWR_TUNING_FILE, when set, names a file the table is read from once and
// written back to after every swr_autotune.
struct TuneChoice {
  int depth = 1, tile = 16, order = 0;
  double ms = 0.0;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune;
bool g_tune_loaded = false;

std::string tune_key(swr_handle h) {
  int dev = 0;
  hipDeviceProp_t p{};
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
    arch = p.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  const Geometry& g = h->g;
  int bands[5] = {0, 0, 0, 0, 0};
  for (int s = 0; s < g.n_items; ++s) ++bands[std::min(4, (g.K[s] - 1) / 64)];
  std::ostringstream k;
  k << arch << " " << (h->block ? "block" : h->wide ? "wide" : "narrow") << " D" << g.D << " e"
    << g.desc.n_elec << " items" << g.n_items << " steps" << h->n_T << " K64";
  for (int b : bands) k << ":" << b;
  return k.str();
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("SWR_TUNING_FILE");
  if (!path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t tab = line.find('\t');
    if (tab == std::string::npos) continue;
    std::istringstream v(line.substr(0, tab));
    TuneChoice c;
    if (v >> c.depth >> c.tile >> c.order >> c.ms) g_tune[line.substr(tab + 1)] = c;
  }
}

bool tune_lookup(const std::string& key, TuneChoice* c) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load_locked();
  const auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *c = it->second;
  return true;
}

void tune_store(const std::string& key, const TuneChoice& c) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load_locked();
  g_tune[key] = c;
  const char* path = std::getenv("SWR_TUNING_FILE");
  if (!path) return;
  std::ofstream f(path, std::ios::trunc);
  for (const auto& e : g_tune)
    f << e.second.depth << " " << e.second.tile << " " << e.second.order << " " << e.second.ms
      << "\t" << e.first << "\n";
}

int check_flags(swr_handle h, hipStream_t st) {
  int flags = 0;
  HIPCHECK(h, hipMemcpyAsync(&flags, h->ptr<int>(h->bFlags), sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(h, hipStreamSynchronize(st));
  if (flags) {
    HIPCHECK(h, hipMemsetAsync(h->ptr<int>(h->bFlags), 0, sizeof(int), st));
    HIPCHECK(h, hipStreamSynchronize(st));
    if (flags & 2) return fail(h, SWR_E_SINGULAR, "zero pivot in a device factorisation");
    return fail(h, SWR_E_NAN, "non-finite value produced on the device");
  }
  return SWR_OK;
}

// The field's first (or only) component at time t, and the second of a
// circular pulse (Section 5 Test 3).
double field(const swr_desc& d, double t) {
  if (d.field_shape == SWR_FIELD_CIRCULAR)
    return d.E0 * std::cos(d.omega * t + d.phase) *
           std::exp(-d.pulse_nu * (t - d.pulse_center) * (t - d.pulse_center));
  return d.E0 * std::sin(d.omega * t + d.phase);
}
double field2(const swr_desc& d, double t) {
  return d.E0 * std::sin(d.omega * t + d.phase) *
         std::exp(-d.pulse_nu * (t - d.pulse_center) * (t - d.pulse_center));
}

// kinds of timed launches
enum { kTFactor = 0, kTTransmit = 1, kTRecur = 2, kTResidual = 3 };

// Record the opening event of a timed launch (no-op unless timing).
hipError_t tbegin(swr_handle h, hipStream_t st, int kind) {
  if (!h->timing) return hipSuccess;
  if (2 * h->tused + 2 > h->tev.size()) {
    for (int q = 0; q < 64; ++q) {
      hipEvent_t e;
      const hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      h->tev.push_back(e);
    }
    h->tkind.resize(h->tev.size() / 2);
  }
  h->tkind[h->tused] = kind;
  return hipEventRecord(h->tev[2 * h->tused], st);
}

hipError_t tend(swr_handle h, hipStream_t st) {
  if (!h->timing) return hipSuccess;
  const hipError_t r = hipEventRecord(h->tev[2 * h->tused + 1], st);
  ++h->tused;
  return r;
}

// Sum the recorded durations by kind into the run statistics.
hipError_t tcollect(swr_handle h, swr_run_stats* s) {
  if (!h->timing || h->tused == 0) return hipSuccess;
  hipError_t r = hipEventSynchronize(h->tev[2 * h->tused - 1]);
  if (r != hipSuccess) return r;
  double* ms[4] = {&s->ms_factor, &s->ms_transmit, &s->ms_recur, &s->ms_residual};
  int32_t* n[4] = {&s->n_factor, &s->n_transmit, &s->n_recur, &s->n_residual};
  for (size_t q = 0; q < h->tused; ++q) {
    float t = 0.0f;
    r = hipEventElapsedTime(&t, h->tev[2 * q], h->tev[2 * q + 1]);
    if (r != hipSuccess) return r;
    *ms[h->tkind[q]] += t;
    *n[h->tkind[q]] += 1;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Block path (block.hip): host side.

constexpr int kBlkDepth = swr::kBlkCols - 1;  // iterates in flight, + the one they follow
constexpr int kBlkPotBatch = 16;               // items per four-dimensional potential batch

// least number of series terms K + 1 with rho^{K+1}/(1 - rho) <= 2^-53; 0
// when more than max_terms would be needed
int series_terms(double rho, int max_terms) {
  if (!(rho < 0.5)) return 0;
  int t = 1;
  for (double tail = rho / (1.0 - rho); tail > 0x1p-53 && t <= max_terms; ++t) tail *= rho;
  return t > max_terms ? 0 : t;
}

// Empty when the block path can take the description, else the reason.
std::string blk_unsupported(const Geometry& g) {
  const swr_desc& d = g.desc;
  if (!(g.D == 2 || g.D == 4)) return "the block path takes two or four configuration dimensions";
  if (d.mode != SWR_TDSE) return "the block path is for real time";
  if (d.field_shape != SWR_FIELD_SINE) return "the block path takes the sine field";
  if (d.mu_im > 0.0) return "the block path needs Im mu <= 0 (the field series)";
  if (g.K_max > swr::kBlkK) return "basis size per subdomain above 1536 (block path)";
  const int nt = 2 * d.face_nodes_band + d.face_nodes_mid;
  if (nt > swr::kBlkNt) return "more than 32 face nodes per tangential dimension (block path)";
  int face = 1;
  for (int k = 1; k < g.D; ++k) face *= nt;
  if (face > swr::kBlkFace) return "more than 512 nodes per face (block path)";
  for (int k = 0; k < g.D; ++k) {
    const double width = g.hi1[k][0] - g.lo1[k][0];
    if (g.L[k] > 1 && !(g.eps[k] > 0.0 && 2.0 * g.eps[k] < width))
      return "the block path needs overlaps 0 < eps < core width";
  }
  for (int s = 0; s < g.n_items; ++s)
    for (int k = 0; k < g.D; ++k) {
      if (g.nb[(size_t)s * 4 + k] > swr::kBlkN) return "more than 8 Gaussians per dimension (block path)";
      if (g.qn[(size_t)s * 4 + k] > 4096) return "potential quadrature too fine (block path)";
    }
  if (g.D == 4)
    for (int s = 0; s < g.n_items; ++s) {
      const int q1 = g.qn[(size_t)s * 4 + 1], n3 = g.nb[(size_t)s * 4 + 3];
      if (q1 > swr::kEeQ || q1 * n3 * n3 > swr::kEeZ)
        return "potential quadrature too fine for the four-dimensional stage (block path)";
    }
  return "";
}

void plan_block_layout(swr_handle h) {
  const Geometry& g = h->g;
  const size_t NI = g.n_items;
  Layout& L = h->lay;
  L = Layout();
  h->bK = L.add(NI * 4);
  h->bOff1 = L.add((NI + 1) * 8);
  h->bOff2 = L.add((NI + 1) * 8);
  h->bOffP = L.add((NI + 1) * 8);
  h->bIdx = L.add(NI * 16);
  h->bNb = L.add(NI * 16);
  h->bL = L.add(16);
  h->bLo = L.add(NI * 32);
  h->bHi = L.add(NI * 32);
  h->bEps = L.add(32);
  h->bDelta = L.add(NI * 32);
  h->bAoff = L.add(NI * 32);
  h->bAlpha = L.add(g.alpha.size() * 8);
  h->bQoff = L.add(NI * 32);
  h->bQn = L.add(NI * 16);
  h->bQx = L.add(g.qx.size() * 8);
  h->bQw = L.add(g.qw.size() * 8);
  h->bPos = L.add(std::max<size_t>(1, g.nuc_pos.size()) * 8);
  h->bCharge = L.add(std::max<size_t>(1, g.nuc_charge.size()) * 8);
  h->bCenter = L.add(32);
  h->bFlags = L.add(8);
  h->bResOut = L.add(8);
  h->bResv = L.add(64 * 8);
  h->bE = L.add((h->n_T + 1) * 8);
  h->bBd = L.add(NI * 4 * sizeof(swr::BlkDim));
  h->bBlkPotOff = L.add((NI + 1) * 8);
  h->bBlkVp = L.add(h->sum_K2 * 8);
  h->bBlkY0 = L.add(h->sum_K * 16);
  h->bBlkF0 = L.add(h->sum_K * 16);
  h->bBlkF1 = L.add(h->sum_K * 16);
  h->bBlkRing = L.add((size_t)h->blk_slots * 2 * h->sum_K * 16);
  h->bBlkPart = L.add((size_t)h->blk_slots * NI * (h->n_T + 1) * 8);
  h->bBlkRb = L.add(h->sum_K * swr::kBlkCols * 16);
  h->bBlkTr = L.add((size_t)swr::kBlkCols * NI * g.D * swr::kBlkPos * h->blk_fstride * 16);
  h->bBlkFrag = L.add((size_t)h->blk_chunks * h->blk_foff.back() * 16);
  h->bBlkTerms = L.add(NI * 4);
  h->bBlkFoff = L.add((NI + 1) * 8);
  h->bBlkTileOff = L.add((NI + 1) * 8);
  h->bBlkEa = L.add((size_t)h->blk_chunks * 8);
  h->bBlkCp = L.add((size_t)h->blk_chunks * swr::kBlkGJ * h->sum_K * 16);
  h->bBlkRp = L.add((size_t)h->blk_chunks * swr::kBlkGJ * h->sum_K * 16);
  h->bBlkCvec = L.add(h->sum_K * 16);
  // one region for the iterates' histories, reused (outside a window's
  // iterations) by the potential's scratch at assembly and by the anchor
  // matrices and series products at factorisation
  const size_t hist = (size_t)h->blk_slots * (h->n_T + 1) * h->sum_K * 16;
  const size_t pot = (size_t)(h->blk_pot_total + (int64_t)h->blk_pot_batch * h->blk_stage_item) * 8 + 256;
  const size_t fac = (size_t)3 * h->blk_chunks * h->sum_K2 * 16;
  h->bBlkRegion = L.add(std::max({hist, pot, fac}));
}

// Per-item sizes the block path derives at creation.
int blk_prepare(swr_handle h, std::string* msg) {
  const Geometry& g = h->g;
  const int NI = g.n_items;
  h->block = true;
  h->blk_depth = kBlkDepth;
  h->blk_slots = kBlkDepth + 1;
  // anchors per window: the field moves by at most E0 |omega| per unit time,
  // so a chunk of T_c has a half range <= E0 |omega| T_c / 2
  const double tau = 0.5 * g.desc.dt;
  const double slope = std::fabs(g.desc.E0 * g.desc.omega);
  int nc = 1;
  for (; nc <= 64; ++nc) {
    const int64_t cl = (h->n_T + nc - 1) / nc;
    const double half = 0.5 * slope * cl * g.desc.dt;
    if (series_terms(tau * half * h->dipole_max, swr::kBlkTerms) > 0) break;
  }
  if (nc > 64) {
    *msg = "the field varies too fast for the block path's series (64 anchors per window)";
    return SWR_E_SIZE;
  }
  h->blk_chunk_len = (int)((h->n_T + nc - 1) / nc);
  h->blk_chunks = (int)((h->n_T + h->blk_chunk_len - 1) / h->blk_chunk_len);
  // potential scratch, packed terms, tiles, face stride
  h->pot_off.assign(NI + 1, 0);
  h->blk_foff.assign(NI + 1, 0);
  h->blk_toff.assign(NI + 1, 0);
  h->blk_stage_item = 0;
  h->blk_qmax = h->blk_qqmax = 1;
  for (int s = 0; s < NI; ++s) {
    int32_t nb[4], qn[4];
    for (int k = 0; k < 4; ++k) {
      nb[k] = k < g.D ? g.nb[(size_t)s * 4 + k] : 1;
      qn[k] = k < g.D ? g.qn[(size_t)s * 4 + k] : 1;
      h->blk_qmax = std::max(h->blk_qmax, qn[k]);
    }
    if (g.D == 4) h->blk_qqmax = std::max(h->blk_qqmax, qn[0] * qn[2]);
    h->pot_off[s + 1] = h->pot_off[s] + swr::blk_pot_item_doubles(nb, qn, g.D);
    h->blk_stage_item =
        std::max(h->blk_stage_item, swr::blk_pot_stage_doubles(nb, qn, g.D, g.desc.n_elec));
    const int K = g.K[s];
    const int64_t fs = (int64_t)((K + 15) / 16) * ((K + 3) / 4) * 64;
    h->blk_foff[s + 1] = h->blk_foff[s] + swr::kBlkTerms * fs;
    const int64_t t = (K + 63) / 64;
    h->blk_toff[s + 1] = h->blk_toff[s] + t * t;
  }
  h->blk_pot_total = h->pot_off.back();
  h->blk_pot_batch = std::max(1, std::min(NI, kBlkPotBatch));
  const int nt = 2 * g.desc.face_nodes_band + g.desc.face_nodes_mid;
  h->blk_fstride = 1;
  for (int k = 1; k < g.D; ++k) h->blk_fstride *= nt;
  h->blk_terms.assign(NI, 1);
  h->depth = h->depth_run = h->blk_depth;
  plan_block_layout(h);
  return SWR_OK;
}

int32_t blk_assemble(swr_handle h, hipStream_t st) {
  const Geometry& g = h->g;
  const int NI = g.n_items;
  std::vector<int32_t> L4(4, 1);
  std::vector<double> eps4(4, 0.0), cen4(4, 0.0);
  for (int k = 0; k < g.D; ++k) {
    L4[k] = g.L[k];
    eps4[k] = g.eps[k];
    cen4[k] = g.desc.init_center[k];
  }
  std::vector<int64_t> zoffp(NI + 1, 0);
  HIPCHECK(h, upload(h, h->bK, g.K, st));
  HIPCHECK(h, upload(h, h->bOff1, g.off1, st));
  HIPCHECK(h, upload(h, h->bOff2, g.off2, st));
  HIPCHECK(h, upload(h, h->bOffP, zoffp, st));
  HIPCHECK(h, upload(h, h->bIdx, g.idx, st));
  HIPCHECK(h, upload(h, h->bNb, g.nb, st));
  HIPCHECK(h, upload(h, h->bL, L4, st));
  HIPCHECK(h, upload(h, h->bLo, g.lo, st));
  HIPCHECK(h, upload(h, h->bHi, g.hi, st));
  HIPCHECK(h, upload(h, h->bEps, eps4, st));
  HIPCHECK(h, upload(h, h->bDelta, g.delta, st));
  HIPCHECK(h, upload(h, h->bAoff, g.aoff, st));
  HIPCHECK(h, upload(h, h->bAlpha, g.alpha, st));
  HIPCHECK(h, upload(h, h->bQoff, g.qoff, st));
  HIPCHECK(h, upload(h, h->bQn, g.qn, st));
  HIPCHECK(h, upload(h, h->bQx, g.qx, st));
  HIPCHECK(h, upload(h, h->bQw, g.qw, st));
  HIPCHECK(h, upload(h, h->bPos, g.nuc_pos, st));
  HIPCHECK(h, upload(h, h->bCharge, g.nuc_charge, st));
  HIPCHECK(h, upload(h, h->bCenter, cen4, st));
  // per (item, dimension) one-dimensional data: sizes and the face rule
  h->bdim.assign((size_t)NI * 4, swr::BlkDim{});
  for (int s = 0; s < NI; ++s)
    for (int k = 0; k < g.D; ++k) {
      swr::BlkDim& d = h->bdim[(size_t)s * 4 + k];
      d.n = g.nb[(size_t)s * 4 + k];
      d.band = g.desc.face_nodes_band;
      d.mid = g.desc.face_nodes_mid;
      d.nt = 2 * d.band + d.mid;
      d.lo = g.lo[(size_t)s * 4 + k];
      d.hi = g.hi[(size_t)s * 4 + k];
      d.eps = g.eps[k];
      std::vector<double> x, w;
      swr::face_rule_1d(g, s, k, &x, &w);
      for (int t = 0; t < d.nt; ++t) {
        d.tx[t] = x[t];
        d.tw[t] = w[t];
      }
    }
  HIPCHECK(h, upload(h, h->bBd, h->bdim, st));
  HIPCHECK(h, upload(h, h->bBlkPotOff, h->pot_off, st));
  HIPCHECK(h, upload(h, h->bBlkFoff, h->blk_foff, st));
  HIPCHECK(h, upload(h, h->bBlkTileOff, h->blk_toff, st));
  HIPCHECK(h, upload(h, h->bBlkTerms, h->blk_terms, st));
  HIPCHECK(h, hipMemsetAsync(h->ptr<int>(h->bFlags), 0, 8, st));
  HIPCHECK(h, hipMemsetAsync(h->ptr<double2>(h->bBlkRb), 0, h->bBlkRb.bytes, st));
  const swr::Items it = h->items();
  HIPCHECK(h, swr::launch_blk_dims(it, h->ptr<swr::BlkDim>(h->bBd), g.desc.mu_re, g.desc.mu_im,
                                   g.desc.init_alpha, h->ptr<double>(h->bCenter),
                                   h->ptr<int>(h->bFlags), st));
  const swr::BlkItems b = h->blk_items();
  swr::Potential pot{g.desc.n_nuc, h->ptr<double>(h->bPos), h->ptr<double>(h->bCharge),
                     g.desc.eps_en, g.desc.eps_ee};
  double* scratch = h->ptr<double>(h->bBlkRegion);
  HIPCHECK(h, swr::launch_blk_potential(b, pot, h->ptr<int64_t>(h->bBlkPotOff), scratch,
                                        scratch + h->blk_pot_total, h->blk_stage_item,
                                        h->blk_pot_batch, h->blk_qmax, h->blk_qqmax, g.K_max,
                                        h->ptr<double>(h->bBlkVp), st));
  HIPCHECK(h, hipStreamSynchronize(st));
  const int rc = check_flags(h, st);
  if (rc != SWR_OK)
    return fail(h, rc, "a one-dimensional Gram matrix is not positive definite (Cholesky)");
  h->assembled = true;
  h->initial = h->warm = h->factored = false;
  h->blk_k = 0;
  return SWR_OK;
}

int32_t blk_set_initial(swr_handle h, const void* c0_dev, hipStream_t st) {
  const swr::BlkItems b = h->blk_items();
  double2* y0 = h->ptr<double2>(h->bBlkY0);
  if (c0_dev) {
    HIPCHECK(h, swr::launch_blk_kron(b, 0, (const double2*)c0_dev, 1, 0, y0, 1, 1, st));
  } else {
    const double norm = std::pow(2.0 * h->g.desc.init_alpha / 3.14159265358979323846, 0.25 * h->g.D);
    HIPCHECK(h, swr::launch_blk_project(b, norm, h->g.K_max, y0, st));
  }
  h->initial = true;
  h->warm = false;
  h->blk_k = 0;
  return SWR_OK;
}

swr::BlkTx blk_tx_one(int slot, int step, int prev, int dst) {
  swr::BlkTx tx{};
  tx.n = 1;
  tx.slot[0] = slot;
  tx.step[0] = step;
  tx.prev[0] = prev;
  tx.dst[0] = dst;
  return tx;
}

int32_t blk_warm_start(swr_handle h, int mode, hipStream_t st) {
  if (mode == SWR_WARM_GIVEN)
    return fail(h, SWR_E_ARG, "the block path takes the plain or the zero warm start");
  if (mode != SWR_WARM_PLAIN && mode != SWR_WARM_ZERO) return fail(h, SWR_E_ARG, "unknown warm start");
  const swr::BlkItems b = h->blk_items();
  const swr::BlkState S = h->blk_state();
  // F0: Robin data of the initial state (every iterate's step 0 after the
  // first; the plain guess holds it for the first iterate's whole window)
  HIPCHECK(h, swr::launch_blk_transmit(b, S, blk_tx_one(-1, 0, -2, swr::kBlkF0),
                                       h->ptr<double2>(h->bBlkTr), h->g.K_max,
                                       h->ptr<int>(h->bFlags), st));
  if (mode == SWR_WARM_PLAIN)
    HIPCHECK(h, hipMemcpyAsync(S.F1, S.F0, h->sum_K * 16, hipMemcpyDeviceToDevice, st));
  else
    HIPCHECK(h, hipMemsetAsync(S.F1, 0, h->sum_K * 16, st));
  h->blk_warm = mode;
  h->blk_k = 0;
  h->warm = true;
  return SWR_OK;
}

int32_t blk_factor(swr_handle h, double t0, hipStream_t st) {
  const Geometry& g = h->g;
  HIPCHECK(h, hipStreamSynchronize(st));
  h->E_host.assign(h->n_T + 1, 0.0);
  for (int64_t n = 0; n <= h->n_T; ++n) h->E_host[n] = field(g.desc, t0 + n * g.desc.dt);
  HIPCHECK(h, upload(h, h->bE, h->E_host, st));
  const double tau = 0.5 * g.desc.dt;
  const int nc = h->blk_chunks, cl = h->blk_chunk_len;
  h->blk_Ea.assign(nc, 0.0);
  double half = 0.0;
  for (int c = 0; c < nc; ++c) {
    const int64_t n0 = (int64_t)c * cl, n1 = std::min<int64_t>(n0 + cl, h->n_T);
    double lo = h->E_host[n0 + 1], hi = lo;
    for (int64_t n = n0; n < n1; ++n) {
      lo = std::min(lo, h->E_host[n + 1]);
      hi = std::max(hi, h->E_host[n + 1]);
    }
    h->blk_Ea[c] = 0.5 * (lo + hi);
    half = std::max(half, 0.5 * (hi - lo));
  }
  int t_max = 1;
  for (int s = 0; s < g.n_items; ++s) {
    const int t = series_terms(tau * half * h->dipole[s], swr::kBlkTerms);
    if (t == 0)
      return fail(h, SWR_E_SIZE, "the field varies too much per anchor for the block path's "
                                 "series (the workspace was sized for the creation's field)");
    h->blk_terms[s] = t;
    t_max = std::max(t_max, t);
  }
  HIPCHECK(h, upload(h, h->bBlkEa, h->blk_Ea, st));
  HIPCHECK(h, upload(h, h->bBlkTerms, h->blk_terms, st));
  HIPCHECK(h, tbegin(h, st, kTFactor));
  const swr::BlkItems b = h->blk_items();
  const int64_t cs = h->sum_K2;
  double2* Z = h->ptr<double2>(h->bBlkRegion);
  double2* Zq = Z + (size_t)nc * cs;
  double2* Pk = Zq + (size_t)nc * cs;
  const int64_t* toff = h->ptr<int64_t>(h->bBlkTileOff);
  const int64_t nt = h->blk_toff.back();
  const int64_t fcs = h->blk_foff.back();
  double2* frag = h->ptr<double2>(h->bBlkFrag);
  HIPCHECK(h, swr::launch_blk_anchor(b, h->ptr<double>(h->bBlkVp), h->ptr<double>(h->bBlkEa), nc,
                                     cs, Z, g.K_max, st));
  HIPCHECK(h, swr::launch_blk_invert(b, nc, cs, Z, h->ptr<double2>(h->bBlkCp),
                                     h->ptr<double2>(h->bBlkRp), (int64_t)swr::kBlkGJ * h->sum_K,
                                     toff, nt, g.K_max, h->ptr<int>(h->bFlags), st));
  HIPCHECK(h, swr::launch_blk_pack(b, nc, cs, Z, 0, fcs, frag, g.K_max, st));
  for (int k = 1; k < t_max; ++k) {
    HIPCHECK(h, swr::launch_blk_qapply(b, nc, cs, k == 1 ? Z : Pk, Zq, g.K_max, st));
    HIPCHECK(h, swr::launch_gemm_wide(b.it, toff, nt, nc, Z, Zq, nullptr, make_double2(1.0, 0.0),
                                      nullptr, cs, Pk, st));
    HIPCHECK(h, swr::launch_blk_pack(b, nc, cs, Pk, k, fcs, frag, g.K_max, st));
  }
  HIPCHECK(h, tend(h, st));
  h->factor_terms = t_max - 1;
  h->factored = true;
  h->t0 = t0;
  return SWR_OK;
}

// Iterates k0 .. k0 + P - 1 of the window, all in flight: launch l advances
// iterate k0 + i from step l - i (lag one step: iterate k at step n needs
// iterate k - 1's Robin data up to step n + 1).  Iterate k0 - 1, complete,
// sends its data one step ahead as an extra transmission column.  With
// tol >= 0 the launches stop once an iterate k >= 2 has Res(k) <= tol.
int32_t blk_batch(swr_handle h, int k0, int P, double tol, hipStream_t st, swr_run_stats* out,
                  bool* stop) {
  const Geometry& g = h->g;
  const int NS = h->blk_slots;
  const int nT = (int)h->n_T;
  auto slot = [NS](int k) { return k % NS; };
  const swr::BlkItems b = h->blk_items();
  const swr::BlkState S = h->blk_state();
  double2* Tr = h->ptr<double2>(h->bBlkTr);
  double2* Rb = h->ptr<double2>(h->bBlkRb);
  const double2* frag = h->ptr<double2>(h->bBlkFrag);
  const int64_t fcs = h->blk_foff.back();
  double* resv = h->ptr<double>(h->bResv);
  int* flags = h->ptr<int>(h->bFlags);
  if (!h->res_pinned) HIPCHECK(h, hipHostMalloc((void**)&h->res_pinned, 64 * sizeof(double), 0));
  if (!h->ev_ready) {
    for (auto& e : h->ev) HIPCHECK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->ev_ready = true;
  }
  // every iterate of the batch starts from the window's initial state
  for (int i = 0; i < P; ++i) {
    HIPCHECK(h, hipMemsetAsync(S.part + slot(k0 + i) * S.pstride, 0, S.pstride * 8, st));
    HIPCHECK(h, swr::launch_blk_kron(b, 3, S.y0, 1, 0, S.hist + slot(k0 + i) * S.hstride,
                                     h->n_T + 1, 1, st));
  }
  const bool pseudo = k0 > 1;
  if (pseudo && nT >= 1) {
    HIPCHECK(h, tbegin(h, st, kTTransmit));
    HIPCHECK(h, swr::launch_blk_transmit(b, S, blk_tx_one(slot(k0 - 1), 1, -2, 2 * slot(k0) + 1),
                                         Tr, g.K_max, flags, st));
    HIPCHECK(h, tend(h, st));
  }
  std::vector<int> pending;  // completed iterates not yet checked
  int k_done = k0 - 1, k_stop = 0;
  auto check = [&](bool wait_all) -> int32_t {
    while (!pending.empty()) {
      const int k = pending.front();
      hipEvent_t e = h->ev[k % kResEvents];
      if (!wait_all && pending.size() < 3) {
        const hipError_t q = hipEventQuery(e);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return fail(h, SWR_E_DEVICE, "hipEventQuery failed");
      } else {
        HIPCHECK(h, hipEventSynchronize(e));
      }
      pending.erase(pending.begin());
      const double r = h->res_pinned[k % 64];
      if (k <= 64) out->res[k - 1] = r;
      out->iters = k;
      h->blk_last_res = r;
      if (tol >= 0.0 && k >= 2 && r <= tol) {
        out->converged = 1;
        k_stop = k;
        return SWR_OK;
      }
    }
    return SWR_OK;
  };
  const int n_launch = nT + P - 1;
  for (int l = 0; l < n_launch && !k_stop; ++l) {
    // columns grouped by series chunk (one solve launch per chunk present)
    std::vector<swr::BlkCols> cols;
    std::vector<int> cchunk;
    swr::BlkTx tx{};
    for (int i = 0; i < P; ++i) {
      const int n = l - i;
      if (n < 0 || n >= nT) continue;
      const int k = k0 + i;
      const int ch = n / h->blk_chunk_len;
      size_t gsel = 0;
      while (gsel < cchunk.size() && cchunk[gsel] != ch) ++gsel;
      if (gsel == cchunk.size()) {
        cchunk.push_back(ch);
        cols.push_back(swr::BlkCols{});
      }
      swr::BlkCols& c = cols[gsel];
      const int j = c.n++;
      c.step[j] = n;
      c.slot[j] = slot(k);
      c.fa[j] = k == 1 ? swr::kBlkF1 : (n == 0 ? swr::kBlkF0 : 2 * slot(k) + (n & 1));
      c.fb[j] = k == 1 ? swr::kBlkF1 : 2 * slot(k) + ((n + 1) & 1);
      c.dE[j] = h->E_host[n + 1] - h->E_host[n];
      const double d = h->E_host[n + 1] - h->blk_Ea[ch];
      double pw = 1.0;
      for (int q = 0; q < swr::kBlkTerms; ++q) {
        c.w[q][j] = pw;
        pw *= -d;
      }
      const int t = tx.n++;
      tx.slot[t] = slot(k);
      tx.step[t] = n + 1;
      tx.prev[t] = k == 1 ? -1 : slot(k - 1);
      tx.dst[t] = 2 * slot(k + 1) + ((n + 1) & 1);
    }
    if (pseudo && l + 2 <= nT) {
      const int t = tx.n++;
      tx.slot[t] = slot(k0 - 1);
      tx.step[t] = l + 2;
      tx.prev[t] = -2;
      tx.dst[t] = 2 * slot(k0) + ((l + 2) & 1);
    }
    HIPCHECK(h, tbegin(h, st, kTRecur));
    for (size_t q = 0; q < cols.size(); ++q)
      HIPCHECK(h, swr::launch_blk_step(b, S, cols[q], frag + (size_t)cchunk[q] * fcs, Rb,
                                       g.K_max, st));
    HIPCHECK(h, tend(h, st));
    HIPCHECK(h, tbegin(h, st, kTTransmit));
    HIPCHECK(h, swr::launch_blk_transmit(b, S, tx, Tr, g.K_max, flags, st));
    HIPCHECK(h, tend(h, st));
    const int i_done = l - (nT - 1);
    if (i_done >= 0 && i_done < P) {
      const int k = k0 + i_done;
      HIPCHECK(h, tbegin(h, st, kTResidual));
      HIPCHECK(h, swr::launch_blk_res_reduce(S.part + slot(k) * S.pstride, g.n_items, nT,
                                             g.desc.dt, resv + (k % 64), st));
      HIPCHECK(h, tend(h, st));
      HIPCHECK(h, hipMemcpyAsync(h->res_pinned + (k % 64), resv + (k % 64), 8,
                                 hipMemcpyDeviceToHost, st));
      HIPCHECK(h, hipEventRecord(h->ev[k % kResEvents], st));
      pending.push_back(k);
      k_done = k;
      if (tol >= 0.0) {
        const int32_t rc = check(false);
        if (rc) return rc;
      }
    }
  }
  {
    const int32_t rc = check(true);
    if (rc) return rc;
  }
  const int k_last = k_stop ? k_stop : k_done;
  h->blk_k = k_last;
  h->blk_cur = slot(k_last);
  *stop = k_stop != 0;
  return SWR_OK;
}

int32_t blk_run(swr_handle h, const swr_run_opts* o, swr_run_stats* stats, hipStream_t st) {
  int32_t rc = blk_factor(h, o->t0, st);
  if (rc) return rc;
  rc = blk_warm_start(h, o->warm, st);
  if (rc) return rc;
  swr_run_stats s{};
  int P = o->depth > 0 ? std::min(o->depth, h->blk_depth) : h->depth_run;
  P = std::max(1, std::min(P, o->k_max));
  bool stop = false;
  for (int k0 = 1; k0 <= o->k_max && !stop;) {
    const int Pb = std::min(P, o->k_max - k0 + 1);
    rc = blk_batch(h, k0, Pb, o->tol, st, &s, &stop);
    if (rc) return rc;
    k0 += Pb;
  }
  rc = check_flags(h, st);
  if (rc) return rc;
  HIPCHECK(h, tcollect(h, &s));
  if (stats) *stats = s;
  if (o->tol > 0.0 && !s.converged)
    return fail(h, SWR_E_NOCONV, "iteration cap reached above the residual target");
  return SWR_OK;
}

}  // namespace

extern "C" {

int32_t swr_create(const swr_desc* desc, swr_handle* out) {
  if (!desc || !out) {
    g_create_error = "null argument";
    return SWR_E_ARG;
  }
  swr_handle h = new (std::nothrow) swr_handle_s();
  if (!h) {
    g_create_error = "out of host memory";
    return SWR_E_ARG;
  }
  int code = SWR_OK;
  std::string msg = swr::build_geometry(*desc, &h->g, &code);
  if (code != SWR_OK) {
    g_create_error = msg;
    delete h;
    return code;
  }
  Geometry& g = h->g;
  double cond_1d = 1.0;
  const double gram_cond = max_gram_condition(g, &cond_1d);
  if (!(cond_1d <= kSingularLimit)) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "a subdomain's one-dimensional Gram matrix is singular to working precision "
                  "(condition %.3g): its Gaussians are linearly dependent at this width", cond_1d);
    g_create_error = buf;
    delete h;
    return SWR_E_SINGULAR;
  }
  if (g.desc.factor_mode == SWR_FACTOR_BLOCK || (g.D == 4 && g.K_max > swr::kSmallK)) {
    const std::string why = blk_unsupported(g);
    if (!why.empty()) {
      g_create_error = why;
      delete h;
      return SWR_E_SIZE;
    }
    if (g.desc.n_steps > 16384) {
      g_create_error = "n_steps above 16384";
      delete h;
      return SWR_E_SIZE;
    }
    h->sum_K = g.off1[g.n_items];
    h->sum_K2 = g.off2[g.n_items];
    h->n_T = g.desc.n_steps;
    h->n_mats = g.desc.n_steps;
    h->offp.assign(g.n_items + 1, 0);
    for (int s = 0; s < g.n_items; ++s) {
      double x = 0.0;
      for (int el = 0; el < g.desc.n_elec; ++el) {
        const int k = el * g.desc.dim + g.desc.axis;
        x += std::max(std::fabs(g.lo[(size_t)s * 4 + k]), std::fabs(g.hi[(size_t)s * 4 + k]));
      }
      h->dipole_max = std::max(h->dipole_max, x);
      h->dipole.push_back(x);
    }
    std::string msg;
    const int rc = blk_prepare(h, &msg);
    if (rc) {
      g_create_error = msg;
      delete h;
      return rc;
    }
    *out = h;
    return SWR_OK;
  }
  const bool wide_ok =
      g.desc.dim == 1 && g.desc.n_elec == 1 && g.desc.mode == SWR_TDSE && g.te_ok;
  if (g.K_max > (wide_ok ? swr::kWideK : swr::kSmallK)) {
    g_create_error = wide_ok ? "basis size per subdomain exceeds 256"
                             : "basis size per subdomain exceeds 64 (256 for one electron in "
                               "one dimension in real time)";
    delete h;
    return SWR_E_SIZE;
  }
  if (g.desc.factor_mode == SWR_FACTOR_WIDE && !wide_ok) {
    g_create_error = "the wide-basis path is for one electron in one dimension in real time";
    delete h;
    return SWR_E_ARG;
  }
  h->wide = wide_ok && (g.K_max > swr::kSmallK || g.desc.factor_mode == SWR_FACTOR_WIDE);
  if (h->wide && (g.desc.factor_mode == SWR_FACTOR_DIRECT || g.desc.mu_im > 0.0)) {
    g_create_error = "bases above 64 take the field series: factor_mode direct and Im mu > 0 "
                     "are not available";
    delete h;
    return SWR_E_SIZE;
  }
  // Local Slater determinants are not a tensor basis: their Gram matrices
  // are checked once assembled (swr_assemble), the orbitals being computed
  // there.
  if (g.desc.basis_kind != SWR_BASIS_LSD && g.desc.basis_kind != SWR_BASIS_LO) {
    const double cond = gram_cond;
    if (!(cond <= kCondLimit)) {
      char buf[200];
      std::snprintf(buf, sizeof buf,
                    "a subdomain's Gram matrix has condition %.3g, above the %.0e the "
                    "stored-inverse recurrence keeps to 1e-10 (widen the Gaussians or use "
                    "fewer per subdomain)", cond, kCondLimit);
      g_create_error = buf;
      delete h;
      return SWR_E_COND;
    }
  }
  if (g.desc.n_steps > 16384) {
    g_create_error = "n_steps above 16384 (the field table of a window is staged in LDS)";
    delete h;
    return SWR_E_SIZE;
  }
  if (g.desc.dim > 2 || g.desc.n_elec > 2) {
    g_create_error = "the library assembles at most two space dimensions per electron and 2 electrons";
    delete h;
    return SWR_E_SIZE;
  }
  h->offp.assign(g.n_items + 1, 0);
  for (int q = 0; q < g.n_items; ++q) {
    const int64_t T8 = (g.K[q] + 7) / 8;
    h->offp[q + 1] = h->offp[q] + 32 * T8 * (T8 + 1);
  }
  h->sum_K = g.off1[g.n_items];
  h->sum_K2 = g.off2[g.n_items];
  h->n_T = g.desc.n_steps;
  h->n_nodes_t = g.desc.learned_nodes > 0 ? g.desc.learned_nodes : 8;
  h->n_mats = g.desc.mode == SWR_TDSE ? g.desc.n_steps : 1;
  for (int s = 0; s < g.n_items; ++s) {
    double x = 0.0;
    for (int el = 0; el < g.desc.n_elec; ++el) {
      const int k = el * g.desc.dim + g.desc.axis;
      x += std::max(std::fabs(g.lo[(size_t)s * 4 + k]), std::fabs(g.hi[(size_t)s * 4 + k]));
    }
    h->dipole_max = std::max(h->dipole_max, x);
    h->dipole.push_back(x);
  }
  h->n_res_tiles = (int)((h->n_T + 1 + 15) / 16);
  if (h->wide) h->n_res_tiles = std::max(h->n_res_tiles, swr::tx_wide_tiles((int)h->n_T, 8));
  h->s1off.assign((size_t)g.n_items * 4, 0);
  h->scratch_off.assign(g.n_items, 0);
  int64_t s1 = 0, scr = 0;
  for (int s = 0; s < g.n_items; ++s) {
    for (int k = 0; k < g.D; ++k) {
      h->s1off[(size_t)s * 4 + k] = s1;
      const int n = g.nb[(size_t)s * 4 + k];
      s1 += (int64_t)n * n;
    }
    h->scratch_off[s] = scr;
    if (g.desc.basis_kind == SWR_BASIS_SLATER || g.desc.basis_kind == SWR_BASIS_LSD) {
      // staged electron-electron term over the extended pairs (Gaussians,
      // or local orbitals)
      const int half =
          g.desc.basis_kind == SWR_BASIS_LSD ? swr::lsd_functions(g.desc) : g.nb[(size_t)s * 4];
      scr += swr::slater_pot_scratch(half, g.qn[(size_t)s * 4 + 1]);
    } else if (g.desc.dim == 2) {
      int32_t nb[4], qn[4];
      for (int k = 0; k < 4; ++k) {
        nb[k] = k < g.D ? g.nb[(size_t)s * 4 + k] : 1;
        qn[k] = k < g.D ? g.qn[(size_t)s * 4 + k] : 1;
      }
      int64_t off[11];
      swr::pot2_layout(nb, qn, g.desc.n_elec, off);
      scr += off[10];
    } else if (g.desc.n_elec == 2) {
      const int n1 = g.nb[(size_t)s * 4 + 1];
      scr += (int64_t)g.qn[(size_t)s * 4 + 0] * n1 * n1;
    }
  }
  h->s1_total = s1;
  h->scratch_total = scr;
  if (!h->wide) {
    // iterates in flight: enough blocks of one per item to fill the chip
    const int per_cu = g.desc.mode == SWR_TISE ? kIePerCU : kRecPerCU;
    const int fill = (per_cu * kGpuCUs + g.n_items - 1) / g.n_items;
    h->depth = std::max(1, std::min({kMaxDepth, fill, (int)h->n_T}));
  }
  if (h->wide) {
    h->order.resize(g.n_items);
    for (int q = 0; q < g.n_items; ++q) h->order[q] = q;
    h->order_natural = h->order;
    std::stable_sort(h->order.begin(), h->order.end(),
                     [&](int a, int b) { return g.K[a] > g.K[b]; });
    h->tile_off.assign(g.n_items + 1, 0);
    for (int q = 0; q < g.n_items; ++q) {
      const int64_t t = (g.K[q] + 63) / 64;
      h->tile_off[q + 1] = h->tile_off[q] + t * t;
    }
  }
  // pipelined: depth iterates in flight, the one they read, and the one
  // before it (the residual of iterate k-1 reads iterate k-2)
  h->n_slots = h->depth > 1 ? h->depth + 2 : 2;
  if (g.D == 2)
    for (int q = 0; q < g.n_items; ++q)
      h->nbt = std::max({h->nbt, g.nb[(size_t)q * 4], g.nb[(size_t)q * 4 + 1]});
  if (g.te_ok) {
    h->te_blob_off.assign(g.n_items + 1, 0);
    h->te_sdesc.assign(g.te_sidx.size() * swr::kTxDesc, 0);
    for (int j = 0; j < g.n_items; ++j) {
      int64_t b = 0;
      for (int64_t q = g.te_soff[j]; q < g.te_soff[j + 1]; ++q) {
        const int e = g.te_sidx[q];
        const int p = g.te_pair[e];
        const int i = g.pair_i[p], jj = g.pair_j[p];
        const int kf = g.te_face[e] >> 1;
        const int na = g.nb[(size_t)jj * 4 + kf];
        const int nx = g.D == 2 ? g.nb[(size_t)i * 4 + (1 - kf)] * g.nb[(size_t)jj * 4 + (1 - kf)] : 1;
        const int nbj1 = g.D == 2 ? g.nb[(size_t)jj * 4 + 1] : 1;
        int32_t* d = &h->te_sdesc[(size_t)q * swr::kTxDesc];
        d[0] = e;
        d[1] = kf;
        d[2] = na;                                                       // sender normal size
        d[3] = g.D == 2 ? g.nb[(size_t)jj * 4 + (1 - kf)] : 1;           // sender tangential
        d[4] = g.D == 2 ? g.nb[(size_t)i * 4 + (1 - kf)] : 1;            // receiver tangential
        d[5] = (g.D == 2 && kf == 0) ? nbj1 : 1;                         // stride of m_k
        d[6] = (g.D == 2 && kf == 1) ? nbj1 : 1;                         // stride of m_t
        d[7] = (int32_t)(b / 16);                                        // a in the blob
        b += 16 * (na + (nx + 1) / 2);
      }
      h->te_max_send = std::max<int>(h->te_max_send, (int)(g.te_soff[j + 1] - g.te_soff[j]));
      h->te_pieces = std::max(h->te_pieces, b);
      h->te_blob_off[j + 1] = h->te_blob_off[j] + b / 16;
      h->te_max_recv = std::max<int>(h->te_max_recv, (int)(g.te_off[j + 1] - g.te_off[j]));
    }
    // factored face Gram pieces and the node run of every face
    h->te_gram_off.assign(g.n_items + 1, 0);
    h->te_fnode.assign((size_t)g.n_items * 16, 0);
    for (int j = 0; j < g.n_items; ++j) {
      int64_t n = 0;
      for (int f = 0; f < 2 * g.D; ++f) {
        const int kf = f >> 1;
        const int nt = g.D == 2 ? g.nb[(size_t)j * 4 + (1 - kf)] : 1;
        n += g.nb[(size_t)j * 4 + kf] + nt * nt;
      }
      n += n & 1;
      h->te_gram_off[j + 1] = h->te_gram_off[j] + n;
      h->te_gram_max = std::max<int64_t>(h->te_gram_max, 8 * n);
      for (int64_t q = g.node_off[j]; q < g.node_off[j + 1]; ++q) {
        const int f = g.nodes[q].face;
        int64_t* r = &h->te_fnode[((size_t)j * 8 + f) * 2];
        if (r[1] == 0) r[0] = q;
        ++r[1];
      }
    }
    h->tx_tt = swr::transmit_tile_steps(h->nbt, h->te_pieces, h->te_max_send, h->te_gram_max);
    h->tx_tt_max = h->tx_tt;
    if (h->wide)
      h->tx_tt = 16;  // the wide path has a transmission of its own
    else if (h->te_max_recv > 64 || h->te_max_send > 64 || h->tx_tt == 0)
      g.te_ok = false;  // dense fallback
  }
  // residual partials for the smallest tile, so that either tile may be used
  if (g.te_ok && !h->wide) h->part_stride = parts_needed(h, h->depth, 16);
  h->depth_run = h->depth;
  plan_layout(h);
  *out = h;
  return SWR_OK;
}

void swr_destroy(swr_handle h) { delete h; }

const char* swr_last_error(swr_handle h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

int32_t swr_query(swr_handle h, swr_info* info) {
  if (!h || !info) return fail(h, SWR_E_ARG, "null argument");
  swr_info r{};
  r.D = h->g.D;
  r.n_sub = h->g.n_sub;
  r.n_items = h->g.n_items;
  r.K_max = h->g.K_max;
  r.sum_K = h->sum_K;
  r.sum_K2 = h->sum_K2;
  r.n_face_nodes = (int64_t)h->g.nodes.size();
  r.n_pairs = (int64_t)h->g.pair_i.size();
  r.depth = h->depth;
  r.learned_nodes = h->n_nodes_t;
  r.factor_terms = h->factor_terms;
  r.tx_tile = h->block ? 0 : h->wide ? h->wide_tile : (h->g.te_ok ? h->tx_tt : 0);
  r.wide_order = h->wide_order;
  r.tuned = h->tuned_cached ? 1 : 0;
  r.rec_series = h->rec_series ? 1 : 0;
  r.wide = h->wide ? 1 : 0;
  r.block = h->block ? 1 : 0;
  r.depth_run = h->depth_run;
  r.sum_KK_pairs = h->g.pair_toff.back();
  r.n_steps = (int32_t)h->n_T;
  r.workspace_bytes = h->lay.total;
  *info = r;
  return SWR_OK;
}

int32_t swr_workspace_bytes(swr_handle h, uint64_t* bytes) {
  if (!h || !bytes) return fail(h, SWR_E_ARG, "null argument");
  *bytes = h->lay.total;
  return SWR_OK;
}

int32_t swr_bind_workspace(swr_handle h, void* dev, uint64_t bytes) {
  if (!h || !dev) return fail(h, SWR_E_ARG, "null argument");
  if (((uintptr_t)dev & 255) != 0) return fail(h, SWR_E_ARG, "workspace must be 256-byte aligned");
  if (bytes < h->lay.total) return fail(h, SWR_E_SIZE, "workspace smaller than swr_workspace_bytes");
  h->ws = (char*)dev;
  h->ws_bytes = bytes;
  h->bound = true;
  if (h->gexec) {  // its kernels hold addresses in the old workspace
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  h->assembled = h->initial = h->warm = h->factored = false;
  return SWR_OK;
}

namespace {
// Takes a schedule (tuning table or autotuner): depth, transmission tile and,
// on the wide path, the recurrence order (re-uploaded when it changes).
int32_t apply_schedule(swr_handle h, const TuneChoice& c, hipStream_t st) {
  h->g_kmax = -1;  // a captured window holds the old tile's kernels: capture again
  h->depth_run = std::max(1, std::min(c.depth, h->depth));
  if (h->wide) {
    h->wide_tile = (c.tile == 8 || c.tile == 32) ? c.tile : 16;
    const int order = c.order ? 1 : 0;
    if (order != h->wide_order) {
      h->wide_order = order;
      HIPCHECK(h, upload(h, h->bOrder, order ? h->order_natural : h->order, st));
    }
  } else if (h->g.te_ok) {
    h->tx_tt = (c.tile == 32 && h->tx_tt_max == 32) ? 32 : 16;
  }
  return SWR_OK;
}
}  // namespace

int32_t swr_assemble(swr_handle h, void* stream) {
  if (!h) return SWR_E_ARG;
  if (!h->bound) return fail(h, SWR_E_STATE, "no workspace bound");
  hipStream_t st = (hipStream_t)stream;
  if (h->block) return blk_assemble(h, st);
  const Geometry& g = h->g;
  const size_t NI = g.n_items;
  std::vector<int32_t> L4(4, 1);
  std::vector<double> eps4(4, 0.0), cen4(4, 0.0);
  for (int k = 0; k < g.D; ++k) {
    L4[k] = g.L[k];
    eps4[k] = g.eps[k];
    cen4[k] = g.desc.init_center[k];
  }
  std::vector<int32_t> nitem, nface, ncount, ncover;
  std::vector<double> nx, nw;
  for (const auto& n : g.nodes) {
    nitem.push_back(n.item);
    nface.push_back(n.face);
    ncount.push_back(n.count);
    for (int c = 0; c < swr::kMaxCover; ++c) ncover.push_back(n.cover[c]);
    for (int k = 0; k < 4; ++k) nx.push_back(n.x[k]);
    nw.push_back(n.w);
  }
  HIPCHECK(h, upload(h, h->bK, g.K, st));
  HIPCHECK(h, upload(h, h->bOff1, g.off1, st));
  HIPCHECK(h, upload(h, h->bOff2, g.off2, st));
  HIPCHECK(h, upload(h, h->bOffP, h->offp, st));
  HIPCHECK(h, upload(h, h->bIdx, g.idx, st));
  HIPCHECK(h, upload(h, h->bNb, g.nb, st));
  HIPCHECK(h, upload(h, h->bL, L4, st));
  HIPCHECK(h, upload(h, h->bLo, g.lo, st));
  HIPCHECK(h, upload(h, h->bHi, g.hi, st));
  HIPCHECK(h, upload(h, h->bEps, eps4, st));
  HIPCHECK(h, upload(h, h->bDelta, g.delta, st));
  HIPCHECK(h, upload(h, h->bAoff, g.aoff, st));
  HIPCHECK(h, upload(h, h->bAlpha, g.alpha, st));
  HIPCHECK(h, upload(h, h->bQoff, g.qoff, st));
  HIPCHECK(h, upload(h, h->bQn, g.qn, st));
  HIPCHECK(h, upload(h, h->bQx, g.qx, st));
  HIPCHECK(h, upload(h, h->bQw, g.qw, st));
  if (g.desc.basis_kind == SWR_BASIS_LSD) {
    HIPCHECK(h, upload(h, h->bLoQx, g.lo_qx, st));
    HIPCHECK(h, upload(h, h->bLoQw, g.lo_qw, st));
    HIPCHECK(h, upload(h, h->bLoQoff, g.lo_qoff, st));
    HIPCHECK(h, upload(h, h->bLoMx, g.lo_mx, st));
    HIPCHECK(h, upload(h, h->bLoMw, g.lo_mw, st));
  }
  if (g.desc.basis_kind == SWR_BASIS_LO) {
    HIPCHECK(h, upload(h, h->bLoQx, g.lo_qx, st));
    HIPCHECK(h, upload(h, h->bLoQw, g.lo_qw, st));
    HIPCHECK(h, upload(h, h->bLoQoff, g.lo_qoff, st));
    HIPCHECK(h, upload(h, h->bLoAng, h->lo_ang, st));
    HIPCHECK(h, upload(h, h->bKG, h->lo_kg, st));
    HIPCHECK(h, upload(h, h->bOff2G, h->lo_off2g, st));
  }
  HIPCHECK(h, upload(h, h->bNItem, nitem, st));
  HIPCHECK(h, upload(h, h->bNFace, nface, st));
  HIPCHECK(h, upload(h, h->bNCount, ncount, st));
  HIPCHECK(h, upload(h, h->bNCover, ncover, st));
  // barycentric Lagrange rows of the learned warm start's time nodes
  const int M = h->n_nodes_t;
  if (distinct_time_nodes((int)h->n_T, M)) {
    const std::vector<int> tn = time_nodes((int)h->n_T, M);
    std::vector<double> ts(M), wb(M);
    for (int m = 0; m < M; ++m) ts[m] = tn[m] * g.desc.dt;
    for (int m = 0; m < M; ++m) {
      double p = 1.0;
      for (int k2 = 0; k2 < M; ++k2)
        if (k2 != m) p *= ts[m] - ts[k2];
      wb[m] = 1.0 / p;
    }
    h->lag_host.assign((size_t)(h->n_T + 1) * M, 0.0);
    for (int64_t n = 0; n <= h->n_T; ++n) {
      const double tt = n * g.desc.dt;
      double* row = &h->lag_host[(size_t)n * M];
      int hit = -1;
      for (int m = 0; m < M; ++m)
        if (tt - ts[m] == 0.0) hit = m;
      if (hit >= 0) {
        row[hit] = 1.0;
      } else {
        double sum = 0.0;
        for (int m = 0; m < M; ++m) sum += (row[m] = wb[m] / (tt - ts[m]));
        for (int m = 0; m < M; ++m) row[m] /= sum;
      }
    }
    HIPCHECK(h, upload(h, h->bLag, h->lag_host, st));
  }
  HIPCHECK(h, upload(h, h->bNX, nx, st));
  HIPCHECK(h, upload(h, h->bNW, nw, st));
  HIPCHECK(h, upload(h, h->bNOff, g.node_off, st));
  HIPCHECK(h, upload(h, h->bPI, g.pair_i, st));
  HIPCHECK(h, upload(h, h->bPJ, g.pair_j, st));
  HIPCHECK(h, upload(h, h->bPOff, g.pair_off, st));
  HIPCHECK(h, upload(h, h->bTOff, g.pair_toff, st));
  HIPCHECK(h, upload(h, h->bPNode, g.pnode, st));
  HIPCHECK(h, upload(h, h->bPNOff, g.pnode_off, st));
  if (g.te_ok) {
    HIPCHECK(h, upload(h, h->bTePair, g.te_pair, st));
    HIPCHECK(h, upload(h, h->bTeFace, g.te_face, st));
    HIPCHECK(h, upload(h, h->bTeT0, g.te_t0, st));
    HIPCHECK(h, upload(h, h->bTeT1, g.te_t1, st));
    HIPCHECK(h, upload(h, h->bTeOff, g.te_off, st));
    HIPCHECK(h, upload(h, h->bTeBoff, g.te_boff, st));
    HIPCHECK(h, upload(h, h->bTeAoff, g.te_aoff, st));
    HIPCHECK(h, upload(h, h->bTeXoff, g.te_xoff, st));
    HIPCHECK(h, upload(h, h->bTeSoff, g.te_soff, st));
    HIPCHECK(h, upload(h, h->bTeSidx, g.te_sidx, st));
    HIPCHECK(h, upload(h, h->bTeBlobOff, h->te_blob_off, st));
    HIPCHECK(h, upload(h, h->bTeSdesc, h->te_sdesc, st));
    HIPCHECK(h, upload(h, h->bTeGramOff, h->te_gram_off, st));
    HIPCHECK(h, upload(h, h->bTeFnode, h->te_fnode, st));
  }
  HIPCHECK(h, upload(h, h->bPos, g.nuc_pos, st));
  HIPCHECK(h, upload(h, h->bCharge, g.nuc_charge, st));
  HIPCHECK(h, upload(h, h->bS1Off, h->s1off, st));
  HIPCHECK(h, upload(h, h->bScrOff, h->scratch_off, st));
  HIPCHECK(h, upload(h, h->bCenter, cen4, st));
  if (h->wide) {
    HIPCHECK(h, upload(h, h->bOrder, h->wide_order ? h->order_natural : h->order, st));
    HIPCHECK(h, upload(h, h->bTileOff, h->tile_off, st));
  }
  HIPCHECK(h, hipMemsetAsync(h->ptr<int>(h->bFlags), 0, 8, st));

  const swr::Items it = h->items();
  const swr::Nodes nd = h->nodes();
  const swr::Pairs pr = h->pairs();
  swr::Potential pot{g.desc.n_nuc, h->ptr<double>(h->bPos), h->ptr<double>(h->bCharge),
                     g.desc.eps_en, g.desc.eps_ee};
  const bool lsd = g.desc.basis_kind == SWR_BASIS_LSD;
  const bool lo = g.desc.basis_kind == SWR_BASIS_LO;
  const bool slater = g.desc.basis_kind == SWR_BASIS_SLATER || lsd;
  if (lsd) {
    // Section 3: the local orbitals of every interval, then the items'
    // one-dimensional orbital integrals (slater.hip)
    const int order = g.desc.lsd_moll_order;
    double sig = 1.0;  // sigma_M = (2M+1)! / (2^(2M+1) (M!)^2)
    for (int j = 1; j <= order; ++j) sig *= (2.0 * j + 1.0) / (2.0 * j);
    sig *= 0.5;
    const swr::LoParams lp{g.desc.lsd_barrier, g.desc.lsd_barrier_width, g.desc.lsd_v_inf,
                           g.desc.lsd_moll_eps, sig, order, g.desc.lsd_orbitals};
    HIPCHECK(h, swr::launch_lo_orbitals(it, g.L[0], pot, lp, h->ptr<double>(h->bLoQx),
                                        h->ptr<double>(h->bLoQw), h->ptr<int64_t>(h->bLoQoff),
                                        h->ptr<double>(h->bLoMx), h->ptr<double>(h->bLoMw),
                                        (int)g.lo_mx.size(), h->ptr<double>(h->bLoC),
                                        h->ptr<int>(h->bFlags), st));
    HIPCHECK(h, swr::launch_lo_tables(it, h->ptr<double>(h->bLoTab), st));
  }
  if (slater) {
    // Section 2 eq. (LSD): the antisymmetrised pairs (slater.hip)
    HIPCHECK(h, swr::launch_slater_assemble(it, h->ptr<double>(h->bA), h->ptr<double>(h->bKin),
                                            h->ptr<double>(h->bQ), h->ptr<double>(h->bB),
                                            h->ptr<double>(h->bW), g.K_max, st));
    int n_max = 1, q_max = 1;
    for (int s = 0; s < g.n_items; ++s) {
      n_max = std::max(n_max, lsd ? swr::lsd_functions(g.desc) : (int)g.nb[(size_t)s * 4]);
      q_max = std::max(q_max, (int)g.qn[(size_t)s * 4 + 1]);
    }
    HIPCHECK(h, swr::launch_slater_potential(it, pot, h->ptr<int64_t>(h->bScrOff),
                                             h->ptr<double>(h->bScr), n_max, q_max,
                                             h->ptr<double>(h->bV), g.K_max, st));
  } else if (lo) {
    // Section 3 in d = 2: the box's Gaussian matrices, its orbitals, then
    // every matrix as C^T (Gaussian matrix) C
    const swr::Items itg = h->items_gaussian();
    int kg_max = 1;
    for (const int k : h->lo_kg) kg_max = std::max(kg_max, k);
    HIPCHECK(h, swr::launch_assemble(itg, h->ptr<double>(h->bAG), h->ptr<double>(h->bKinG),
                                     h->ptr<double>(h->bQG), nullptr, h->ptr<double>(h->bBG),
                                     h->ptr<double>(h->bWG), h->ptr<double>(h->bS1),
                                     h->ptr<int64_t>(h->bS1Off), kg_max, st));
    HIPCHECK(h, swr::launch_potential(itg, pot, h->ptr<double>(h->bS1),
                                      h->ptr<int64_t>(h->bS1Off), h->ptr<double>(h->bVG),
                                      h->ptr<double>(h->bScr), h->ptr<int64_t>(h->bScrOff), st));
    const int order = g.desc.lsd_moll_order;
    const double e = g.desc.lsd_moll_eps;
    // 2 sigma 2^(2M+1) (M!)^2 / ((2M+1)! eps^(2M+2)), sigma = (M+1) / pi, and
    // 2^(2M+1) (M!)^2 / (2M+1)! = 2 prod_{j <= M} 2j / (2j + 1)
    double pref = 2.0 * (order + 1) / 3.14159265358979323846 * 2.0;
    for (int j = 1; j <= order; ++j) pref *= (2.0 * j) / (2.0 * j + 1.0);
    pref /= std::pow(e, 2 * order + 2);
    int64_t nq1 = 1;
    for (int s = 0; s < g.n_items; ++s)
      nq1 = std::max(nq1, g.lo_qoff[2 * s + 2] - g.lo_qoff[2 * s + 1]);
    const swr::LoParams lp{g.desc.lsd_barrier, g.desc.lsd_barrier_width, g.desc.lsd_v_inf, e,
                           pref, order, g.desc.lsd_orbitals};
    HIPCHECK(h, swr::launch_lo2_orbitals(it, pot, lp, h->ptr<double>(h->bLoQx),
                                         h->ptr<double>(h->bLoQw), h->ptr<int64_t>(h->bLoQoff),
                                         h->ptr<double2>(h->bLoAng), (int)g.lo_mx.size(), nq1,
                                         h->ptr<double>(h->bLoGt), h->ptr<double>(h->bLoTab),
                                         h->ptr<double>(h->bLoPP), h->ptr<double>(h->bLoC),
                                         h->ptr<int>(h->bFlags), st));
    const int64_t* og = h->ptr<int64_t>(h->bOff2G);
    const std::pair<Buf, Buf> mats[] = {{h->bAG, h->bA},   {h->bKinG, h->bKin}, {h->bVG, h->bV},
                                        {h->bQG, h->bQ},   {h->bBG, h->bB},     {h->bWG, h->bW}};
    for (const auto& m : mats)
      HIPCHECK(h, swr::launch_lo2_transform(it, og, h->ptr<double>(m.first),
                                            h->ptr<double>(m.second), st));
  } else {
    HIPCHECK(h, swr::launch_assemble(it, h->ptr<double>(h->bA), h->ptr<double>(h->bKin),
                                     h->ptr<double>(h->bQ), it.Q2 ? h->ptr<double>(h->bQ2) : nullptr,
                                     h->ptr<double>(h->bB), h->ptr<double>(h->bW),
                                     h->ptr<double>(h->bS1),
                                     h->ptr<int64_t>(h->bS1Off), g.K_max, st));
  }
  if (slater || lo) {
    // V assembled above
  } else if (h->wide)
    HIPCHECK(h, swr::launch_potential_wide(it, pot, h->ptr<double>(h->bV), g.K_max, st));
  else
    HIPCHECK(h, swr::launch_potential(it, pot, h->ptr<double>(h->bS1),
                                      h->ptr<int64_t>(h->bS1Off), h->ptr<double>(h->bV),
                                      h->ptr<double>(h->bScr), h->ptr<int64_t>(h->bScrOff), st));
  const double dt = g.desc.dt;
  const int tise = g.desc.mode == SWR_TISE;
  HIPCHECK(h, swr::launch_cn_matrices(h->sum_K2, h->ptr<double>(h->bA), h->ptr<double>(h->bKin),
                                      h->ptr<double>(h->bV), h->ptr<double>(h->bB), 0.5 * dt,
                                      g.desc.mu_re, g.desc.mu_im, h->ptr<double>(h->bAr),
                                      h->ptr<double>(h->bAp), h->ptr<double>(h->bHr), tise, dt, st));
  if (h->wide) {
    HIPCHECK(h, swr::launch_add_wide(h->sum_K2, h->ptr<double>(h->bAr), h->ptr<double>(h->bAp),
                                     h->ptr<double>(h->bScrW), st));
    HIPCHECK(h, swr::launch_pack_wide(it, h->ptr<double>(h->bScrW), h->ptr<double>(h->bS2P), st));
  }
  if (g.te_ok) {
    const swr::TEnt te = h->te();
    HIPCHECK(h, swr::launch_transfer_tensor(it, nd, pr, te, g.desc.mu_re, g.desc.mu_im,
                                            h->ptr<double>(h->bTeBeta), h->ptr<double2>(h->bTeA),
                                            h->ptr<double>(h->bTeX), st));
    HIPCHECK(h, swr::launch_tx_pack(it, pr, te, h->ptr<double2>(h->bTeBlob), st));
    HIPCHECK(h, swr::launch_gram_tensor(it, nd, te, h->ptr<double>(h->bTeGram), st));
  } else {
    HIPCHECK(h, swr::launch_transfer(it, nd, pr, g.desc.mu_re, g.desc.mu_im,
                                     h->ptr<double2>(h->bT), g.K_max, st));
  }
  HIPCHECK(h, swr::launch_face_gram(it, nd, h->ptr<double>(h->bG), g.K_max, st));
  // the uploads above read host vectors local to this call
  HIPCHECK(h, hipStreamSynchronize(st));
  if (lsd || lo) {
    // the determinants' (orbitals') Gram matrices A against the same limit
    // as the tensor bases' at swr_create
    std::vector<double> A(h->sum_K2);
    HIPCHECK(h, hipMemcpy(A.data(), h->ptr<double>(h->bA), h->sum_K2 * 8, hipMemcpyDeviceToHost));
    double worst = 1.0;
    for (int s = 0; s < g.n_items; ++s) {
      const double c = spd_condition(&A[g.off2[s]], g.K[s]);
      worst = std::isnan(c) ? c : std::max(worst, c);
    }
    if (!(worst <= kCondLimit)) {
      char buf[240];
      std::snprintf(buf, sizeof buf,
                    "a subdomain's %s Gram matrix has condition %.3g, above the %.0e "
                    "the stored-inverse recurrence keeps to 1e-10 (fewer orbitals or added "
                    "Gaussians, or wider overlaps)", lo ? "orbital" : "determinant", worst,
                    kCondLimit);
      return fail(h, worst <= kSingularLimit ? SWR_E_COND : SWR_E_SINGULAR, buf);
    }
  }
  h->assembled = true;
  h->initial = h->warm = h->factored = false;
  // a schedule measured earlier for this kind of problem
  TuneChoice c;
  if (tune_lookup(tune_key(h), &c)) {
    const int rc = apply_schedule(h, c, st);
    if (rc) return rc;
    h->tuned_cached = true;
  }
  return SWR_OK;
}

int32_t swr_set_initial(swr_handle h, const void* c0_dev, void* stream) {
  if (!h) return SWR_E_ARG;
  if (!h->assembled) return fail(h, SWR_E_STATE, "swr_assemble first");
  hipStream_t st = (hipStream_t)stream;
  if (h->block) return blk_set_initial(h, c0_dev, st);
  const swr::Items it = h->items();
  if (c0_dev) {
    HIPCHECK(h, hipMemcpyAsync(h->ptr<double2>(h->bC0), c0_dev, h->sum_K * 16,
                               hipMemcpyDeviceToDevice, st));
  } else if (h->wide) {
    HIPCHECK(h, swr::launch_project_wide(it, h->ptr<double>(h->bA), h->g.desc.init_alpha,
                                         h->ptr<double>(h->bCenter), h->ptr<double>(h->bScrW),
                                         h->ptr<double2>(h->bC0), h->ptr<int>(h->bFlags), st));
  } else {
    if (it.slater)
      HIPCHECK(h, swr::launch_slater_project(it, h->ptr<double>(h->bA), h->g.desc.init_alpha,
                                             h->ptr<double>(h->bCenter), h->ptr<double2>(h->bC0),
                                             h->ptr<int>(h->bFlags), st));
    else
      HIPCHECK(h, swr::launch_project(it, h->ptr<double>(h->bA), h->g.desc.init_alpha,
                                      h->ptr<double>(h->bCenter), h->ptr<double2>(h->bC0),
                                      h->ptr<int>(h->bFlags), st));
  }
  if (h->g.desc.mode == SWR_TISE && !h->g.desc.unnormalized)
    HIPCHECK(h, swr::launch_global_normalise(it, h->ptr<double>(h->bW), h->ptr<double2>(h->bC0),
                                             h->iepart_of(0), st));
  h->initial = true;
  int rc = swr_warm_start(h, SWR_WARM_PLAIN, nullptr, stream);
  return rc;
}

namespace {

// one job over the whole window: Robin data of iterate k+1 from iterate k
swr::TxJobs full_tx(const double2* src, double2* dst, int n_T) {
  swr::TxJobs j{};
  j.n = 1;
  j.src[0] = src;
  j.dst[0] = dst;
  j.n_lo[0] = 0;
  j.n_hi[0] = n_T;
  return j;
}

}  // namespace

int32_t swr_warm_start(swr_handle h, int32_t mode, const void* g_dev, void* stream) {
  if (!h) return SWR_E_ARG;
  if (!h->initial) return fail(h, SWR_E_STATE, "swr_set_initial first");
  if (mode == SWR_WARM_GIVEN && !g_dev) return fail(h, SWR_E_ARG, "GIVEN warm start needs g_dev");
  if (mode != SWR_WARM_PLAIN && mode != SWR_WARM_ZERO && mode != SWR_WARM_GIVEN)
    return fail(h, SWR_E_ARG, "unknown warm start mode");
  hipStream_t st = (hipStream_t)stream;
  if (h->block) return blk_warm_start(h, mode, st);
  const swr::Items it = h->items();
  const int nT = (int)h->n_T;
  // iterate 0 (residual reference) = the window's initial state held constant
  HIPCHECK(h, swr::launch_fill_history(it, nT, h->ptr<double2>(h->bC0), h->hist_of(0), st));
  double2* F = h->F_of(1);
  if (mode == SWR_WARM_PLAIN && h->wide) {
    HIPCHECK(h, swr::launch_tx_wide(it, h->pairs(), h->te(), nT, h->hist_of(0), F, nullptr,
                                    nullptr, h->g.desc.dt, h->wide_tile, st));
  } else if (mode == SWR_WARM_PLAIN) {
    HIPCHECK(h, swr::launch_transmit(it, h->pairs(), h->te(), nT, h->ptr<double2>(h->bT),
                                     full_tx(h->hist_of(0), F, nT), h->nbt,
                                     h->te_pieces, h->te_max_recv, h->te_max_send,
                                     h->te_gram_max, h->tx_tt, st));
  } else if (mode == SWR_WARM_ZERO) {
    HIPCHECK(h, hipMemsetAsync(F, 0, h->bF[0].bytes, st));
  } else {
    HIPCHECK(h, swr::launch_forcing_from_nodes(it, h->nodes(), nT, (const double2*)g_dev, F, st));
  }
  h->cur = 0;
  h->k = 0;
  h->warm = true;
  return SWR_OK;
}

int32_t swr_factor(swr_handle h, double t0, void* stream) {
  if (!h) return SWR_E_ARG;
  if (!h->assembled) return fail(h, SWR_E_STATE, "swr_assemble first");
  hipStream_t st = (hipStream_t)stream;
  if (h->block) return blk_factor(h, t0, st);
  // the previous upload of the field table must have been consumed
  HIPCHECK(h, hipStreamSynchronize(st));
  h->E_host.assign(h->n_T + 1, 0.0);
  for (int64_t n = 0; n <= h->n_T; ++n) h->E_host[n] = field(h->g.desc, t0 + n * h->g.desc.dt);
  HIPCHECK(h, upload(h, h->bE, h->E_host, st));
  const bool circular = h->g.desc.field_shape == SWR_FIELD_CIRCULAR;
  if (circular) {
    h->E2_host.assign(h->n_T + 1, 0.0);
    for (int64_t n = 0; n <= h->n_T; ++n)
      h->E2_host[n] = field2(h->g.desc, t0 + n * h->g.desc.dt);
    HIPCHECK(h, upload(h, h->bE2, h->E2_host, st));
  }
  const int tise = h->g.desc.mode == SWR_TISE;
  const double tau = 0.5 * h->g.desc.dt;
  // series around the midpoint of each chunk's field range (TDSE)
  int terms = 0;
  const int n_chunks = (int)((h->n_mats + swr::kSeriesChunk - 1) / swr::kSeriesChunk);
  const int max_terms = h->wide ? swr::kWideTerms : kSeriesMaxTerms;
  if (!tise && !circular && (h->g.desc.factor_mode == SWR_FACTOR_AUTO || h->wide) &&
      h->g.desc.mu_im <= 0.0) {
    h->Ea_host.assign(n_chunks, 0.0);
    double half = 0.0;
    for (int c = 0; c < n_chunks; ++c) {
      const int64_t n0 = (int64_t)c * swr::kSeriesChunk;
      const int64_t n1 = std::min<int64_t>(n0 + swr::kSeriesChunk, h->n_mats);
      double lo = h->E_host[n0 + 1], hi = lo;
      for (int64_t n = n0; n < n1; ++n) {
        lo = std::min(lo, h->E_host[n + 1]);
        hi = std::max(hi, h->E_host[n + 1]);
      }
      h->Ea_host[c] = 0.5 * (lo + hi);
      half = std::max(half, 0.5 * (hi - lo));
    }
    // least K with rho^{K+1} / (1 - rho) <= 2^-53, as a number of terms K + 1
    // (0: more than max_terms)
    auto terms_for = [&](double rho) {
      if (!(rho < 0.5)) return 0;
      int t = 1;
      for (double tail = rho / (1.0 - rho); tail > 0x1p-53 && t <= max_terms; ++t) tail *= rho;
      return t > max_terms ? 0 : t;
    };
    terms = terms_for(tau * half * h->dipole_max);
    if (h->wide && terms > 0) {
      // the bound holds item by item with the item's own dipole extent
      h->terms_item.resize(h->g.n_items);
      for (int q = 0; q < h->g.n_items; ++q)
        h->terms_item[q] = std::max(1, terms_for(tau * half * h->dipole[q]));
    }
  }
  const swr::Items it = h->items();
  if (h->wide && terms == 0)
    return fail(h, SWR_E_SIZE, "the field varies too much within a chunk for the wide-basis "
                               "series (more than 6 terms)");
  if (terms > 0) HIPCHECK(h, upload(h, h->bEanchor, h->Ea_host, st));
  if (!h->wide && terms > 0 && terms <= swr::kRecSeriesMax) {
    // the offsets of the series evaluated in the step, rounded as the
    // assembly of the inverses rounds them
    h->D_host.resize(h->n_mats);
    for (int64_t n = 0; n < h->n_mats; ++n)
      h->D_host[n] = h->Ea_host[n / swr::kSeriesChunk] - h->E_host[n + 1];
    HIPCHECK(h, upload(h, h->bDser, h->D_host, st));
  }
  if (h->wide) HIPCHECK(h, upload(h, h->bTermsW, h->terms_item, st));
  HIPCHECK(h, tbegin(h, st, kTFactor));
  if (h->wide) {
    // per chunk: X = M_c^{-1} (Gauss-Jordan), R = I - M_c X (compensated),
    // P_0 = X + X R, G = i tau P_0 Q, P_k = G P_{k-1}
    const int64_t cstride = (int64_t)kWideSlots * h->sum_K2;
    double2* G = h->ptr<double2>(h->bSeries);
    double2* X = G + h->sum_K2;
    double2* P = G + 2 * h->sum_K2;
    const int64_t nt = h->tile_off.back();
    const int64_t* toff = h->ptr<int64_t>(h->bTileOff);
    const double* Ea = h->ptr<double>(h->bEanchor);
    HIPCHECK(h, swr::launch_invert_wide(it, n_chunks, h->ptr<double>(h->bAr),
                                        h->ptr<double>(h->bHr), h->ptr<double>(h->bQ), Ea, tau, X,
                                        cstride, h->ptr<int>(h->bFlags), st));
    HIPCHECK(h, swr::launch_residual_wide(it, toff, nt, n_chunks, h->ptr<double>(h->bAr),
                                          h->ptr<double>(h->bHr), h->ptr<double>(h->bQ), Ea, tau,
                                          X, cstride, G, st));
    HIPCHECK(h, swr::launch_gemm_wide(it, toff, nt, n_chunks, X, G, nullptr,
                                      make_double2(1.0, 0.0), X, cstride, P, st));
    if (terms > 1)
      HIPCHECK(h, swr::launch_gemm_wide(it, toff, nt, n_chunks, P, nullptr, h->ptr<double>(h->bQ),
                                        make_double2(0.0, tau), nullptr, cstride, G, st));
    for (int k = 1; k < terms; ++k)
      HIPCHECK(h, swr::launch_gemm_wide(it, toff, nt, n_chunks, G, P + (k - 1) * h->sum_K2,
                                        nullptr, make_double2(1.0, 0.0), nullptr, cstride,
                                        P + k * h->sum_K2, st));
    const int64_t np = h->offp.back();
    HIPCHECK(h, swr::launch_pack_wide(it, n_chunks, terms, P, cstride, h->sum_K2,
                                      h->ptr<double2>(h->bSeriesP), swr::kWideTerms * np, np, st));
  } else if (terms > 0) {
    const int64_t cstride = (int64_t)(kSeriesMaxTerms + 1) * h->sum_K2;
    double2* G = h->ptr<double2>(h->bSeries);
    double2* P = G + h->sum_K2;  // chunk c: P_k at P + c cstride + k sum_K2
    HIPCHECK(h, swr::launch_invert(it, n_chunks, h->ptr<double>(h->bAr), h->ptr<double>(h->bHr),
                                   h->ptr<double>(h->bQ), h->ptr<double>(h->bEanchor), cstride,
                                   tau, 2, P, h->ptr<int>(h->bFlags), st, h->g.K_max));
    // one refinement step of each anchor inverse: R = I - M_c P_0 (in the G
    // slot), P_0 += P_0 R
    HIPCHECK(h, swr::launch_series_residual(it, n_chunks, h->ptr<double>(h->bAr),
                                            h->ptr<double>(h->bHr), h->ptr<double>(h->bQ),
                                            h->ptr<double>(h->bEanchor), tau, P, cstride, G, st));
    HIPCHECK(h, swr::launch_series_product(it, n_chunks, P, G, nullptr, make_double2(1.0, 0.0), P,
                                           cstride, P, st));
    if (terms > 1)
      HIPCHECK(h, swr::launch_series_product(it, n_chunks, P, nullptr, h->ptr<double>(h->bQ),
                                             make_double2(0.0, tau), nullptr, cstride, G, st));
    for (int k = 1; k < terms; ++k)
      HIPCHECK(h, swr::launch_series_product(it, n_chunks, G, P + (k - 1) * h->sum_K2, nullptr,
                                             make_double2(1.0, 0.0), nullptr, cstride,
                                             P + k * h->sum_K2, st));
    if (terms > swr::kRecSeriesMax)
      HIPCHECK(h, swr::launch_series_assemble(it, h->n_mats, terms, P, h->sum_K2, cstride,
                                              h->ptr<double>(h->bE),
                                              h->ptr<double>(h->bEanchor),
                                              h->ptr<double2>(h->bMinv), st));
  } else {
    HIPCHECK(h, swr::launch_invert(it, h->n_mats, h->ptr<double>(h->bAr), h->ptr<double>(h->bHr),
                                   h->ptr<double>(h->bQ), h->ptr<double>(h->bE), 0, tau,
                                   tise ? 1 : 0, h->ptr<double2>(h->bMinv),
                                   h->ptr<int>(h->bFlags), st, h->g.K_max));
  }
  HIPCHECK(h, tend(h, st));
  h->factor_terms = terms - 1;
  h->rec_series = !h->wide && terms > 0 && terms <= swr::kRecSeriesMax;
  h->factored = true;
  h->t0 = t0;
  return SWR_OK;
}

int32_t swr_sweep(swr_handle h, void* stream) {
  if (!h) return SWR_E_ARG;
  if (!h->factored) return fail(h, SWR_E_STATE, "swr_factor first");
  if (!h->warm) return fail(h, SWR_E_STATE, "swr_warm_start (or swr_set_initial) first");
  hipStream_t st = (hipStream_t)stream;
  if (h->block) {
    // one iterate, its transmission and its residual (swr_transmit reports it)
    swr_run_stats s{};
    bool stop = false;
    const int rc = blk_batch(h, h->blk_k + 1, 1, -1.0, st, &s, &stop);
    if (rc) return rc;
    return check_flags(h, st);
  }
  const swr::Items it = h->items();
  const int k = h->k + 1;
  const int nT = (int)h->n_T;
  double2* hist = h->hist_of(k);
  if (h->wide) {
    const int64_t np = h->offp.back();
    HIPCHECK(h, tbegin(h, st, kTRecur));
    HIPCHECK(h, swr::launch_cn_recur_wide(
                    it, h->ptr<int32_t>(h->bOrder), nT, h->ptr<double>(h->bS2P),
                    h->ptr<double>(h->bAr), h->ptr<double>(h->bHr), h->ptr<double>(h->bQ),
                    h->ptr<double>(h->bE), h->ptr<double>(h->bEanchor), 0.5 * h->g.desc.dt,
                    h->ptr<double2>(h->bSeriesP), h->ptr<int32_t>(h->bTermsW), np,
                    (int64_t)swr::kWideTerms * np, h->ptr<double2>(h->bC0), hist, h->F_of(k),
                    h->ptr<int>(h->bFlags), st));
    HIPCHECK(h, tend(h, st));
  } else if (h->g.desc.mode == SWR_TDSE) {
    swr::RecJobs jobs{};
    jobs.n = 1;
    jobs.hist[0] = hist;
    jobs.F[0] = h->F_of(k);
    jobs.n_lo[0] = 0;
    jobs.n_cnt[0] = nT;
    HIPCHECK(h, tbegin(h, st, kTRecur));
    const swr::RecSeries se = h->rec_se();
    HIPCHECK(h, swr::launch_cn_recur(it, nT, h->ptr<double>(h->bAr), h->ptr<double>(h->bAp),
                                     h->ptr<double>(h->bHr), h->ptr<double>(h->bQ),
                                     h->ptr<double>(h->bE), 0.5 * h->g.desc.dt,
                                     h->ptr<double2>(h->bMinv), h->rec_series ? &se : nullptr,
                                     h->ptr<double2>(h->bC0), jobs, h->ptr<int>(h->bFlags), st));
    HIPCHECK(h, tend(h, st));
  } else {
    // step 0 of every item is the (normalised) initial state
    HIPCHECK(h, swr::launch_fill_history(it, nT, h->ptr<double2>(h->bC0), hist, st));
    const int norm = h->g.desc.unnormalized ? 0 : 1;
    HIPCHECK(h, tbegin(h, st, kTRecur));  // the sweep's n_T step launches
    swr::IeJobs jobs{};
    jobs.n = 1;
    jobs.hist[0] = hist;
    jobs.F[0] = h->F_of(k);
    jobs.partial[0] = h->iepart_of(k);
    jobs.nus[0] = h->nus_of(k);
    for (int n = 0; n < nT; ++n) {
      jobs.step[0] = n;
      HIPCHECK(h, swr::launch_ie_step(it, jobs, nT, h->g.desc.dt, h->ptr<double>(h->bA),
                                      h->ptr<double>(h->bW), h->ptr<double2>(h->bMinv), norm,
                                      h->ptr<int>(h->bFlags), st));
    }
    HIPCHECK(h, swr::launch_ie_finish(it, nT, hist, h->iepart_of(k), h->nus_of(k), norm, st));
    HIPCHECK(h, tend(h, st));
  }
  h->cur = k % h->n_slots;
  h->k = k;
  return SWR_OK;
}

namespace {

// Robin data of iterate k+1 from iterate k over the whole window, and the
// residual Res(k) against iterate k-1 into *res_dev (device).  The factored
// transmission computes the residual in the same pass; the dense one uses
// the face Gram matrices separately.
int32_t transmit_and_residual(swr_handle h, int k, const double* scale, double* res_dev,
                              hipStream_t st) {
  const swr::Items it = h->items();
  const int nT = (int)h->n_T;
  if (h->wide) {
    double* part = res_dev ? h->ptr<double>(h->bResPart) : nullptr;
    HIPCHECK(h, tbegin(h, st, kTTransmit));
    HIPCHECK(h, swr::launch_tx_wide(it, h->pairs(), h->te(), nT, h->hist_of(k), h->F_of(k + 1),
                                    res_dev ? h->hist_of(k - 1) : nullptr, part,
                                    h->g.desc.dt, h->wide_tile, st));
    if (res_dev)
      HIPCHECK(h, swr::launch_sum_sqrt(part,
                                       (int64_t)it.n_items * swr::tx_wide_tiles(nT, h->wide_tile),
                                       res_dev, st));
    HIPCHECK(h, tend(h, st));
    (void)scale;
    return SWR_OK;
  }
  swr::TxJobs tx = full_tx(h->hist_of(k), h->F_of(k + 1), nT);
  tx.scale[0] = scale;
  tx.dt = h->g.desc.dt;
  tx.part_stride = h->part_stride;
  if (h->fused_residual() && res_dev) {
    tx.prev[0] = h->hist_of(k - 1);
    tx.part[0] = h->parts_of(k);
    tx.part_base[0] = 0;
  } else if (res_dev) {
    HIPCHECK(h, tbegin(h, st, kTResidual));
    HIPCHECK(h, swr::launch_residual(it, nT, h->g.desc.dt, h->ptr<double>(h->bG), h->hist_of(k),
                                     h->hist_of(k - 1), h->ptr<double>(h->bResPart), res_dev, st));
    HIPCHECK(h, tend(h, st));
  }
  HIPCHECK(h, tbegin(h, st, kTTransmit));
  HIPCHECK(h, swr::launch_transmit(it, h->pairs(), h->te(), nT, h->ptr<double2>(h->bT), tx,
                                   h->nbt, h->te_pieces, h->te_max_recv, h->te_max_send,
                                   h->te_gram_max, h->tx_tt, st));
  if (h->fused_residual() && res_dev)
    HIPCHECK(h, swr::launch_res_reduce(h->parts_of(k), h->g.n_items, h->part_stride, nT, nT, 1,
                                       h->tx_tt, res_dev, st));
  HIPCHECK(h, tend(h, st));
  return SWR_OK;
}

}  // namespace

int32_t swr_transmit(swr_handle h, double* residual_host, void* stream) {
  if (!h) return SWR_E_ARG;
  if (h->block) {
    // the block path sends each iterate's Robin data during its own sweep
    if (h->blk_k < 1) return fail(h, SWR_E_STATE, "swr_sweep first");
    HIPCHECK(h, hipStreamSynchronize((hipStream_t)stream));
    if (residual_host) *residual_host = h->blk_last_res;
    return SWR_OK;
  }
  if (h->k < 1) return fail(h, SWR_E_STATE, "swr_sweep first");
  hipStream_t st = (hipStream_t)stream;
  const double* scale = h->g.desc.mode == SWR_TISE ? h->nus_of(h->k) : nullptr;
  int rc = transmit_and_residual(h, h->k, scale, h->ptr<double>(h->bResOut), st);
  if (rc) return rc;
  double res = 0.0;
  HIPCHECK(h, hipMemcpyAsync(&res, h->ptr<double>(h->bResOut), 8, hipMemcpyDeviceToHost, st));
  HIPCHECK(h, hipStreamSynchronize(st));
  rc = check_flags(h, st);
  if (rc != SWR_OK) return rc;
  if (residual_host) *residual_host = res;
  return SWR_OK;
}

namespace {

// Pipelined window (TDSE, depth P > 1).  Chunk c of the window holds the
// Crank-Nicolson steps [c S, min((c+1) S, n_T)).  Launch d advances every
// iterate k with c = d - (k - 1) in [0, n_chunks) by its chunk c: first the
// Robin data of iterate k on the chunk's steps from iterate k-1 (complete
// there since launch d-1) -- the same pass adds the chunk's share of the
// residual Res(k-1) -- then the recurrence of the chunk from the state the
// previous launch left at step c S.  Res(k-1) is complete once chunk
// n_chunks-1 of iterate k has been transmitted; it is reduced and copied to
// pinned host memory before that launch's recurrence, so the host reads it
// while the recurrence runs and never idles the GPU.
// capture: only enqueue (the stream is being captured into a graph): no host
// reads of the residuals, every iterate up to k_max, no flag check.
// Imaginary-time chunks of one pipelined launch: each job is a Schwarz
// iterate (rec_k) at its chunk [n_lo, n_lo + n_cnt); an iterate starting
// (n_lo = 0) gets the initial state in its history and factors of 1; then
// one launch per step for all jobs, and the final normalisation of the
// iterates that reach the window's end.
int32_t ie_chunks(swr_handle h, const swr::RecJobs& rec, const int* rec_k, int S, hipStream_t st) {
  const swr::Items it = h->items();
  const int nT = (int)h->n_T;
  const int norm = h->g.desc.unnormalized ? 0 : 1;
  for (int j = 0; j < rec.n; ++j)
    if (rec.n_lo[j] == 0) {
      HIPCHECK(h, swr::launch_fill_history(it, nT, h->ptr<double2>(h->bC0), rec.hist[j], st));
      HIPCHECK(h, swr::launch_fill_f64(h->nus_of(rec_k[j]), nT + 1, 1.0, st));
    }
  HIPCHECK(h, tbegin(h, st, kTRecur));
  for (int q = 0; q < S; ++q) {
    swr::IeJobs ie{};
    for (int j = 0; j < rec.n; ++j) {
      if (q >= rec.n_cnt[j]) continue;
      ie.hist[ie.n] = rec.hist[j];
      ie.F[ie.n] = rec.F[j];
      ie.partial[ie.n] = h->iepart_of(rec_k[j]);
      ie.nus[ie.n] = h->nus_of(rec_k[j]);
      ie.step[ie.n] = rec.n_lo[j] + q;
      ++ie.n;
    }
    if (ie.n == 0) break;
    HIPCHECK(h, swr::launch_ie_step(it, ie, nT, h->g.desc.dt, h->ptr<double>(h->bA),
                                    h->ptr<double>(h->bW), h->ptr<double2>(h->bMinv), norm,
                                    h->ptr<int>(h->bFlags), st));
  }
  for (int j = 0; j < rec.n; ++j)
    if (rec.n_lo[j] + rec.n_cnt[j] == nT)
      HIPCHECK(h, swr::launch_ie_finish(it, nT, rec.hist[j], h->iepart_of(rec_k[j]),
                                        h->nus_of(rec_k[j]), norm, st));
  HIPCHECK(h, tend(h, st));
  return SWR_OK;
}

int32_t run_pipelined(swr_handle h, const swr_run_opts* o, int P, swr_run_stats* out,
                      hipStream_t st, bool capture = false) {
  const swr::Items it = h->items();
  const int nT = (int)h->n_T;
  const int S = (nT + P - 1) / P;
  const int n_chunks = (nT + S - 1) / S;
  // Imaginary time: one launch per step, every iterate in flight in it; the
  // residual of an iterate is taken once it is complete (and normalised)
  const bool tise = h->g.desc.mode == SWR_TISE;
  const bool fused = h->fused_residual() && !tise;
  if (fused && parts_needed(h, P, h->tx_tt) > h->part_stride)
    return fail(h, SWR_E_SIZE, "residual partials exceed their buffer");
  if (!capture && !h->ev_ready) {
    for (auto& e : h->ev) HIPCHECK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->ev_ready = true;
  }
  if (!capture && !h->res_pinned)
    HIPCHECK(h, hipHostMalloc((void**)&h->res_pinned, 64 * sizeof(double), 0));
  swr_run_stats s{};
  int k_final = 0;
  auto queue_read = [&](int k) -> int {  // Res(k) (already in bResv) to the host
    if (capture) return SWR_OK;
    double* dev = h->ptr<double>(h->bResv) + k % 64;
    HIPCHECK(h, hipMemcpyAsync(h->res_pinned + k % 64, dev, 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(h, hipEventRecord(h->ev[k % kResEvents], st));
    return SWR_OK;
  };
  auto read = [&](int k) -> int {
    if (capture) return SWR_OK;
    HIPCHECK(h, hipEventSynchronize(h->ev[k % kResEvents]));
    const double r = h->res_pinned[k % 64];
    if (k <= 64) s.res[k - 1] = r;
    if (k >= 2 && r <= o->tol) {
      k_final = k;
      s.converged = 1;
    }
    if (h->growth.step(r) && k_final == 0) k_final = k;  // the caller falls back
    return SWR_OK;
  };
  int last_read = 0;
  for (int d = 0; k_final == 0; ++d) {
    swr::TxJobs tx{};
    tx.dt = h->g.desc.dt;
    tx.part_stride = h->part_stride;
    swr::RecJobs rec{};
    int rec_k[swr::kMaxJobs] = {};
    for (int k = std::max(1, d - n_chunks + 2); k <= std::min(d + 1, o->k_max); ++k) {
      const int c = d - (k - 1);
      const int lo = c * S, cnt = std::min(S, nT - lo), hi = lo + cnt;
      if (k >= 2) {
        tx.src[tx.n] = h->hist_of(k - 1);
        tx.dst[tx.n] = h->F_of(k);
        tx.n_lo[tx.n] = c == 0 ? 0 : lo + 1;
        tx.n_hi[tx.n] = hi;
        // imaginary time: the Robin data of the unnormalised states; step
        // hi of iterate k - 1 is normalised only by its next chunk, which
        // runs after this transmission, and its factor there is still 1
        tx.scale[tx.n] = tise ? h->nus_of(k - 1) : nullptr;
        if (fused) {
          tx.prev[tx.n] = h->hist_of(k - 2);
          tx.part[tx.n] = h->parts_of(k - 1);
          tx.part_base[tx.n] = c * ((S + 1 + h->tx_tt - 1) / h->tx_tt);
        }
        ++tx.n;
      }
      rec.hist[rec.n] = h->hist_of(k);
      rec.F[rec.n] = h->F_of(k);
      rec.carry[rec.n] = h->carry_of(k);
      rec.n_lo[rec.n] = lo;
      rec.n_cnt[rec.n] = cnt;
      rec_k[rec.n] = k;
      ++rec.n;
    }
    if (rec.n == 0) break;
    // Res(kr) is complete after this launch's transmission (fused), or its
    // iterate completed in the previous launch (dense residual kernel)
    const int kr = d - n_chunks + 1;
    const bool res_now = kr >= 1 && kr + 1 <= o->k_max;
    if (tx.n > 0) {
      HIPCHECK(h, tbegin(h, st, kTTransmit));
      HIPCHECK(h, swr::launch_transmit(it, h->pairs(), h->te(), nT, h->ptr<double2>(h->bT), tx,
                                       h->nbt, h->te_pieces, h->te_max_recv, h->te_max_send,
                                       h->te_gram_max, h->tx_tt, st));
      HIPCHECK(h, tend(h, st));
    }
    if (res_now) {
      double* dev = h->ptr<double>(h->bResv) + kr % 64;
      HIPCHECK(h, tbegin(h, st, kTResidual));
      if (fused)
        HIPCHECK(h, swr::launch_res_reduce(h->parts_of(kr), it.n_items, h->part_stride, nT, S,
                                           n_chunks, h->tx_tt, dev, st));
      else
        HIPCHECK(h, swr::launch_residual(it, nT, h->g.desc.dt, h->ptr<double>(h->bG),
                                         h->hist_of(kr), h->hist_of(kr - 1),
                                         h->ptr<double>(h->bResPart), dev, st));
      HIPCHECK(h, tend(h, st));
      const int rc = queue_read(kr);
      if (rc) return rc;
    }
    if (tise) {
      const int rc = ie_chunks(h, rec, rec_k, S, st);
      if (rc) return rc;
    } else {
      HIPCHECK(h, tbegin(h, st, kTRecur));
      const swr::RecSeries se = h->rec_se();
      HIPCHECK(h, swr::launch_cn_recur(it, nT, h->ptr<double>(h->bAr), h->ptr<double>(h->bAp),
                                       h->ptr<double>(h->bHr), h->ptr<double>(h->bQ),
                                       h->ptr<double>(h->bE), 0.5 * h->g.desc.dt,
                                       h->ptr<double2>(h->bMinv), h->rec_series ? &se : nullptr,
                                       h->ptr<double2>(h->bC0), rec, h->ptr<int>(h->bFlags),
                                       st));
      HIPCHECK(h, tend(h, st));
    }
    if (res_now) {
      const int rc = read(kr);
      if (rc) return rc;
      last_read = kr;
    }
  }
  // iterates not checked inside the loop (the last one needs a transmission
  // of its own: iterate k_max + 1 is never started)
  for (int k = last_read + 1; k_final == 0 && k <= o->k_max; ++k) {
    const int rc0 = transmit_and_residual(h, k, tise ? h->nus_of(k) : nullptr,
                                          h->ptr<double>(h->bResv) + k % 64, st);
    if (rc0) return rc0;
    int rc = queue_read(k);
    if (rc) return rc;
    rc = read(k);
    if (rc) return rc;
  }
  if (k_final == 0) k_final = o->k_max;
  s.iters = k_final;
  // state as after sweep + transmit of iterate k_final at depth 1
  h->k = k_final;
  h->cur = k_final % h->n_slots;
  const int rc0 = transmit_and_residual(h, k_final, tise ? h->nus_of(k_final) : nullptr, nullptr,
                                        st);
  if (rc0) return rc0;
  if (!capture) {
    const int rc = check_flags(h, st);
    if (rc != SWR_OK) return rc;
  }
  *out = s;
  return SWR_OK;
}

// One iterate at a time, launches only (captured into the window's graph at
// depth 1): every iterate's sweep, then its Robin data and Res(k) into the
// device residual ring; the host reads them after the window.
int32_t run_steps_launches(swr_handle h, const swr_run_opts* o, hipStream_t st) {
  for (int k = 1; k <= o->k_max; ++k) {
    int rc = swr_sweep(h, st);
    if (rc) return rc;
    rc = transmit_and_residual(h, k, nullptr, h->ptr<double>(h->bResv) + k % 64, st);
    if (rc) return rc;
  }
  return SWR_OK;
}

// Fixed-iteration window through a HIP graph (pipelined, or one iterate at a
// time): captured on the first call for (k_max, P) and replayed afterwards;
// the residuals are read once, after the window.
int32_t run_graph(swr_handle h, const swr_run_opts* o, int P, swr_run_stats* out,
                  hipStream_t st) {
  if (!h->res_pinned) HIPCHECK(h, hipHostMalloc((void**)&h->res_pinned, 64 * sizeof(double), 0));
  if (!h->gexec || h->g_kmax != o->k_max || h->g_P != P) {
    if (h->gexec) {
      HIPCHECK(h, hipGraphExecDestroy(h->gexec));
      h->gexec = nullptr;
    }
    // captured on a stream of the library's own (default priority): nothing
    // runs there, the graph is launched on the caller's stream below
    if (!h->cap_stream) HIPCHECK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIPCHECK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    swr_run_stats dummy{};
    const int rc = P > 1 ? run_pipelined(h, o, P, &dummy, h->cap_stream, true)
                         : run_steps_launches(h, o, h->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    HIPCHECK(h, e);
    const hipError_t ei = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHECK(h, ei);
    h->g_kmax = o->k_max;
    h->g_P = P;
  } else {
    // the state the captured window leaves (as run_pipelined sets it)
    h->k = o->k_max;
    h->cur = o->k_max % h->n_slots;
  }
  HIPCHECK(h, hipGraphLaunch(h->gexec, st));
  HIPCHECK(h, hipMemcpyAsync(h->res_pinned, h->ptr<double>(h->bResv), 64 * sizeof(double),
                             hipMemcpyDeviceToHost, st));
  const int rc = check_flags(h, st);  // synchronises the stream
  if (rc != SWR_OK) return rc;
  swr_run_stats s{};
  s.iters = o->k_max;
  for (int k = std::max(1, o->k_max - 63); k <= o->k_max; ++k)
    if (k <= 64) s.res[k - 1] = h->res_pinned[k % 64];
  *out = s;
  return SWR_OK;
}

}  // namespace

namespace {
int32_t run_steps(swr_handle h, const swr_run_opts* o, swr_run_stats* out, void* stream);
}  // namespace

int32_t swr_run(swr_handle h, const swr_run_opts* o, swr_run_stats* stats, void* stream) {
  if (!h || !o) return fail(h, SWR_E_ARG, "null argument");
  if (o->k_max < 1) return fail(h, SWR_E_ARG, "k_max must be >= 1");
  h->timing = o->timing != 0;
  h->tused = 0;
  struct TimingOff {  // timing covers this call only
    swr_handle h;
    ~TimingOff() { h->timing = false; }
  } timing_off{h};
  if (h->block) {
    if (!h->initial) return fail(h, SWR_E_STATE, "swr_set_initial first");
    return blk_run(h, o, stats, (hipStream_t)stream);
  }
  int rc = swr_factor(h, o->t0, stream);
  if (rc) return rc;
  rc = swr_warm_start(h, o->warm, o->g_dev, stream);
  if (rc) return rc;
  swr_run_stats s{};
  const int P = o->depth <= 0 ? h->depth_run : std::min(o->depth, h->depth);
  const bool tise = h->g.desc.mode == SWR_TISE;
  const bool graph = o->graph != 0 && o->tol < 0.0 && !h->timing;
  h->growth = Growth{};
  if (o->warm == SWR_WARM_GIVEN) h->growth.limit = o->growth_guard == 0 ? 2 : std::max(0, o->growth_guard);
  auto iterate = [&]() -> int32_t {
    if (graph) {
      const int32_t r = run_graph(h, o, P, &s, (hipStream_t)stream);
      // a replayed window's residuals arrive after it: the guard looks at them now
      for (int k = 1; r == SWR_OK && k <= std::min(s.iters, 64); ++k) h->growth.step(s.res[k - 1]);
      return r;
    }
    return P > 1 ? run_pipelined(h, o, P, &s, (hipStream_t)stream) : run_steps(h, o, &s, stream);
  };
  rc = iterate();
  if (rc) return rc;
  if (h->growth.hit) {
    // the given Robin data made the iteration grow: the window again from
    // the plain warm start (the factorisation stands)
    rc = swr_warm_start(h, SWR_WARM_PLAIN, nullptr, stream);
    if (rc) return rc;
    h->growth = Growth{};
    s = swr_run_stats{};
    rc = iterate();
    if (rc) return rc;
    s.fallback = 1;
  }
  if (tise) {
    double nu = 1.0;
    HIPCHECK(h, hipMemcpyAsync(&nu, h->nus_of(h->k) + h->n_T, 8, hipMemcpyDeviceToHost,
                               (hipStream_t)stream));
    HIPCHECK(h, hipStreamSynchronize((hipStream_t)stream));
    s.energy = h->g.desc.unnormalized ? std::nan("") : (1.0 / nu - 1.0) / h->g.desc.dt;
  }
  HIPCHECK(h, tcollect(h, &s));
  if (stats) *stats = s;
  if (o->tol > 0.0 && !s.converged)
    return fail(h, SWR_E_NOCONV, "iteration cap reached above the residual target");
  return SWR_OK;
}

namespace {

// One Schwarz iterate at a time: sweep, then transmission and residual.
int32_t run_steps(swr_handle h, const swr_run_opts* o, swr_run_stats* out, void* stream) {
  swr_run_stats& s = *out;
  int rc = SWR_OK;
  for (int k = 1; k <= o->k_max; ++k) {
    rc = swr_sweep(h, stream);
    if (rc) return rc;
    double r = 0.0;
    rc = swr_transmit(h, &r, stream);
    if (rc) return rc;
    if (k <= 64) s.res[k - 1] = r;
    s.iters = k;
    if (k >= 2 && r <= o->tol) {
      s.converged = 1;
      break;
    }
    if (h->growth.step(r)) break;  // the caller falls back
  }
  return SWR_OK;
}

}  // namespace

static int32_t copy_out(swr_handle h, const Buf& b, size_t bytes, void* dst, uint64_t cap,
                        void* stream) {
  if (!h || !dst) return fail(h, SWR_E_ARG, "null argument");
  if (!h->bound) return fail(h, SWR_E_STATE, "no workspace bound");
  if (cap < bytes) return fail(h, SWR_E_SIZE, "destination too small");
  HIPCHECK(h, hipMemcpyAsync(dst, h->ws + b.off, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SWR_OK;
}

int32_t swr_get_history(swr_handle h, void* dst_dev, uint64_t bytes, void* stream) {
  if (!h) return SWR_E_ARG;
  if (h->block) {
    if (!dst_dev) return fail(h, SWR_E_ARG, "null argument");
    if (h->blk_k < 1) return fail(h, SWR_E_STATE, "no iterate computed yet");
    if (bytes < (uint64_t)(h->n_T + 1) * h->sum_K * 16) return fail(h, SWR_E_SIZE, "destination too small");
    const swr::BlkState S = h->blk_state();
    HIPCHECK(h, swr::launch_blk_kron(h->blk_items(), 1, S.hist + h->blk_cur * S.hstride, h->n_T + 1,
                                     0, (double2*)dst_dev, h->n_T + 1, (int)h->n_T + 1,
                                     (hipStream_t)stream));
    return SWR_OK;
  }
  return copy_out(h, h->bH[h->cur], h->bH[h->cur].bytes, dst_dev, bytes, stream);
}

int32_t swr_get_forcing(swr_handle h, void* dst_dev, uint64_t bytes, void* stream) {
  if (!h) return SWR_E_ARG;
  if (h->block)
    return fail(h, SWR_E_STATE, "the block path keeps only the two latest Robin data vectors");
  if (!h->warm) return fail(h, SWR_E_STATE, "no Robin data yet");
  const Buf& b = h->bF[(h->k + 1) % h->n_slots];
  return copy_out(h, b, b.bytes, dst_dev, bytes, stream);
}

int32_t swr_get_initial(swr_handle h, void* dst_dev, uint64_t bytes, void* stream) {
  if (!h) return SWR_E_ARG;
  if (h->block) {
    if (!dst_dev) return fail(h, SWR_E_ARG, "null argument");
    if (!h->initial) return fail(h, SWR_E_STATE, "swr_set_initial first");
    if (bytes < (uint64_t)h->sum_K * 16) return fail(h, SWR_E_SIZE, "destination too small");
    HIPCHECK(h, swr::launch_blk_kron(h->blk_items(), 1, h->ptr<double2>(h->bBlkY0), 1, 0,
                                     (double2*)dst_dev, 1, 1, (hipStream_t)stream));
    return SWR_OK;
  }
  return copy_out(h, h->bC0, h->bC0.bytes, dst_dev, bytes, stream);
}

int32_t swr_get_matrix(swr_handle h, int32_t which, void* dst_dev, uint64_t bytes, void* stream) {
  if (!h) return SWR_E_ARG;
  const Buf* bs[] = {&h->bA, &h->bKin, &h->bV, &h->bQ, &h->bB, &h->bW, &h->bG, &h->bQ2};
  if (which < 0 || which > 7) return fail(h, SWR_E_ARG, "matrix index out of range");
  if (h->block) {
    if (!dst_dev) return fail(h, SWR_E_ARG, "null argument");
    if (which > 4) return fail(h, SWR_E_ARG, "the block path forms A, Kin, V, Q and B only");
    if (!h->assembled) return fail(h, SWR_E_STATE, "swr_assemble first");
    if (bytes < (uint64_t)h->sum_K2 * 8) return fail(h, SWR_E_SIZE, "destination too small");
    HIPCHECK(h, swr::launch_blk_dense(h->blk_items(), which, h->ptr<double>(h->bBlkVp),
                                      (double*)dst_dev, h->g.K_max, (hipStream_t)stream));
    return SWR_OK;
  }
  if (which == 7 && h->g.desc.field_shape != SWR_FIELD_CIRCULAR)
    return fail(h, SWR_E_ARG, "Q2 exists for a circular field only");
  return copy_out(h, *bs[which], bs[which]->bytes, dst_dev, bytes, stream);
}

int32_t swr_get_items(swr_handle h, int32_t* dst, uint64_t n) {
  if (!h || !dst) return fail(h, SWR_E_ARG, "null argument");
  const Geometry& g = h->g;
  if (n < (uint64_t)g.n_items * 10) return fail(h, SWR_E_SIZE, "destination too small");
  for (int s = 0; s < g.n_items; ++s) {
    int32_t* r = dst + (size_t)s * 10;
    r[0] = g.K[s];
    r[1] = (int32_t)(g.node_off[s + 1] - g.node_off[s]);
    for (int k = 0; k < 4; ++k) {
      r[2 + k] = k < g.D ? g.idx[(size_t)s * 4 + k] : 0;
      r[6 + k] = k < g.D ? g.nb[(size_t)s * 4 + k] : 0;
    }
  }
  return SWR_OK;
}

int32_t swr_get_terms(swr_handle h, int32_t* dst, uint64_t n) {
  if (!h || !dst) return fail(h, SWR_E_ARG, "null argument");
  if (!h->factored) return fail(h, SWR_E_STATE, "swr_factor first");
  if (n < (uint64_t)h->g.n_items) return fail(h, SWR_E_SIZE, "destination too small");
  for (int s = 0; s < h->g.n_items; ++s)
    dst[s] = h->block ? h->blk_terms[s] : (h->wide ? h->terms_item[s] : h->factor_terms + 1);
  return SWR_OK;
}

int32_t swr_get_boxes(swr_handle h, double* dst, uint64_t n) {
  if (!h || !dst) return fail(h, SWR_E_ARG, "null argument");
  const Geometry& g = h->g;
  if (n < (uint64_t)g.n_items * 8) return fail(h, SWR_E_SIZE, "destination too small");
  for (int s = 0; s < g.n_items; ++s)
    for (int k = 0; k < 4; ++k) {
      dst[(size_t)s * 8 + 2 * k] = k < g.D ? g.lo[(size_t)s * 4 + k] : 0.0;
      dst[(size_t)s * 8 + 2 * k + 1] = k < g.D ? g.hi[(size_t)s * 4 + k] : 0.0;
    }
  return SWR_OK;
}

int32_t swr_get_index_maps(swr_handle h, int32_t* dst, uint64_t n) {
  if (!h || !dst) return fail(h, SWR_E_ARG, "null argument");
  const Geometry& g = h->g;
  if (n < (uint64_t)g.nodes.size() * 16) return fail(h, SWR_E_SIZE, "destination too small");
  for (size_t q = 0; q < g.nodes.size(); ++q) {
    const auto& fn = g.nodes[q];
    int32_t* r = dst + q * 16;
    r[0] = fn.is_global ? -1 : fn.count;
    for (int c = 0; c < swr::kMaxCover; ++c)
      r[1 + c] = (c < fn.count) ? fn.cover[c] % g.n_sub : -1;
  }
  return SWR_OK;
}

int32_t swr_get_face_nodes(swr_handle h, double* coords, double* weights, uint64_t n) {
  if (!h || !coords || !weights) return fail(h, SWR_E_ARG, "null argument");
  const Geometry& g = h->g;
  if (n < (uint64_t)g.nodes.size()) return fail(h, SWR_E_SIZE, "destination too small");
  for (size_t q = 0; q < g.nodes.size(); ++q) {
    for (int k = 0; k < 4; ++k) coords[q * 4 + k] = g.nodes[q].x[k];
    weights[q] = g.nodes[q].w;
  }
  return SWR_OK;
}

static int32_t reconstruct(swr_handle h, int32_t geom, int32_t step, const void* pts_dev,
                           int64_t n_pts, int antisym, void* out_dev, void* stream) {
  if (!h || (n_pts > 0 && (!pts_dev || !out_dev))) return fail(h, SWR_E_ARG, "null argument");
  if (geom < 0 || geom >= h->g.desc.n_geom) return fail(h, SWR_E_ARG, "geometry out of range");
  if (step < 0 || step > h->n_T) return fail(h, SWR_E_ARG, "step out of range");
  if (antisym && h->g.desc.n_elec != 2)
    return fail(h, SWR_E_ARG, "antisymmetric reconstruction needs two electrons");
  if (!h->initial) return fail(h, SWR_E_STATE, "no coefficients yet");
  if (h->block) {
    if (h->blk_k < 1) return fail(h, SWR_E_STATE, "no iterate computed yet");
    // the step's coefficients in the Gaussians' basis, then the common kernel
    const swr::BlkState S = h->blk_state();
    double2* cv = h->ptr<double2>(h->bBlkCvec);
    HIPCHECK(h, swr::launch_blk_kron(h->blk_items(), 1, S.hist + h->blk_cur * S.hstride,
                                     h->n_T + 1, step, cv, 1, 1, (hipStream_t)stream));
    HIPCHECK(h, swr::launch_reconstruct(h->items(), geom, 0, 0, cv, (const double*)pts_dev, n_pts,
                                        antisym, (double2*)out_dev, (hipStream_t)stream));
    return SWR_OK;
  }
  HIPCHECK(h, swr::launch_reconstruct(h->items(), geom, step, (int)h->n_T, h->hist(h->cur),
                                      (const double*)pts_dev, n_pts, antisym, (double2*)out_dev,
                                      (hipStream_t)stream));
  return SWR_OK;
}

int32_t swr_reconstruct(swr_handle h, int32_t geom, int32_t step, const void* pts_dev,
                        int64_t n_pts, void* out_dev, void* stream) {
  return reconstruct(h, geom, step, pts_dev, n_pts, 0, out_dev, stream);
}

int32_t swr_reconstruct_antisym(swr_handle h, int32_t geom, int32_t step, const void* pts_dev,
                                int64_t n_pts, void* out_dev, void* stream) {
  return reconstruct(h, geom, step, pts_dev, n_pts, 1, out_dev, stream);
}

int32_t swr_local_eigen(swr_handle h, void* lambda_dev, void* vectors_dev, void* stream) {
  if (!h || !lambda_dev || !vectors_dev) return fail(h, SWR_E_ARG, "null argument");
  if (!h->assembled) return fail(h, SWR_E_STATE, "swr_assemble first");
  if (h->block) return fail(h, SWR_E_STATE, "the block path is for real time");
  if (h->g.desc.mu_im != 0.0) return fail(h, SWR_E_ARG, "local eigenproblems need a real mu");
  if (h->g.K_max > swr::kSmallK) return fail(h, SWR_E_SIZE, "local eigenproblems need K <= 64");
  hipStream_t st = (hipStream_t)stream;
  HIPCHECK(h, swr::launch_geneig(h->items(), h->ptr<double>(h->bA), h->ptr<double>(h->bHr),
                                 (double*)lambda_dev, (double*)vectors_dev, h->ptr<int>(h->bFlags),
                                 st));
  return check_flags(h, st);
}

int32_t swr_get_norms(swr_handle h, void* dst_dev, uint64_t bytes, void* stream) {
  if (!h) return SWR_E_ARG;
  if (h->block) return fail(h, SWR_E_STATE, "the block path is for real time");
  const Buf& b = h->bNus[h->k % h->n_slots];
  return copy_out(h, b, b.bytes, dst_dev, bytes, stream);
}

int32_t swr_set_field(swr_handle h, double E0, double omega, double phase) {
  if (!h) return SWR_E_ARG;
  h->g.desc.E0 = E0;
  h->g.desc.omega = omega;
  h->g.desc.phase = phase;
  h->factored = false;
  return SWR_OK;
}

int32_t swr_advance_window(swr_handle h, void* stream) {
  if (!h) return SWR_E_ARG;
  if (h->block) {
    if (!h->initial || h->blk_k < 1) return fail(h, SWR_E_STATE, "no iterate to advance from");
    const swr::BlkState S = h->blk_state();
    HIPCHECK(h, swr::launch_blk_kron(h->blk_items(), 3, S.hist + h->blk_cur * S.hstride,
                                     h->n_T + 1, (int)h->n_T, h->ptr<double2>(h->bBlkY0), 1, 1,
                                     (hipStream_t)stream));
    return blk_warm_start(h, SWR_WARM_PLAIN, (hipStream_t)stream);
  }
  if (!h->initial || h->k < 1) return fail(h, SWR_E_STATE, "no iterate to advance from");
  HIPCHECK(h, swr::launch_last_step(h->items(), (int)h->n_T, h->hist(h->cur),
                                    h->ptr<double2>(h->bC0), (hipStream_t)stream));
  return swr_warm_start(h, SWR_WARM_PLAIN, nullptr, stream);
}

int32_t swr_time_nodes(swr_handle h, int32_t* steps_host) {
  if (!h || !steps_host) return fail(h, SWR_E_ARG, "null argument");
  if (!distinct_time_nodes((int)h->n_T, h->n_nodes_t)) return fail(h, SWR_E_ARG, kShortWindow);
  const std::vector<int> tn = time_nodes((int)h->n_T, h->n_nodes_t);
  for (int m = 0; m < h->n_nodes_t; ++m) steps_host[m] = tn[m];
  return SWR_OK;
}

int32_t swr_face_data(swr_handle h, int32_t n_sel, const int32_t* steps_host, void* g_dev,
                      void* stream) {
  if (!h || !steps_host || !g_dev) return fail(h, SWR_E_ARG, "null argument");
  if (n_sel < 1 || n_sel > 64) return fail(h, SWR_E_ARG, "n_sel must be in 1..64");
  if (h->block) return fail(h, SWR_E_STATE, "the learned warm start is not on the block path");
  if (!h->initial) return fail(h, SWR_E_STATE, "no coefficients yet");
  swr::StepList sl{};
  sl.n = n_sel;
  for (int i = 0; i < n_sel; ++i) {
    if (steps_host[i] < 0 || steps_host[i] > h->n_T) return fail(h, SWR_E_ARG, "step out of range");
    sl.step[i] = steps_host[i];
  }
  HIPCHECK(h, swr::launch_face_data(h->items(), h->nodes(), h->ptr<int32_t>(h->bNCover), sl,
                                    (int)h->n_T, h->g.desc.mu_re, h->g.desc.mu_im,
                                    h->hist(h->cur), (double2*)g_dev, (hipStream_t)stream));
  return SWR_OK;
}

static int max_item_nodes(swr_handle h) {
  int64_t mx = 0;
  for (int s = 0; s < h->g.n_items; ++s)
    mx = std::max<int64_t>(mx, h->g.node_off[s + 1] - h->g.node_off[s]);
  return (int)mx;
}

int32_t swr_learned_features(swr_handle h, const void* g0_dev, double t0, int32_t n_in,
                             float* x_dev, double* scale_dev, void* stream) {
  if (!h || !g0_dev || !x_dev || !scale_dev) return fail(h, SWR_E_ARG, "null argument");
  if (h->block) return fail(h, SWR_E_STATE, "the learned warm start is not on the block path");
  if (!h->assembled) return fail(h, SWR_E_STATE, "swr_assemble first");
  if (!distinct_time_nodes((int)h->n_T, h->n_nodes_t)) return fail(h, SWR_E_ARG, kShortWindow);
  const int M = h->n_nodes_t;
  if (n_in < 2 * max_item_nodes(h) + M + 8) return fail(h, SWR_E_SIZE, "n_in too small");
  swr::FieldFeat ff{};
  ff.n = M;
  const std::vector<int> tn = time_nodes((int)h->n_T, M);
  for (int m = 0; m < M; ++m) ff.v[m] = kFieldScale * field(h->g.desc, t0 + tn[m] * h->g.desc.dt);
  for (int k = 0; k < 4; ++k) {
    ff.mid[k] = 0.5 * (h->g.desc.box_lo[k] + h->g.desc.box_hi[k]);
    ff.half[k] = k < h->g.D ? 0.5 * (h->g.desc.box_hi[k] - h->g.desc.box_lo[k]) : 1.0;
  }
  ff.t0w = t0 / (8.0 * h->n_T * h->g.desc.dt);
  HIPCHECK(h, swr::launch_learned_features(h->items(), h->nodes(), (const double2*)g0_dev, ff,
                                           n_in, x_dev, scale_dev, h->ptr<double>(h->bLMax),
                                           (hipStream_t)stream));
  return SWR_OK;
}

int32_t swr_learned_targets(swr_handle h, const void* g_nodes_dev, const double* scale_dev,
                            int32_t n_out, float* y_dev, void* stream) {
  if (!h || !g_nodes_dev || !scale_dev || !y_dev) return fail(h, SWR_E_ARG, "null argument");
  if (h->block) return fail(h, SWR_E_STATE, "the learned warm start is not on the block path");
  if (!h->assembled) return fail(h, SWR_E_STATE, "swr_assemble first");
  if (!distinct_time_nodes((int)h->n_T, h->n_nodes_t)) return fail(h, SWR_E_ARG, kShortWindow);
  if (n_out < 2 * h->n_nodes_t * max_item_nodes(h)) return fail(h, SWR_E_SIZE, "n_out too small");
  HIPCHECK(h, swr::launch_learned_targets(h->items(), h->nodes(), (const double2*)g_nodes_dev,
                                          h->n_nodes_t, scale_dev, n_out, y_dev, (hipStream_t)stream));
  return SWR_OK;
}

int32_t swr_learned_apply(swr_handle h, const float* y_dev, const double* scale_dev,
                          const void* g0_dev, int32_t n_out, void* g_all_dev, void* stream) {
  if (!h || !y_dev || !scale_dev || !g0_dev || !g_all_dev) return fail(h, SWR_E_ARG, "null argument");
  if (h->block) return fail(h, SWR_E_STATE, "the learned warm start is not on the block path");
  if (!h->assembled) return fail(h, SWR_E_STATE, "swr_assemble first");
  if (!distinct_time_nodes((int)h->n_T, h->n_nodes_t)) return fail(h, SWR_E_ARG, kShortWindow);
  if (n_out < 2 * h->n_nodes_t * max_item_nodes(h)) return fail(h, SWR_E_SIZE, "n_out too small");
  HIPCHECK(h, swr::launch_learned_apply(h->items(), h->nodes(), y_dev, scale_dev,
                                        (const double2*)g0_dev, h->ptr<double>(h->bLag), h->n_nodes_t,
                                        n_out, (int)h->n_T, (double2*)g_all_dev,
                                        (hipStream_t)stream));
  return SWR_OK;
}

int32_t swr_status_sync(swr_handle h, void* stream) {
  if (!h) return SWR_E_ARG;
  if (!h->bound) return fail(h, SWR_E_STATE, "no workspace bound");
  return check_flags(h, (hipStream_t)stream);
}

}  // extern "C"

int32_t swr_set_schedule(swr_handle h, int32_t depth, int32_t tx_tile, int32_t order,
                         void* stream) {
  if (!h) return SWR_E_ARG;
  if (!h->assembled) return fail(h, SWR_E_STATE, "swr_assemble first");
  const int max_depth = h->block ? h->blk_depth : h->depth;
  if (depth < 1 || depth > max_depth) return fail(h, SWR_E_ARG, "depth out of range");
  bool tile_ok, order_ok = order == 0;
  if (h->block) {
    tile_ok = tx_tile == 0;
  } else if (h->wide) {
    tile_ok = tx_tile == 8 || tx_tile == 16 || tx_tile == 32;
    order_ok = order == 0 || order == 1;
  } else if (h->g.te_ok) {
    tile_ok = tx_tile == 16 || (tx_tile == 32 && h->tx_tt_max == 32);
  } else {
    tile_ok = tx_tile == h->tx_tt;
  }
  if (!tile_ok) return fail(h, SWR_E_ARG, "transmission tile not available on this path");
  if (!order_ok) return fail(h, SWR_E_ARG, "recurrence order not available on this path");
  if (h->block) {
    h->depth_run = depth;
    return SWR_OK;
  }
  TuneChoice c;
  c.depth = depth;
  c.tile = tx_tile;
  c.order = order;
  return apply_schedule(h, c, (hipStream_t)stream);
}

int32_t swr_autotune(swr_handle h, int32_t k_iters, double t0, swr_tuning* out, void* stream) {
  if (!h || !out) return fail(h, SWR_E_ARG, "null argument");
  if (k_iters < 1) return fail(h, SWR_E_ARG, "k_iters must be >= 1");
  if (!h->assembled || !h->initial) return fail(h, SWR_E_STATE, "swr_assemble and swr_set_initial first");
  if (h->block) {
    // nothing to reorder on the block path: time one window at its depth
    swr_run_opts o{};
    o.k_max = k_iters;
    o.tol = -1.0;
    o.t0 = t0;
    o.warm = SWR_WARM_PLAIN;
    hipEvent_t e0, e1;
    HIPCHECK(h, hipEventCreate(&e0));
    HIPCHECK(h, hipEventCreate(&e1));
    HIPCHECK(h, hipEventRecord(e0, (hipStream_t)stream));
    swr_run_stats rs{};
    const int rc = swr_run(h, &o, &rs, stream);
    HIPCHECK(h, hipEventRecord(e1, (hipStream_t)stream));
    HIPCHECK(h, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHECK(h, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    out->depth = h->blk_depth;
    out->tx_tile = 0;
    out->ms_per_window = ms;
    out->candidates = 1;
    return SWR_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  std::vector<int> depths, tiles, orders{0};
  for (int d = 1; d <= h->depth; ++d) depths.push_back(d);
  if (h->wide) {
    tiles = {8, 16, 32};
    orders = {0, 1};
  } else if (h->g.te_ok) {
    tiles.push_back(16);
    if (h->tx_tt_max == 32) tiles.push_back(32);
  } else {
    tiles.push_back(h->tx_tt);
  }
  hipEvent_t e0, e1;
  HIPCHECK(h, hipEventCreate(&e0));
  HIPCHECK(h, hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } ev{e0, e1};
  TuneChoice best;
  best.ms = -1.0;
  for (const int od : orders)
    for (const int t : tiles)
      for (const int d : depths) {
        TuneChoice c;
        c.depth = d;
        c.tile = t;
        c.order = od;
        int rc = apply_schedule(h, c, st);
        if (rc) return rc;
        swr_run_opts o{};
        o.k_max = k_iters;
        o.tol = -1.0;
        o.t0 = t0;
        o.warm = SWR_WARM_PLAIN;
        o.depth = d;
        swr_run_stats s{};
        rc = swr_run(h, &o, &s, stream);  // warm-up
        if (rc) return rc;
        HIPCHECK(h, hipEventRecord(e0, st));
        rc = swr_run(h, &o, &s, stream);
        if (rc) return rc;
        HIPCHECK(h, hipEventRecord(e1, st));
        HIPCHECK(h, hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHECK(h, hipEventElapsedTime(&ms, e0, e1));
        if (best.ms < 0.0 || ms < best.ms) {
          best = c;
          best.ms = ms;
        }
      }
  const int rc = apply_schedule(h, best, st);
  if (rc) return rc;
  tune_store(tune_key(h), best);
  out->depth = h->depth_run;
  out->tx_tile = h->wide ? h->wide_tile : (h->g.te_ok ? h->tx_tt : 0);
  out->order = h->wide_order;
  out->ms_per_window = best.ms;
  out->candidates = (int32_t)(depths.size() * tiles.size() * orders.size());
  return SWR_OK;
}
