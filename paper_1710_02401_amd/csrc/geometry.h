// Host-side decomposition, local bases, face quadrature and covering sets.
//
// Section 5 (opening paragraph) gives the uniform decomposition of the
// global box into L^{dN} overlapping hypercubes; Section 4.1 defines the
// interfaces Gamma_{i;j} = boundary(Omega_i) cap Omega_j and the averaging
// over the set O of subdomains sharing a multi-overlap zone.  Everything here
// is exact integer/FP64 bookkeeping done once per handle; geometry.cpp is
// compiled without floating-point contraction so that box ends and centres
// follow the formulas operation by operation.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/swr.h"

namespace swr {

constexpr int kMaxD = 4;
constexpr int kMaxCover = 15;  // 2^4 - 1

struct FaceNode {
  int32_t item;        // receiving item
  int32_t face;        // 2*k + side
  int32_t is_global;   // face lies on the global boundary
  int32_t count;       // |O(y)| (0 on global faces)
  int32_t cover[kMaxCover];  // global item indices of O(y), increasing
  double x[kMaxD];
  double w;            // tangential quadrature weight
};

struct Geometry {
  swr_desc desc{};
  std::vector<int32_t> nbasis_in;     // copy of desc.nbasis
  std::vector<double> nuc_pos, nuc_charge;

  int D = 0, n_sub = 0, n_items = 0, K_max = 0;
  int L[kMaxD]{}, stride[kMaxD]{};
  double eps[kMaxD]{};
  std::vector<double> lo1[kMaxD], hi1[kMaxD];

  // per item
  std::vector<int32_t> idx;      // [n_items][kMaxD]
  std::vector<int32_t> nb;       // [n_items][kMaxD]
  std::vector<int32_t> K;        // [n_items]
  std::vector<int64_t> off1;     // prefix sums of K   (n_items + 1)
  std::vector<int64_t> off2;     // prefix sums of K^2 (n_items + 1)
  std::vector<double> lo, hi;    // [n_items][kMaxD]
  std::vector<double> delta;     // [n_items][kMaxD]
  std::vector<int64_t> aoff;     // [n_items][kMaxD] offsets into alpha
  std::vector<double> alpha;     // centres, concatenated

  // receiving face nodes, item-major then face then node (oracle order)
  std::vector<FaceNode> nodes;
  std::vector<int64_t> node_off; // (n_items + 1)

  // neighbour pairs (i, j) with j in some O(y) of i's nodes
  std::vector<int32_t> pair_i, pair_j;
  std::vector<int64_t> pair_off;  // (n_items + 1): pairs of item i
  std::vector<int64_t> pair_toff; // offset of T_ij entries (n_pairs + 1)
  // nodes of i whose covering set holds j: list per pair
  std::vector<int32_t> pnode;     // node indices
  std::vector<int64_t> pnode_off; // (n_pairs + 1)
  // Factored transfer operators (D <= 2): one entry per (pair, face of the
  // receiving item that the sender covers); the entry's nodes are the run
  // [te_t0, te_t1) of the pair's node list.  Per entry: beta (receiver's
  // normal-dimension basis at the face), a (sender's Robin trace, complex)
  // and X (tangential weighted overlap, receiver x sender rows).
  bool te_ok = false;
  std::vector<int32_t> te_pair, te_face;
  std::vector<int64_t> te_t0, te_t1;
  std::vector<int64_t> te_off;    // (n_items + 1): entries of item i
  std::vector<int64_t> te_soff;   // (n_items + 1): entries whose sender is item j
  std::vector<int32_t> te_sidx;   // entry indices grouped by sender
  std::vector<int64_t> te_boff, te_aoff, te_xoff;  // offsets of beta, a, X
  int64_t te_nb = 0, te_na = 0, te_nx = 0;         // totals

  // potential quadrature: per item per dim composite Gauss-Legendre rule
  std::vector<double> qx, qw;     // concatenated
  std::vector<int64_t> qoff;      // [n_items][kMaxD] offsets, plus count
  std::vector<int32_t> qn;        // [n_items][kMaxD] node counts
  // local orbitals (SWR_BASIS_LSD): per interval i of the first dimension
  // (item i) the orbital problem's rule over [x_c - R, x_c + R], R =
  // barrier + width/2 + 10/sqrt(delta), composite 16-point Gauss-Legendre
  // with breaks at the barrier's transition edges and panels no wider than
  // 0.25/sqrt(delta); and the 64-point rule on [-1, 1] of the mollifier
  std::vector<double> lo_qx, lo_qw;
  std::vector<int64_t> lo_qoff;   // (L[0] + 1)
  std::vector<double> lo_mx, lo_mw;
};

// One-electron functions per interval of a local-orbital basis (Section 3):
// the orbitals, then the Gaussians added at each end (Section 3.3).
inline int lsd_functions(const swr_desc& d) { return d.lsd_orbitals + 2 * d.lsd_augment; }

// Returns an empty string on success, else the error message; *code gets
// the SWR_E_* status.
std::string build_geometry(const swr_desc& d, Geometry* g, int* code);

// Tangential face rule of item s in dimension t (composite Gauss-Legendre
// over [lo, lo + eps], [lo + eps, hi - eps], [hi - eps, hi]), the same
// nodes and weights as the face nodes of the geometry.
void face_rule_1d(const Geometry& g, int s, int t, std::vector<double>* x, std::vector<double>* w);

// n-point Gauss-Legendre rule on [-1, 1], ascending nodes (Newton on the
// three-term recurrence of the Legendre polynomials).
void gauss_legendre(int n, std::vector<double>* t, std::vector<double>* w);

}  // namespace swr
