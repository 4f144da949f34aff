// Host geometry of the SWR decomposition (see geometry.h).
// Compiled with -ffp-contract=off: every box end, centre and width follows
// the defining formulas one IEEE operation at a time.
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <set>

namespace swr {

void gauss_legendre(int n, std::vector<double>* t, std::vector<double>* w) {
  t->assign(n, 0.0);
  w->assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    // i-th largest root, initial guess from the asymptotic formula
    double x = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p0 = 1.0; p1 = x; }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    (*t)[n - 1 - i] = x;
    (*w)[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  // symmetrise about 0
  std::vector<double> ts = *t, ws = *w;
  for (int i = 0; i < n; ++i) {
    (*t)[i] = 0.5 * (ts[i] - ts[n - 1 - i]);
    (*w)[i] = 0.5 * (ws[i] + ws[n - 1 - i]);
  }
}

namespace {

void composite(const std::vector<double>& edges, const std::vector<int>& counts,
               std::vector<double>* x, std::vector<double>* w) {
  x->clear();
  w->clear();
  for (size_t p = 0; p + 1 < edges.size(); ++p) {
    std::vector<double> t, tw;
    gauss_legendre(counts[p], &t, &tw);
    const double a = edges[p], b = edges[p + 1];
    const double half = 0.5 * (b - a);
    const double mid = 0.5 * (a + b);
    for (int j = 0; j < counts[p]; ++j) {
      x->push_back(mid + half * t[j]);
      w->push_back(half * tw[j]);
    }
  }
}

}  // namespace

void face_rule_1d(const Geometry& g, int s, int t, std::vector<double>* x, std::vector<double>* w) {
  const double lo = g.lo[(size_t)s * kMaxD + t], hi = g.hi[(size_t)s * kMaxD + t];
  std::vector<double> edges = {lo, lo + g.eps[t], hi - g.eps[t], hi};
  composite(edges, {g.desc.face_nodes_band, g.desc.face_nodes_mid, g.desc.face_nodes_band}, x, w);
}

std::string build_geometry(const swr_desc& d, Geometry* g, int* code) {
  *code = SWR_E_ARG;
  if (d.n_elec < 1 || d.dim < 1) return "n_elec and dim must be >= 1";
  const int D = d.n_elec * d.dim;
  if (D > kMaxD) return "configuration dimension D = n_elec*dim must be <= 4";
  if (d.n_geom < 1) return "n_geom must be >= 1";
  if (d.mode != SWR_TDSE && d.mode != SWR_TISE) return "mode must be SWR_TDSE or SWR_TISE";
  if (d.mode == SWR_TISE && d.mu_im != 0.0) return "imaginary time needs a real Robin coefficient";
  if (d.mode == SWR_TISE && d.n_geom != 1)
    return "imaginary time takes one geometry (its normalisation spans every subdomain)";
  if (!(d.dt != 0.0) || d.n_steps < 1) return "dt must be non-zero and n_steps >= 1";
  if (d.axis < 0 || d.axis >= d.dim) return "field axis out of range";
  if (d.n_nuc < 0 || (d.n_nuc > 0 && (!d.nuc_pos || !d.nuc_charge))) return "nuclei arrays missing";
  if (!d.nbasis) return "nbasis missing";
  if (d.face_nodes_band < 1 || d.face_nodes_mid < 1 || d.quad_nodes < 1) return "node counts must be >= 1";
  if (d.learned_nodes != 0 && (d.learned_nodes < 2 || d.learned_nodes > 64))
    return "learned_nodes must be 0 (default 8) or in 2..64";
  if (d.factor_mode < 0 || d.factor_mode > 3)
    return "factor_mode must be 0 (auto), 1 (direct), 2 (wide) or 3 (block)";
  if (d.unnormalized != 0 && d.unnormalized != 1) return "unnormalized must be 0 or 1";
  if (d.unnormalized && d.mode != SWR_TISE) return "unnormalized applies to imaginary time only";
  if (d.field_shape != SWR_FIELD_SINE && d.field_shape != SWR_FIELD_CIRCULAR)
    return "field_shape must be SWR_FIELD_SINE or SWR_FIELD_CIRCULAR";
  if (d.field_shape == SWR_FIELD_CIRCULAR) {
    if (d.mode != SWR_TDSE) return "a circular field applies to real time only";
    const int all = (1 << D) - 1;
    const int m0 = d.field_mask[0], m1 = d.field_mask[1];
    if (m0 <= 0 || m1 <= 0 || (m0 & ~all) || (m1 & ~all) || (m0 & m1))
      return "field_mask must be two non-empty, disjoint sets of the D coordinates";
    if (!(d.pulse_nu >= 0.0) || !std::isfinite(d.pulse_center))
      return "pulse_nu must be >= 0 and pulse_center finite";
  }
  if (!(d.eps_en > 0.0) || !(d.eps_ee > 0.0)) return "soft-Coulomb eps must be > 0";
  if (!(d.width > 0.0) && !(d.width_ratio > 0.0)) return "width or width_ratio must be > 0";
  if (d.basis_extend < 0) return "basis_extend must be >= 0";
  if (d.basis_kind != SWR_BASIS_GAUSSIAN && d.basis_kind != SWR_BASIS_SLATER &&
      d.basis_kind != SWR_BASIS_LSD && d.basis_kind != SWR_BASIS_LO)
    return "basis_kind must be SWR_BASIS_GAUSSIAN, SWR_BASIS_SLATER, SWR_BASIS_LSD or SWR_BASIS_LO";
  if (d.basis_kind == SWR_BASIS_LO) {
    if (d.n_elec != 1 || d.dim != 2)
      return "local orbitals (SWR_BASIS_LO) are for one electron in two dimensions";
    if (!d.nbasis || d.nbasis[0] < 1 || d.nbasis[1] < 1 || d.nbasis[0] > 8 || d.nbasis[1] > 8)
      return "local orbitals take 1..8 Gaussians per dimension";
    if (!(d.lsd_orbitals >= 1 && d.lsd_orbitals <= d.nbasis[0] * d.nbasis[1]))
      return "lsd_orbitals must be in 1..(Gaussians per box)";
    if (!(d.lsd_barrier > 0.0) || !(d.lsd_barrier_width > 0.0) || !(d.lsd_v_inf >= 0.0) ||
        !(d.lsd_moll_eps > 0.0) || d.lsd_moll_order < 2 || d.lsd_moll_order > 8)
      return "local orbitals need lsd_barrier, lsd_barrier_width, lsd_moll_eps > 0, "
             "lsd_v_inf >= 0 and lsd_moll_order in 2..8";
    if (d.lsd_augment != 0) return "lsd_augment applies to local Slater determinants only";
    if (d.n_geom != 1) return "local orbitals take one geometry";
    if (d.field_shape != SWR_FIELD_SINE) return "local orbitals take the sine field";
    if (d.factor_mode == SWR_FACTOR_BLOCK || d.factor_mode == SWR_FACTOR_WIDE)
      return "local orbitals run on the narrow path";
  }
  if (d.basis_kind == SWR_BASIS_LSD) {
    if (!(d.lsd_orbitals >= 2 && d.lsd_orbitals <= 8 && d.nbasis && d.lsd_orbitals <= d.nbasis[0]))
      return "lsd_orbitals must be in 2..8 and at most the Gaussians per interval";
    if (!(d.lsd_barrier > 0.0) || !(d.lsd_barrier_width > 0.0) || !(d.lsd_v_inf >= 0.0) ||
        !(d.lsd_moll_eps > 0.0) || d.lsd_moll_order < 1 || d.lsd_moll_order > 8)
      return "local orbitals need lsd_barrier, lsd_barrier_width, lsd_moll_eps > 0, "
             "lsd_v_inf >= 0 and lsd_moll_order in 1..8";
    if (d.nbasis && d.nbasis[0] > 16) return "local orbitals take at most 16 Gaussians per interval";
    if (d.lsd_augment < 0 || lsd_functions(d) > 8 || lsd_functions(d) > d.nbasis[0])
      return "lsd_augment must be >= 0 with lsd_orbitals + 2 lsd_augment at most 8 and at most "
             "the Gaussians per interval";
  }
  if (d.basis_kind == SWR_BASIS_SLATER || d.basis_kind == SWR_BASIS_LSD) {
    if (d.n_elec != 2 || d.dim != 1)
      return "the Slater basis is for two electrons in one dimension each";
    if (d.per_subdomain_basis || d.nbasis[0] != d.nbasis[1] || d.nbasis[0] < 2)
      return "the Slater basis takes one basis size (>= 2) for every interval";
    if (d.L[0] != d.L[1] || d.box_lo[0] != d.box_lo[1] || d.box_hi[0] != d.box_hi[1] ||
        d.overlap[0] != d.overlap[1])
      return "the Slater basis needs a decomposition symmetric under the exchange of the coordinates";
    if (d.field_shape != SWR_FIELD_SINE) return "the Slater basis takes the sine field";
    if (d.factor_mode == SWR_FACTOR_WIDE || d.factor_mode == SWR_FACTOR_BLOCK)
      return "the Slater basis runs on the narrow path (factor_mode auto or direct)";
    if (d.n_geom != 1) return "the Slater basis takes one geometry";
    if (!(d.init_center[0] != d.init_center[1]))
      return "the antisymmetrised initial state needs two distinct centres";
  }
  g->desc = d;
  g->D = D;
  int n_sub = 1;
  for (int k = 0; k < D; ++k) {
    if (d.L[k] < 1) return "L must be >= 1";
    if (!(d.box_hi[k] > d.box_lo[k])) return "box_hi must exceed box_lo";
    if (d.overlap[k] < 0.0) return "overlap must be >= 0";
    g->L[k] = d.L[k];
    g->stride[k] = n_sub;
    n_sub *= d.L[k];
    g->eps[k] = d.overlap[k];
  }
  g->n_sub = n_sub;
  g->n_items = n_sub * d.n_geom;
  const int nb_len = d.per_subdomain_basis ? n_sub * D : D;
  g->nbasis_in.assign(d.nbasis, d.nbasis + nb_len);
  g->nuc_pos.assign(d.nuc_pos, d.nuc_pos + (size_t)d.n_geom * d.n_nuc * d.dim);
  g->nuc_charge.assign(d.nuc_charge, d.nuc_charge + d.n_nuc);
  g->desc.nbasis = g->nbasis_in.data();
  g->desc.nuc_pos = g->nuc_pos.data();
  g->desc.nuc_charge = g->nuc_charge.data();

  // per-dimension interval ends (Section 5): a = lo + eps/2, b = hi - eps/2
  for (int k = 0; k < D; ++k) {
    const double a = d.box_lo[k] + 0.5 * d.overlap[k];
    const double b = d.box_hi[k] - 0.5 * d.overlap[k];
    const double h = (b - a) / g->L[k];
    if (g->L[k] > 1 && !(d.overlap[k] < h)) return "overlap must be smaller than the core width";
    g->lo1[k].resize(g->L[k]);
    g->hi1[k].resize(g->L[k]);
    for (int i = 0; i < g->L[k]; ++i) {
      g->lo1[k][i] = (a + i * h) - 0.5 * d.overlap[k];
      g->hi1[k][i] = (a + (i + 1) * h) + 0.5 * d.overlap[k];
    }
  }

  const int NI = g->n_items;
  g->idx.assign((size_t)NI * kMaxD, 0);
  g->nb.assign((size_t)NI * kMaxD, 0);
  g->K.assign(NI, 0);
  g->off1.assign(NI + 1, 0);
  g->off2.assign(NI + 1, 0);
  g->lo.assign((size_t)NI * kMaxD, 0.0);
  g->hi.assign((size_t)NI * kMaxD, 0.0);
  g->delta.assign((size_t)NI * kMaxD, 0.0);
  g->aoff.assign((size_t)NI * kMaxD, 0);
  g->alpha.clear();
  g->qoff.assign((size_t)NI * kMaxD, 0);
  g->qn.assign((size_t)NI * kMaxD, 0);
  g->qx.clear();
  g->qw.clear();
  g->K_max = 0;
  for (int s = 0; s < NI; ++s) {
    const int i = s % n_sub;
    int rem = i;
    int K = 1;
    for (int k = 0; k < D; ++k) {
      const int ik = rem % g->L[k];
      rem /= g->L[k];
      g->idx[(size_t)s * kMaxD + k] = ik;
      const int n = d.per_subdomain_basis ? g->nbasis_in[(size_t)i * D + k] : g->nbasis_in[k];
      if (n < 1) return "nbasis must be >= 1";
      if (n > 1 && n - 1 - 2 * d.basis_extend < 1) return "basis_extend too large for nbasis";
      g->nb[(size_t)s * kMaxD + k] = n;
      K *= n;
      const double lo = g->lo1[k][ik], hi = g->hi1[k][ik];
      g->lo[(size_t)s * kMaxD + k] = lo;
      g->hi[(size_t)s * kMaxD + k] = hi;
      double sp;
      g->aoff[(size_t)s * kMaxD + k] = (int64_t)g->alpha.size();
      if (n == 1) {
        sp = hi - lo;
        g->alpha.push_back(0.5 * (lo + hi));
      } else {
        sp = (hi - lo) / (n - 1 - 2 * d.basis_extend);
        const double first = lo - d.basis_extend * sp;
        for (int j = 0; j < n; ++j) g->alpha.push_back(first + j * sp);
      }
      const double sigma = d.width > 0.0 ? d.width : d.width_ratio * sp;
      const double delta = 0.5 / (sigma * sigma);
      g->delta[(size_t)s * kMaxD + k] = delta;
      // potential quadrature panels of width <= min(eps_en, eps_ee, sigma)
      const double sig = std::sqrt(0.5 / delta);
      const double hmax = std::min(std::min(d.eps_en, d.eps_ee), sig);
      const int npan = std::max(1, (int)std::ceil((hi - lo) / hmax));
      const double wdt = (hi - lo) / npan;
      std::vector<double> edges;
      for (int p = 0; p < npan; ++p) edges.push_back(lo + p * wdt);
      edges.push_back(hi);
      std::vector<double> x, w;
      composite(edges, std::vector<int>(npan, d.quad_nodes), &x, &w);
      g->qoff[(size_t)s * kMaxD + k] = (int64_t)g->qx.size();
      g->qn[(size_t)s * kMaxD + k] = (int32_t)x.size();
      g->qx.insert(g->qx.end(), x.begin(), x.end());
      g->qw.insert(g->qw.end(), w.begin(), w.end());
    }
    if (d.basis_kind == SWR_BASIS_LO) K = d.lsd_orbitals;  // Section 3, d = 2
    if (d.basis_kind == SWR_BASIS_SLATER || d.basis_kind == SWR_BASIS_LSD) {
      // Section 2 eq. (LSD): antisymmetrised pairs of Gaussians (or, Section
      // 3, of local orbitals); l < p on the diagonal
      const int n = d.basis_kind == SWR_BASIS_LSD ? lsd_functions(d) : g->nb[(size_t)s * kMaxD];
      K = g->idx[(size_t)s * kMaxD] == g->idx[(size_t)s * kMaxD + 1] ? n * (n - 1) / 2 : n * n;
    }
    g->K[s] = K;
    g->K_max = std::max(g->K_max, K);
    g->off1[s + 1] = g->off1[s] + K;
    g->off2[s + 1] = g->off2[s] + (int64_t)K * K;
  }

  // receiving face nodes and covering sets O(y) (closed membership)
  g->nodes.clear();
  g->node_off.assign(NI + 1, 0);
  for (int s = 0; s < NI; ++s) {
    const int geom = s / n_sub;
    const int32_t* ix = &g->idx[(size_t)s * kMaxD];
    const double* slo = &g->lo[(size_t)s * kMaxD];
    const double* shi = &g->hi[(size_t)s * kMaxD];
    for (int k = 0; k < D; ++k) {
      for (int side = 0; side < 2; ++side) {
        const int is_global = (side == 0 && ix[k] == 0) || (side == 1 && ix[k] == g->L[k] - 1);
        // tangential rules, increasing dimension, last fastest
        std::vector<int> tang;
        for (int t = 0; t < D; ++t)
          if (t != k) tang.push_back(t);
        std::vector<std::vector<double>> tx(tang.size()), tw(tang.size());
        for (size_t c = 0; c < tang.size(); ++c) {
          const int t = tang[c];
          std::vector<double> edges = {slo[t], slo[t] + g->eps[t], shi[t] - g->eps[t], shi[t]};
          composite(edges, {d.face_nodes_band, d.face_nodes_mid, d.face_nodes_band}, &tx[c], &tw[c]);
        }
        size_t n_y = 1;
        for (auto& v : tx) n_y *= v.size();
        for (size_t q = 0; q < n_y; ++q) {
          FaceNode fn{};
          fn.item = s;
          fn.face = 2 * k + side;
          fn.is_global = is_global;
          fn.x[k] = side ? shi[k] : slo[k];
          double w = 1.0;
          size_t rem2 = q;
          for (int c = (int)tang.size() - 1; c >= 0; --c) {
            const size_t nn = tx[c].size();
            const size_t j = rem2 % nn;
            rem2 /= nn;
            fn.x[tang[c]] = tx[c][j];
          }
          rem2 = q;
          std::vector<double> wj(tang.size());
          for (int c = (int)tang.size() - 1; c >= 0; --c) {
            const size_t nn = tx[c].size();
            wj[c] = tw[c][rem2 % nn];
            rem2 /= nn;
          }
          for (size_t c = 0; c < tang.size(); ++c) w = w * wj[c];
          fn.w = w;
          fn.count = 0;
          for (int c = 0; c < kMaxCover; ++c) fn.cover[c] = -1;
          if (!is_global) {
            // candidates: 3^D neighbourhood (sufficient since eps < h)
            int total = 1;
            for (int t = 0; t < D; ++t) total *= 3;
            std::vector<int> found;
            for (int cnd = 0; cnd < total; ++cnd) {
              int r = cnd, lin = 0;
              bool ok = true;
              for (int t = 0; t < D && ok; ++t) {
                const int jt = ix[t] + (r % 3) - 1;
                r /= 3;
                if (jt < 0 || jt >= g->L[t]) { ok = false; break; }
                if (!(g->lo1[t][jt] <= fn.x[t] && fn.x[t] <= g->hi1[t][jt])) ok = false;
                lin += jt * g->stride[t];
              }
              if (ok && lin != (s % n_sub)) found.push_back(lin);
            }
            std::sort(found.begin(), found.end());
            if ((int)found.size() > kMaxCover) { *code = SWR_E_SIZE; return "covering set too large"; }
            fn.count = (int32_t)found.size();
            for (size_t c = 0; c < found.size(); ++c) fn.cover[c] = geom * n_sub + found[c];
          }
          g->nodes.push_back(fn);
        }
      }
    }
    g->node_off[s + 1] = (int64_t)g->nodes.size();
  }

  // neighbour pairs and their node lists
  g->pair_i.clear();
  g->pair_j.clear();
  g->pair_off.assign(NI + 1, 0);
  g->pair_toff.assign(1, 0);
  g->pnode.clear();
  g->pnode_off.assign(1, 0);
  for (int s = 0; s < NI; ++s) {
    std::set<int> nb;
    for (int64_t q = g->node_off[s]; q < g->node_off[s + 1]; ++q)
      for (int c = 0; c < g->nodes[q].count; ++c) nb.insert(g->nodes[q].cover[c]);
    for (int j : nb) {
      g->pair_i.push_back(s);
      g->pair_j.push_back(j);
      g->pair_toff.push_back(g->pair_toff.back() + (int64_t)g->K[s] * g->K[j]);
      for (int64_t q = g->node_off[s]; q < g->node_off[s + 1]; ++q)
        for (int c = 0; c < g->nodes[q].count; ++c)
          if (g->nodes[q].cover[c] == j) g->pnode.push_back((int32_t)q);
      g->pnode_off.push_back((int64_t)g->pnode.size());
    }
    g->pair_off[s + 1] = (int64_t)g->pair_i.size();
  }

  // local orbitals: the orbital problem's rule per interval (Section 3)
  g->lo_qx.clear();
  g->lo_qw.clear();
  g->lo_qoff.assign(1, 0);
  g->lo_mx.clear();
  g->lo_mw.clear();
  if (d.basis_kind == SWR_BASIS_LSD) {
    for (int i = 0; i < g->L[0]; ++i) {  // item i: interval i in the first dimension
      const double lo = g->lo[(size_t)i * kMaxD], hi = g->hi[(size_t)i * kMaxD];
      const double xc = 0.5 * (lo + hi), dl = g->delta[(size_t)i * kMaxD];
      const double xb = d.lsd_barrier, eb = d.lsd_barrier_width;
      const double R = xb + 0.5 * eb + 10.0 / std::sqrt(dl), h = 0.25 / std::sqrt(dl);
      std::vector<double> br = {xc - R, xc - xb - 0.5 * eb, xc - xb + 0.5 * eb,
                                xc + xb - 0.5 * eb, xc + xb + 0.5 * eb, xc + R};
      std::sort(br.begin(), br.end());
      br.erase(std::unique(br.begin(), br.end()), br.end());
      std::vector<double> edges;
      for (size_t k = 0; k + 1 < br.size(); ++k) {
        const int np = std::max(1, (int)std::ceil((br[k + 1] - br[k]) / h));
        for (int j = 0; j < np; ++j) edges.push_back(br[k] + (br[k + 1] - br[k]) * j / np);
      }
      edges.push_back(br.back());
      std::vector<double> x, w;
      composite(edges, std::vector<int>(edges.size() - 1, 16), &x, &w);
      g->lo_qx.insert(g->lo_qx.end(), x.begin(), x.end());
      g->lo_qw.insert(g->lo_qw.end(), w.begin(), w.end());
      g->lo_qoff.push_back((int64_t)g->lo_qx.size());
    }
    gauss_legendre(64, &g->lo_mx, &g->lo_mw);
  }
  if (d.basis_kind == SWR_BASIS_LO) {
    // one electron in two dimensions: the rule per (item s, dimension k) at
    // lo_qoff[2 s + k] (the same recipe as the oracle's): composite
    // 16-point Gauss-Legendre on [x_c - R, x_c + R], R = x_b + eps_b / 2 +
    // 7 / sqrt(delta), breaks at the barrier's transition edges and at every
    // nucleus +- eps inside the range, panels no wider than 0.4 / sqrt(delta)
    for (int s = 0; s < NI; ++s)
      for (int k = 0; k < 2; ++k) {
        const size_t q = (size_t)s * kMaxD + k;
        const double xc = 0.5 * (g->lo[q] + g->hi[q]), dl = g->delta[q];
        const double xb = d.lsd_barrier, eb = d.lsd_barrier_width, em = d.lsd_moll_eps;
        const double R = xb + 0.5 * eb + 7.0 / std::sqrt(dl), h = 0.4 / std::sqrt(dl);
        std::vector<double> br = {xc - R, xc - xb - 0.5 * eb, xc - xb + 0.5 * eb,
                                  xc + xb - 0.5 * eb, xc + xb + 0.5 * eb, xc + R};
        for (int a = 0; a < d.n_nuc; ++a)
          for (const double e : {d.nuc_pos[a * 2 + k] - em, d.nuc_pos[a * 2 + k] + em})
            if (xc - R < e && e < xc + R) br.push_back(e);
        std::sort(br.begin(), br.end());
        br.erase(std::unique(br.begin(), br.end()), br.end());
        std::vector<double> edges;
        for (size_t b = 0; b + 1 < br.size(); ++b) {
          const int np = std::max(1, (int)std::ceil((br[b + 1] - br[b]) / h));
          for (int j = 0; j < np; ++j) edges.push_back(br[b] + (br[b + 1] - br[b]) * j / np);
        }
        edges.push_back(br.back());
        std::vector<double> x, w;
        composite(edges, std::vector<int>(edges.size() - 1, 16), &x, &w);
        g->lo_qx.insert(g->lo_qx.end(), x.begin(), x.end());
        g->lo_qw.insert(g->lo_qw.end(), w.begin(), w.end());
        g->lo_qoff.push_back((int64_t)g->lo_qx.size());
      }
    gauss_legendre(64, &g->lo_mx, &g->lo_mw);
  }

  // factored transfer entries: runs of equal face in each pair's node list
  g->te_ok = D <= 2 && d.basis_kind == SWR_BASIS_GAUSSIAN;
  g->te_pair.clear();
  g->te_face.clear();
  g->te_t0.clear();
  g->te_t1.clear();
  g->te_boff.clear();
  g->te_aoff.clear();
  g->te_xoff.clear();
  g->te_off.assign(NI + 1, 0);
  g->te_soff.assign(NI + 1, 0);
  g->te_sidx.clear();
  g->te_nb = g->te_na = g->te_nx = 0;
  if (g->te_ok) {
    for (int s = 0; s < NI; ++s) {
      for (int64_t p = g->pair_off[s]; p < g->pair_off[s + 1]; ++p) {
        const int j = g->pair_j[p];
        int64_t t = g->pnode_off[p];
        while (t < g->pnode_off[p + 1]) {
          const int face = g->nodes[g->pnode[t]].face;
          int64_t t1 = t;
          while (t1 < g->pnode_off[p + 1] && g->nodes[g->pnode[t1]].face == face) ++t1;
          const int kf = face >> 1;
          const int nbi_k = g->nb[(size_t)s * kMaxD + kf], nbj_k = g->nb[(size_t)j * kMaxD + kf];
          int nx = 1;
          if (D == 2) nx = g->nb[(size_t)s * kMaxD + (1 - kf)] * g->nb[(size_t)j * kMaxD + (1 - kf)];
          g->te_pair.push_back((int32_t)p);
          g->te_face.push_back(face);
          g->te_t0.push_back(t);
          g->te_t1.push_back(t1);
          g->te_boff.push_back(g->te_nb);
          g->te_aoff.push_back(g->te_na);
          g->te_xoff.push_back(g->te_nx);
          g->te_nb += nbi_k;
          g->te_na += nbj_k;
          g->te_nx += nx;
          t = t1;
        }
      }
      g->te_off[s + 1] = (int64_t)g->te_pair.size();
    }
    // the same entries grouped by sending item (counting sort, stable)
    const size_t ne = g->te_pair.size();
    g->te_soff.assign(NI + 1, 0);
    for (size_t e = 0; e < ne; ++e) ++g->te_soff[g->pair_j[g->te_pair[e]] + 1];
    for (int q = 0; q < NI; ++q) g->te_soff[q + 1] += g->te_soff[q];
    g->te_sidx.assign(ne, 0);
    std::vector<int64_t> fill(g->te_soff.begin(), g->te_soff.end() - 1);
    for (size_t e = 0; e < ne; ++e) g->te_sidx[fill[g->pair_j[g->te_pair[e]]]++] = (int32_t)e;
  }
  *code = SWR_OK;
  return "";
}

}  // namespace swr
