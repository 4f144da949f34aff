"""Local Galerkin matrices of one subdomain.

Paper passages followed:
  * Section 1.2: Galerkin form i A c' = (H_0 + T(t)) c with the Gram matrix
    A, the Born-Oppenheimer Hamiltonian H_0 and the dipole term
    T_jl = sum_i <x_i w_j, w_l> E(t) (length gauge, eq. (LG)).
  * Section 4.1, local expansion (eq. (exp2)) and eq. (Q): matrices
    A_i, H~_i = <v, (H_0 + R_i) v> including the Robin operator R_i, and
    Q_i = sum over electrons m of <x_m v_j, v_l>, computed once per
    subdomain.  (The printed T_i(t) = H~_i + E Q double counts H~_i; it is
    read as T_i(t) = E(t) Q_i.  The printed y/z rows drop the sum over m;
    the sum is read as included.)
  * Robin operator (Section 4.1, eq. (RTC)): from the weak form of
    -1/2 Laplacian with d_n psi = g - mu psi on the boundary,
      int(-1/2 Lap psi) v = 1/2 int grad psi . grad v + mu/2 int_bdry psi v
                            - 1/2 int_bdry g v,
    so H~_i = Kin + V + (mu/2) B with the boundary mass B, and the data g
    enters through f_l = int_bdry g v_l (the paper is silent on this term;
    the design notes list it as a reading).
  * Potential: soft-Coulomb -Z/sqrt(r^2 + eps^2) and 1/sqrt(r^2 + eps^2)
    as in eq. (pseudo) of Section 5 (Test 2.a); no nuclear repulsion.
    Integrated with composite Gauss-Legendre panels of width at most
    min(eps_en, eps_ee, sigma), quad_nodes nodes each.
  * Section 4.2 (imaginary time normalisation): the norm of the
    reconstructed function is taken with partition-of-unity weights
    1/#cover(x), giving the matrix W (reading listed in the design notes).
  * Section 4.4 step 1 and Test 1.a: projection of phi_0 restricted to
    Omega_i, c~_l = <phi_0, v_l>_{Omega_i}, then A c = c~ (a direct dense
    solve stands in for GMRES).

Pinned by: closed forms of the one-dimensional factors, the co-centred
soft-Coulomb identity with the modified Bessel function K_0, harmonic
oscillator spectra (the oracle also accepts a harmonic potential for that
pin), Gram-matrix symmetry/positivity, and, in more than one
configuration dimension, adaptive two-dimensional quadrature of the
two-electron potential on an off-diagonal subdomain and the unstaged sum
over the whole four-dimensional grid of the two-electron, two-dimension
potential (tests/test_oracle_potential_md.py).
"""
import math

import numpy as np

from . import gauss1d, lo2, quadrature, slater


def kron_all(mats):
    out = np.array([[1.0]])
    for m in mats:
        out = np.kron(out, m)
    return out


class LocalSystem:
    """All matrices of one subdomain, real FP64 (B and W included)."""

    def __init__(self, dec, s):
        cfg = dec.cfg
        D = dec.D
        self.sub = s
        self.D = D
        if slater.is_slater(s) or lo2.is_lo2(s):
            # Section 2, eq. (LSD): M = T M_E T^T over the extended tensor
            # basis; Section 3 in d = 2: over the box's own Gaussians
            if lo2.is_lo2(s):
                ext = LocalSystem(dec, lo2.gaussians(s))
                T = lo2.transform(s)
            else:
                ext = LocalSystem(dec, slater.extended(s))
                T = slater.transform(s)
            for name in ("A", "Kin", "B", "W", "Q", "V"):
                setattr(self, name, T @ getattr(ext, name) @ T.T)
            if hasattr(ext, "Q2"):
                self.Q2 = T @ ext.Q2 @ T.T
            self.mu = ext.mu
            self.Htilde = self.Kin + self.V + 0.5 * self.mu * self.B
            self.K = s.K
            return
        S, Kin, X, Bk, Wk = [], [], [], [], []
        for k in range(D):
            a, d = s.alpha[k], s.delta[k]
            lo, hi = s.lo[k], s.hi[k]
            S.append(gauss1d.overlap(a, d, lo, hi))
            Kin.append(gauss1d.kinetic(a, d, lo, hi))
            X.append(gauss1d.position(a, d, lo, hi))
            elo = gauss1d.values(a, d, [lo])[0]
            ehi = gauss1d.values(a, d, [hi])[0]
            Bk.append(np.outer(elo, elo) + np.outer(ehi, ehi))
            # partition-of-unity mass: halve the overlap bands that another
            # subdomain shares (points there are covered twice in this dim)
            w = S[k].copy()
            eps = dec.eps[k]
            if s.idx[k] > 0:
                w -= 0.5 * gauss1d.overlap(a, d, lo, lo + eps)
            if s.idx[k] < dec.L[k] - 1:
                w -= 0.5 * gauss1d.overlap(a, d, hi - eps, hi)
            Wk.append(w)
        self.S1, self.Kin1, self.X1, self.B1, self.W1 = S, Kin, X, Bk, Wk

        def embed(k, m):
            return kron_all([m if kk == k else S[kk] for kk in range(D)])

        self.A = kron_all(S)
        self.Kin = sum(embed(k, Kin[k]) for k in range(D))
        self.B = sum(embed(k, Bk[k]) for k in range(D))
        self.W = kron_all(Wk)
        # dipole matrices: x_k summed over the coordinates the field couples
        # to -- the field axis of every electron (eq. (LG)), or for the
        # circular field of Section 5, Test 3, each component's own list of
        # configuration coordinates k = electron * dim + axis
        f = cfg["field"]
        if f.get("shape", "sine") == "circular":
            self.Q, self.Q2 = (sum(embed(k, X[k]) for k in f["coords"][c]) for c in range(2))
        else:
            ax, dim = int(f["axis"]), cfg["dim"]
            self.Q = sum(embed(m * dim + ax, X[m * dim + ax]) for m in range(cfg["n_elec"]))
        self.V = potential_matrix(dec, s)
        mu = complex(cfg["mu"][0], cfg["mu"][1])
        self.mu = mu
        self.Htilde = self.Kin + self.V + 0.5 * mu * self.B
        self.K = s.K


def _panel_rule(dec, s, k, hmax):
    edges = quadrature.potential_panels(s.lo[k], s.hi[k], hmax)
    return quadrature.composite(edges, int(dec.cfg["quad_nodes"]))


def _term(dec, s, dims, rules, fvals):
    """int over the subdomain of U(x_dims) v_l v_m, with U sampled on the
    tensor grid of `rules` (fvals has one axis per dim in `dims`); every
    other dimension contributes its overlap matrix."""
    D = dec.D
    T = fvals.copy()
    for c in range(len(dims)):
        shape = [1] * len(dims)
        shape[c] = -1
        T = T * rules[c][1].reshape(shape)
    # contract one grid axis at a time with F_k[a, b, q] = phi_a(x_q) phi_b(x_q)
    cur = T
    for c, k in enumerate(dims):
        ph = gauss1d.values(s.alpha[k], s.delta[k], rules[c][0])  # (q, n)
        F = np.einsum("qa,qb->abq", ph, ph)
        n_done = 2 * c
        cur = np.tensordot(F, cur, axes=([2], [n_done]))
        perm = list(range(2, 2 + n_done)) + [0, 1] + list(range(2 + n_done, cur.ndim))
        cur = np.transpose(cur, perm)
    # cur axes: (a, b) pairs in the order of `dims`; append the other dims
    order = list(dims)
    for k in range(D):
        if k not in dims:
            cur = np.multiply.outer(cur, gauss1d.overlap(s.alpha[k], s.delta[k],
                                                         s.lo[k], s.hi[k]))
            order.append(k)
    pos = {k: i for i, k in enumerate(order)}
    perm = [2 * pos[k] for k in range(D)] + [2 * pos[k] + 1 for k in range(D)]
    cur = np.transpose(cur, perm)
    return cur.reshape(s.K, s.K)


# Grids above this many points are summed one node of their first dimension
# at a time (the same sum, split to bound memory: a four-dimensional grid of
# 176 nodes per dimension would need tens of GB at once).
_SLICE_POINTS = 30_000_000


def _grid_term(dec, s, dims, rules, ufunc):
    """int over the subdomain of U(x_dims) v_l v_m on the tensor grid of
    `rules`, with U = ufunc(grids) evaluated on the grid."""
    n_pts = int(np.prod([len(r[0]) for r in rules]))
    if n_pts <= _SLICE_POINTS:
        grids = np.meshgrid(*[r[0] for r in rules], indexing="ij")
        return _term(dec, s, dims, rules, ufunc(grids))
    x0, w0 = rules[0]
    out = np.zeros((s.K, s.K))
    for q in range(len(x0)):
        r0 = (x0[q:q + 1], w0[q:q + 1])
        sub = [r0] + list(rules[1:])
        grids = np.meshgrid(*[r[0] for r in sub], indexing="ij")
        out += _term(dec, s, dims, sub, ufunc(grids))
    return out


def potential_matrix(dec, s):
    cfg = dec.cfg
    D = dec.D
    N, d = cfg["n_elec"], cfg["dim"]
    K = s.K
    V = np.zeros((K, K))
    kind = cfg.get("potential", "soft_coulomb")
    sig = [float(np.sqrt(0.5 / s.delta[k][0])) for k in range(D)]
    if kind == "harmonic":
        # U = 1/2 w^2 |x|^2, separable: one term per dimension
        w2 = float(cfg["omega_ho"]) ** 2
        for k in range(D):
            rule = _panel_rule(dec, s, k, sig[k])
            V += _term(dec, s, [k], [rule], 0.5 * w2 * rule[0] ** 2)
        return V
    if kind != "soft_coulomb":
        raise ValueError(kind)
    eps_en, eps_ee = float(cfg["eps_en"]), float(cfg["eps_ee"])
    nuc = [np.asarray(p, dtype=np.float64) for p in cfg["nuclei"]]
    Z = [float(z) for z in cfg["charges"]]
    rules = [_panel_rule(dec, s, k, min(eps_en, eps_ee, sig[k])) for k in range(D)]
    # electron-nucleus: one d-dimensional term per electron
    if nuc:
        def u_en(grids):
            U = np.zeros(grids[0].shape)
            for RA, ZA in zip(nuc, Z):
                r2 = sum((grids[a] - RA[a]) ** 2 for a in range(d))
                U -= ZA / np.sqrt(r2 + eps_en * eps_en)
            return U
        for m in range(N):
            dims = [m * d + a for a in range(d)]
            V += _grid_term(dec, s, dims, [rules[k] for k in dims], u_en)
    # electron-electron: one 2d-dimensional term per pair

    def u_ee(grids):
        r2 = sum((grids[a] - grids[d + a]) ** 2 for a in range(d))
        return 1.0 / np.sqrt(r2 + eps_ee * eps_ee)
    for m in range(N):
        for mp in range(m + 1, N):
            dims = [m * d + a for a in range(d)] + [mp * d + a for a in range(d)]
            V += _grid_term(dec, s, dims, [rules[k] for k in dims], u_ee)
    return V


def projection_rhs(dec, s):
    """c~_l = <phi_0, v_l>_{Omega_i} for the Gaussian initial state (or, in
    the Slater basis, its antisymmetrised form)."""
    cfg = dec.cfg
    D = dec.D
    alpha0 = float(cfg["init"]["alpha"])
    cen = [float(c) for c in cfg["init"]["center"]]
    if lo2.is_lo2(s):
        return lo2.transform(s) @ projection_rhs(dec, lo2.gaussians(s))
    if slater.is_slater(s):
        ext = slater.extended(s)
        proj = [[gauss1d.gaussian_projection(ext.alpha[k], ext.delta[k], s.lo[k], s.hi[k],
                                             alpha0, c) for c in cen] for k in range(2)]
        b = np.kron(proj[0][0], proj[1][1]) - np.kron(proj[0][1], proj[1][0])
        return slater.transform(s) @ (slater.initial_norm(alpha0, cen[0], cen[1]) * b)
    norm = (2.0 * alpha0 / math.pi) ** (0.25 * D)
    vecs = [gauss1d.gaussian_projection(s.alpha[k], s.delta[k], s.lo[k], s.hi[k],
                                        alpha0, cen[k]) for k in range(D)]
    out = np.array([norm])
    for v in vecs:
        out = np.kron(out, v)
    return out


def project_initial(dec, s, A):
    """Local Cauchy data: solve A c = c~ (Section 4.4 step 1)."""
    return np.linalg.solve(A, projection_rhs(dec, s))
