"""Domain decomposition, local Gaussian bases, faces and covering sets.

Paper passages followed:
  * Section 4 (SWR): R^{dN} is decomposed into L^{dN} overlapping
    hypercubes; interfaces Gamma_{i;j} = boundary(Omega_i) cap Omega_j.
  * Section 5 (opening paragraph): global box
    [a - eps/2, b + eps/2], a_i = a + (i-1)(b-a)/L, b_i = a + i(b-a)/L,
    Omega_{i+Lj} = [a_i - eps/2, b_i + eps/2] x [c_j - eps/2, d_j + eps/2]
    (the printed c_i = c + i(d-c)/L is read as c + (i-1)(d-c)/L).
  * Section 3.4 (notations): Lambda_{i,j} is re-indexed Omega_{i+jL}; the
    linear index generalises with the first dimension fastest.
  * Section 2 / Test 1.a: tensor products of 1-D Gaussians whose centres
    are "uniformly distributed" in the subdomain (read: equispaced,
    including both ends, so that interface traces are not negligible).
    Optionally (basis_extend = e > 0) the equispaced centres run e spacings
    beyond each end, in the spirit of the augmented bases of Section 3.3
    (Gaussians added around the subdomain so that transmission is
    represented well).
  * Section 4.1, multi-subdomain overlapping zones: the set O of
    subdomains other than Omega_i sharing a zone with it, with
    Card O = 2^{dN} - 1 in interior corner zones.  Read with closed
    membership y in closure(Omega_j).

Readings (listed in the design notes): the stated box is the outer box
[a - eps/2, b + eps/2]; centres equispaced with both ends; sigma from
`width` or `width_ratio * spacing`; faces on the global boundary carry the
Robin operator with zero data (absorbing).

Pinned by: hand-enumerated decompositions (2x2 and 3x3) and the Card O
count of the paper's corner zone (tests/golden/).
"""
import itertools

import numpy as np

from . import quadrature


class Subdomain:
    """One hypercube Omega_i with its local tensor Gaussian basis."""

    def __init__(self, lin, idx, lo, hi, alpha, delta):
        self.lin = lin                  # linear index (first dim fastest)
        self.idx = tuple(idx)           # multi-index
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.alpha = [np.asarray(a, dtype=np.float64) for a in alpha]
        self.delta = [np.asarray(d, dtype=np.float64) for d in delta]
        self.nb = tuple(len(a) for a in alpha)
        self.K = int(np.prod(self.nb))
        self.faces = []

    @property
    def D(self):
        return len(self.lo)


class Face:
    """Face x_k = lo_k (side 0) or x_k = hi_k (side 1) of a subdomain."""

    def __init__(self, k, side, is_global, nodes, weights, cover):
        self.k = k
        self.side = side
        self.is_global = is_global
        self.nodes = nodes              # (n_y, D) points on the face
        self.weights = weights          # (n_y,) tangential quadrature weights
        self.cover = cover              # list (per node) of sorted lists of j
        self.normal_sign = 1.0 if side == 1 else -1.0


class Decomposition:
    def __init__(self, cfg):
        self.cfg = cfg
        D = cfg["n_elec"] * cfg["dim"]
        self.D = D
        self.L = [int(v) for v in cfg["L"]]
        self.n_sub = int(np.prod(self.L))
        self.strides = [int(np.prod(self.L[:k])) for k in range(D)]
        eps = [float(e) for e in cfg["overlap"]]
        self.eps = eps
        # per-dimension interval ends lo[k][i], hi[k][i]
        self.lo1, self.hi1 = [], []
        for k in range(D):
            a = float(cfg["box_lo"][k]) + 0.5 * eps[k]
            b = float(cfg["box_hi"][k]) - 0.5 * eps[k]
            h = (b - a) / self.L[k]
            self.lo1.append([(a + i * h) - 0.5 * eps[k] for i in range(self.L[k])])
            self.hi1.append([(a + (i + 1) * h) + 0.5 * eps[k] for i in range(self.L[k])])
        self.subs = []
        for lin in range(self.n_sub):
            idx = self.multi_index(lin)
            lo = [self.lo1[k][idx[k]] for k in range(D)]
            hi = [self.hi1[k][idx[k]] for k in range(D)]
            nb = self.nbasis(lin)
            alpha, delta = [], []
            for k in range(D):
                n = nb[k]
                ext = int(cfg.get("basis_extend", 0))
                if n == 1:
                    cen = np.array([0.5 * (lo[k] + hi[k])])
                    sp = hi[k] - lo[k]
                else:
                    sp = (hi[k] - lo[k]) / (n - 1 - 2 * ext)
                    first = lo[k] - ext * sp
                    cen = np.array([first + j * sp for j in range(n)])
                if cfg.get("width") is not None:
                    sigma = float(cfg["width"])
                else:
                    sigma = float(cfg["width_ratio"]) * sp
                alpha.append(cen)
                delta.append(np.full(n, 0.5 / (sigma * sigma)))
            self.subs.append(Subdomain(lin, idx, lo, hi, alpha, delta))
        if cfg.get("basis", "gaussian") == "slater":
            # Section 2, eq. (LSD): antisymmetrised pairs (oracle/slater.py)
            from . import slater
            for s in self.subs:
                s.slater = True
                s.K = len(slater.pairs(s))
        if cfg.get("basis", "gaussian") == "lsd":
            # Section 3: determinants of local orbitals (oracle/lsd.py); the
            # orbitals of interval i from its Gaussians in the first
            # dimension (the decomposition is exchange-symmetric)
            from . import lsd, slater
            orb = {}
            for s in self.subs:
                for k in range(2):
                    i = s.idx[k]
                    if i not in orb and k == 0:
                        orb[i] = lsd.orbitals(cfg, s.alpha[0], s.delta[0], s.lo[0], s.hi[0])
            self.orbital_energies = {i: v[0] for i, v in orb.items()}
            for s in self.subs:
                s.slater = True
                s.lsd = True
                s.lo_coef = [orb[s.idx[0]][1], orb[s.idx[1]][1]]
                s.K = len(slater.pairs(s))
        if cfg.get("basis", "gaussian") == "lo":
            # Section 3 in d = 2, one electron: each box's local orbitals in
            # its tensor Gaussians (oracle/lo2.py)
            from . import lo2
            self.orbital_energies = {}
            for s in self.subs:
                lam, C = lo2.orbitals2(cfg, s)
                s.lo2 = True
                s.lo_coef = C
                s.K = C.shape[1]
                self.orbital_energies[s.lin] = lam
        for s in self.subs:
            s.faces = self._faces(s)

    # -- indexing ---------------------------------------------------------
    def multi_index(self, lin):
        idx = []
        for k in range(self.D):
            idx.append(lin % self.L[k])
            lin //= self.L[k]
        return tuple(idx)

    def linear_index(self, idx):
        return int(sum(i * s for i, s in zip(idx, self.strides)))

    def nbasis(self, lin):
        nb = self.cfg["nbasis"]
        if isinstance(nb[0], (list, tuple)):
            return [int(v) for v in nb[lin]]
        return [int(v) for v in nb]

    # -- faces --------------------------------------------------------------
    def _tangential_rule(self, s, t):
        cfgn = self.cfg["face_nodes"]
        edges = quadrature.face_panels(s.lo[t], s.hi[t], self.eps[t])
        return quadrature.composite(edges, [cfgn[0], cfgn[1], cfgn[0]])

    def face_rule(self, s, k, side):
        """Tensor Gauss-Legendre nodes on face (k, side): last tangential
        dimension fastest."""
        D = self.D
        tang = [t for t in range(D) if t != k]
        xk = s.hi[k] if side == 1 else s.lo[k]
        if not tang:
            return np.array([[xk]]), np.array([1.0])
        rules = [self._tangential_rule(s, t) for t in tang]
        grids = np.meshgrid(*[r[0] for r in rules], indexing="ij")
        wgrid = np.meshgrid(*[r[1] for r in rules], indexing="ij")
        n_y = grids[0].size
        nodes = np.empty((n_y, D))
        nodes[:, k] = xk
        w = np.ones(n_y)
        for c, t in enumerate(tang):
            nodes[:, t] = grids[c].ravel()
            w = w * wgrid[c].ravel()
        return nodes, w

    def covers(self, lin, ys):
        """O(y) for every point y of ys: each j != lin with y in the closure
        of Omega_j, checked against all subdomains, increasing linear index."""
        LO = np.array([j.lo for j in self.subs])
        HI = np.array([j.hi for j in self.subs])
        inside = np.all((LO[None, :, :] <= ys[:, None, :]) &
                        (ys[:, None, :] <= HI[None, :, :]), axis=2)
        inside[:, lin] = False
        return [list(np.nonzero(row)[0]) for row in inside]

    def _faces(self, s):
        faces = []
        for k in range(self.D):
            for side in (0, 1):
                is_global = (side == 0 and s.idx[k] == 0) or \
                            (side == 1 and s.idx[k] == self.L[k] - 1)
                nodes, w = self.face_rule(s, k, side)
                cover = None if is_global else self.covers(s.lin, nodes)
                faces.append(Face(k, side, is_global, nodes, w, cover))
        return faces

    def cover_count(self, x):
        """Number of subdomains whose closure holds the point x."""
        return sum(1 for j in self.subs if np.all(j.lo <= x) and np.all(x <= j.hi))
