"""Local orbitals and local Slater determinants (test infrastructure: the
CPU oracle, never called by the product path).

Paper passages followed: Section 3 (local orbitals and local Slater
determinants), eqs. (GEPS), (Beps), (BARPOT), and the one-electron
eigenproblem of Section 3.2; eq. (LSD) for the determinants.

Local orbitals.  For every interval D_i of the one-dimensional
decomposition, with centre x_c (the middle of the interval's box), the
orbitals are the M lowest eigenfunctions of

    h = -1/2 d/dx (a(x) d/dx) + V_n(x) + V_b(x),
    a(x) = 1 - s(|x - x_c| - x_b),   V_b(x) = V_inf s(|x - x_c| - x_b),

with s the smooth step from 0 (at t = -eps_b/2) to 1 (at t = +eps_b/2),
discretised in the interval's Gaussians (a generalised eigenproblem with
the overlap S and h's matrix H over the real line).  V_n sums the nuclei:
for a nucleus inside the interval's box the soft-Coulomb attraction of eq.
(pseudo) smoothed by the polynomial mollifier,

    G(x) = (V * B_eps)(x),   B_eps(x) = (sigma_M / eps) (1 - (x/eps)^2)^M
    on |x| <= eps (zero outside), sigma_M = 1 / int_{-1}^{1} (1 - t^2)^M dt,

and the soft-Coulomb attraction itself for the other nuclei.  Each orbital
is S-normalised and signed so that sum_u (u + 1) C[u, l] > 0.

Determinants.  On the two-dimensional subdomain of intervals (i, j), with
orbitals phi_l of the first and psi_p of the second,

    v_{l,p}(x1, x2) = (phi_l(x1) psi_p(x2) - phi_l(x2) psi_p(x1)) / sqrt(2),

l slowest; l < p when i = j (v_{l,p} = -v_{p,l}).  In the extended tensor
basis E_{a,b} = U_a(x1) U_b(x2) of the two intervals' Gaussians
(oracle/slater.py) v_{l,p} = sum_{u,w} C_i[u,l] C_j[w,p] (E_{u,n+w} -
E_{n+w,u}) / sqrt(2), so the Galerkin matrices are T M_E T^T as for the
Slater-like Gaussian basis.

Augmented local bases (Section 3.3): the orbitals vanish near the ends of
their interval, so the determinants are small in the overlaps and transmit
little.  The interval's g Gaussians nearest each end of its box (its
centres are equispaced with both ends, so g = 1 adds the Gaussians centred
on the box's ends) join the orbitals as further one-electron functions; the
pairs then run over the M + 2g functions, which keeps every basis function
antisymmetric and puts functions along all four edges of the subdomain.

Readings (listed in the design notes): the barrier is symmetric about the
interval's centre; the garbled step definition is read as a C^2 quintic
from 0 to 1 across [-eps_b/2, eps_b/2]; the one-dimensional Coulomb kernel
-1/|x| is not locally integrable, so the mollifier smooths the
soft-Coulomb term of eq. (pseudo) (the two-electron Hamiltonian keeps the
soft-Coulomb terms); a nucleus counts as inside an interval when it lies in
the interval's box; the orbital problem is posed on the real line in the
interval's Gaussians.

Pinned by (tests/test_oracle_lsd.py): the mollifier's normalisations
against the values the paper prints (3/4, 15/16, 315/256); the O(eps^2)
approach of the mollified potential to the unmollified one; every entry of
the orbital problem's S and H against adaptive quadrature of its
definition; the orbitals' residual and S-orthonormality; the determinants'
antisymmetry and their matrices against two-dimensional adaptive
quadrature; and, with as many orbitals as Gaussians (the same function
space as the Slater-like basis), SWR windows equal to the Slater basis's.
"""
import math

import numpy as np
import scipy.linalg

_GL16 = np.polynomial.legendre.leggauss(16)
_GL64 = np.polynomial.legendre.leggauss(64)


def sigma(order):
    """sigma_M = 1 / int_{-1}^{1} (1 - t^2)^M dt = (2M+1)! / (2^(2M+1) (M!)^2)."""
    return math.factorial(2 * order + 1) / (2.0 ** (2 * order + 1) * math.factorial(order) ** 2)


def mollifier(x, eps, order):
    """B_eps(x) of eq. (Beps)."""
    x = np.asarray(x, dtype=float)
    t = x / eps
    return np.where(np.abs(x) <= eps, sigma(order) / eps * (1.0 - t * t) ** order, 0.0)


def soft_coulomb(x, Z, eta):
    return -Z / np.sqrt(x * x + eta * eta)


def mollified(x, Z, eta, eps, order):
    """(V * B_eps)(x) for the soft-Coulomb V = -Z / sqrt(x^2 + eta^2),
    by 64-point Gauss-Legendre over the mollifier's support."""
    t, w = _GL64
    y = eps * t
    x = np.asarray(x, dtype=float)
    vals = soft_coulomb(x[..., None] - y, Z, eta) * mollifier(y, eps, order)
    return (vals * (eps * w)).sum(axis=-1)


def smooth_step(t, width):
    """0 below -width/2, 1 above width/2, the C^2 quintic between."""
    u = np.clip(np.asarray(t, dtype=float) / width + 0.5, 0.0, 1.0)
    return u * u * u * (10.0 - 15.0 * u + 6.0 * u * u)


def _params(cfg):
    p = cfg["lsd"]
    return (int(p["orbitals"]), float(p["barrier"]), float(p["barrier_width"]),
            float(p["v_inf"]), float(p["moll_eps"]), int(p["moll_order"]))


def _rule(xc, xb, eb, reach, h):
    """Composite 16-point Gauss-Legendre over [xc - R, xc + R] with breaks
    at the barrier's transition edges and panels no wider than h."""
    R = xb + 0.5 * eb + reach
    edges = sorted({xc - R, xc - xb - 0.5 * eb, xc - xb + 0.5 * eb,
                    xc + xb - 0.5 * eb, xc + xb + 0.5 * eb, xc + R})
    xs, ws = [], []
    t, w = _GL16
    for a, b in zip(edges[:-1], edges[1:]):
        n = max(1, int(math.ceil((b - a) / h)))
        for k in range(n):
            lo, hi = a + (b - a) * k / n, a + (b - a) * (k + 1) / n
            xs.append(0.5 * (hi - lo) * t + 0.5 * (hi + lo))
            ws.append(0.5 * (hi - lo) * w)
    return np.concatenate(xs), np.concatenate(ws)


def nuclear_potential(cfg, x, lo, hi):
    """V_n at x for an interval with box [lo, hi]."""
    eta = float(cfg["eps_en"])
    _, _, _, _, eps, order = _params(cfg)
    out = np.zeros_like(np.asarray(x, dtype=float))
    for R, Z in zip(cfg["nuclei"], cfg["charges"]):
        if lo <= R[0] <= hi:
            out = out + mollified(x - R[0], Z, eta, eps, order)
        else:
            out = out + soft_coulomb(x - R[0], Z, eta)
    return out


def orbital_matrices(cfg, cen, delta, lo, hi):
    """S and H of the orbital problem in the Gaussians (centres cen,
    exponents delta) of the interval with box [lo, hi]."""
    _, xb, eb, vinf, _, _ = _params(cfg)
    xc = 0.5 * (lo + hi)
    reach = 10.0 / math.sqrt(float(np.min(delta)))
    x, w = _rule(xc, xb, eb, reach, 0.25 / math.sqrt(float(np.max(delta))))
    g = np.exp(-delta[None, :] * (x[:, None] - cen[None, :]) ** 2)
    dg = -2.0 * delta[None, :] * (x[:, None] - cen[None, :]) * g
    step = smooth_step(np.abs(x - xc) - xb, eb)
    a = 1.0 - step
    v = nuclear_potential(cfg, x, lo, hi) + vinf * step
    S = (g * w[:, None]).T @ g
    H = 0.5 * (dg * (w * a)[:, None]).T @ dg + (g * (w * v)[:, None]).T @ g
    return S, H


def augment(cfg):
    """Gaussians added per end of each interval (Section 3.3); 0 if absent."""
    return int(cfg["lsd"].get("augment", 0))


def orbitals(cfg, cen, delta, lo, hi):
    """C (n x M'): the M lowest orbitals, S-normalised, signed, then (Section
    3.3, augmented local bases) the interval's g Gaussians nearest each end
    of its box as unit columns (the first g, then the last g from the end
    inwards); M' = M + 2g."""
    M = _params(cfg)[0]
    g = augment(cfg)
    S, H = orbital_matrices(cfg, cen, delta, lo, hi)
    lam, C = scipy.linalg.eigh(H, S)
    C = C[:, :M].copy()
    wts = np.arange(1, C.shape[0] + 1, dtype=float)
    for l in range(M):
        if wts @ C[:, l] < 0.0:
            C[:, l] = -C[:, l]
    n = C.shape[0]
    extra = [a for a in range(g)] + [n - 1 - a for a in range(g)]
    E = np.zeros((n, len(extra)))
    for c, u in enumerate(extra):
        E[u, c] = 1.0
    return lam[:M], np.concatenate([C, E], axis=1)


def is_lsd(s):
    return getattr(s, "lsd", False)


def pairs(s):
    M = s.lo_coef[0].shape[1]
    if s.idx[0] == s.idx[1]:
        return [(l, p) for l in range(M) for p in range(l + 1, M)]
    return [(l, p) for l in range(M) for p in range(M)]


def transform(s):
    """T with v = T E over the extended tensor basis (oracle/slater.py)."""
    n = len(s.alpha[0])
    m2 = 2 * n
    C1, C2 = s.lo_coef
    r = 1.0 / math.sqrt(2.0)
    pr = pairs(s)
    T = np.zeros((len(pr), m2 * m2))
    for m, (l, p) in enumerate(pr):
        c = r * np.outer(C1[:, l], C2[:, p])  # [u, w]
        blk = np.zeros((m2, m2))
        blk[:n, n:] += c
        blk[n:, :n] -= c.T
        T[m] = blk.ravel()
    return T
