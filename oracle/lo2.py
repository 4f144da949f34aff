"""Local orbitals of one electron in two dimensions (test infrastructure: the
CPU oracle, never called by the product path).

Paper passages followed: Section 3 (local orbital construction: the
mollified nuclear attraction, eqs. (GEPS), (Beps), the barrier of eq.
(BARPOT) with its kinetic coefficient a_eps, and the one-electron
eigenproblem per subdomain), taken in d = 2, where the bare Coulomb kernel
-1/|x| is locally integrable and its convolution with B_eps is finite.

The basis of a subdomain (a box with centre x_c and tensor Gaussians
g_u(x) = g_{u0}(x_0) g_{u1}(x_1), last index fastest) is its M lowest
orbitals, the eigenfunctions of

    h = -1/2 div(a grad) + V_n + V_b,
    a(x)   = prod_k (1 - s(|x_k - x_ck| - x_b)),
    V_b(x) = V_inf sum_k s(|x_k - x_ck| - x_b),
    V_n(x) = sum_A -Z_A G(|x - R_A|),   G = (1/|.|) * B_eps,
    B_eps(y) = (sigma / eps^2) (1 - |y|^2 / eps^2)^M on |y| <= eps,
    sigma = (M + 1) / pi  (so that B_eps integrates to one over the plane),

discretised in the box's Gaussians over the plane (a generalised symmetric
eigenproblem with the overlap S and h's matrix H), S-normalised and signed
so that sum_u (u + 1) C[u, l] > 0.  Every matrix of the subdomain is then
T M_G T^T with T = C^T and M_G the box's Gaussian matrices (oracle/assemble.py).

G is radial.  With s the distance of the mollifier's mass from its centre,
averaging 1/|x - y| over the circle of radius s gives a complete elliptic
integral of the first kind (parameter m = 4 rho s / (rho + s)^2):

    G(rho) = int_0^eps B(s) s 4 K(m) / (rho + s) ds,

evaluated by double-exponential (tanh-sinh) quadrature split at s = rho,
where K has a logarithmic singularity (K is taken as K(1 - p) with
p = ((rho - s) / (rho + s))^2 formed from the distance |rho - s|).

Readings (listed in the design notes): the one-dimensional barrier and
coefficient become a tensor product and a sum over the coordinates (so that
S, the kinetic and the barrier terms are products of one-dimensional
integrals); every nucleus enters mollified (d = 2 makes V * B_eps finite
everywhere, and the orbital problem is posed on the plane, where the other
boxes' nuclei also lie); the 1 / (4 pi) of eq. (GEPS) belongs to the
three-dimensional Poisson scaling and is dropped, so that G tends to the
Coulomb attraction as eps -> 0.

Pinned by (tests/test_oracle_lo2.py): G(0) in closed form; the far-field
expansion G(rho) = 1/rho (1 + eps^2 / (4 (M + 2) rho^2)) + O(eps^4 / rho^5);
G at points inside and outside the support against two-dimensional adaptive
quadrature of the convolution; every entry of S and H against adaptive
quadrature of its definition; the orbitals' eigen-residual and
S-orthonormality; and, with every orbital kept (M = n_0 n_1), SWR windows
equal to the Gaussian basis's (the same function space).
"""
import math

import numpy as np
import scipy.linalg
import scipy.special

from . import lsd


def _params(cfg):
    p = cfg["lo"]
    return (int(p["orbitals"]), float(p["barrier"]), float(p["barrier_width"]),
            float(p["v_inf"]), float(p["moll_eps"]), int(p["moll_order"]))


def sigma2(order):
    """sigma with int_{R^2} B_eps = 1: (order + 1) / pi."""
    return (order + 1) / math.pi


def mollifier2(r, eps, order):
    """B_eps at distance r from its centre."""
    r = np.asarray(r, dtype=float)
    t = r / eps
    return np.where(r <= eps, sigma2(order) / (eps * eps) * (1.0 - t * t) ** order, 0.0)


def _tanh_sinh(n_half=60, h=1.0 / 16.0):
    """Nodes of the double-exponential rule on [-1, 1] as distances to the
    two ends (1 + x, 1 - x) and weights."""
    t = h * np.arange(-n_half, n_half + 1)
    u = 0.5 * math.pi * np.sinh(t)
    w = h * 0.5 * math.pi * np.cosh(t) / np.cosh(u) ** 2
    # 1 - x and 1 + x without cancellation
    one_minus = 2.0 / (1.0 + np.exp(2.0 * u))
    one_plus = 2.0 / (1.0 + np.exp(-2.0 * u))
    return one_plus, one_minus, w


_TS = _tanh_sinh()


def _panel(rho, a, b, eps, order, toward):
    """int_a^b B(s) s 4 K / (rho + s) ds for one rho; the singular end
    s = rho is b when toward == 'hi', a when 'lo' (or none)."""
    if b <= a:
        return 0.0
    one_plus, one_minus, w = _TS
    half = 0.5 * (b - a)
    if toward == "hi":
        d = half * one_minus          # distance to b = rho
        s = b - d
    else:
        d = half * one_plus           # distance to a
        s = a + d
    if toward in ("hi", "lo"):
        p = (d / (rho + s)) ** 2      # 1 - m, m = 4 rho s / (rho + s)^2
    else:
        p = ((rho - s) / (rho + s)) ** 2
    K = scipy.special.ellipkm1(p)
    f = mollifier2(s, eps, order) * s * 4.0 * K / (rho + s)
    return float(half * np.sum(w * f))


def coulomb_mollified2(rho, eps, order):
    """(1/|.| * B_eps)(x) at |x| = rho (positive; the attraction of a charge
    Z is -Z times it)."""
    rho = float(rho)
    if rho == 0.0:
        # 4 K(0) / s = 2 pi / s: G(0) = 2 pi int_0^eps B(s) ds
        return 2.0 * math.pi * _plain(lambda s: mollifier2(s, eps, order), 0.0, eps)
    if rho <= eps:
        return (_panel(rho, 0.0, rho, eps, order, "hi")
                + _panel(rho, rho, eps, eps, order, "lo"))
    return _panel(rho, 0.0, eps, eps, order, "none")


def _plain(f, a, b):
    one_plus, _, w = _TS
    half = 0.5 * (b - a)
    return float(half * np.sum(w * f(a + half * one_plus)))


def coulomb_mollified2_many(rho, eps, order, chunk=4096):
    """coulomb_mollified2 at every entry of rho (the same quadrature)."""
    rho = np.asarray(rho, dtype=float)
    flat = rho.ravel()
    out = np.empty_like(flat)
    one_plus, one_minus, w = _TS
    g0 = coulomb_mollified2(0.0, eps, order)

    def f(s, r, p):
        return mollifier2(s, eps, order) * s * 4.0 * scipy.special.ellipkm1(p) / (r + s)

    for a in range(0, flat.size, chunk):
        r = flat[a:a + chunk][:, None]
        res = np.empty(r.shape[0])
        zero = r[:, 0] == 0.0
        inside = (r[:, 0] <= eps) & ~zero
        ri = r[inside]
        if ri.size:
            h1 = 0.5 * ri
            d1 = h1 * one_minus
            s1 = ri - d1
            v1 = np.sum(w * f(s1, ri, (d1 / (ri + s1)) ** 2), axis=1) * h1[:, 0]
            v2 = np.zeros_like(v1)
            wide = ri[:, 0] < eps       # the panel [rho, eps] is empty at rho = eps
            rw = ri[wide]
            if rw.size:
                h2 = 0.5 * (eps - rw)
                d2 = h2 * one_plus
                s2 = rw + d2
                v2[wide] = np.sum(w * f(s2, rw, (d2 / (rw + s2)) ** 2), axis=1) * h2[:, 0]
            res[inside] = v1 + v2
        outside = r[:, 0] > eps
        ro = r[outside]
        if ro.size:
            s3 = 0.5 * eps * one_plus
            res[outside] = 0.5 * eps * np.sum(w * f(s3, ro, ((ro - s3) / (ro + s3)) ** 2), axis=1)
        res[zero] = g0
        out[a:a + chunk] = res
    return out.reshape(rho.shape)


def nuclear_potential2(cfg, x0, x1):
    """V_n on the grid x0 (n0) x x1 (n1): every nucleus mollified."""
    _, _, _, _, eps, order = _params(cfg)
    X0, X1 = np.meshgrid(x0, x1, indexing="ij")
    out = np.zeros_like(X0)
    for R, Z in zip(cfg["nuclei"], cfg["charges"]):
        rho = np.hypot(X0 - R[0], X1 - R[1])
        out = out - Z * coulomb_mollified2_many(rho, eps, order)
    return out


_GL16 = np.polynomial.legendre.leggauss(16)


def _rule(s, k, cfg):
    """Composite 16-point Gauss-Legendre on [x_c - R, x_c + R] in dimension
    k, R = x_b + eps_b / 2 + 7 / sqrt(min delta), with breaks at the
    barrier's transition edges and at every nucleus +- eps (inside the
    range), panels no wider than 0.4 / sqrt(max delta)."""
    _, xb, eb, _, eps, _ = _params(cfg)
    d = s.delta[k]
    xc = 0.5 * (s.lo[k] + s.hi[k])
    R = xb + 0.5 * eb + 7.0 / math.sqrt(float(np.min(d)))
    h = 0.4 / math.sqrt(float(np.max(d)))
    edges = {xc - R, xc - xb - 0.5 * eb, xc - xb + 0.5 * eb, xc + xb - 0.5 * eb,
             xc + xb + 0.5 * eb, xc + R}
    for nuc in cfg["nuclei"]:
        for e in (nuc[k] - eps, nuc[k] + eps):
            if xc - R < e < xc + R:
                edges.add(e)
    edges = sorted(edges)
    xs, ws = [], []
    t, wt = _GL16
    for a, b in zip(edges[:-1], edges[1:]):
        n = max(1, int(math.ceil((b - a) / h)))
        for q in range(n):
            lo, hi = a + (b - a) * q / n, a + (b - a) * (q + 1) / n
            xs.append(0.5 * (hi - lo) * t + 0.5 * (hi + lo))
            ws.append(0.5 * (hi - lo) * wt)
    return np.concatenate(xs), np.concatenate(ws)


def orbital_matrices2(cfg, s):
    """S and H of the box's orbital problem in its tensor Gaussians."""
    _, xb, eb, vinf, _, _ = _params(cfg)
    one = []
    grids = []
    for k in range(2):
        x, w = _rule(s, k, cfg)
        cen, dl = s.alpha[k], s.delta[k]
        xc = 0.5 * (s.lo[k] + s.hi[k])
        g = np.exp(-dl[None, :] * (x[:, None] - cen[None, :]) ** 2)
        dg = -2.0 * dl[None, :] * (x[:, None] - cen[None, :]) * g
        st = lsd.smooth_step(np.abs(x - xc) - xb, eb)
        a = 1.0 - st
        one.append(dict(S=(g * w[:, None]).T @ g, A=(g * (w * a)[:, None]).T @ g,
                        Ad=(dg * (w * a)[:, None]).T @ dg, Bs=(g * (w * st)[:, None]).T @ g))
        grids.append((x, w, g))
    o0, o1 = one
    S = np.kron(o0["S"], o1["S"])
    H = 0.5 * (np.kron(o0["Ad"], o1["A"]) + np.kron(o0["A"], o1["Ad"]))
    H = H + vinf * (np.kron(o0["Bs"], o1["S"]) + np.kron(o0["S"], o1["Bs"]))
    (x0, w0, g0), (x1, w1, g1) = grids
    V = nuclear_potential2(cfg, x0, x1) * w0[:, None] * w1[None, :]
    # N[(u0,u1),(w0,w1)] = sum_{q0,q1} V[q0,q1] g0[q0,u0] g0[q0,w0] g1[q1,u1] g1[q1,w1]
    N = np.einsum("pq,pa,pc,qb,qd->abcd", V, g0, g0, g1, g1, optimize=True)
    n0, n1 = g0.shape[1], g1.shape[1]
    H = H + N.reshape(n0 * n1, n0 * n1)
    return S, H


def orbitals2(cfg, s):
    """C (n0 n1 x M): the M lowest orbitals, S-normalised, signed."""
    M = _params(cfg)[0]
    S, H = orbital_matrices2(cfg, s)
    lam, C = scipy.linalg.eigh(H, S)
    C = C[:, :M].copy()
    wts = np.arange(1, C.shape[0] + 1, dtype=float)
    for l in range(M):
        if wts @ C[:, l] < 0.0:
            C[:, l] = -C[:, l]
    return lam[:M], C


def is_lo2(s):
    return getattr(s, "lo2", False)


def gaussians(s):
    """The box's own tensor Gaussian basis (a plain Subdomain)."""
    from .geometry import Subdomain
    return Subdomain(s.lin, s.idx, s.lo, s.hi, s.alpha, s.delta)


def transform(s):
    """T with v = T g (rows: orbitals, columns: tensor Gaussians)."""
    return s.lo_coef.T
