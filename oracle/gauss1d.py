"""Integrals of products of one-dimensional Gaussians over a bounded interval.

Paper: Section 2, eq. (gauss1d) defines the local Gaussians
phi_j(x) = exp(-delta (x - alpha_j)^2); Section 4.1 (local expansion and
the matrices A_i, H_i, Q_i) takes every inner product over the subdomain
Omega_i itself (Section 5.1, Test 1.a, writes the Gram matrix as an L2 inner
product on Omega_i).  For a tensor-product basis the D-dimensional integrals
factor into the one-dimensional ones computed here.

Closed forms (Gaussian product rule): phi_a phi_b = E exp(-p (x-P)^2) with
p = d_a + d_b, P = (d_a a_a + d_b a_b)/p, E = exp(-d_a d_b (a_a-a_b)^2/p);
the moments of exp(-p (x-P)^2) over [lo, hi] are expressed with erf.

Pinned by: adaptive quadrature of the defining integrals, and the
whole-line limits (Gaussian product theorem) when [lo, hi] is wide.
"""
import numpy as np
from scipy.special import erf, erfc


def _erf_diff(ul, uh):
    """erf(uh) - erf(ul) for ul <= uh, without cancellation in the tails."""
    ul = np.asarray(ul, dtype=np.float64)
    uh = np.asarray(uh, dtype=np.float64)
    right = erfc(ul) - erfc(uh)          # both arguments positive
    left = erfc(-uh) - erfc(-ul)         # both arguments negative
    mid = erf(uh) - erf(ul)
    return np.where(ul > 0.0, right, np.where(uh < 0.0, left, mid))


def moments(p, P, lo, hi):
    """Moments I0, I1, I2 of exp(-p (x-P)^2) over [lo, hi] about P."""
    sp = np.sqrt(p)
    ul = sp * (lo - P)
    uh = sp * (hi - P)
    I0 = 0.5 * np.sqrt(np.pi / p) * _erf_diff(ul, uh)
    el = np.exp(-ul * ul)
    eh = np.exp(-uh * uh)
    I1 = (el - eh) / (2.0 * p)
    I2 = I0 / (2.0 * p) - ((hi - P) * eh - (lo - P) * el) / (2.0 * p)
    return I0, I1, I2


def _pair(alpha_a, delta_a, alpha_b, delta_b):
    aa = np.asarray(alpha_a, dtype=np.float64)[:, None]
    da = np.broadcast_to(np.asarray(delta_a, dtype=np.float64), np.shape(alpha_a))[:, None]
    ab = np.asarray(alpha_b, dtype=np.float64)[None, :]
    db = np.broadcast_to(np.asarray(delta_b, dtype=np.float64), np.shape(alpha_b))[None, :]
    p = da + db
    P = (da * aa + db * ab) / p
    E = np.exp(-da * db * (aa - ab) ** 2 / p)
    return aa, da, ab, db, p, P, E


def overlap(alpha, delta, lo, hi, alpha_b=None, delta_b=None):
    """S_ab = int_lo^hi phi_a phi_b dx."""
    if alpha_b is None:
        alpha_b, delta_b = alpha, delta
    _, _, _, _, p, P, E = _pair(alpha, delta, alpha_b, delta_b)
    I0, _, _ = moments(p, P, lo, hi)
    return E * I0


def position(alpha, delta, lo, hi):
    """X_ab = int_lo^hi x phi_a phi_b dx (dipole matrix, eq. (Q))."""
    _, _, _, _, p, P, E = _pair(alpha, delta, alpha, delta)
    I0, I1, _ = moments(p, P, lo, hi)
    return E * (P * I0 + I1)


def kinetic(alpha, delta, lo, hi):
    """Kin_ab = 1/2 int_lo^hi phi_a' phi_b' dx (weak form of -1/2 d^2/dx^2)."""
    aa, da, ab, db, p, P, E = _pair(alpha, delta, alpha, delta)
    I0, I1, I2 = moments(p, P, lo, hi)
    return 2.0 * da * db * E * (I2 + (2.0 * P - aa - ab) * I1 + (P - aa) * (P - ab) * I0)


def values(alpha, delta, x):
    """phi_a(x) for every centre a and point x: array (len(x), n)."""
    x = np.asarray(x, dtype=np.float64)[:, None]
    a = np.asarray(alpha, dtype=np.float64)[None, :]
    d = np.broadcast_to(np.asarray(delta, dtype=np.float64), np.shape(alpha))[None, :]
    return np.exp(-d * (x - a) ** 2)


def derivatives(alpha, delta, x):
    """phi_a'(x) = -2 delta (x - alpha_a) phi_a(x): array (len(x), n)."""
    x = np.asarray(x, dtype=np.float64)[:, None]
    a = np.asarray(alpha, dtype=np.float64)[None, :]
    d = np.broadcast_to(np.asarray(delta, dtype=np.float64), np.shape(alpha))[None, :]
    return -2.0 * d * (x - a) * np.exp(-d * (x - a) ** 2)


def gaussian_projection(alpha, delta, lo, hi, g_alpha, g_center):
    """int_lo^hi exp(-g_alpha (x-g_center)^2) phi_a(x) dx for every centre a."""
    S = overlap(np.asarray(alpha), delta, lo, hi,
                alpha_b=np.array([g_center], dtype=np.float64),
                delta_b=np.array([g_alpha], dtype=np.float64))
    return S[:, 0]
