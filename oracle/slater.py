"""Slater-like antisymmetric Gaussian basis (test infrastructure: the CPU
oracle, never called by the product path).

Paper passage followed: Section 2, eq. (LSD): for two electrons in one
dimension each, the local basis function built from the one-dimensional
Gaussians phi_l of the first coordinate's interval and phi_p of the second
coordinate's interval is

    v_{l,p}(x1, x2) = (phi_l(x1) phi_p(x2) - phi_l(x2) phi_p(x1)) / sqrt(2),

antisymmetric under the exchange x1 <-> x2.  On a subdomain off the
diagonal (the two intervals differ) the n^2 functions are independent; on
a diagonal subdomain (the same interval, hence the same Gaussians in both
coordinates) v_{l,p} = -v_{p,l} and v_{l,l} = 0, so the basis is the
n(n-1)/2 functions with l < p.

Every v is a signed pair of tensor products of Gaussians from the combined
list U = (phi_1..phi_n of the first interval, phi_1..phi_n of the second),
used in both coordinates: with E_{a,b}(x1, x2) = U_a(x1) U_b(x2) (index
a * 2n + b, first coordinate slowest),

    v_{l,p} = (E_{l, n+p} - E_{n+p, l}) / sqrt(2),

so the Galerkin matrices are M = T M_E T^T with M_E those of the extended
tensor basis on the same box (closed forms and quadrature as for any
tensor basis) and T the K x (2n)^2 signed selection.  The antisymmetric
initial state is phi_0 = N (g_{c1}(x1) g_{c2}(x2) - g_{c2}(x1) g_{c1}(x2))
with g_c(x) = exp(-alpha (x - c)^2), normalised on the whole plane.

Readings (listed in the design notes): the pair order is l slowest; the
exchanged term uses the same widths; the initial state's normalisation is
taken on R^2 (as for the tensor Gaussian initial state).

Pinned by (tests/test_oracle_slater.py): exchange antisymmetry of the basis
functions; every assembled matrix against adaptive two-dimensional
quadrature of its definition on an off-diagonal subdomain; on a diagonal
subdomain the projection of an antisymmetric function onto the Slater
basis equals its projection onto the (exchange-symmetric) tensor basis;
and converged SWR in the Slater basis against a brute-force
finite-difference solution started from the same antisymmetric state.
"""
import math

import numpy as np

from . import lsd
from .geometry import Subdomain


def is_slater(s):
    return getattr(s, "slater", False)


def pairs(s):
    """(l, p) of every basis function of subdomain s, in basis order."""
    if lsd.is_lsd(s):
        return lsd.pairs(s)
    n = len(s.alpha[0])
    if s.idx[0] == s.idx[1]:
        return [(l, p) for l in range(n) for p in range(l + 1, n)]
    return [(l, p) for l in range(n) for p in range(n)]


def extended(s):
    """The tensor basis U x U on the same box (a plain Subdomain)."""
    U = np.concatenate([s.alpha[0], s.alpha[1]])
    dU = np.concatenate([s.delta[0], s.delta[1]])
    return Subdomain(s.lin, s.idx, s.lo, s.hi, [U, U], [dU, dU])


def transform(s):
    """T with v = T E (rows: basis functions, columns: extended tensor);
    for local Slater determinants oracle/lsd.py's."""
    if lsd.is_lsd(s):
        return lsd.transform(s)
    n = len(s.alpha[0])
    m2 = 2 * n
    pr = pairs(s)
    T = np.zeros((len(pr), m2 * m2))
    r = 1.0 / math.sqrt(2.0)
    for m, (l, p) in enumerate(pr):
        T[m, l * m2 + (n + p)] += r
        T[m, (n + p) * m2 + l] -= r
    return T


def initial_norm(alpha0, c1, c2):
    """N of phi_0 = N (g_c1 g_c2 - g_c2 g_c1) with unit norm on R^2."""
    g2 = math.sqrt(math.pi / (2.0 * alpha0))
    return 1.0 / math.sqrt(2.0 * g2 * g2 * (1.0 - math.exp(-alpha0 * (c1 - c2) ** 2)))
