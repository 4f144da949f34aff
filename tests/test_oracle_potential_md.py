"""Pins of the oracle's soft-Coulomb matrix (Section 5, eq. pseudo) in more
than one configuration dimension, against evaluations that do not go
through its staged contraction (`assemble._term`, one grid axis at a time):

  * two electrons in one dimension each (D = 2: the nucleus terms of each
    electron and the electron-electron term): adaptive two-dimensional
    quadrature (scipy dblquad) of U(x1, x2) v_l v_m over an off-diagonal
    subdomain whose two dimensions differ in box, size and basis, so that
    exchanging the two electrons' axes, a transposed table or a dropped
    term changes the value;
  * two electrons in two dimensions each (D = 4: the two-dimensional
    nucleus term of each electron and the four-dimensional
    electron-electron term): the same tensor Gauss-Legendre rule summed
    over the whole four-dimensional grid at once, with the integrand formed
    pointwise (no contraction order), on a subdomain of unequal sizes.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import assemble, gauss1d
from oracle.geometry import Decomposition
from workloads import get_config, tiny_configs


def _potential(cfg, x):
    """U(x) of eq. (pseudo) at one configuration point x (length D)."""
    N, d = cfg["n_elec"], cfg["dim"]
    u = 0.0
    for m in range(N):
        r = x[m * d:(m + 1) * d]
        for R, Z in zip(cfg["nuclei"], cfg["charges"]):
            u -= Z / math.sqrt(sum((r[a] - R[a]) ** 2 for a in range(d)) + cfg["eps_en"] ** 2)
    for m in range(N):
        for mp in range(m + 1, N):
            r1, r2 = x[m * d:(m + 1) * d], x[mp * d:(mp + 1) * d]
            u += 1.0 / math.sqrt(sum((r1[a] - r2[a]) ** 2 for a in range(d)) + cfg["eps_ee"] ** 2)
    return u


def _phi(s, k, a, x):
    return math.exp(-s.delta[k][a] * (x - s.alpha[k][a]) ** 2)


def test_two_electron_potential_matches_adaptive_2d_quadrature():
    cfg = [c for c in tiny_configs() if c["name"] == "tiny-2d"][0]
    dec = Decomposition(cfg)
    s = dec.subs[1]                        # multi-index (1, 0): off the diagonal
    assert s.idx == (1, 0) and s.nb == (5, 4)
    V = assemble.potential_matrix(dec, s)
    n1 = s.nb[1]
    for l, m in [(0, 0), (3, 14), (14, 3), (7, 19), (12, 5), (19, 19)]:
        a0, a1 = divmod(l, n1)
        b0, b1 = divmod(m, n1)
        f = lambda y, x: (_potential(cfg, (x, y)) * _phi(s, 0, a0, x) * _phi(s, 0, b0, x)
                          * _phi(s, 1, a1, y) * _phi(s, 1, b1, y))
        ref, _ = integrate.dblquad(f, s.lo[0], s.hi[0], s.lo[1], s.hi[1],
                                   epsabs=1e-15, epsrel=1e-13)
        assert V[l, m] == pytest.approx(ref, rel=1e-12, abs=1e-14), (l, m)
    # the two dimensions differ in box and basis here, so reading a basis
    # table along the other electron's axis changes the value
    assert s.lo[0] != s.lo[1] and s.hi[0] != s.hi[1]
    l, m = 7, 19
    a0, a1 = divmod(l, n1)
    b0, b1 = divmod(m, n1)
    g = lambda y, x: (_potential(cfg, (x, y)) * _phi(s, 0, a0, y) * _phi(s, 0, b0, y)
                      * _phi(s, 1, a1, x) * _phi(s, 1, b1, x))
    swapped, _ = integrate.dblquad(g, s.lo[0], s.hi[0], s.lo[1], s.hi[1],
                                   epsabs=1e-15, epsrel=1e-13)
    assert abs(swapped - V[l, m]) > 1e-3 * abs(V[l, m])


def _rule(dec, s, k):
    sig = math.sqrt(0.5 / s.delta[k][0])
    cfg = dec.cfg
    h = min(float(cfg["eps_en"]), float(cfg["eps_ee"]), sig)
    from oracle import quadrature
    edges = quadrature.potential_panels(s.lo[k], s.hi[k], h)
    return quadrature.composite(edges, int(cfg["quad_nodes"]))


def test_four_dimensional_potential_matches_unstaged_grid_sum():
    cfg = get_config("c5-mini")
    dec = Decomposition(cfg)
    s = dec.subs[5]                        # multi-index (1, 0, 1, 0)
    assert s.idx == (1, 0, 1, 0)
    V = assemble.potential_matrix(dec, s)
    rules = [_rule(dec, s, k) for k in range(4)]
    X = np.meshgrid(*[r[0] for r in rules], indexing="ij")
    W = np.ones(X[0].shape)
    for k in range(4):
        shape = [1, 1, 1, 1]
        shape[k] = -1
        W = W * rules[k][1].reshape(shape)
    # U on the whole grid, pointwise
    U = np.zeros(X[0].shape)
    for m in range(2):
        for R, Z in zip(cfg["nuclei"], cfg["charges"]):
            U -= Z / np.sqrt((X[2 * m] - R[0]) ** 2 + (X[2 * m + 1] - R[1]) ** 2
                             + cfg["eps_en"] ** 2)
    U += 1.0 / np.sqrt((X[0] - X[2]) ** 2 + (X[1] - X[3]) ** 2 + cfg["eps_ee"] ** 2)
    UW = U * W
    nb = s.nb
    for l, m in [(0, 0), (5, 30), (30, 5), (17, 2), (35, 35), (11, 24)]:
        li = np.unravel_index(l, nb)
        mi = np.unravel_index(m, nb)
        integrand = UW.copy()
        for k in range(4):
            shape = [1, 1, 1, 1]
            shape[k] = -1
            pk = (np.exp(-s.delta[k][li[k]] * (rules[k][0] - s.alpha[k][li[k]]) ** 2)
                  * np.exp(-s.delta[k][mi[k]] * (rules[k][0] - s.alpha[k][mi[k]]) ** 2))
            integrand = integrand * pk.reshape(shape)
        ref = float(np.sum(integrand))
        assert V[l, m] == pytest.approx(ref, rel=1e-11, abs=1e-13), (l, m)
