"""Composite Gauss-Legendre rules used for the potential and for face integrals.

The paper evaluates its inner products by quadrature on uniform grids
(Section 5, grids N^(x1) x N^(x2)); here the same integrals are taken with
composite Gauss-Legendre rules instead, which the design notes record as a
reading.  The Legendre nodes come from NumPy's Golub-Welsch routine
(`leggauss`), a library primitive.

Pinned by: exact integration of polynomials up to degree 2n-1, and
panel-doubling convergence of the soft-Coulomb matrix elements.
"""
import math

import numpy as np


def gauss_legendre(n):
    """Nodes and weights of the n-point rule on [-1, 1]."""
    t, w = np.polynomial.legendre.leggauss(n)
    return t.astype(np.float64), w.astype(np.float64)


def composite(edges, nodes_per_panel):
    """Composite rule over consecutive panels [edges[p], edges[p+1]].

    nodes_per_panel is an int or one count per panel.
    Returns (x, w) concatenated panel by panel.
    """
    edges = [float(e) for e in edges]
    npan = len(edges) - 1
    if isinstance(nodes_per_panel, int):
        counts = [nodes_per_panel] * npan
    else:
        counts = list(nodes_per_panel)
    xs, ws = [], []
    for p in range(npan):
        t, w = gauss_legendre(counts[p])
        a, b = edges[p], edges[p + 1]
        half = 0.5 * (b - a)
        mid = 0.5 * (a + b)
        xs.append(mid + half * t)
        ws.append(half * w)
    return np.concatenate(xs), np.concatenate(ws)


def potential_panels(lo, hi, hmax):
    """Equal panels of width at most hmax covering [lo, hi]."""
    npan = max(1, int(math.ceil((hi - lo) / hmax)))
    width = (hi - lo) / npan
    return [lo + p * width for p in range(npan)] + [hi]


def face_panels(lo, hi, eps):
    """Panels [lo, lo+eps], [lo+eps, hi-eps], [hi-eps, hi] of a tangential
    direction: their breaks are where the set of covering subdomains
    changes (edges of the overlap bands)."""
    return [lo, lo + eps, hi - eps, hi]
