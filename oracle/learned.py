"""Reference of the learned warm start's data plumbing (FP64).

The paper leaves the Schwarz initial guess psi^(0) of a window free
(Section 4.1, eq. (S1): "psi_i^(k=0) is a given function").  The plain guess
holds the window's initial Robin data constant in time.  The learned guess
adds a correction predicted by a network at M time nodes and interpolates
it to every time step.  Definitions (readings, since the paper has no
learned part):

* time nodes: steps n_m = round(n_T (1 - cos(pi m / (M-1))) / 2),
  m = 0..M-1 (Chebyshev-Lobatto positions rounded to the time grid; the
  interpolation needs them distinct, which bounds n_T from below);
* window scale S = the largest item RMS of g0 over the window's items
  (RMS over an item's receiving face nodes), or 1 if g0 vanishes: one
  scale per window, so that the loss weighs every item by its amplitude,
  as the interface residual does;
* features of item i: (Re, Im) of g0 / S, node by node, zero padded to
  n_in - (M + 8) entries, then a tail of M + 8 entries: 10 E(t0 + t_m) for
  the M nodes; the item's box centre in global box coordinates,
  (c_k - mid_k) / half_k for k < D, zero padded to four; RMS_i / S;
  t0 / (8 T) with T the window length (the window's place in a run of
  eight); two zeros;
* targets: (g(t_m) - g0) / S, node-major within each time node
  ([m][node][re, im]);
* applied guess: g(t_n) = g0 + S sum_m l_m(t_n) y_m, with l_m the
  Lagrange basis on the node times in barycentric form.

Pinned by: exact reproduction of polynomials of degree <= M-1 by the
interpolation, and identity at the nodes (tests/test_oracle_learned.py).
"""
import math

import numpy as np

N_NODES_T = 8          # default number of time nodes
FIELD_SCALE = 10.0


def time_nodes(n_T, M=N_NODES_T):
    n = [int(round(n_T * (1.0 - math.cos(math.pi * m / (M - 1))) / 2.0)) for m in range(M)]
    if any(b <= a for a, b in zip(n, n[1:])):
        raise ValueError(f"{M} distinct time nodes need a longer window than {n_T} steps")
    return n


def tail_len(M=N_NODES_T):
    return M + 8


def bary_weights(ts):
    ts = np.asarray(ts, dtype=np.float64)
    w = np.empty(len(ts))
    for m in range(len(ts)):
        w[m] = 1.0 / np.prod([ts[m] - ts[k] for k in range(len(ts)) if k != m])
    return w


def lagrange_row(t, ts, w):
    """l_m(t) for all m (barycentric second form)."""
    ts = np.asarray(ts, dtype=np.float64)
    d = t - ts
    hit = np.nonzero(d == 0.0)[0]
    if hit.size:
        out = np.zeros(len(ts))
        out[hit[0]] = 1.0
        return out
    q = w / d
    return q / q.sum()


def item_rms(g0):
    return math.sqrt(float(np.mean(np.abs(g0) ** 2))) if g0.size else 0.0


def window_scale(g0_items):
    s = max(item_rms(g) for g in g0_items)
    return s if s > 0.0 else 1.0


def item_positions(prob):
    """(c_k - mid_k) / half_k of every subdomain's box centre, padded to 4."""
    lo = np.asarray(prob.cfg["box_lo"], dtype=np.float64)
    hi = np.asarray(prob.cfg["box_hi"], dtype=np.float64)
    out = np.zeros((prob.n_sub, 4))
    for i, sub in enumerate(prob.dec.subs):
        c = 0.5 * (sub.lo + sub.hi)
        out[i, :len(c)] = (c - 0.5 * (lo + hi)) / (0.5 * (hi - lo))
    return out


def features(g0_items, field_vals, n_in, positions, t0_over_T=0.0):
    """g0_items: list per item of complex (n_nodes_i,); field_vals: (M,);
    positions: (n_items, 4); t0_over_T: window start / window length.
    Returns (X, per-item scales, all equal)."""
    M = len(field_vals)
    S = window_scale(g0_items)
    X = np.zeros((len(g0_items), n_in))
    for i, g0 in enumerate(g0_items):
        z = g0 / S
        X[i, 0:2 * z.size:2] = z.real
        X[i, 1:2 * z.size:2] = z.imag
        t = n_in - tail_len(M)
        X[i, t:t + M] = FIELD_SCALE * np.asarray(field_vals)
        X[i, t + M:t + M + 4] = positions[i]
        X[i, t + M + 4] = item_rms(g0) / S
        X[i, t + M + 5] = t0_over_T / 8.0
    return X, np.full(len(g0_items), S)


def targets(g_nodes_items, scales, n_out):
    """g_nodes_items: list per item of complex (M, n_nodes_i) at the time
    nodes; returns (n_items, n_out)."""
    Y = np.zeros((len(g_nodes_items), n_out))
    for i, g in enumerate(g_nodes_items):
        d = (g - g[0][None, :]) / scales[i]
        n = g.shape[1]
        for m in range(g.shape[0]):
            Y[i, m * 2 * n:(m + 1) * 2 * n:2] = d[m].real
            Y[i, m * 2 * n + 1:(m + 1) * 2 * n:2] = d[m].imag
    return Y


def apply(Y, scales, g0_items, n_T, dt, M=N_NODES_T):
    """Robin data at every step: list per item of complex (n_T+1, n_nodes_i)."""
    nodes = time_nodes(n_T, M)
    ts = np.array(nodes, dtype=np.float64) * dt
    w = bary_weights(ts)
    L = np.array([lagrange_row(k * dt, ts, w) for k in range(n_T + 1)])  # (n_T+1, M)
    out = []
    for i, g0 in enumerate(g0_items):
        n = g0.size
        corr = np.zeros((M, n), dtype=np.complex128)
        for m in range(M):
            corr[m] = Y[i, m * 2 * n:(m + 1) * 2 * n:2] + 1j * Y[i, m * 2 * n + 1:(m + 1) * 2 * n:2]
        out.append(g0[None, :] + scales[i] * (L @ corr))
    return out
