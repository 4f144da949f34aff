"""Reconstruction of the global wavefunction from the local ones.

Paper passages followed: Section 4.3 (wavefunction reconstruction): in a
zone shared by Omega_i and the subdomains of O, the global function is
(phi_i + sum_j phi_j)/(Card O + 1); elsewhere it is phi_i.  Test 1.a
(Section 5.1) writes the same rule as the mean over all subdomains that
contain the point.  Closed membership is used, as for the covering sets.

Antisymmetric reconstruction of two electrons (Appendix A: the subdomain
holding the exchanged point sigma(x) carries minus the local function, read
off at the exchanged point; Section 5 applies the same antisymmetrisation a
posteriori to a reconstructed state): psi_A(x) = psi(x) where electron 2's
coordinates do not come after electron 1's (lexicographically over the space
dimensions), psi_A(x) = -psi(sigma x) where they do.

Pinned by: reconstruction of a function that every local basis represents
exactly (a single Gaussian that is itself a basis function of every
subdomain is not available in general, so the pin uses the projected
initial state of a one-subdomain decomposition, which reduces to the
local expansion) and by the partition-of-unity identity: the squared norm
of the reconstruction equals sum_i c_i^T W_i c_i when the local functions
agree on the overlaps.
"""
import numpy as np

from .swr import basis_values


def reconstruct(prob, coeffs, pts):
    """psi(x) = mean over {i : x in closure(Omega_i)} of psi_i(x)."""
    pts = np.asarray(pts, dtype=np.float64)
    out = np.zeros(pts.shape[0], dtype=np.result_type(coeffs[0].dtype, np.float64))
    cnt = np.zeros(pts.shape[0])
    for s in prob.dec.subs:
        inside = np.all((s.lo[None, :] <= pts) & (pts <= s.hi[None, :]), axis=1)
        rows = np.nonzero(inside)[0]
        if rows.size == 0:
            continue
        out[rows] += basis_values(s, pts[rows]) @ coeffs[s.lin]
        cnt[rows] += 1.0
    covered = cnt > 0
    out[covered] /= cnt[covered]
    return out


def exchange(pts, dim):
    """sigma(x): the two electrons' coordinates swapped (points [n][2 dim])."""
    pts = np.asarray(pts, dtype=np.float64)
    return np.concatenate([pts[:, dim:2 * dim], pts[:, :dim]], axis=1)


def after(pts, dim):
    """Electron 2's coordinates come after electron 1's, lexicographically."""
    out = np.zeros(pts.shape[0], dtype=bool)
    undecided = np.ones(pts.shape[0], dtype=bool)
    for a in range(dim):
        u, v = pts[:, a], pts[:, dim + a]
        out |= undecided & (v > u)
        undecided &= v == u
    return out


def reconstruct_antisym(prob, coeffs, pts):
    """psi_A(x) = psi(x), or -psi(sigma x) where electron 2 comes after 1."""
    dim = prob.cfg["dim"]
    if prob.cfg["n_elec"] != 2:
        raise ValueError("two electrons")
    pts = np.asarray(pts, dtype=np.float64)
    flip = after(pts, dim)
    src = pts.copy()
    src[flip] = exchange(pts[flip], dim)
    out = reconstruct(prob, coeffs, src)
    out[flip] = -out[flip]
    return out
