"""Reconstruction of the global wavefunction from the local ones.

Paper passages followed: Section 4.3 (wavefunction reconstruction): in a
zone shared by Omega_i and the subdomains of O, the global function is
(phi_i + sum_j phi_j)/(Card O + 1); elsewhere it is phi_i.  Test 1.a
(Section 5.1) writes the same rule as the mean over all subdomains that
contain the point.  Closed membership is used, as for the covering sets.

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
