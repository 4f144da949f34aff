"""Pins of the oracle's decomposition, covering sets and partition-of-unity
weights against hand-enumerated fixtures (tests/golden/) and closed forms."""
import math
import os

import numpy as np
import pytest

from oracle import assemble, gauss1d
from oracle.geometry import Decomposition

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid_cfg(L, nb=(4, 4), eps=(0.5, 0.5), box=3.0, face_nodes=(3, 5)):
    D = len(L)
    return dict(name="grid", mode="tdse", n_elec=D, dim=1, L=list(L),
                box_lo=[-box] * D, box_hi=[box] * D, overlap=list(eps), nbasis=list(nb),
                width=None, width_ratio=0.7, nuclei=[], charges=[], eps_en=1.0,
                eps_ee=1.0, dt=0.01, n_steps=1, mu=[0.0, -1.0],
                field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0),
                init=dict(alpha=1.0, center=[0.0] * D), iters=1, tol=1e-8,
                face_nodes=list(face_nodes), quad_nodes=8)


def _zone(dec, s, F, y):
    t = [d for d in range(dec.D) if d != F.k][0]
    if y[t] < s.lo[t] + dec.eps[t]:
        return "low"
    if y[t] > s.hi[t] - dec.eps[t]:
        return "high"
    return "mid"


def test_c1_subdomains_match_hand_computed_fixture():
    from workloads import get_config
    dec = Decomposition(get_config("c1-1e-1d"))
    rows = [l.split() for l in open(os.path.join(GOLDEN, "c1_subdomains.txt"))
            if l.strip() and not l.startswith("#")]
    for r, s in zip(rows, dec.subs):
        assert s.lo[0] == float(r[1]) and s.hi[0] == float(r[2])


def test_cover_sets_3x3_match_hand_enumeration():
    dec = Decomposition(_grid_cfg((3, 3)))
    s = dec.subs[4]
    assert s.idx == (1, 1)
    expect = {}
    for l in open(os.path.join(GOLDEN, "cover_3x3.txt")):
        if not l.strip() or l.startswith("#"):
            continue
        p = l.split()
        expect[(int(p[0]), int(p[1]), p[2])] = [int(v) for v in p[3:]]
    seen = set()
    for F in s.faces:
        assert not F.is_global
        for y, cov in zip(F.nodes, F.cover):
            key = (F.k, F.side, _zone(dec, s, F, y))
            assert [int(c) for c in cov] == expect[key], key
            seen.add(key)
    assert seen == set(expect)


def test_cover_counts_2x2_and_global_faces():
    """Corner zones of a 2x2 decomposition: the only interior corner sees
    all 3 = 2^2 - 1 other subdomains; global faces are flagged."""
    dec = Decomposition(_grid_cfg((2, 2)))
    s = dec.subs[0]
    flags = {(F.k, F.side): F.is_global for F in s.faces}
    assert flags == {(0, 0): True, (0, 1): False, (1, 0): True, (1, 1): False}
    right = [F for F in s.faces if (F.k, F.side) == (0, 1)][0]
    counts = sorted({len(c) for c in right.cover})
    assert counts == [1, 3]
    assert max(len(c) for F in s.faces if not F.is_global for c in F.cover) == 2 ** 2 - 1


def test_linear_index_first_dimension_fastest():
    dec = Decomposition(_grid_cfg((3, 2)))
    assert [s.idx for s in dec.subs] == [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (2, 1)]


def test_partition_of_unity_weights_sum_to_global_integral():
    """sum_i int_{Omega_i} G^2 / #cover = int_Omega G^2 for a Gaussian G
    that is not a basis function: pins the halving of the overlap bands."""
    cfg = _grid_cfg((4,), nb=(3,), eps=(0.8,), box=5.0)
    cfg["n_elec"] = 1
    dec = Decomposition(cfg)
    g_a, g_d = 0.37, 0.45
    tot = 0.0
    for s in dec.subs:
        s.alpha = [np.array([g_a])]
        s.delta = [np.array([g_d])]
        s.nb = (1,)
        s.K = 1
        sy = assemble.LocalSystem(dec, s)
        tot += sy.W[0, 0]
    ref = math.sqrt(math.pi / (2 * g_d)) * 0.5 * (
        math.erf(math.sqrt(2 * g_d) * (5.0 - g_a)) - math.erf(math.sqrt(2 * g_d) * (-5.0 - g_a)))
    assert tot == pytest.approx(ref, rel=1e-13)


def test_face_rule_integrates_tangential_gaussian():
    """Face Gauss-Legendre weights integrate a smooth function across the
    panel breaks at the overlap bands."""
    dec = Decomposition(_grid_cfg((3, 3), eps=(0.6, 0.6), face_nodes=(10, 16)))
    s = dec.subs[4]
    F = s.faces[1]
    y = F.nodes[:, 1]
    v = np.sum(F.weights * np.exp(-(y - 0.1) ** 2))
    lo, hi = s.lo[1], s.hi[1]
    ref = 0.5 * math.sqrt(math.pi) * (math.erf(hi - 0.1) - math.erf(lo - 0.1))
    assert v == pytest.approx(ref, rel=1e-13)
