"""Pins of the oracle's local orbitals and local Slater determinants
(Section 3; oracle/lsd.py), against values and evaluations that do not go
through its quadrature rules or its extended-basis transform:

  * the mollifier's normalisations are the values the paper prints for
    sigma(1), sigma(2) and (in the determinant tests) sigma_1 = 315/256, and
    each B_eps integrates to one;
  * the mollified potential approaches the unmollified one as eps^2, and
    equals the convolution integral evaluated adaptively;
  * every entry of the orbital problem's S and H equals adaptive quadrature
    of its definition (smooth step, barrier, coefficient a(x) and the
    mollified nuclei written out here);
  * the orbitals solve the generalised eigenproblem and are S-orthonormal;
  * the determinants are antisymmetric, and every matrix of an off-diagonal
    subdomain equals two-dimensional adaptive quadrature of its definition;
  * with as many orbitals as Gaussians the determinants span the Slater-like
    basis's space: the SWR window reconstructs the same function;
  * augmented bases (Section 3.3): the added functions are Gaussians of the
    interval's exponent centred on its box's ends (built here from the box
    and the exponent alone), their determinants' matrices equal quadrature,
    and orbitals plus added Gaussians as many as the Gaussians span the
    Slater-like basis's space again.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads
from oracle import lsd, reconstruct, slater, swr

CF = {c["name"]: c for c in workloads.lsd_configs()}


def test_mollifier_normalisation_matches_the_printed_values():
    # Section 3.2 prints sigma(1) = 3/4, sigma(2) = 15/16; the determinant
    # tests use sigma_1 = 315/256 (the order-4 mollifier)
    assert lsd.sigma(1) == pytest.approx(3 / 4, rel=1e-15)
    assert lsd.sigma(2) == pytest.approx(15 / 16, rel=1e-15)
    assert lsd.sigma(4) == pytest.approx(315 / 256, rel=1e-15)
    for order in (1, 2, 3, 4):
        for eps in (0.1, 0.5):
            tot = integrate.quad(lambda x: float(lsd.mollifier(x, eps, order)), -eps, eps,
                                 epsabs=1e-15, epsrel=1e-14)[0]
            assert tot == pytest.approx(1.0, abs=1e-13)
            assert float(lsd.mollifier(1.0001 * eps, eps, order)) == 0.0
            assert float(lsd.mollifier(0.3 * eps, eps, order)) == \
                float(lsd.mollifier(-0.3 * eps, eps, order))


def test_mollified_potential_is_the_convolution_and_approaches_v_as_eps_squared():
    Z, eta, order = 1.0, 0.5, 4
    xs = np.array([-1.3, -0.2, 0.0, 0.05, 0.7, 2.4])
    for eps in (0.1, 0.3):
        got = lsd.mollified(xs, Z, eta, eps, order)
        for x, g in zip(xs, got):
            ref = integrate.quad(
                lambda y: -Z / math.sqrt((x - y) ** 2 + eta ** 2)
                * lsd.sigma(order) / eps * (1 - (y / eps) ** 2) ** order,
                -eps, eps, epsabs=1e-15, epsrel=1e-14)[0]
            assert g == pytest.approx(ref, rel=1e-13, abs=1e-15)
    v = lsd.soft_coulomb(xs, Z, eta)
    e1 = np.max(np.abs(lsd.mollified(xs, Z, eta, 0.2, order) - v))
    e2 = np.max(np.abs(lsd.mollified(xs, Z, eta, 0.1, order) - v))
    assert 3.8 < e1 / e2 < 4.2


def _step(t, w):
    u = min(max(t / w + 0.5, 0.0), 1.0)
    return u ** 3 * (10 - 15 * u + 6 * u * u)


def test_orbital_matrices_match_adaptive_quadrature():
    cfg = CF["tiny-lsd"]
    p = cfg["lsd"]
    prob = swr.Problem(cfg)
    s = prob.dec.subs[1]                     # first coordinate: interval 1
    cen, dl, lo, hi = s.alpha[0], s.delta[0], s.lo[0], s.hi[0]
    S, H = lsd.orbital_matrices(cfg, cen, dl, lo, hi)
    xc = 0.5 * (lo + hi)

    def nuc(x):
        u = 0.0
        for R, Z in zip(cfg["nuclei"], cfg["charges"]):
            if lo <= R[0] <= hi:
                e = p["moll_eps"]
                u += integrate.quad(
                    lambda y: -Z / math.sqrt((x - R[0] - y) ** 2 + cfg["eps_en"] ** 2)
                    * lsd.sigma(p["moll_order"]) / e * (1 - (y / e) ** 2) ** p["moll_order"],
                    -e, e, epsabs=1e-15, epsrel=1e-13)[0]
            else:
                u += -Z / math.sqrt((x - R[0]) ** 2 + cfg["eps_en"] ** 2)
        return u

    def g(u, x):
        return math.exp(-dl[u] * (x - cen[u]) ** 2)

    def dg(u, x):
        return -2 * dl[u] * (x - cen[u]) * g(u, x)

    pts = [xc - p["barrier"] - 0.5 * p["barrier_width"], xc - p["barrier"] + 0.5 * p["barrier_width"],
           xc + p["barrier"] - 0.5 * p["barrier_width"], xc + p["barrier"] + 0.5 * p["barrier_width"]]
    for u, w in [(0, 0), (1, 4), (5, 2), (3, 3)]:
        s_ref = integrate.quad(lambda x: g(u, x) * g(w, x), -np.inf, np.inf,
                               epsabs=1e-15, epsrel=1e-13)[0]
        assert S[u, w] == pytest.approx(s_ref, rel=1e-12, abs=1e-15)

        def h(x):
            st = _step(abs(x - xc) - p["barrier"], p["barrier_width"])
            return (0.5 * (1 - st) * dg(u, x) * dg(w, x)
                    + (nuc(x) + p["v_inf"] * st) * g(u, x) * g(w, x))
        h_ref = integrate.quad(h, xc - 12.0, xc + 12.0, points=pts, limit=400,
                               epsabs=1e-14, epsrel=1e-12)[0]
        assert H[u, w] == pytest.approx(h_ref, rel=1e-10, abs=1e-13), (u, w)


def test_orbitals_solve_the_eigenproblem_and_are_orthonormal():
    cfg = CF["tiny-lsd"]
    prob = swr.Problem(cfg)
    s = prob.dec.subs[4]                      # the middle interval (the nuclei)
    S, H = lsd.orbital_matrices(cfg, s.alpha[0], s.delta[0], s.lo[0], s.hi[0])
    lam, C = lsd.orbitals(cfg, s.alpha[0], s.delta[0], s.lo[0], s.hi[0])
    assert np.all(np.diff(lam) > 0)
    assert np.max(np.abs(H @ C - S @ C * lam)) <= 1e-12 * np.max(np.abs(H))
    assert np.max(np.abs(C.T @ S @ C - np.eye(C.shape[1]))) <= 1e-13
    assert np.all(np.arange(1, C.shape[0] + 1) @ C > 0)
    # the lowest orbital is bound by the nuclei in the middle interval
    assert lam[0] < prob.dec.orbital_energies[0][0]


def _phi(C, cen, dl, l, x):
    g = np.exp(-dl * (x - cen) ** 2)
    return float(C[:, l] @ g), float(C[:, l] @ (-2 * dl * (x - cen) * g))


@pytest.mark.parametrize("name,K,checks", [
    ("tiny-lsd", 16, [(0, 0), (5, 9), (15, 2)]),
    # 3 orbitals + 2 end Gaussians: pairs (l, p) = m // 5, m % 5, functions
    # 3 and 4 the added Gaussians
    ("tiny-lsd-aug", 25, [(24, 0), (4, 23), (19, 12), (18, 18)])])
def test_determinants_antisymmetric_and_matrices_match_quadrature(name, K, checks):
    cfg = CF[name]
    prob = swr.Problem(cfg)
    s = prob.dec.subs[1]                       # intervals 1 (x1) and 0 (x2)
    assert s.idx[0] != s.idx[1] and s.K == K
    sy = prob.sys[1]
    pts = np.random.default_rng(3).uniform(-6, 6, size=(30, 2))
    v = swr.basis_values(s, pts)
    assert np.max(np.abs(v + swr.basis_values(s, pts[:, ::-1]))) <= 1e-15
    (lo1, lo2), (hi1, hi2) = s.lo, s.hi
    C1, C2 = s.lo_coef
    c1, d1, c2, d2 = s.alpha[0], s.delta[0], s.alpha[1], s.delta[1]
    pr = slater.pairs(s)
    r = 1 / math.sqrt(2)

    def vfun(m, x1, x2):
        l, p = pr[m]
        a1, da1 = _phi(C1, c1, d1, l, x1)
        a2, da2 = _phi(C1, c1, d1, l, x2)
        b1, db1 = _phi(C2, c2, d2, p, x1)
        b2, db2 = _phi(C2, c2, d2, p, x2)
        return (r * (a1 * b2 - a2 * b1), r * (da1 * b2 - a2 * db1), r * (a1 * db2 - da2 * b1))

    def U(x1, x2):
        u = 1.0 / math.sqrt((x1 - x2) ** 2 + cfg["eps_ee"] ** 2)
        for R, Z in zip(cfg["nuclei"], cfg["charges"]):
            u -= Z / math.sqrt((x1 - R[0]) ** 2 + cfg["eps_en"] ** 2)
            u -= Z / math.sqrt((x2 - R[0]) ** 2 + cfg["eps_en"] ** 2)
        return u

    for m, n in checks:
        def prod(x1, x2, kind):
            vm, am, bm = vfun(m, x1, x2)
            vn, an, bn = vfun(n, x1, x2)
            return {"A": vm * vn, "Kin": 0.5 * (am * an + bm * bn),
                    "Q": (x1 + x2) * vm * vn, "V": U(x1, x2) * vm * vn}[kind]
        for kind in ("A", "Kin", "Q", "V"):
            ref = integrate.dblquad(lambda x2, x1: prod(x1, x2, kind), lo1, hi1, lo2, hi2,
                                    epsabs=1e-13, epsrel=1e-12)[0]
            got = getattr(sy, kind)[m, n]
            assert abs(got - ref) <= 1e-10 * np.max(np.abs(getattr(sy, kind))), (kind, m, n)


@pytest.mark.parametrize("name", ["tiny-lsd-all", "tiny-lsd-aug-all"])
def test_all_orbitals_span_the_slater_basis_space(name):
    """With M = n orbitals per interval (or M + 2 = n with the two end
    Gaussians added) the determinants span exactly the Slater-like pairs of
    the same Gaussians, so every SWR iterate is the same function; compared
    through the reconstruction."""
    cfg = CF[name]
    cfg_s = dict(cfg, basis="slater")
    cfg_s.pop("lsd")
    out = []
    pts = np.random.default_rng(5).uniform(-5.7, 5.7, size=(200, 2))
    for c in (cfg, cfg_s):
        prob = swr.Problem(c)
        h, res = swr.swr_window(prob, prob.initial_coeffs(), iters=3)
        out.append((reconstruct.reconstruct(prob, [hh[c["n_steps"]] for hh in h], pts), res))
    (f_l, r_l), (f_s, r_s) = out
    scale = np.max(np.abs(f_s))
    assert np.max(np.abs(f_l - f_s)) <= 1e-10 * scale
    assert np.allclose(r_l, r_s, rtol=1e-8, atol=1e-14)


def test_augmented_functions_are_the_gaussians_on_the_box_ends():
    """Section 3.3: with augment = 1 the one-electron functions of an
    interval are its orbitals and the Gaussians exp(-delta (x - e)^2) centred
    on its box's ends e = lo, hi (delta the interval's exponent, 1/(2 w^2)
    for the workload's width ratio); checked pointwise on the determinants of
    a diagonal and an off-diagonal subdomain against those Gaussians written
    out from the box alone, and the counts M + 2 per interval."""
    cfg = CF["tiny-lsd-aug"]
    prob = swr.Problem(cfg)
    pts = np.random.default_rng(8).uniform(-6, 6, size=(40, 2))
    r = 1 / math.sqrt(2)
    M = cfg["lsd"]["orbitals"]
    for lin in (0, 1):                          # (0, 0) diagonal, (1, 0) off it
        s = prob.dec.subs[lin]
        i, j = s.idx
        n = cfg["nbasis"][0]

        def fns(k, x):
            lo, hi = prob.dec.lo1[0][s.idx[k]], prob.dec.hi1[0][s.idx[k]]
            sp = (hi - lo) / (n - 1)
            dl = 0.5 / (cfg["width_ratio"] * sp) ** 2
            orb = s.lo_coef[k][:, :M].T @ np.exp(-s.delta[k][:, None] * (x[None, :] - s.alpha[k][:, None]) ** 2)
            ends = np.exp(-dl * (x[None, :] - np.array([lo, hi])[:, None]) ** 2)
            return np.concatenate([orb, ends])      # (M + 2, npts)

        f1a, f1b = fns(0, pts[:, 0]), fns(0, pts[:, 1])
        f2a, f2b = fns(1, pts[:, 0]), fns(1, pts[:, 1])
        m5 = M + 2
        pr = [(l, p) for l in range(m5) for p in range(m5) if i != j or l < p]
        assert s.K == len(pr) == (25 if i != j else 10)
        ref = np.stack([r * (f1a[l] * f2b[p] - f1b[l] * f2a[p]) for l, p in pr], axis=1)
        got = swr.basis_values(s, pts)
        assert np.max(np.abs(got - ref)) <= 1e-14, lin
