"""Pins of the oracle's local orbitals of one electron in two dimensions
(Section 3 with d = 2; oracle/lo2.py), against values and evaluations that do
not go through its quadrature rules or its elliptic-integral form of G:

  * B_eps integrates to one over the plane;
  * G = (1/|.|) * B_eps: G(0) in closed form, 2 pi sigma / eps times
    int_0^1 (1 - t^2)^M dt = 2^(2M) (M!)^2 / (2M + 1)!; the far-field
    expansion 1/rho (1 + eps^2 / (4 (M + 2) rho^2)) (the second moment of
    B_eps is eps^2 / (M + 2), and the circle average of 1/|x - y| is
    1/rho (1 + s^2 / (4 rho^2) + ...)); and G inside, on and outside the
    support against two-dimensional adaptive quadrature of the convolution
    in polar coordinates about the evaluation point (no singularity there);
  * every S entry against the closed-form Gaussian overlaps over the plane,
    the kinetic and barrier terms against adaptive quadrature of their
    one-dimensional factors, and the nuclear term against two-dimensional
    adaptive quadrature of V_n g_u g_w;
  * the orbitals solve the generalised eigenproblem and are S-orthonormal;
  * with all 25 orbitals the basis spans the box's Gaussians: the SWR window
    reconstructs the Gaussian basis's iterates.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads
from oracle import lo2, reconstruct, swr

CF = {c["name"]: c for c in workloads.lo_configs()}


@pytest.fixture(scope="module")
def prob():
    return swr.Problem(CF["tiny-lo"])


def test_mollifier_integrates_to_one():
    for order in (1, 2, 4):
        for eps in (0.1, 0.3):
            tot = integrate.quad(lambda r: 2 * math.pi * r * float(lo2.mollifier2(r, eps, order)),
                                 0, eps, epsabs=1e-15, epsrel=1e-14)[0]
            assert tot == pytest.approx(1.0, abs=1e-13)
            assert float(lo2.mollifier2(1.0001 * eps, eps, order)) == 0.0


@pytest.mark.parametrize("order", [1, 4])
def test_mollified_coulomb_closed_forms(order):
    eps = 0.3
    im = 2.0 ** (2 * order) * math.factorial(order) ** 2 / math.factorial(2 * order + 1)
    assert lo2.coulomb_mollified2(0.0, eps, order) == pytest.approx(
        2 * math.pi * lo2.sigma2(order) / eps * im, rel=1e-14)
    for ratio in (20.0, 40.0):
        rho = ratio * eps
        g = lo2.coulomb_mollified2(rho, eps, order)
        c = (g * rho - 1.0) / (eps * eps / (4 * (order + 2) * rho * rho))
        assert c == pytest.approx(1.0, abs=3.0 / ratio ** 2)


@pytest.mark.parametrize("rho", [0.03, 0.2, 0.3, 0.31, 0.6, 2.0])
def test_mollified_coulomb_matches_polar_quadrature(rho):
    eps, order = 0.3, 4

    def chord(th, sign):
        b = rho * math.cos(th)
        D = eps * eps - (rho * math.sin(th)) ** 2
        return max(0.0, -b + sign * math.sqrt(D)) if D > 0 else 0.0

    f = lambda r, th: float(lo2.mollifier2(math.hypot(rho + r * math.cos(th), r * math.sin(th)),
                                           eps, order))
    ref = integrate.dblquad(f, 0, 2 * math.pi, lambda th: chord(th, -1), lambda th: chord(th, 1),
                            epsabs=1e-15, epsrel=1e-13)[0]
    assert lo2.coulomb_mollified2(rho, eps, order) == pytest.approx(ref, rel=1e-13)
    assert float(lo2.coulomb_mollified2_many(np.array([rho]), eps, order)[0]) == \
        lo2.coulomb_mollified2(rho, eps, order)


def _step(t, w):
    u = min(max(t / w + 0.5, 0.0), 1.0)
    return u ** 3 * (10 - 15 * u + 6 * u * u)


def test_orbital_matrices_match_quadrature(prob):
    cfg = CF["tiny-lo"]
    p = cfg["lo"]
    s = prob.dec.subs[1]
    S, H = lo2.orbital_matrices2(cfg, s)
    (c0, c1), (d0, d1) = s.alpha, s.delta
    n1 = len(c1)
    xc = [0.5 * (s.lo[k] + s.hi[k]) for k in range(2)]

    def g(c, d, x):
        return math.exp(-d * (x - c) ** 2)

    def dg(c, d, x):
        return -2 * d * (x - c) * g(c, d, x)

    def one(k, u, w, kind):
        c, d = (c0, d0) if k == 0 else (c1, d1)
        edge = [xc[k] + sg * p["barrier"] + e * 0.5 * p["barrier_width"] for sg in (-1, 1) for e in (-1, 1)]

        def f(x):
            st = _step(abs(x - xc[k]) - p["barrier"], p["barrier_width"])
            if kind == "S":
                return g(c[u], d[u], x) * g(c[w], d[w], x)
            if kind == "A":
                return (1 - st) * g(c[u], d[u], x) * g(c[w], d[w], x)
            if kind == "Ad":
                return (1 - st) * dg(c[u], d[u], x) * dg(c[w], d[w], x)
            return st * g(c[u], d[u], x) * g(c[w], d[w], x)
        return integrate.quad(f, xc[k] - 25, xc[k] + 25, points=edge, limit=400,
                              epsabs=1e-15, epsrel=1e-13)[0]

    eps, order = p["moll_eps"], p["moll_order"]
    R = cfg["nuclei"][0]

    def vn(x0, x1):
        return -cfg["charges"][0] * lo2.coulomb_mollified2(math.hypot(x0 - R[0], x1 - R[1]), eps, order)

    for ua, wa in [(0, 0), (6, 13), (24, 3)]:
        u0, u1, w0, w1 = ua // n1, ua % n1, wa // n1, wa % n1
        s_ref = one(0, u0, w0, "S") * one(1, u1, w1, "S")
        assert S[ua, wa] == pytest.approx(s_ref, rel=1e-12, abs=1e-15)
        kin = 0.5 * (one(0, u0, w0, "Ad") * one(1, u1, w1, "A") + one(0, u0, w0, "A") * one(1, u1, w1, "Ad"))
        bar = p["v_inf"] * (one(0, u0, w0, "B") * one(1, u1, w1, "S") + one(0, u0, w0, "S") * one(1, u1, w1, "B"))
        nuc = integrate.dblquad(
            lambda x1, x0: vn(x0, x1) * g(c0[u0], d0[u0], x0) * g(c0[w0], d0[w0], x0)
            * g(c1[u1], d1[u1], x1) * g(c1[w1], d1[w1], x1),
            xc[0] - 12, xc[0] + 12, xc[1] - 12, xc[1] + 12, epsabs=1e-12, epsrel=1e-10)[0]
        assert H[ua, wa] == pytest.approx(kin + bar + nuc, rel=1e-9, abs=1e-11), (ua, wa)


def test_orbitals_solve_the_eigenproblem(prob):
    cfg = CF["tiny-lo"]
    s = prob.dec.subs[2]
    S, H = lo2.orbital_matrices2(cfg, s)
    lam, C = lo2.orbitals2(cfg, s)
    assert np.all(np.diff(lam) > 0)
    assert np.max(np.abs(H @ C - S @ C * lam)) <= 1e-11 * np.max(np.abs(H))
    assert np.max(np.abs(C.T @ S @ C - np.eye(C.shape[1]))) <= 1e-12
    assert np.all(np.arange(1, C.shape[0] + 1) @ C > 0)
    assert prob.sys[2].K == 8 and prob.sys[2].A.shape == (8, 8)


def test_all_orbitals_span_the_gaussian_basis():
    cfg = CF["tiny-lo-all"]
    cfg_g = dict(cfg, basis="gaussian")
    cfg_g.pop("lo")
    pts = np.random.default_rng(6).uniform(-5.5, 5.5, size=(200, 2))
    out = []
    for c in (cfg, cfg_g):
        p = swr.Problem(c)
        h, res = swr.swr_window(p, p.initial_coeffs(), iters=3)
        out.append((reconstruct.reconstruct(p, [hh[c["n_steps"]] for hh in h], pts), res))
    (f_l, r_l), (f_g, r_g) = out
    scale = np.max(np.abs(f_g))
    assert np.max(np.abs(f_l - f_g)) <= 1e-9 * scale
    assert np.allclose(r_l, r_g, rtol=1e-7, atol=1e-14)
