"""Pins of the oracle's one-dimensional integrals and quadrature rules
against definitions they do not share code with: adaptive quadrature of
the defining integrals, whole-line closed forms (Gaussian product
theorem), exactness of Gauss-Legendre rules on polynomials, and the
co-centred soft-Coulomb identity with the modified Bessel function K_0."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import gauss1d, quadrature, assemble
from oracle.geometry import Decomposition

RNG = np.random.default_rng(20171006)


def _cases(n=12):
    for _ in range(n):
        lo = RNG.uniform(-5, 0)
        hi = lo + RNG.uniform(0.5, 6)
        aa, ab = RNG.uniform(lo, hi, size=2)
        da, db = RNG.uniform(0.2, 4.0, size=2)
        yield lo, hi, aa, ab, da, db


def _quad(f, lo, hi):
    v, err = integrate.quad(f, lo, hi, epsabs=1e-15, epsrel=1e-13, limit=200)
    return v


@pytest.mark.parametrize("case", list(_cases()))
def test_truncated_integrals_match_adaptive_quadrature(case):
    lo, hi, aa, ab, da, db = case
    al = np.array([aa, ab])
    de = np.array([da, db])
    S = gauss1d.overlap(al, de, lo, hi)
    X = gauss1d.position(al, de, lo, hi)
    T = gauss1d.kinetic(al, de, lo, hi)
    pa = lambda x: math.exp(-da * (x - aa) ** 2)
    pb = lambda x: math.exp(-db * (x - ab) ** 2)
    dpa = lambda x: -2 * da * (x - aa) * pa(x)
    dpb = lambda x: -2 * db * (x - ab) * pb(x)
    assert S[0, 1] == pytest.approx(_quad(lambda x: pa(x) * pb(x), lo, hi), abs=1e-14)
    assert X[0, 1] == pytest.approx(_quad(lambda x: x * pa(x) * pb(x), lo, hi), abs=1e-13)
    assert T[0, 1] == pytest.approx(_quad(lambda x: 0.5 * dpa(x) * dpb(x), lo, hi), abs=1e-13)
    assert T[1, 1] == pytest.approx(_quad(lambda x: 0.5 * dpb(x) ** 2, lo, hi), abs=1e-13)
    # symmetry
    assert S[0, 1] == S[1, 0]
    assert T[0, 1] == pytest.approx(T[1, 0], abs=1e-15)


def test_tail_interval_without_cancellation():
    """Product centre far to the left of [lo, hi]: erf(uh)-erf(ul) would
    cancel; the erfc branch must keep relative accuracy."""
    lo, hi = 3.0, 4.0
    v = gauss1d.gaussian_projection(np.array([3.0]), 1.0, lo, hi, 1.5, -2.0)[0]
    ref = _quad(lambda x: math.exp(-1.5 * (x + 2) ** 2 - (x - 3) ** 2), lo, hi)
    assert v == pytest.approx(ref, rel=1e-10)


def test_whole_line_limits():
    al = np.array([-0.7, 0.4])
    de = np.array([0.9, 1.7])
    S = gauss1d.overlap(al, de, -60, 60)
    T = gauss1d.kinetic(al, de, -60, 60)
    X = gauss1d.position(al, de, -60, 60)
    p = de[0] + de[1]
    mr = de[0] * de[1] / p
    R2 = (al[0] - al[1]) ** 2
    S_ref = math.sqrt(math.pi / p) * math.exp(-mr * R2)
    assert S[0, 1] == pytest.approx(S_ref, rel=1e-14)
    assert T[0, 1] == pytest.approx(mr * (1 - 2 * mr * R2) * S_ref, rel=1e-13)
    P = (de[0] * al[0] + de[1] * al[1]) / p
    assert X[0, 1] == pytest.approx(P * S_ref, rel=1e-13)
    assert S[0, 0] == pytest.approx(math.sqrt(math.pi / (2 * de[0])), rel=1e-14)


@pytest.mark.parametrize("n", [2, 5, 16, 32])
def test_gauss_legendre_exact_on_polynomials(n):
    x, w = quadrature.composite([-1.3, 0.2, 2.0], n)
    for deg in range(2 * n):
        exact = (2.0 ** (deg + 1) - (-1.3) ** (deg + 1)) / (deg + 1)
        assert np.dot(w, x ** deg) == pytest.approx(exact, rel=1e-12, abs=1e-12)


def _single_gaussian_cfg(width, eps, quad_nodes=16):
    return dict(name="one", mode="tdse", n_elec=1, dim=1, L=[1], box_lo=[-12.0],
                box_hi=[12.0], overlap=[0.0], nbasis=[1], width=width, width_ratio=None,
                nuclei=[[0.0]], charges=[1.0], eps_en=eps, eps_ee=eps, dt=0.01,
                n_steps=1, mu=[0.0, 0.0], field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0),
                init=dict(alpha=1.0, center=[0.0]), iters=1, tol=1e-8,
                face_nodes=[4, 4], quad_nodes=quad_nodes)


@pytest.mark.parametrize("width,eps", [(0.5, 1.0), (0.8, 1.0), (0.3, 0.5)])
def test_cocentred_soft_coulomb_bessel_identity(width, eps):
    """int_R exp(-p y^2)/sqrt(y^2+eps^2) dy = exp(p eps^2/2) K_0(p eps^2/2)."""
    cfg = _single_gaussian_cfg(width, eps)
    dec = Decomposition(cfg)
    V = assemble.potential_matrix(dec, dec.subs[0])
    p = 1.0 / width ** 2          # phi^2 = exp(-2 delta y^2), delta = 1/(2 w^2)
    z = 0.5 * p * eps * eps
    ref = -math.exp(z) * special.k0(z)
    assert V[0, 0] == pytest.approx(ref, rel=1e-13)


def test_potential_panel_doubling_converged():
    from workloads import get_config
    cfg = get_config("c2-2e-1d")
    dec = Decomposition(cfg)
    s = dec.subs[27]
    V16 = assemble.potential_matrix(dec, s)
    cfg32 = get_config("c2-2e-1d", quad_nodes=32)
    dec32 = Decomposition(cfg32)
    V32 = assemble.potential_matrix(dec32, dec32.subs[27])
    assert np.max(np.abs(V16 - V32)) < 1e-13 * np.max(np.abs(V32))
