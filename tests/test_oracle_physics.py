"""Physics pins of the oracle: textbook closed forms, invariants of the
time integrators, and brute-force solutions of the same boundary value
problems by an independent finite-difference discretisation."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import workloads
from oracle import reconstruct, swr, tise


def base(**kw):
    c = dict(name="pin", mode="tdse", n_elec=1, dim=1, L=[1], box_lo=[-12.0], box_hi=[12.0],
             overlap=[0.0], nbasis=[1], width=1.0, width_ratio=None, nuclei=[], charges=[],
             eps_en=1.0, eps_ee=1.0, dt=0.01, n_steps=10, mu=[0.0, 0.0],
             field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0),
             init=dict(alpha=0.25, center=[0.0]), iters=1, tol=1e-8, face_nodes=[4, 4],
             quad_nodes=16)
    c.update(kw)
    return c


# --- Hamiltonian / eigen path -------------------------------------------------

def test_single_gaussian_harmonic_ground_state_is_exact():
    """exp(-x^2/2) is the exact ground state of -1/2 d^2 + x^2/2: E0 = 1/2."""
    p = swr.Problem(base(potential="harmonic", omega_ho=1.0))
    lam, _ = tise.local_eigen(p, 0)
    assert lam[0] == pytest.approx(0.5, abs=1e-13)


def test_harmonic_spectrum_n_plus_half():
    p = swr.Problem(base(potential="harmonic", omega_ho=1.0, box_lo=[-9.0], box_hi=[9.0],
                         nbasis=[40], width=None, width_ratio=1.0))
    lam, X = tise.local_eigen(p, 0)
    assert np.allclose(lam[:4], np.arange(4) + 0.5, atol=1e-8)
    # A-orthonormal eigenvectors
    assert np.allclose(X.T @ p.sys[0].A @ X, np.eye(40), atol=1e-8)


def test_two_dimensional_harmonic_is_sum_of_one_dimensional():
    p = swr.Problem(base(potential="harmonic", omega_ho=1.0, n_elec=2, L=[1, 1],
                         box_lo=[-7.0, -7.0], box_hi=[7.0, 7.0], overlap=[0.0, 0.0],
                         nbasis=[24, 22], width=None, width_ratio=1.0,
                         init=dict(alpha=0.25, center=[0.0, 0.0])))
    lam, _ = tise.local_eigen(p, 0)
    assert lam[0] == pytest.approx(1.0, abs=1e-7)
    assert lam[1] == pytest.approx(2.0, abs=1e-6) and lam[2] == pytest.approx(2.0, abs=1e-6)


# --- Crank-Nicolson ---------------------------------------------------------

def _free(**kw):
    return base(box_lo=[-20.0], box_hi=[20.0], nbasis=[81], width=None, width_ratio=1.0,
                dt=0.005, n_steps=200, **kw)


def test_free_gaussian_packet_spreading():
    """psi(x,t) = (2 pi s^2)^(-1/4) a^(-1/2) exp(-x^2/(4 s^2 a)), a = 1 + i t/(2 s^2)."""
    p = swr.Problem(_free())
    c0 = p.initial_coeffs()
    h, _ = swr.swr_window(p, c0, iters=1)
    x = np.linspace(-6, 6, 49)
    T, s0 = 1.0, 1.0
    a = 1 + 1j * T / (2 * s0 ** 2)
    exact = (2 * np.pi * s0 ** 2) ** -0.25 * a ** -0.5 * np.exp(-x ** 2 / (4 * s0 ** 2 * a))
    psi = reconstruct.reconstruct(p, [h[0][-1]], x[:, None])
    assert np.max(np.abs(psi - exact)) < 5e-7
    # variance s0^2 (1 + t^2/(4 s0^4)) from the Galerkin moments
    A = p.sys[0].A
    c = h[0][-1]
    n = np.real(np.conj(c) @ A @ c)
    xs = np.linspace(-20, 20, 4001)
    dens = np.abs(reconstruct.reconstruct(p, [c], xs[:, None])) ** 2
    var = np.trapezoid(xs ** 2 * dens, xs) / np.trapezoid(dens, xs)
    assert var == pytest.approx(s0 ** 2 * (1 + T ** 2 / (4 * s0 ** 4)), rel=1e-6)
    assert n == pytest.approx(1.0, abs=1e-7)


def test_ehrenfest_drift_in_uniform_field():
    """V = 0, E = E0 sin(w t): <x>(t) = -E0 (t/w - sin(w t)/w^2)."""
    E0, w = 0.5, 2.0
    p = swr.Problem(_free(field=dict(E0=E0, omega=w, phase=0.0, axis=0)))
    c0 = p.initial_coeffs()
    h, _ = swr.swr_window(p, c0, iters=1)
    A, Q = p.sys[0].A, p.sys[0].Q
    xs = np.array([np.real(np.conj(c) @ Q @ c) / np.real(np.conj(c) @ A @ c) for c in h[0]])
    t = p.times()
    assert np.max(np.abs(xs + E0 * (t / w - np.sin(w * t) / w ** 2))) < 3e-6


def _circular(**kw):
    f = dict(shape="circular", E0=1.0, omega=3.0, phase=0.3, nu=2.0, center=0.5,
             coords=[[0], [1]], axis=0)
    f.update(kw)
    return f


def test_ehrenfest_drift_in_circular_field():
    """Section 5, Test 3's circular pulse on a free particle in two
    dimensions: each mean coordinate follows its own component,
    <x_c>(t) = x_c(0) - int_0^t (t - s) E_c(s) ds (quadrature), the two
    drifts differing (a swapped component, sign or envelope fails)."""
    from scipy.integrate import quad
    cfg = base(dim=2, L=[1, 1], box_lo=[-8.0, -8.0], box_hi=[8.0, 8.0], overlap=[0.0, 0.0],
               nbasis=[17, 17], width=None, width_ratio=1.0, dt=0.01, n_steps=100,
               field=_circular(), init=dict(alpha=0.5, center=[0.5, -0.3]))
    p = swr.Problem(cfg)
    h, _ = swr.swr_window(p, p.initial_coeffs(), iters=1)
    sy = p.sys[0]
    t = p.times()
    drift = []
    for c, Qc in enumerate((sy.Q, sy.Q2)):
        xs = np.array([np.real(np.conj(v) @ Qc @ v) / np.real(np.conj(v) @ sy.A @ v) for v in h[0]])
        ref = np.array([cfg["init"]["center"][c] -
                        quad(lambda s: (tt - s) * swr.field(cfg, s)[c], 0.0, tt,
                             epsabs=1e-13, epsrel=1e-12)[0] for tt in t])
        assert np.max(np.abs(xs - ref)) < 2e-4, c
        drift.append(ref[-1] - ref[0])
    assert abs(drift[0] - drift[1]) > 0.1


def test_cn_time_reversal_with_circular_field():
    """The two-component field term in both Crank-Nicolson matrices: stepping
    back over the reversed field and data recovers c0 (one electron in two
    dimensions with a nucleus, one component per axis)."""
    cfg = workloads.get_config("c5-mini-1e", field=_circular(E0=0.7, omega=5.0, center=0.05))
    p = swr.Problem(cfg)
    sy = p.sys[2]
    rng = np.random.default_rng(5)
    c0 = p.initial_coeffs()[2]
    f = rng.standard_normal((p.n_T + 1, sy.K)) + 1j * rng.standard_normal((p.n_T + 1, sy.K))
    E = swr.field(cfg, p.times())
    assert E.shape == (p.n_T + 1, 2) and np.ptp(E[:, 0]) > 0.1 and np.ptp(E[:, 1]) > 0.1
    h = swr.local_cn(sy, c0, f, E, p.dt)
    back = swr.local_cn(sy, h[-1], f[::-1], E[::-1], -p.dt)
    assert np.max(np.abs(back[-1] - c0)) < 1e-11 * np.max(np.abs(c0))


def test_cn_conserves_a_norm_for_hermitian_static_hamiltonian():
    from workloads import tiny_configs
    cfg = tiny_configs()[0]
    cfg.update(mu=[0.0, 0.0], n_steps=400, field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0))
    p = swr.Problem(cfg)
    sy = p.sys[1]
    c0 = p.initial_coeffs()[1]
    f = np.zeros((cfg["n_steps"] + 1, sy.K), dtype=complex)
    h = swr.local_cn(sy, c0, f, np.zeros(cfg["n_steps"] + 1), p.dt)
    norms = np.real(np.einsum("ni,ij,nj->n", np.conj(h), sy.A, h))
    assert np.max(np.abs(norms - norms[0])) < 1e-12 * norms[0]


def test_cn_time_reversal_with_field_and_robin_data():
    """Stepping back with -dt over the reversed field and data recovers c0:
    each step's left and right matrices are each other's reverse step."""
    from workloads import tiny_configs
    cfg = tiny_configs()[0]
    p = swr.Problem(cfg)
    sy = p.sys[1]
    rng = np.random.default_rng(3)
    c0 = p.initial_coeffs()[1]
    f = rng.standard_normal((p.n_T + 1, sy.K)) + 1j * rng.standard_normal((p.n_T + 1, sy.K))
    E = swr.field(cfg, p.times())
    h = swr.local_cn(sy, c0, f, E, p.dt)
    back = swr.local_cn(sy, h[-1], f[::-1], E[::-1], -p.dt)
    assert np.max(np.abs(back[-1] - c0)) < 1e-11 * np.max(np.abs(c0))


def test_cn_second_order_in_time_with_strong_field():
    """Richardson: halving dt divides the error by ~4 (second order); a field
    frozen at t_n on both sides would give first order."""
    errs = []
    cfg0 = base(box_lo=[-10.0], box_hi=[10.0], nbasis=[30], width=None, width_ratio=1.0,
                nuclei=[[0.0]], charges=[1.0], field=dict(E0=2.0, omega=3.0, phase=0.3, axis=0))
    ref = None
    for dt in (0.00125, 0.02, 0.01, 0.005):
        cfg = dict(cfg0, dt=dt, n_steps=int(round(0.6 / dt)))
        p = swr.Problem(cfg)
        h, _ = swr.swr_window(p, p.initial_coeffs(), iters=1)
        if ref is None:
            ref = h[0][-1]
            A = p.sys[0].A
            continue
        d = h[0][-1] - ref
        errs.append(math.sqrt(np.real(np.conj(d) @ A @ d)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5


# --- Imaginary time ---------------------------------------------------------

def test_ngf_energy_decreases_monotonically_to_lowest_eigenvalue():
    cfg = base(box_lo=[-10.0], box_hi=[10.0], nbasis=[30], width=None, width_ratio=1.0,
               nuclei=[[0.4]], charges=[1.0], mu=[2.0, 0.0], dt=0.1, n_steps=300,
               init=dict(alpha=0.3, center=[1.0]), mode="tise")
    p = swr.Problem(cfg)
    c0 = tise.initial_state(p)
    f = [np.zeros((p.n_T + 1, p.sys[0].K))]
    h, nus = tise.ngf_iteration(p, c0, f)
    H, A = tise.real_H(p, 0), p.sys[0].A
    en = np.array([c @ H @ c / (c @ A @ c) for c in h[0]])
    assert np.all(np.diff(en) <= 1e-13)
    lam, _ = tise.local_eigen(p, 0)
    assert en[-1] == pytest.approx(lam[0], abs=1e-10)
    # energy from the normaliser at the fixed point
    assert tise.energy_from_nu(nus[-1], p.dt) == pytest.approx(lam[0], abs=1e-10)


# --- SWR against brute force ------------------------------------------------

def _fd_laplacian_robin(x, mu):
    """Second-order central differences with ghost points eliminated by the
    Robin condition d_n psi + mu psi = 0 at both ends."""
    M = len(x)
    h = x[1] - x[0]
    main = np.full(M, -2.0) / h ** 2
    off = np.ones(M - 1) / h ** 2
    D2 = sp.diags([off, main, off], [-1, 0, 1], format="lil", dtype=complex)
    D2[0, 1] = 2 / h ** 2
    D2[0, 0] = -(2 + 2 * h * mu) / h ** 2
    D2[M - 1, M - 2] = 2 / h ** 2
    D2[M - 1, M - 1] = -(2 + 2 * h * mu) / h ** 2
    return D2.tocsc()


def _swr_fd_cfg(nb):
    return dict(name="swr-fd", mode="tdse", n_elec=1, dim=1, L=[3], box_lo=[-8.0],
                box_hi=[8.0], overlap=[1.5], nbasis=[nb], basis_extend=2, width=None,
                width_ratio=0.8, nuclei=[[0.3]], charges=[1.0], eps_en=1.0, eps_ee=1.0,
                dt=0.01, n_steps=100, mu=[0.0, -4.0],
                field=dict(E0=0.3, omega=1.1, phase=0.2, axis=0),
                init=dict(alpha=0.7, center=[0.4]), iters=30, tol=1e-12,
                face_nodes=[4, 4], quad_nodes=16)


def _fd_tdse(c, M=3201):
    x = np.linspace(c["box_lo"][0], c["box_hi"][0], M)
    mu = complex(*c["mu"])
    V = sum(-Z / np.sqrt((x - R[0]) ** 2 + c["eps_en"] ** 2) for R, Z in zip(c["nuclei"], c["charges"]))
    H0 = -0.5 * _fd_laplacian_robin(x, mu) + sp.diags(V)
    a, x0 = c["init"]["alpha"], c["init"]["center"][0]
    psi = (2 * a / np.pi) ** 0.25 * np.exp(-a * (x - x0) ** 2) + 0j
    dt = c["dt"]
    tau = dt / 2
    I = sp.identity(M, format="csc")
    f = c["field"]
    E = lambda t: f["E0"] * np.sin(f["omega"] * t + f["phase"])
    for n in range(c["n_steps"]):
        Hn = H0 + sp.diags(x * E(n * dt))
        Hn1 = H0 + sp.diags(x * E((n + 1) * dt))
        psi = spl.spsolve((I + 1j * tau * Hn1).tocsc(), (I - 1j * tau * Hn) @ psi)
    return x, psi


@pytest.mark.slow
def test_converged_swr_matches_finite_difference_solution():
    """Converged Robin-SWR (3 overlapping subdomains, soft-Coulomb well,
    laser field, absorbing outer boundary) vs CN + finite differences on a
    fine grid of the whole box: agreement at the level of the Galerkin
    error, shrinking as the local bases grow."""
    xs = np.linspace(-7.5, 7.5, 61)
    x, psi = _fd_tdse(_swr_fd_cfg(16))
    ref = np.interp(xs, x, psi.real) + 1j * np.interp(xs, x, psi.imag)
    errs = []
    for nb in (16, 24):
        p = swr.Problem(_swr_fd_cfg(nb))
        h, res = swr.swr_window(p, p.initial_coeffs(), tol=1e-12)
        assert res[-1] < 1e-12
        out = reconstruct.reconstruct(p, [hh[-1] for hh in h], xs[:, None])
        errs.append(np.max(np.abs(out - ref)))
    assert errs[1] < 3e-5 and errs[1] < errs[0]


def test_swr_residual_decreases_and_single_domain_needs_one_iteration():
    from workloads import tiny_configs
    cfg = tiny_configs()[0]
    cfg["iters"] = 8
    p = swr.Problem(cfg)
    _, res = swr.swr_window(p, p.initial_coeffs())
    assert all(b < a for a, b in zip(res[1:], res[2:]))
    cfg1 = dict(cfg, L=[1], overlap=[0.0])
    p1 = swr.Problem(cfg1)
    _, res1 = swr.swr_window(p1, p1.initial_coeffs(), iters=3)
    assert res1[1] == 0.0 and res1[2] == 0.0


def _fd_ground_energy(c, M=2001):
    x = np.linspace(c["box_lo"][0], c["box_hi"][0], M)
    V = sum(-Z / np.sqrt((x - R[0]) ** 2 + c["eps_en"] ** 2) for R, Z in zip(c["nuclei"], c["charges"]))
    H = (-0.5 * _fd_laplacian_robin(x, complex(*c["mu"])) + sp.diags(V)).toarray().real
    # the ghost-point rows are scaled by 2 at the ends: symmetrise with the
    # trapezoid weights
    w = np.ones(M)
    w[0] = w[-1] = 0.5
    Hs = np.sqrt(w)[:, None] * H / np.sqrt(w)[None, :]
    return float(np.min(np.linalg.eigvals(Hs).real))


@pytest.mark.slow
def test_swr_imaginary_time_energy_matches_finite_difference_ground_state():
    cfg = dict(_swr_fd_cfg(24), mode="tise", mu=[3.0, 0.0], dt=0.1, n_steps=250,
               field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0), iters=40, tol=1e-11)
    p = swr.Problem(cfg)
    _, res, en = tise.swr_tise(p, tol=1e-11)
    e_fd = _fd_ground_energy(cfg)
    assert en[-1] == pytest.approx(e_fd, abs=2e-5)


def _two_electron_states():
    """Tiny two-electron decomposition (symmetric under exchange: the same
    boxes and bases for both coordinates) with random local coefficients,
    and their exchange-symmetrised copy."""
    cfg = dict([c for c in workloads.tiny_configs() if c["name"] == "tiny-2d"][0],
               L=[3, 3], box_lo=[-6.0, -6.0], box_hi=[6.0, 6.0], overlap=[0.8, 0.8],
               nbasis=[4, 4])
    p = swr.Problem(cfg)
    rng = np.random.default_rng(5)
    c = [rng.standard_normal(s.K) + 1j * rng.standard_normal(s.K) for s in p.dec.subs]
    # subdomain (i, j) <-> (j, i), basis (a, b) <-> (b, a): the exchanged state
    L = 3
    cs = []
    for s in p.dec.subs:
        i, j = s.lin % L, s.lin // L
        m = p.dec.subs[j + L * i]
        cm = c[m.lin].reshape(4, 4).T.reshape(-1)
        cs.append(0.5 * (c[s.lin] + cm))
    return p, c, cs


def test_antisymmetric_reconstruction_is_antisymmetric():
    """Appendix A: psi_A(sigma x) = -psi_A(x) off the diagonal, for any local
    coefficients; on the side where electron 2 does not come after electron
    1 it is the plain reconstruction."""
    p, c, _ = _two_electron_states()
    x = np.random.default_rng(6).uniform(-6.0, 6.0, size=(300, 2))
    x = x[np.abs(x[:, 0] - x[:, 1]) > 1e-3]
    a = reconstruct.reconstruct_antisym(p, c, x)
    b = reconstruct.reconstruct_antisym(p, c, reconstruct.exchange(x, 1))
    assert np.allclose(a, -b, rtol=0, atol=1e-14 * np.max(np.abs(a)))
    keep = ~reconstruct.after(x, 1)
    assert np.array_equal(a[keep], reconstruct.reconstruct(p, c, x[keep]))
    assert np.any(keep) and np.any(~keep)


def test_antisymmetrisation_of_a_symmetric_state_is_the_sign_change():
    """For an exchange-symmetric state the construction is Section 5's
    a posteriori operator: psi where x2 <= x1, -psi where x2 > x1."""
    p, _, cs = _two_electron_states()
    x = np.random.default_rng(7).uniform(-6.0, 6.0, size=(300, 2))
    plain = reconstruct.reconstruct(p, cs, x)
    assert np.allclose(plain, reconstruct.reconstruct(p, cs, reconstruct.exchange(x, 1)),
                       rtol=0, atol=1e-13 * np.max(np.abs(plain)))
    sign = np.where(x[:, 1] > x[:, 0], -1.0, 1.0)
    assert np.allclose(reconstruct.reconstruct_antisym(p, cs, x), sign * plain,
                       rtol=0, atol=1e-13 * np.max(np.abs(plain)))


def test_unnormalized_flow_is_the_heat_equation():
    """Without normalisation and without potential, the imaginary-time steps
    solve phi_t = 1/2 Lap phi (Test 1.b's phi_t = Lap phi in the time 2t):
    exp(-a x^2) spreads as (1 + 2 a t)^(-1/2) exp(-a x^2 / (1 + 2 a t)).  One
    subdomain on a box wide enough for the absorbing faces not to matter;
    the error at t = 1 falls by about half when the step halves (implicit
    Euler), so the flow, not just its shape, is the heat flow."""
    a, T = 0.5, 1.0
    base = dict(mode="tise", unnormalized=True, n_elec=1, dim=1, L=[1], box_lo=[-14.0],
                box_hi=[14.0], overlap=[0.0], nbasis=[60], width=None, width_ratio=0.7,
                nuclei=[], charges=[], eps_en=1.0, eps_ee=1.0, mu=[1.0, 0.0],
                field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0),
                init=dict(alpha=a, center=[0.0]), iters=1, tol=None, face_nodes=[1, 1],
                quad_nodes=16, name="heat-pin")
    x = np.linspace(-3.0, 3.0, 61)
    norm0 = (2.0 * a / math.pi) ** 0.25
    exact = norm0 * (1 + 2 * a * T) ** -0.5 * np.exp(-a * x ** 2 / (1 + 2 * a * T))
    errs = []
    for n in (20, 40, 80):
        cfg = dict(base, dt=T / n, n_steps=n)
        p = swr.Problem(cfg)
        h, _, en = tise.swr_tise(p, iters=1)
        assert math.isnan(en[0])
        psi = reconstruct.reconstruct(p, [hh[-1] for hh in h], x[:, None])
        errs.append(float(np.max(np.abs(psi - exact)) / np.max(exact)))
    assert errs[0] < 2e-2
    for e1, e2 in zip(errs, errs[1:]):
        assert 1.7 < e1 / e2 < 2.3
