"""Workload parameter sets (plain data, JSON-compatible).

Every workload is a dict with these keys:

  name          label
  mode          "tdse" (real time, Crank-Nicolson) or "tise" (imaginary time)
  n_elec, dim   N electrons in d space dimensions; configuration space has
                D = N*d dimensions, electron m owns dims m*d .. m*d+d-1
  L             subdomains per configuration dimension (length D)
  box_lo/box_hi global box per configuration dimension (length D)
  overlap       overlap width eps per configuration dimension (length D)
  nbasis        Gaussians per dimension in every subdomain (length D), or a
                list of per-subdomain lists (uneven bases)
  basis_extend  optional: centres run this many spacings past each end of
                the subdomain (default 0: centres span the subdomain)
  width         absolute Gaussian width sigma (delta = 1/(2 sigma^2)), or None
  width_ratio   sigma = width_ratio * centre spacing, used when width is None
  nuclei        list of nuclear positions (each of length d)
  charges       nuclear charges
  eps_en/eps_ee soft-Coulomb regularisation of e-n and e-e terms
  dt, n_steps   time step and steps per window
  mu            Robin coefficient as [re, im]
  field         E(t) = E0 sin(omega t + phase) along spatial axis `axis`
  init          initial state exp(-alpha |x - center|^2), L2-normalised on R^D
  iters         Schwarz iterations (fixed count) and tol the residual target
  face_nodes    Gauss-Legendre nodes per tangential panel: [band, middle]
  quad_nodes    Gauss-Legendre nodes per panel for the potential quadrature
"""
import copy
import math

_C1 = dict(
    name="c1-1e-1d", mode="tdse", n_elec=1, dim=1,
    L=[4], box_lo=[-20.0], box_hi=[20.0], overlap=[2.0],
    nbasis=[16], width=0.8, width_ratio=None,
    nuclei=[[0.0]], charges=[1.0], eps_en=1.0, eps_ee=1.0,
    dt=0.01, n_steps=200, mu=[0.0, -10.0],
    field=dict(E0=0.05, omega=0.057, phase=0.0, axis=0),
    init=dict(alpha=1.0, center=[0.0]),
    iters=30, tol=1e-8, face_nodes=[16, 32], quad_nodes=16,
)

_C2 = dict(
    name="c2-2e-1d", mode="tdse", n_elec=2, dim=1,
    L=[8, 8], box_lo=[-15.0, -15.0], box_hi=[15.0, 15.0],
    overlap=[0.375, 0.375],
    nbasis=[8, 8], width=None, width_ratio=0.7,
    nuclei=[[-1.4], [1.4]], charges=[1.0, 1.0], eps_en=1.0, eps_ee=1.0,
    dt=0.005, n_steps=1000, mu=[0.0, -10.0],
    field=dict(E0=0.05, omega=0.057, phase=0.0, axis=0),
    init=dict(alpha=1.0, center=[0.0, 0.0]),
    iters=20, tol=1e-8, face_nodes=[16, 32], quad_nodes=16,
)

_C2_TISE = dict(_C2, name="c2-2e-1d-tise", mode="tise", mu=[10.0, 0.0],
                dt=0.05, n_steps=400,
                field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0))

# Learned warm start runs on the two-electron system with several windows;
# 32 time nodes (windows of at least 195 steps).
_C4 = dict(_C2, name="c4-2e-1d-learned", iters=60, tol=1e-8, learned_nodes=32)

_C5 = dict(
    name="c5-2e-2d", mode="tdse", n_elec=2, dim=2,
    L=[4, 4, 4, 4], box_lo=[-10.0] * 4, box_hi=[10.0] * 4, overlap=[0.5] * 4,
    nbasis=[6, 6, 6, 6], width=None, width_ratio=0.7,
    nuclei=[[-1.0, 0.0], [1.0, 0.0]], charges=[1.0, 1.0],
    eps_en=0.5, eps_ee=0.5,
    dt=0.01, n_steps=500, mu=[0.0, -10.0],
    field=dict(E0=0.05, omega=0.057, phase=0.0, axis=0),
    init=dict(alpha=1.0, center=[0.0, 0.0, 0.0, 0.0]),
    iters=30, tol=1e-8, face_nodes=[2, 4], quad_nodes=16,
)

def _uneven_geometries(n_geom, L, box, k_lo, k_span, seed=1710):
    """Seeded geometries of the batched one-electron workload: two unit
    charges at +-R_g/2 with R_g = 1 + 2 u_g (u_g uniform), and per-subdomain
    basis sizes round(k_lo + k_span exp(-d^2 / 8)) with d the distance from
    the subdomain centre to the nearest nucleus (a density rule: more
    Gaussians where the wells are).  The sizes of geometry 0 apply to all
    geometries (one decomposition, batched)."""
    import numpy as np
    u = np.random.default_rng(seed).random(n_geom)
    R = 1.0 + 2.0 * u
    geoms = [[[float(-0.5 * r)], [float(0.5 * r)]] for r in R]
    h = (box[1] - box[0]) / L
    centres = box[0] + h * (np.arange(L) + 0.5)
    d = np.min(np.abs(centres[:, None] - np.array([-0.5 * R[0], 0.5 * R[0]])[None, :]), axis=1)
    nb = [[int(round(k_lo + k_span * np.exp(-di * di / 8.0)))] for di in d]
    return geoms, nb


_C3_GEOMS, _C3_NB = _uneven_geometries(64, 256, (-20.0, 20.0), 32, 224)
_C3 = dict(
    name="c3-1e-1d-batched", mode="tdse", n_elec=1, dim=1,
    L=[256], box_lo=[-20.0], box_hi=[20.0], overlap=[0.2 * 40.0 / 256],
    nbasis=_C3_NB, width=None, width_ratio=0.7, geometries=_C3_GEOMS,
    nuclei=_C3_GEOMS[0], charges=[1.0, 1.0], eps_en=1.0, eps_ee=1.0,
    dt=0.01, n_steps=200, mu=[0.0, -10.0],
    field=dict(E0=0.05, omega=0.057, phase=0.0, axis=0),
    init=dict(alpha=1.0, center=[0.0]),
    iters=30, tol=1e-8, face_nodes=[16, 32], quad_nodes=16,
)

# The same recipe at sizes the narrow path takes (K <= 64): 4 geometries, 16
# subdomains, K from 8 to 40.
_C3M_GEOMS, _C3M_NB = _uneven_geometries(4, 16, (-20.0, 20.0), 8, 32)
_C3_MINI = dict(_C3, name="c3-mini", L=[16], overlap=[0.5], nbasis=_C3M_NB,
                geometries=_C3M_GEOMS, nuclei=_C3M_GEOMS[0], iters=8)

# Wide bases (the wide-basis path) at a size the oracle runs in seconds: two
# geometries of the batched recipe on 8 subdomains with 33 to 256 Gaussians
# (one to four 64-wide tiles, ragged ends), 200 steps (two chunks of the
# field series, the second one ragged).
_C3W_GEOMS, _ = _uneven_geometries(2, 8, (-20.0, 20.0), 32, 224)
_C3_WIDE = dict(_C3, name="c3-wide", L=[8], overlap=[1.0],
                nbasis=[[40], [72], [130], [256], [201], [97], [65], [33]],
                geometries=_C3W_GEOMS, nuclei=_C3W_GEOMS[0], iters=3)

# Two electrons in two dimensions at a size the oracle assembles in under a
# minute: 2^4 subdomains of 3x2x2x3 Gaussians, unequal boxes, overlaps and
# per-dimension sizes, field along the second spatial axis.
_C5_MINI = dict(
    name="c5-mini", mode="tdse", n_elec=2, dim=2,
    L=[2, 2, 2, 2], box_lo=[-5.0, -4.0, -5.0, -4.5], box_hi=[5.0, 4.0, 4.5, 4.0],
    overlap=[0.8, 0.7, 0.8, 0.6],
    nbasis=[3, 2, 2, 3], width=None, width_ratio=0.7,
    nuclei=[[-1.0, 0.0], [1.0, 0.2]], charges=[1.0, 1.0], eps_en=0.5, eps_ee=0.6,
    dt=0.01, n_steps=6, mu=[0.3, -5.0],
    field=dict(E0=0.2, omega=0.9, phase=0.1, axis=1),
    init=dict(alpha=0.5, center=[0.2, -0.1, -0.2, 0.1]),
    iters=3, tol=1e-8, face_nodes=[2, 2], quad_nodes=8,
)

# The four-dimensional workload's decomposition (4^4 subdomains: interior
# subdomains with all 80 neighbours) at a size the oracle runs in minutes:
# 2^4 Gaussians per subdomain, coarser potential panels, 10 steps.
_C5_K16 = dict(_C5, name="c5-k16", nbasis=[2, 2, 2, 2], quad_nodes=4, n_steps=10, iters=5)

# One electron in two dimensions (D = 2 with a two-dimensional nucleus term),
# field along the second axis.
_C5_MINI_1E = dict(
    _C5_MINI, name="c5-mini-1e", n_elec=1, L=[3, 2], box_lo=[-6.0, -5.0], box_hi=[6.0, 5.5],
    overlap=[0.8, 0.7], nbasis=[5, 4], init=dict(alpha=0.6, center=[0.3, -0.2]), n_steps=10,
)

# The paper's imaginary-time ground-state experiments (Section 5, Tests 2.a
# and 2.b): H2 with two electrons in one dimension each, 5x5 subdomains with
# 6x6 Gaussians, mu = 10.  Readings where the paper is silent: overlap 10 %
# of box/L (it says "about 10 %"), softening 0.2 for both the nucleus and
# the electron-electron terms (Test 2.a's eta; Test 2.b gives none), and a
# fixed imaginary-time window (18 for 2.a, 4 for 2.b) instead of the
# variable converged time.
_T2A = dict(
    name="paper-test-2a", mode="tise", n_elec=2, dim=1,
    L=[5, 5], box_lo=[-15.0, -15.0], box_hi=[15.0, 15.0], overlap=[0.6, 0.6],
    nbasis=[6, 6], width=1.0, width_ratio=None,            # delta = 0.5
    nuclei=[[-1.25], [1.25]], charges=[1.0, 1.0], eps_en=0.2, eps_ee=0.2,
    dt=0.45, n_steps=40, mu=[10.0, 0.0],
    field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0),
    init=dict(alpha=1.0, center=[0.0, 0.0]),
    iters=30, tol=1e-8, face_nodes=[16, 32], quad_nodes=16,
)
# The paper's determinant Test 2.a (Section 6): 5 x 5 subdomains of [-8, 8]^2
# with overlap 0.32, nuclei at +-0.5, imaginary time with mu = 1 and
# dt = 1.4e-3; 8 local orbitals per interval from 10 Gaussians (64
# determinants off the diagonal, 28 on it: the paper's K = 28), the order-4
# mollifier of width 0.1 (sigma = 315/256, eps = 0.1 as printed), a barrier
# 0.32 beyond each box edge; eta = 0.5 for both soft-Coulomb terms (the test
# gives none), the antisymmetrised Gaussian pair at +-1 as the start, 200
# steps per window.
_T2A_LSD = dict(
    name="paper-lsd-test-2a", mode="tise", n_elec=2, dim=1, basis="lsd",
    L=[5, 5], box_lo=[-8.0, -8.0], box_hi=[8.0, 8.0], overlap=[0.32, 0.32],
    nbasis=[10, 10], width=None, width_ratio=0.7,
    nuclei=[[-0.5], [0.5]], charges=[1.0, 1.0], eps_en=0.5, eps_ee=0.5,
    dt=1.4e-3, n_steps=200, mu=[1.0, 0.0],
    field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0),
    init=dict(alpha=0.5, center=[-1.0, 1.0]),
    lsd=dict(orbitals=8, barrier=2.0, barrier_width=0.4, v_inf=30.0, moll_eps=0.1,
             moll_order=4),
    iters=20, tol=1e-8, face_nodes=[16, 32], quad_nodes=16,
)
# Section 5, determinant Test 2.b: H2 with x_A, x_B = -/+0.1 and eta = 0.6 in
# eq. (pseudo) on (-4, 4)^2, 25 subdomains, mu = 10, the local basis
# augmented (Section 3.3) by Gaussians of exponent 3 at the subdomains'
# boundaries, 15 determinants on the diagonal subdomains.  Readings: the
# intervals' Gaussians all have exponent 3 (width 1/sqrt(6)), so the added
# ones are each interval's first and last Gaussian, centred on its box's
# ends (augment = 1), and 15 = 6 * 5 / 2 gives 4 orbitals + 2 Gaussians
# (36 determinants off the diagonal); 7 Gaussians per interval (the test
# does not give the count; 6 would make the basis the Slater-like one);
# Test 2.a's overlap 0.32 (0.16 puts the determinants' Gram condition at
# 1.1e6, above the recurrence's limit; 0.32 gives 7.8e5); the barrier scaled with the
# interval (half-width 1.0, transition 0.2); the printed initial guess
# exp(-4 (x1^2 + x2^2)) is symmetric, so the antisymmetrised product of two
# such Gaussians centred at -/+0.5; Test 2.a's time step.
_T2B_LSD = dict(
    _T2A_LSD, name="paper-lsd-test-2b", box_lo=[-4.0, -4.0], box_hi=[4.0, 4.0],
    overlap=[0.32, 0.32], nbasis=[7, 7], width=1.0 / math.sqrt(6.0),
    nuclei=[[-0.1], [0.1]], eps_en=0.6, eps_ee=0.6, mu=[10.0, 0.0],
    init=dict(alpha=4.0, center=[-0.5, 0.5]),
    lsd=dict(orbitals=4, augment=1, barrier=1.0, barrier_width=0.2, v_inf=30.0, moll_eps=0.1,
             moll_order=4),
)
# Local orbitals of one electron in two dimensions (Section 3 with d = 2):
# 4 x 4 boxes of [-8, 8]^2 (overlap 0.5), 8 x 8 Gaussians per box at 0.7 x
# spacing, the 16 lowest orbitals of each box (barrier half-width 2.6 about
# its centre, transition 0.4, height 30, order-4 mollifier of radius 0.2)
# for a one-electron molecule with two unit charges at (-/+0.7, 0); real
# time with a complex Robin constant and a sine field, 200 steps, 20
# iterations.
_LO_2D = dict(
    name="lo-1e-2d", mode="tdse", n_elec=1, dim=2, basis="lo",
    L=[4, 4], box_lo=[-8.0, -8.0], box_hi=[8.0, 8.0], overlap=[0.5, 0.5],
    nbasis=[8, 8], width=None, width_ratio=0.7,
    nuclei=[[-0.7, 0.0], [0.7, 0.0]], charges=[1.0, 1.0], eps_en=0.5, eps_ee=0.5,
    dt=0.01, n_steps=200, mu=[0.0, -4.0],
    field=dict(E0=0.1, omega=0.5, phase=0.0, axis=0),
    init=dict(alpha=0.5, center=[0.3, -0.2]),
    iters=20, tol=1e-8, face_nodes=[16, 32], quad_nodes=16,
    lo=dict(orbitals=16, barrier=2.6, barrier_width=0.4, v_inf=30.0, moll_eps=0.2,
            moll_order=4),
)
_T2B = dict(_T2A, name="paper-test-2b", box_lo=[-6.5, -6.5], box_hi=[6.5, 6.5],
            overlap=[0.26, 0.26], width=0.5,                  # delta = 2
            nuclei=[[-0.5], [0.5]], dt=0.01, n_steps=400,
            init=dict(alpha=0.8, center=[0.0, 0.0]))

# Section 5, Test 1.b: the heat equation phi_t = Lap phi on (-15, 15)^2, 5x5
# subdomains of 6x6 Gaussians, mu = 1, phi_0 = exp(-0.2 |x|^2), T = 16 with
# steps of about 0.213 (75 steps).  It is run as the imaginary-time flow
# without normalisation and without potential, d_t phi = 1/2 Lap phi, over
# the time 2t (so dt = 2 x 16/75).  Readings: overlap 10 % of box/L, widths
# 0.7 x spacing (the test gives neither).
_T1B = dict(
    name="paper-test-1b", mode="tise", unnormalized=True, n_elec=1, dim=2,
    L=[5, 5], box_lo=[-15.0, -15.0], box_hi=[15.0, 15.0], overlap=[0.6, 0.6],
    nbasis=[6, 6], width=None, width_ratio=0.7,
    nuclei=[], charges=[], eps_en=1.0, eps_ee=1.0,
    dt=2.0 * 16.0 / 75.0, n_steps=75, mu=[1.0, 0.0],
    field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0),
    init=dict(alpha=0.2, center=[0.0, 0.0]),
    iters=30, tol=1e-8, face_nodes=[16, 32], quad_nodes=16,
)

# Section 5, Test 3 (real time): two electrons in one dimension each on
# (-10, 10)^2, 5x5 subdomains of 6x6 Gaussians, mu = -10i, steps of 0.05 to
# T = 2.5, phi_0 = exp(-|x|^2), softening eta = 0.5, and the circular pulse
# E0 = 1, omega = 8, nu = 10 centred at T/2 whose two components act on the
# two coordinates of the configuration plane (x1 and x2).  Readings where the
# test is silent: the H2 nuclei at -0.5 and 0.5 (Section 6 places H2
# there), widths 0.7 x spacing as for Test 1.b (Test 2.a's delta = 0.5 on
# these smaller boxes makes the Gram matrices nearly singular, condition
# 1.6e8), overlap 10 % of box/L, eta for both the nucleus and the
# electron-electron terms.
_T3 = dict(
    name="paper-test-3", mode="tdse", n_elec=2, dim=1,
    L=[5, 5], box_lo=[-10.0, -10.0], box_hi=[10.0, 10.0], overlap=[0.4, 0.4],
    nbasis=[6, 6], width=None, width_ratio=0.7,
    nuclei=[[-0.5], [0.5]], charges=[1.0, 1.0], eps_en=0.5, eps_ee=0.5,
    dt=0.05, n_steps=50, mu=[0.0, -10.0],
    field=dict(shape="circular", E0=1.0, omega=8.0, phase=0.0, nu=10.0, center=1.25,
               coords=[[0], [1]], axis=0),
    init=dict(alpha=1.0, center=[0.0, 0.0]),
    iters=30, tol=1e-8, face_nodes=[16, 32], quad_nodes=16,
)

# The two-electron workload in the Slater-like antisymmetric basis of
# Section 2 (eq. (LSD)): the same decomposition, 8 Gaussians per interval
# (64 antisymmetrised pairs off the diagonal, 28 on it), started from the
# antisymmetrised product of two Gaussians at -1 and +1.
_C2_SLATER = dict(_C2, name="c2-2e-1d-slater", basis="slater",
                  init=dict(alpha=1.0, center=[-1.0, 1.0]))
_C2_SLATER_TISE = dict(_C2_TISE, name="c2-2e-1d-slater-tise", basis="slater",
                       init=dict(alpha=1.0, center=[-1.0, 1.0]))

CONFIGS = {c["name"]: c for c in (_C1, _C2, _C2_TISE, _C3, _C3_MINI, _C3_WIDE, _C4, _C5, _T2A_LSD,
                                   _T2B_LSD, _LO_2D,
                                   _C5_K16, _C5_MINI, _C5_MINI_1E, _T1B, _T2A, _T2B, _T3,
                                   _C2_SLATER, _C2_SLATER_TISE)}


def get_config(name, **overrides):
    """Deep copy of a named workload with optional top-level overrides."""
    cfg = copy.deepcopy(CONFIGS[name])
    cfg.update(copy.deepcopy(overrides))
    return cfg


def tiny_configs():
    """Small workloads the oracle runs in well under a second each.

    They cover one and two configuration dimensions, unequal L and basis
    sizes per dimension (to catch transposed indices), a basis size that is
    not a multiple of any tile, complex and real Robin coefficients.
    """
    t1 = dict(
        name="tiny-1d", mode="tdse", n_elec=1, dim=1,
        L=[3], box_lo=[-8.0], box_hi=[8.0], overlap=[1.5],
        nbasis=[7], width=None, width_ratio=0.8,
        nuclei=[[0.3]], charges=[1.0], eps_en=1.0, eps_ee=1.0,
        dt=0.02, n_steps=12, mu=[0.0, -4.0],
        field=dict(E0=0.3, omega=1.1, phase=0.2, axis=0),
        init=dict(alpha=0.7, center=[0.4]),
        iters=6, tol=1e-8, face_nodes=[4, 6], quad_nodes=16,
    )
    t2 = dict(
        name="tiny-2d", mode="tdse", n_elec=2, dim=1,
        L=[3, 2], box_lo=[-6.0, -5.0], box_hi=[6.0, 5.5], overlap=[0.8, 0.7],
        nbasis=[5, 4], width=None, width_ratio=0.7,
        nuclei=[[-0.7], [0.9]], charges=[1.0, 0.8], eps_en=1.0, eps_ee=0.9,
        dt=0.01, n_steps=8, mu=[0.5, -6.0],
        field=dict(E0=0.2, omega=0.9, phase=0.1, axis=0),
        init=dict(alpha=0.6, center=[0.2, -0.3]),
        iters=4, tol=1e-8, face_nodes=[4, 6], quad_nodes=16,
    )
    t3 = dict(t2, name="tiny-2d-tise", mode="tise", mu=[6.0, 0.0],
              dt=0.05, n_steps=10,
              field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0))
    return [copy.deepcopy(t) for t in (t1, t2, t3)]


def slater_configs():
    """Small workloads in the Slater-like antisymmetric Gaussian basis of
    Section 2 (eq. (LSD)): two electrons in one dimension each on a
    decomposition symmetric under the exchange of the two coordinates (3 x 3
    subdomains of equal intervals, 4 Gaussians per interval: 16 functions
    off the diagonal, 6 on it), started from the antisymmetrised product of
    two Gaussians; real and imaginary time."""
    t1 = dict(
        name="tiny-slater", mode="tdse", n_elec=2, dim=1, basis="slater",
        L=[3, 3], box_lo=[-6.0, -6.0], box_hi=[6.0, 6.0], overlap=[0.8, 0.8],
        nbasis=[4, 4], width=None, width_ratio=0.7,
        nuclei=[[-0.7], [0.9]], charges=[1.0, 0.8], eps_en=1.0, eps_ee=0.9,
        dt=0.01, n_steps=8, mu=[0.5, -6.0],
        field=dict(E0=0.2, omega=0.9, phase=0.1, axis=0),
        init=dict(alpha=0.6, center=[-0.8, 0.9]),
        iters=4, tol=1e-8, face_nodes=[4, 6], quad_nodes=16,
    )
    t2 = dict(t1, name="tiny-slater-tise", mode="tise", mu=[6.0, 0.0], dt=0.05, n_steps=10,
              field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0))
    return [copy.deepcopy(t) for t in (t1, t2)]


def lsd_configs():
    """Small workloads in the local Slater determinant basis of Section 3:
    the tiny Slater workloads' decomposition (3 x 3 equal intervals on
    [-6, 6]^2, 6 Gaussians per interval) with 4 local orbitals per interval
    (16 determinants off the diagonal, 6 on it), a barrier of half-width 2.8
    about each interval's centre (the box's half-width is 2.4), transition
    width 0.6, height 30, and the mollifier of order 4 (sigma = 315/256, as
    in the paper's determinant tests) of width 0.3; real and imaginary time.
    tiny-lsd-all keeps all 6 orbitals: the same function space as the
    Slater-like basis of the same Gaussians.  tiny-lsd-aug and
    tiny-lsd-aug-tise take 3 orbitals augmented (Section 3.3) by the first
    and last Gaussian of each interval (5 functions: 25 determinants off the
    diagonal, 10 on it); tiny-lsd-aug-all 4 orbitals and the same 2
    Gaussians, the Slater-like basis's space again."""
    lsd = dict(orbitals=4, barrier=2.8, barrier_width=0.6, v_inf=30.0, moll_eps=0.3,
               moll_order=4)
    t1 = dict(slater_configs()[0], name="tiny-lsd", basis="lsd", nbasis=[6, 6], lsd=lsd)
    t2 = dict(slater_configs()[1], name="tiny-lsd-tise", basis="lsd", nbasis=[6, 6], lsd=lsd)
    t3 = dict(t1, name="tiny-lsd-all", lsd=dict(lsd, orbitals=6))
    t4 = dict(t1, name="tiny-lsd-aug", lsd=dict(lsd, orbitals=3, augment=1))
    t5 = dict(t2, name="tiny-lsd-aug-tise", lsd=dict(lsd, orbitals=3, augment=1))
    t6 = dict(t1, name="tiny-lsd-aug-all", lsd=dict(lsd, orbitals=4, augment=1))
    return [copy.deepcopy(t) for t in (t1, t2, t3, t4, t5, t6)]


def lo_configs():
    """Small workloads in the local orbital basis of one electron in two
    dimensions (Section 3 with d = 2): 2 x 2 boxes of [-6, 6]^2 (overlap
    1.0), 5 x 5 Gaussians per box (25), 8 orbitals per box, one nucleus of
    charge 1 at (0.3, -0.2) (the SWR Hamiltonian keeps its soft-Coulomb
    attraction, eps_en 0.5), a barrier of half-width 3.6 about each box's
    centre (the boxes' half-width is 3.25), transition width 0.6, height 30,
    the order-4 mollifier of radius 0.3; real time (complex Robin
    constant, sine field) and imaginary time (real Robin constant).
    tiny-lo-all keeps all 25 orbitals: the Gaussian basis's space."""
    lo = dict(orbitals=8, barrier=3.6, barrier_width=0.6, v_inf=30.0, moll_eps=0.3,
              moll_order=4)
    t1 = dict(
        name="tiny-lo", mode="tdse", n_elec=1, dim=2, basis="lo",
        L=[2, 2], box_lo=[-6.0, -6.0], box_hi=[6.0, 6.0], overlap=[1.0, 1.0],
        nbasis=[5, 5], width=None, width_ratio=0.8,
        nuclei=[[0.3, -0.2]], charges=[1.0], eps_en=0.5, eps_ee=0.5,
        dt=0.02, n_steps=10, mu=[0.0, -4.0],
        field=dict(E0=0.2, omega=0.9, phase=0.1, axis=0),
        init=dict(alpha=0.5, center=[0.4, -0.3]),
        iters=4, tol=1e-8, face_nodes=[4, 6], quad_nodes=16, lo=lo,
    )
    t2 = dict(t1, name="tiny-lo-tise", mode="tise", mu=[6.0, 0.0], dt=0.05,
              field=dict(E0=0.0, omega=0.0, phase=0.0, axis=0))
    t3 = dict(t1, name="tiny-lo-all", lo=dict(lo, orbitals=25))
    return [copy.deepcopy(t) for t in (t1, t2, t3)]


def random_small_configs(n, seed=4021):
    """Seeded small real-time configurations for broad parity checks: one
    electron in one or two dimensions or two electrons in one, 1 to 3
    subdomains per dimension (one subdomain included), 2 to 6 Gaussians per
    dimension (per subdomain in one dimension), 1 to 33 steps, a complex
    Robin constant of either sign of Im mu, and a sine or (two coordinates)
    circular field; each with a pipeline depth to run it at."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        n_elec, dim = [(1, 1), (2, 1), (1, 2)][q % 3]
        D = n_elec * dim
        L = [int(rng.integers(1, 4)) for _ in range(D)]
        lo = [float(-rng.uniform(5.0, 8.0)) for _ in range(D)]
        hi = [float(rng.uniform(5.0, 8.0)) for _ in range(D)]
        overlap = [float(rng.uniform(0.3, 0.9)) if L[k] > 1 else 0.0 for k in range(D)]
        if D == 1 and L[0] > 1:
            nbasis = [[int(rng.integers(2, 7))] for _ in range(L[0])]
        else:
            nbasis = [int(rng.integers(2, 7)) for _ in range(D)]
        n_nuc = int(rng.integers(0, 3))
        nuclei = [[float(rng.uniform(-1.5, 1.5)) for _ in range(dim)] for _ in range(n_nuc)]
        charges = [float(rng.uniform(0.5, 1.0)) for _ in range(n_nuc)]
        mu = [float(rng.uniform(-0.5, 0.5)), float(rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 8.0))]
        if D >= 2 and q % 2 == 0:
            field = dict(shape="circular", E0=float(rng.uniform(0.1, 0.5)),
                         omega=float(rng.uniform(0.5, 4.0)), phase=float(rng.uniform(0, 6.28)),
                         nu=float(rng.uniform(0.0, 5.0)), center=float(rng.uniform(0.0, 0.2)),
                         coords=[[0], [1]], axis=0)
        else:
            field = dict(E0=float(rng.uniform(0.0, 0.3)), omega=float(rng.uniform(0.5, 2.0)),
                         phase=float(rng.uniform(0, 6.28)), axis=int(rng.integers(0, dim)))
        out.append(dict(
            name=f"random-{q}", mode="tdse", n_elec=n_elec, dim=dim, L=L, box_lo=lo, box_hi=hi,
            overlap=overlap, nbasis=nbasis, width=None, width_ratio=float(rng.uniform(0.6, 0.9)),
            nuclei=nuclei, charges=charges, eps_en=float(rng.uniform(0.5, 1.2)),
            eps_ee=float(rng.uniform(0.5, 1.2)), dt=float(rng.uniform(0.005, 0.03)),
            n_steps=int(rng.choice([1, 2, 7, 16, 33])), mu=mu, field=field,
            init=dict(alpha=float(rng.uniform(0.4, 1.0)),
                      center=[float(rng.uniform(-0.5, 0.5)) for _ in range(D)]),
            iters=3, tol=1e-8, face_nodes=[int(rng.integers(2, 6)), int(rng.integers(2, 8))],
            quad_nodes=12, depth=int(rng.choice([1, 2, 4]))))
    return out
