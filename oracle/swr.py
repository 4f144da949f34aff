"""Schwarz Waveform Relaxation for the TDSE: local Crank-Nicolson solves,
Robin transmission with averaging over multi-overlap zones, residual.

Paper passages followed:
  * Section 4.1, eq. (S1): iteration k solves every local TDSE on
    Omega_i x (0, T) with B psi_i^(k) = B psi_j^(k-1) on the interfaces
    (every subdomain uses the previous iterate of its neighbours), starting
    from a given psi^(0).
  * Section 4.1, multi-subdomain zones: the data imposed at a point is the
    average (1/Card O) sum_{j in O} B_{i;j} psi_j^(k-1).
  * Section 4.1, eq. (RTC): Robin operator B = d_n + mu with n the outward
    normal of the receiving subdomain, mu interface independent.
  * Section 4.4 step 2 (real time): Crank-Nicolson
      (A + i dt/2 H~ + i dt/2 T^{n+1}) c^{n+1} = (A - i dt/2 H~ - i dt/2 T^n) c^n
    extended with the Robin data term of the weak form, (i tau/2)(f^n + f^{n+1})
    with tau = dt/2 (reading), T^n = E(t_n) Q.
  * Section 5, eq. (residueRT): Res(k) = (int_0^T sum_i int_{bdry Omega_i}
    |psi_i^(k) - psi_i^(k-1)|^2)^{1/2}, here with the trapezoid rule in
    time and the face Gauss-Legendre rule in space.
  * Faces on the global boundary: Robin operator with zero data (absorbing;
    the paper imposes absorbing conditions at the global boundary, Section
    3.2) -- a reading.

Pinned by: Crank-Nicolson invariants (A-norm conservation for Hermitian
H~, time reversal -- with the two-component field too -- and second order),
free Gaussian packet spreading, Ehrenfest drift in a uniform field and, per
coordinate, in the circular pulse of Section 5 Test 3, converged SWR
against a brute-force finite-difference solution of the same boundary value
problem in one dimension and, on a 2 x 2 decomposition with corner zones
of three covering neighbours, in two (tests/test_oracle_swr_md.py), and
the residual Res(k) against its closed form for basis functions switched on
with a known time profile (same file).
"""
import numpy as np

from . import assemble, gauss1d, lo2, slater
from .geometry import Decomposition


def field(cfg, t):
    """E(t) = E0 sin(omega t + phase) (dipole approximation, eq. (LG)): one
    value per time.  The circular pulse of Section 5, Test 3, has two
    components, E0 cos(omega t + phase) g(t) and E0 sin(omega t + phase) g(t)
    with the envelope g(t) = exp(-nu (t - center)^2) (the test centres it at
    T/2): an array [n][2]."""
    f = cfg["field"]
    t = np.asarray(t, dtype=np.float64)
    if f.get("shape", "sine") == "circular":
        g = np.exp(-f["nu"] * (t - f["center"]) ** 2)
        arg = f["omega"] * t + f["phase"]
        return np.stack([f["E0"] * np.cos(arg) * g, f["E0"] * np.sin(arg) * g], axis=-1)
    return f["E0"] * np.sin(f["omega"] * t + f["phase"])


def field_term(sy, En):
    """T(t_n) = sum over components of E_c(t_n) Q_c (eq. (Q), the dipole
    matrix of each component's coordinates)."""
    if np.ndim(En) == 0:
        return En * sy.Q
    return En[0] * sy.Q + En[1] * sy.Q2


def basis_values(s, pts):
    """v_l(y) for all points (rows) and local basis functions (columns)."""
    if slater.is_slater(s):
        return basis_values(slater.extended(s), pts) @ slater.transform(s).T
    if lo2.is_lo2(s):
        return basis_values(lo2.gaussians(s), pts) @ lo2.transform(s).T
    out = np.ones((pts.shape[0], 1))
    for k in range(s.D):
        vk = gauss1d.values(s.alpha[k], s.delta[k], pts[:, k])
        out = (out[:, :, None] * vk[:, None, :]).reshape(pts.shape[0], -1)
    return out


def basis_derivative(s, pts, kd):
    """d v_l / d x_kd at the points."""
    if slater.is_slater(s):
        return basis_derivative(slater.extended(s), pts, kd) @ slater.transform(s).T
    if lo2.is_lo2(s):
        return basis_derivative(lo2.gaussians(s), pts, kd) @ lo2.transform(s).T
    out = np.ones((pts.shape[0], 1))
    for k in range(s.D):
        if k == kd:
            vk = gauss1d.derivatives(s.alpha[k], s.delta[k], pts[:, k])
        else:
            vk = gauss1d.values(s.alpha[k], s.delta[k], pts[:, k])
        out = (out[:, :, None] * vk[:, None, :]).reshape(pts.shape[0], -1)
    return out


class _LazySystems:
    """Local systems assembled on first use (a sampled check of a large
    decomposition assembles only the subdomains it touches)."""

    def __init__(self, dec):
        self.dec = dec
        self.cache = {}

    def __len__(self):
        return len(self.dec.subs)

    def __iter__(self):
        return (self[i] for i in range(len(self)))

    def __getitem__(self, i):
        if i not in self.cache:
            self.cache[i] = assemble.LocalSystem(self.dec, self.dec.subs[i])
        return self.cache[i]


class Problem:
    """Decomposition plus every subdomain's local matrices."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.dec = Decomposition(cfg)
        self.sys = _LazySystems(self.dec)
        self.mu = complex(cfg["mu"][0], cfg["mu"][1])
        self.dt = float(cfg["dt"])
        self.n_T = int(cfg["n_steps"])

    @property
    def n_sub(self):
        return self.dec.n_sub

    def neighbours(self, i):
        out = set()
        for F in self.dec.subs[i].faces:
            if F.is_global:
                continue
            for c in F.cover:
                out.update(int(j) for j in c)
        return sorted(out)

    def initial_coeff(self, i):
        s = self.dec.subs[i]
        return assemble.project_initial(self.dec, s, self.sys[s.lin].A).astype(np.complex128)

    def initial_coeffs(self):
        return [self.initial_coeff(s.lin) for s in self.dec.subs]

    def times(self, t0=0.0):
        return t0 + self.dt * np.arange(self.n_T + 1)


def local_cn(sy, c0, f, E, dt):
    """Crank-Nicolson over one window for one subdomain.

    c0: (K,) initial coefficients; f: (n_T+1, K) Robin data vectors;
    E: field at the time nodes, (n_T+1,) or (n_T+1, 2) for a two-component
    field.  Returns (n_T+1, K) history."""
    tau = 0.5 * dt
    n_T = len(E) - 1
    hist = np.empty((n_T + 1, sy.K), dtype=np.complex128)
    hist[0] = c0
    for n in range(n_T):
        M = sy.A + 1j * tau * (sy.Htilde + field_term(sy, E[n + 1]))
        R = sy.A - 1j * tau * (sy.Htilde + field_term(sy, E[n]))
        rhs = R @ hist[n] + 0.5j * tau * (f[n] + f[n + 1])
        hist[n + 1] = np.linalg.solve(M, rhs)
    return hist


def robin_values(prob, j, pts, kd, sign):
    """(sign * d/dx_kd + mu) v_l^j at the points: the Robin operator of the
    receiving face applied to the basis of the sending subdomain j."""
    s = prob.dec.subs[j]
    return sign * basis_derivative(s, pts, kd) + prob.mu * basis_values(s, pts)


def face_data(prob, i, hist_of):
    """Averaged Robin data g(y, t_n) on every face of subdomain i, from the
    histories of the covering subdomains.  Returns a list (one entry per
    face) of (n_T+1, n_y) arrays; global faces get zero data."""
    s = prob.dec.subs[i]
    out = []
    for F in s.faces:
        n_y = F.nodes.shape[0]
        g = np.zeros((prob.n_T + 1, n_y), dtype=np.complex128)
        if not F.is_global:
            counts = np.array([len(c) for c in F.cover], dtype=np.float64)
            sources = sorted({int(j) for c in F.cover for j in c})
            for j in sources:
                mask = np.array([j in c for c in F.cover])
                rows = np.nonzero(mask)[0]
                b = robin_values(prob, j, F.nodes[rows], F.k, F.normal_sign)
                g[:, rows] += (hist_of(j) @ b.T) / counts[rows]
        out.append(g)
    return out


def forcing_from_face_data(prob, i, gfaces):
    """f_i^n[l] = sum over faces and nodes of w_y g(y, t_n) v_l^i(y)."""
    s = prob.dec.subs[i]
    f = np.zeros((prob.n_T + 1, s.K), dtype=np.complex128)
    for F, g in zip(s.faces, gfaces):
        f += (g * F.weights[None, :]) @ basis_values(s, F.nodes)
    return f


def forcing(prob, i, hist_of):
    return forcing_from_face_data(prob, i, face_data(prob, i, hist_of))


def transmit(prob, hists):
    return [forcing(prob, i, lambda j: hists[j]) for i in range(prob.n_sub)]


def trapezoid_weights(n_T, dt):
    w = np.full(n_T + 1, dt)
    w[0] *= 0.5
    w[-1] *= 0.5
    return w


def residual_terms(prob, hists_new, hists_old, subs=None):
    """Per-subdomain contributions to Res(k)^2 (eq. (residueRT))."""
    wt = trapezoid_weights(prob.n_T, prob.dt)
    subs = range(prob.n_sub) if subs is None else subs
    out = {}
    for i in subs:
        s = prob.dec.subs[i]
        acc = 0.0
        d = hists_new[i] - hists_old[i]
        for F in s.faces:
            tr = d @ basis_values(s, F.nodes).T          # (n_T+1, n_y)
            acc += float(np.sum(wt[:, None] * F.weights[None, :] * np.abs(tr) ** 2))
        out[i] = acc
    return out


def residual(prob, hists_new, hists_old):
    return float(np.sqrt(sum(residual_terms(prob, hists_new, hists_old).values())))


def constant_history(prob, c0):
    return [np.repeat(c[None, :], prob.n_T + 1, axis=0) for c in c0]


def warm_forcing(prob, c0, warm="plain", g_faces=None):
    """Robin data for iteration k = 1 from the given psi^(0).

    plain: psi^(0)(t) = the window's initial state for every t;
    zero:  no data;
    given: face data g (list per subdomain of per-face (n_T+1, n_y))."""
    if warm == "plain":
        return transmit(prob, constant_history(prob, c0))
    if warm == "zero":
        return [np.zeros((prob.n_T + 1, s.K), dtype=np.complex128) for s in prob.dec.subs]
    if warm == "given":
        return [forcing_from_face_data(prob, i, g_faces[i]) for i in range(prob.n_sub)]
    raise ValueError(warm)


def swr_window(prob, c0, t0=0.0, iters=None, tol=None, warm="plain", g_faces=None):
    """One time window of SWR.  Returns (histories, residuals).

    Res(k) compares iterate k with iterate k-1; iterate 0 is the window's
    initial state held constant.  With tol, stops at the first k >= 2 with
    Res(k) <= tol."""
    iters = prob.cfg["iters"] if iters is None else iters
    E = field(prob.cfg, prob.times(t0))
    f = warm_forcing(prob, c0, warm, g_faces)
    prev = constant_history(prob, c0)
    res = []
    hists = prev
    for k in range(1, iters + 1):
        hists = [local_cn(prob.sys[i], c0[i], f[i], E, prob.dt) for i in range(prob.n_sub)]
        res.append(residual(prob, hists, prev))
        f = transmit(prob, hists)
        prev = hists
        if tol is not None and k >= 2 and res[-1] <= tol:
            break
    return hists, res


def swr_sampled(prob, c0, targets, k, t0=0.0):
    """Iterate k (plain warm start) of the subdomains in `targets` only,
    computing just the dependency cone (neighbours of neighbours ...).
    c0 may be a list or a mapping holding at least the cone's subdomains.
    Returns dict i -> (n_T+1, K) history."""
    E = field(prob.cfg, prob.times(t0))

    def const(j):
        return np.repeat(c0[j][None, :], prob.n_T + 1, axis=0)
    need = [set(targets)]
    for _ in range(k - 1):
        nxt = set()
        for i in need[-1]:
            nxt.update(prob.neighbours(i))
        need.append(nxt)
    need = need[::-1]        # need[0] = set solved at iteration 1
    prev = {}
    for it in range(k):
        cur = {}
        for i in sorted(need[it]):
            if it == 0:
                fi = forcing(prob, i, const)
            else:
                fi = forcing(prob, i, lambda j: prev[j])
            cur[i] = local_cn(prob.sys[i], c0[i], fi, E, prob.dt)
        prev = cur
    return prev


def a_norm_distance(prob, hA, hB, subs=None, step=-1):
    """Relative L2 distance in function space at one time node:
    sqrt(sum_i dc^H A_i dc / sum_i c^H A_i c)."""
    subs = range(prob.n_sub) if subs is None else subs
    num = den = 0.0
    for i in subs:
        A = prob.sys[i].A
        a = hA[i][step]
        d = a - hB[i][step]
        num += float(np.real(np.conj(d) @ A @ d))
        den += float(np.real(np.conj(a) @ A @ a))
    return float(np.sqrt(num / den))
