"""SWR for the TISE: imaginary time (normalised gradient flow) with global
normalisation, and the local generalized eigenproblems.

Paper passages followed:
  * Section 1.3, eq. (e1bis): gradient flow d_t phi = -H_0 phi with
    normalisation at every t_n (the printed Lap phi - V phi is read as
    -H_0 phi = 1/2 Lap phi - V phi, consistent with eq. (SIT)).
  * Section 4.2, eq. (SIT): SWR in imaginary time; every local solution is
    divided by the norm of the global function at each time step.  The
    transmission condition holds on (t_n, t_{n+1}), i.e. before the
    normalisation at t_{n+1}, so the implicit step takes the neighbours'
    data at t_{n+1}^- (their un-normalised values nu_{n+1} c^{n+1}).  The
    printed norm of the sum of zero extensions double-counts overlaps; it
    is read as the norm of the reconstructed function, i.e.
    nu^2 = sum_i c~_i^T W_i c~_i with partition-of-unity weights.
  * Section 4.4 step 2 (imaginary time): implicit Euler
    (A + dt H~) c~^{n+1} = A c^n, extended with the Robin data term,
    + (dt/2) f^{n+1} (reading); step 4: c^{n+1} = c~^{n+1} / nu.
  * Energy: at a fixed point of the normalised implicit Euler map with
    neighbour data scaled alike, H~ c - f/2 = ((1/nu - 1)/dt) A c, so
    lambda = (1/nu - 1)/dt.
  * Local generalized eigenproblems H~_i x = lambda A_i x (real symmetric,
    A_i positive definite) by LAPACK (scipy.linalg.eigh), eigenvectors
    A-normalised with the largest-magnitude component made positive.
  * Reading for the stopping rule: a fixed number of imaginary steps per
    Schwarz iteration, so that traces exist at every step.
  * Without the normalisation (configuration key "unnormalized"), the same
    steps integrate the heat-type flow d_t phi = -H~ phi; with no potential
    that is Section 5 Test 1.b's heat equation phi_t = Lap phi in the time
    variable 2t.

Pinned by: harmonic-oscillator eigenvalues n + 1/2 (and the exact 1/2 of
a single Gaussian of exponent 1/2), monotone energy decrease of the
normalised flow on one domain (Section 1.3 proposition), agreement of
the SWR energy with a brute-force finite-difference ground state, and,
without normalisation, first-order convergence in the step to the heat
kernel's exact spreading of a Gaussian.
"""
import numpy as np
import scipy.linalg

from . import swr as swr_mod


def global_norm(prob, cs):
    return float(np.sqrt(sum(float(c @ prob.sys[i].W @ c) for i, c in enumerate(cs))))


def normalized(prob):
    return not prob.cfg.get("unnormalized", False)


def initial_state(prob):
    """Projected phi_0, divided by its global (partition-of-unity) norm
    (kept as projected without normalisation)."""
    c0 = [np.real(c) for c in prob.initial_coeffs()]
    nu = global_norm(prob, c0) if normalized(prob) else 1.0
    return [c / nu for c in c0]


def real_H(prob, i):
    H = prob.sys[i].Htilde
    if np.any(np.imag(H) != 0.0):
        raise ValueError("imaginary-time SWR needs a real Robin coefficient")
    return np.real(H)


def ngf_iteration(prob, c0, f):
    """One Schwarz iteration of imaginary time: all subdomains advance
    together because of the global normalisation.

    c0: list of (K,) real; f: list of (n_T+1, K) real Robin data vectors.
    Returns (histories, nus)."""
    dt = prob.dt
    n_T = prob.n_T
    hists = [np.empty((n_T + 1, prob.sys[i].K)) for i in range(prob.n_sub)]
    for i in range(prob.n_sub):
        hists[i][0] = c0[i]
    nus = np.ones(n_T + 1)
    Ms = [prob.sys[i].A + dt * real_H(prob, i) for i in range(prob.n_sub)]
    for n in range(n_T):
        ct = [np.linalg.solve(Ms[i], prob.sys[i].A @ hists[i][n] + 0.5 * dt * f[i][n + 1])
              for i in range(prob.n_sub)]
        nu = global_norm(prob, ct) if normalized(prob) else 1.0
        nus[n + 1] = nu
        for i in range(prob.n_sub):
            hists[i][n + 1] = ct[i] / nu
    return hists, nus


def energy_from_nu(nu, dt):
    return (1.0 / nu - 1.0) / dt


def swr_tise(prob, iters=None, tol=None, warm="plain"):
    """SWR-NGF.  Returns (histories, residuals, energies per iteration)."""
    iters = prob.cfg["iters"] if iters is None else iters
    c0 = initial_state(prob)
    const = swr_mod.constant_history(prob, c0)
    if warm == "plain":
        f = [np.real(x) for x in swr_mod.transmit(prob, const)]
    else:
        f = [np.zeros((prob.n_T + 1, prob.sys[i].K)) for i in range(prob.n_sub)]
    prev = const
    res, energies = [], []
    hists = prev
    for k in range(1, iters + 1):
        hists, nus = ngf_iteration(prob, c0, f)
        res.append(swr_mod.residual(prob, hists, prev))
        energies.append(energy_from_nu(nus[-1], prob.dt) if normalized(prob) else float("nan"))
        # the transmission condition holds on (t_n, t_{n+1}), before the
        # normalisation at t_{n+1}: neighbours send nu_{n+1} c^{n+1}
        pre = [h * nus[:, None] for h in hists]
        f = [np.real(x) for x in swr_mod.transmit(prob, pre)]
        prev = hists
        if tol is not None and k >= 2 and res[-1] <= tol:
            break
    return hists, res, energies


def local_eigen(prob, i):
    """Generalized eigenpairs of (H~_i, A_i): ascending eigenvalues and
    A-orthonormal eigenvectors, sign fixed by the largest component."""
    H = real_H(prob, i)
    lam, X = scipy.linalg.eigh(H, prob.sys[i].A)
    for c in range(X.shape[1]):
        r = int(np.argmax(np.abs(X[:, c])))
        if X[r, c] < 0:
            X[:, c] = -X[:, c]
    return lam, X
