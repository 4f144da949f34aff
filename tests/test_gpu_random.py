"""Seeded small real-time configurations of every shape the narrow path
takes (one electron in one or two dimensions, two electrons in one; one to
three subdomains per dimension; uneven bases in one dimension; 1 to 33
steps; either sign of Im mu, so both the series and the per-step inverses;
sine and circular fields; pipeline depths 1, 2 and 4) against the CPU
oracle through the C ABI: every step of every subdomain and the residuals
of 3 Schwarz iterations."""
import numpy as np
import pytest

import workloads
from oracle import swr as o_swr

pytestmark = pytest.mark.gpu

CASES = workloads.random_small_configs(10)
CASES.append(dict(CASES[1], name="random-1-one-step", n_steps=1))


@pytest.mark.parametrize("cfg", CASES, ids=[c["name"] for c in CASES])
def test_random_small_configuration_matches_oracle(cfg):
    import torch
    from paper_1710_02401_amd import Solver
    print(f"[gpu] {cfg['name']}: D={cfg['n_elec'] * cfg['dim']} L={cfg['L']} "
          f"nbasis={cfg['nbasis']} n_steps={cfg['n_steps']} depth={cfg['depth']}", flush=True)
    iters = 3
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    st = s.run(k_max=iters, tol=-1.0, depth=cfg["depth"])
    torch.cuda.synchronize()
    assert st["iters"] == iters
    h_g = [h.cpu().numpy() for h in s.split_history(s.history())]
    prob = o_swr.Problem(cfg)
    h_o, res_o = o_swr.swr_window(prob, prob.initial_coeffs(), iters=iters)
    num = den = 0.0
    for i in range(prob.n_sub):
        A = prob.sys[i].A
        d = h_g[i] - h_o[i]
        num = num + np.real(np.einsum("nk,kl,nl->n", np.conj(d), A, d))
        den = den + np.real(np.einsum("nk,kl,nl->n", np.conj(h_o[i]), A, h_o[i]))
    err = float(np.max(np.sqrt(num / den)))
    print(f"[gpu] {cfg['name']}: rel A-norm {err:.3e}, terms {s.factor_terms() + 1}", flush=True)
    assert err <= 1e-10
    assert np.allclose(st["res"][:iters], res_o, rtol=1e-7, atol=1e-12)
    s.close()
