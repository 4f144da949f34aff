"""The two headline windows at full size, run exactly as the benchmark runs
them, against stored oracle results (tests/golden/make_headline_fixtures.py,
written by the CPU oracle only).

Real time: the two-electron window (64 subdomains of 8 x 8 Gaussians, 1000
Crank-Nicolson steps, 20 Schwarz iterations) after the library's autotuner
has chosen the schedule, launched as a captured HIP graph and then replayed
from it; every subdomain's state at the last step of iterate 20 within 1e-10
relative A-norm (all subdomains together) and Res(1..20) within 1e-7
relative.  Imaginary time: the benchmark's window of 20 iterations x 400
normalised steps; energy within 1e-10 relative, states at the last step
within 1e-10 relative A-norm, residuals within 1e-7."""
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _cvec(v):
    a = np.asarray(v, dtype=np.float64)
    return a[:, 0] + 1j * a[:, 1] if a.ndim == 2 else a


def _gram(cfg):
    """Per-subdomain Gram matrices from the oracle's closed form."""
    from oracle import assemble, gauss1d
    from oracle.geometry import Decomposition
    dec = Decomposition(cfg)
    return [assemble.kron_all([gauss1d.overlap(sub.alpha[k], sub.delta[k], sub.lo[k], sub.hi[k])
                               for k in range(len(sub.alpha))]) for sub in dec.subs]


def _a_norm_rel(A, got, ref):
    num = den = 0.0
    for Ai, g, r in zip(A, got, ref):
        d = g - r
        num += float(np.real(np.conj(d) @ Ai @ d))
        den += float(np.real(np.conj(r) @ Ai @ r))
    return np.sqrt(num / den)


def _final(s):
    return [h[-1].detach().cpu().numpy() for h in s.split_history(s.history())]


def test_headline_real_time_window_autotuned_graph_replay():
    import torch
    from paper_1710_02401_amd import Solver
    ref = _golden("c2_window.json")
    cfg = workloads.get_config("c2-2e-1d")
    iters = ref["iterations"]
    print(f"[gpu] headline window {cfg['name']}, {iters} iterations, autotuned", flush=True)
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    torch.cuda.synchronize()
    c0 = s.initial().clone()
    s.autotune(k_iters=iters)
    A = _gram(cfg)
    want = [_cvec(ref["final"][str(i)]) for i in range(len(A))]
    for rep in range(2):  # capture, then replay
        s.set_initial(c0)
        st = s.run(k_max=iters, tol=-1.0, graph=True)
        torch.cuda.synchronize()
        assert st["iters"] == iters
        for a, b in zip(st["res"], ref["residuals"]):
            assert a == pytest.approx(b, rel=1e-7)
        err = _a_norm_rel(A, _final(s), want)
        print(f"[gpu] window {rep}: depth {int(s.info.depth_run)}, tile {int(s.info.tx_tile)}, "
              f"relative A-norm {err:.2e}", flush=True)
        assert err <= 1e-10


def test_headline_imaginary_time_window():
    import torch
    from paper_1710_02401_amd import Solver
    ref = _golden("c2_tise_window.json")
    cfg = workloads.get_config("c2-2e-1d-tise")
    iters = ref["iterations"]
    print(f"[gpu] headline window {cfg['name']}, {iters} iterations", flush=True)
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    s.run(k_max=2, tol=-1.0)
    s.set_initial()
    st = s.run(k_max=iters, tol=-1.0, timing=True)
    torch.cuda.synchronize()
    assert st["iters"] == iters
    assert st["energy"] == pytest.approx(ref["energies"][-1], rel=1e-10)
    for a, b in zip(st["res"], ref["residuals"]):
        assert a == pytest.approx(b, rel=1e-7)
    A = _gram(cfg)
    got = [np.real(v) for v in _final(s)]
    want = [np.asarray(ref["final"][str(i)]) for i in range(len(A))]
    err = _a_norm_rel(A, got, want)
    print(f"[gpu] imaginary-time states: relative A-norm {err:.2e}", flush=True)
    assert err <= 1e-10
