"""GPU parity of the block path (tensor bases orthonormalised per dimension,
series steps of every iterate in flight on the matrix cores, averaged Robin
transmission in two and four dimensions) against the CPU oracle, through the
C ABI.  Bars as for the other paths: matrices within 1e-12 of their largest
entry, histories within 1e-10 relative A-norm at every step, residuals within
1e-7 relative."""
import numpy as np
import pytest

import workloads
from oracle import swr as o_swr

pytestmark = pytest.mark.gpu

TINY = {c["name"]: c for c in workloads.tiny_configs()}


def _cfg(name, **kw):
    base = dict(TINY[name]) if name in TINY else workloads.get_config(name)
    base.update(factor="block")
    base.update(kw)
    return base


def _solver(cfg):
    import torch
    from paper_1710_02401_amd import Solver
    print(f"[gpu] block solver {cfg['name']}", flush=True)
    s = Solver(cfg)
    assert s.info.block == 1
    s.assemble()
    s.set_initial()
    torch.cuda.synchronize()
    return s


def _np(t):
    return t.detach().cpu().numpy()


def _a_norm_rel(prob, gpu, ora, items=None):
    items = range(prob.n_sub) if items is None else items
    num = den = 0.0
    for i in items:
        A = prob.sys[i].A
        d = gpu[i] - ora[i]
        num = num + np.real(np.einsum("nk,kl,nl->n", np.conj(d), A, d))
        den = den + np.real(np.einsum("nk,kl,nl->n", np.conj(ora[i]), A, ora[i]))
    return float(np.max(np.sqrt(num / den)))


CASES = ["tiny-2d", "c5-mini", "c5-mini-1e"]


@pytest.mark.parametrize("name", CASES)
def test_block_matrices_and_initial_state(name):
    cfg = _cfg(name)
    s = _solver(cfg)
    prob = o_swr.Problem(cfg)
    for which, attr in [("A", "A"), ("Kin", "Kin"), ("V", "V"), ("Q", "Q"), ("B", "B")]:
        mats = s.matrix(which)
        for i in range(prob.n_sub):
            ref = getattr(prob.sys[i], attr)
            got = _np(mats[i])
            scale = max(np.max(np.abs(ref)), 1e-300)
            assert np.max(np.abs(got - ref)) <= 1e-12 * scale, (which, i)
    c0 = prob.initial_coeffs()
    got = [_np(v) for v in s.split_vector(s.initial())]
    assert _a_norm_rel(prob, [g[None] for g in got], [c[None] for c in c0]) <= 1e-12


@pytest.mark.parametrize("name,depth", [("tiny-2d", 0), ("c5-mini", 0), ("c5-mini-1e", 0),
                                        ("c5-mini", 1), ("c5-mini", 2)])
def test_block_window_matches_oracle(name, depth):
    cfg = _cfg(name)
    s = _solver(cfg)
    prob = o_swr.Problem(cfg)
    c0 = prob.initial_coeffs()
    iters = cfg["iters"]
    st = s.run(k_max=iters, tol=-1.0, depth=depth)
    h_o, res_o = o_swr.swr_window(prob, c0, iters=iters)
    h_g = [_np(h) for h in s.split_history(s.history())]
    assert st["iters"] == iters
    assert _a_norm_rel(prob, h_g, h_o) <= 1e-10
    for a, b in zip(st["res"], res_o):
        assert a == pytest.approx(b, rel=1e-7, abs=1e-12)


def test_block_sweep_by_sweep_matches_oracle():
    """swr_sweep / swr_transmit one iterate at a time (the previous iterate
    sends its data one step ahead inside each sweep)."""
    cfg = _cfg("c5-mini")
    s = _solver(cfg)
    prob = o_swr.Problem(cfg)
    c0 = prob.initial_coeffs()
    s.factor(0.0)
    s.warm_start()
    res = []
    for _ in range(cfg["iters"]):
        s.sweep()
        res.append(s.transmit())
    h_o, res_o = o_swr.swr_window(prob, c0, iters=cfg["iters"])
    h_g = [_np(h) for h in s.split_history(s.history())]
    assert _a_norm_rel(prob, h_g, h_o) <= 1e-10
    assert np.allclose(res, res_o, rtol=1e-7, atol=1e-12)


def test_block_several_anchors_and_a_second_window():
    """A fast field: several series anchors per window, launches whose
    iterates straddle anchors, then swr_advance_window and a second window
    from the first one's last state."""
    cfg = _cfg("tiny-2d", n_steps=40, field=dict(E0=0.5, omega=3.0, phase=0.2, axis=0), iters=4)
    s = _solver(cfg)
    prob = o_swr.Problem(cfg)
    c0 = prob.initial_coeffs()
    st = s.run(k_max=4, tol=-1.0, depth=3)
    h_o, res_o = o_swr.swr_window(prob, c0, iters=4)
    h_g = [_np(h) for h in s.split_history(s.history())]
    assert s.factor_terms() >= 0
    assert _a_norm_rel(prob, h_g, h_o) <= 1e-10
    assert np.allclose(st["res"][:4], res_o, rtol=1e-7, atol=1e-12)
    s.advance_window()
    t1 = cfg["n_steps"] * cfg["dt"]
    st2 = s.run(k_max=3, tol=-1.0, t0=t1)
    c1 = [h[-1] for h in h_o]
    h_o2, res_o2 = o_swr.swr_window(prob, c1, t0=t1, iters=3)
    h_g2 = [_np(h) for h in s.split_history(s.history())]
    assert _a_norm_rel(prob, h_g2, h_o2) <= 1e-10
    assert np.allclose(st2["res"][:3], res_o2, rtol=1e-7, atol=1e-12)


def test_block_reconstruction():
    cfg = _cfg("c5-mini")
    s = _solver(cfg)
    prob = o_swr.Problem(cfg)
    st = s.run(k_max=2, tol=-1.0)
    h_o, _ = o_swr.swr_window(prob, prob.initial_coeffs(), iters=2)
    rng = np.random.default_rng(3)
    lo = np.array(cfg["box_lo"]) + 0.3
    hi = np.array(cfg["box_hi"]) - 0.3
    pts = rng.uniform(lo, hi, size=(200, 4))
    from oracle import reconstruct as o_rec
    ref = o_rec.reconstruct(prob, [h[3] for h in h_o], pts)
    import torch
    got = _np(s.reconstruct(torch.from_numpy(pts), step=3))
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
