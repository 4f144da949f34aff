"""Wide-basis path (one electron in one dimension, up to 256 Gaussians per
subdomain) against the CPU oracle through the C ABI: the batched uneven
workload at a size the oracle runs whole, the same windows on the narrow
path, and the full-size batched workload on sampled subdomains."""
import numpy as np
import pytest

import workloads
from oracle import swr as o_swr

pytestmark = pytest.mark.gpu


def _cfg(name):
    tiny = {c["name"]: c for c in workloads.tiny_configs()}
    if name == "tiny-1d-weak-field":  # a field the wide path's six terms cover
        return dict(tiny["tiny-1d"], name=name, field=dict(tiny["tiny-1d"]["field"], E0=0.03))
    return tiny.get(name) or workloads.get_config(name)


def _solver(cfg):
    import torch
    from paper_1710_02401_amd import Solver
    print(f"[gpu] solver {cfg['name']} factor={cfg.get('factor', 'auto')}", flush=True)
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    torch.cuda.synchronize()
    return s


def _np(t):
    return t.detach().cpu().numpy()


def _a_norm_rel(prob, got, ref, items):
    """max over time steps of sqrt(sum_i dc^H A dc / sum_i c^H A c)."""
    num = den = 0.0
    for i in items:
        A = prob.sys[i].A
        d = got[i] - ref[i]
        num = num + np.real(np.einsum("nk,kl,nl->n", np.conj(d), A, d))
        den = den + np.real(np.einsum("nk,kl,nl->n", np.conj(ref[i]), A, ref[i]))
    return float(np.max(np.sqrt(num / den)))


def test_wide_bases_match_the_oracle():
    """Two geometries x 8 subdomains with 33..256 Gaussians, 200 steps (two
    series chunks), 3 Schwarz iterations: every step of every subdomain
    within 1e-10 (A-norm), and the residuals."""
    cfg = workloads.get_config("c3-wide")
    s = _solver(cfg)
    assert s.info.wide == 1 and s.info.K_max == 256
    iters = cfg["iters"]
    st = s.run(k_max=iters, tol=0.0)
    assert st["iters"] == iters and 1 <= s.factor_terms() + 1 <= 6
    hist = [_np(h) for h in s.split_history(s.history())]
    n_sub = len(cfg["nbasis"])
    res2 = np.zeros(iters)
    for g, nuc in enumerate(cfg["geometries"]):
        prob = o_swr.Problem(dict(cfg, nuclei=nuc, geometries=None))
        h_o, res_o = o_swr.swr_window(prob, prob.initial_coeffs(), iters=iters)
        got = hist[g * n_sub:(g + 1) * n_sub]
        err = _a_norm_rel(prob, got, h_o, range(n_sub))
        print(f"[gpu] c3-wide geometry {g}: rel A-norm {err:.3e}", flush=True)
        assert err <= 1e-10, g
        res2 += np.array(res_o) ** 2
    assert np.allclose(st["res"], np.sqrt(res2), rtol=1e-8, atol=1e-14)


@pytest.mark.parametrize("name", ["tiny-1d-weak-field", "c1-1e-1d", "c3-mini"])
def test_wide_path_equals_narrow_path(name):
    """The wide path asked for at K <= 64 against the narrow path (stored
    inverses) and the oracle on the first geometry: both within 1e-10 of the
    oracle, and the wide path no further from it than the narrow one."""
    cfg = _cfg(name)
    iters = 4
    ref = _solver(cfg)
    st_r = ref.run(k_max=iters, tol=0.0)
    h_r = [_np(h) for h in ref.split_history(ref.history())]
    s = _solver(dict(cfg, factor="wide"))
    assert s.info.wide == 1 and ref.info.wide == 0
    st = s.run(k_max=iters, tol=0.0)
    h = [_np(x) for x in s.split_history(s.history())]
    prob = o_swr.Problem(dict(cfg, nuclei=cfg.get("geometries", [cfg["nuclei"]])[0],
                              geometries=None))
    h_o, _ = o_swr.swr_window(prob, prob.initial_coeffs(), iters=iters)
    n_sub = prob.n_sub
    e_wide = _a_norm_rel(prob, h[:n_sub], h_o, range(n_sub))
    e_narrow = _a_norm_rel(prob, h_r[:n_sub], h_o, range(n_sub))
    print(f"[gpu] {name}: rel A-norm to the oracle: wide {e_wide:.3e}, narrow {e_narrow:.3e}",
          flush=True)
    assert e_wide <= 1e-10 and e_narrow <= 1e-10
    assert e_wide <= max(2.0 * e_narrow, 1e-12)
    assert np.allclose(st["res"], st_r["res"], rtol=1e-8, atol=1e-14)


def test_wide_path_refuses_fields_beyond_its_series():
    """The small one-dimensional case's own field (E0 = 0.3, omega = 1.1)
    needs seven series terms per 128-step chunk: the narrow path inverts
    every step instead, the wide path has no such fallback and says so."""
    from paper_1710_02401_amd.swr import SWRError
    cfg = dict(_cfg("tiny-1d"), factor="wide")
    s = _solver(cfg)
    with pytest.raises(SWRError) as e:
        s.run(k_max=2, tol=0.0)
    assert e.value.code == -2 and "more than 6 terms" in str(e.value)


def test_full_size_batched_workload_sampled_subdomains():
    """Full batched workload (64 geometries x 256 subdomains, K = 32..256,
    200 steps): iterate 2 of sampled subdomains of three geometries -- the
    largest and smallest bases, and a geometry's first and last subdomain --
    computed by the oracle from their dependency cone only."""
    import torch
    cfg = workloads.get_config("c3-1e-1d-batched")
    s = _solver(cfg)
    assert s.info.wide == 1 and s.info.n_items == 64 * 256
    s.factor(0.0)
    for _ in range(2):
        s.sweep()
        s.transmit()
    torch.cuda.synchronize()
    parts = s.split_history(s.history())
    n_sub = 256
    K = [nb[0] for nb in cfg["nbasis"]]
    big = K.index(max(K))
    # each item applies the terms its own box needs: fewer for the large
    # bases near the nuclei than for the outermost boxes
    terms = s.item_terms()
    assert terms.max() == s.factor_terms() + 1 and terms.min() >= 1
    assert terms[big] < terms[0] == terms.max()
    for g, subs in ((0, [big, 0]), (37, [big + 1, 255]), (63, [K.index(min(K)), big])):
        prob = o_swr.Problem(dict(cfg, nuclei=cfg["geometries"][g], geometries=None))
        cone = set(subs)
        for _ in range(2):
            cone |= {j for i in cone for j in prob.neighbours(i)}
        c0 = {j: prob.initial_coeff(j) for j in cone}
        ref = o_swr.swr_sampled(prob, c0, subs, 2)
        got = {i: _np(parts[g * n_sub + i]) for i in subs}
        err = _a_norm_rel(prob, got, ref, subs)
        print(f"[gpu] c3 full geometry {g} subdomains {subs}: rel A-norm {err:.3e}", flush=True)
        assert err <= 1e-10, (g, subs)


def test_full_geometry_of_the_batched_workload_residuals():
    """Every subdomain of geometry 0 of the batched workload (256 subdomains,
    K = 32..256), 6 Schwarz iterations: Res(k) against the oracle's sequence
    (tests/golden/batched_geometry0_residuals.json, written by
    make_batched_residuals.py from the oracle alone).  The sequence grows:
    plain SWR diverges on this decomposition (cores 0.156 wide, overlap
    0.031), and the GPU must follow it."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "batched_geometry0_residuals.json")) as f:
        gold = json.load(f)
    cfg = workloads.get_config("c3-1e-1d-batched")
    g0 = cfg["geometries"][0]
    s = _solver(dict(cfg, geometries=[g0], nuclei=g0))
    assert s.info.n_items == 256
    st = s.run(k_max=gold["iterations"], tol=0.0)
    print("[gpu] batched geometry 0 residuals", st["res"][:gold["iterations"]], flush=True)
    assert np.allclose(st["res"][:gold["iterations"]], gold["residuals"], rtol=1e-8, atol=0)


@pytest.mark.parametrize("K,n_steps", [(256, 37), (97, 130)])
def test_wide_single_subdomain(K, n_steps):
    """One subdomain (both faces global: no Robin data, absorbing Robin
    operator), the largest basis and a ragged one, a window shorter than one
    series chunk with a ragged transmission tile, and one spanning two
    chunks: the oracle's local Crank-Nicolson solve, and a residual of
    exactly zero from iteration 2 on (nothing is transmitted)."""
    base = workloads.get_config("c3-wide")
    g0 = base["geometries"][0]
    cfg = dict(base, name=f"wide-single-{K}", L=[1], nbasis=[[K]], geometries=[g0], nuclei=g0,
               n_steps=n_steps)
    s = _solver(cfg)
    assert s.info.wide == 1 and s.info.n_items == 1
    st = s.run(k_max=3, tol=-1.0)  # all three iterations (the residual reaches 0)
    assert st["iters"] == 3
    h = _np(s.split_history(s.history())[0])
    prob = o_swr.Problem(dict(cfg, geometries=None))
    h_o, res_o = o_swr.swr_window(prob, prob.initial_coeffs(), iters=3)
    err = _a_norm_rel(prob, [h], h_o, [0])
    print(f"[gpu] single subdomain K={K} n_steps={n_steps}: rel A-norm {err:.3e}", flush=True)
    assert err <= 1e-10
    assert st["res"][1] == 0.0 and st["res"][2] == 0.0
    # Res(1) is the change of boundary traces where the state is ~0: a small
    # difference, compared in absolute terms as the narrow tests do below 1e-9
    print(f"[gpu] Res(1) {st['res'][0]:.6e} oracle {res_o[0]:.6e}", flush=True)
    assert abs(st["res"][0] - res_o[0]) <= 1e-7 * res_o[0] + 1e-12


def test_wide_reconstruction_matches_oracle():
    """Reconstruction (Section 4.3) of iterate 1 at the last step of the
    window, second geometry of the wide workload, at seeded points covering
    the box (overlap zones included): the mean of the covering subdomains'
    expansions with 33..256 Gaussians each."""
    import torch
    from oracle import reconstruct as o_rec
    cfg = workloads.get_config("c3-wide")
    s = _solver(cfg)
    s.factor(0.0)
    s.sweep()
    s.transmit()
    g = 1
    prob = o_swr.Problem(dict(cfg, nuclei=cfg["geometries"][g], geometries=None))
    c0 = prob.initial_coeffs()
    pts = np.random.default_rng(11).uniform(-20.0, 20.0, size=(400, 1))
    step = cfg["n_steps"]
    got = _np(s.reconstruct(torch.from_numpy(pts), step, geom=g))
    E = o_swr.field(cfg, prob.times())
    f0 = o_swr.warm_forcing(prob, c0, "plain")
    h_o = [o_swr.local_cn(prob.sys[i], c0[i], f0[i], E, prob.dt) for i in range(prob.n_sub)]
    ref = o_rec.reconstruct(prob, [h[step] for h in h_o], pts)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"[gpu] wide reconstruction: max rel {err:.3e}", flush=True)
    assert err <= 1e-10


def test_wide_window_graph_replay_and_autotuned_schedule():
    """Batching on the wide path: the window (one iterate at a time) captured
    as a HIP graph and replayed, with the program's own eager work between
    the replays, gives the eager window's histories bit for bit and its
    residuals; the autotuner measures the three transmission tiles and both
    recurrence orders, and its choice changes no history bit (the residual
    partials are summed per tile, so residuals agree to rounding); a second
    handle of the same problem takes the choice from the tuning table."""
    import torch
    cfg = dict(_cfg("c3-mini"), factor="wide")
    s = _solver(cfg)
    c0 = s.initial().clone()
    eager = s.run(k_max=4, tol=-1.0)
    h_eager = s.history().clone()
    for rep in range(3):  # capture, then replays
        s.set_initial(c0)
        g = s.run(k_max=4, tol=-1.0, graph=True)
        torch.cuda.synchronize()
        assert g["res"] == eager["res"], rep
        assert torch.equal(s.history(), h_eager), rep
        s.set_initial(c0)
        s.run(k_max=2, tol=-1.0)  # eager work between the replays
    s.set_initial(c0)
    t = s.autotune(k_iters=2)
    print(f"[gpu] wide autotune {t}", flush=True)
    assert t["candidates"] == 6 and t["tx_tile"] in (8, 16, 32) and t["order"] in (0, 1)
    assert s.info.tx_tile == t["tx_tile"] and s.info.wide_order == t["order"]
    s.set_initial(c0)
    tuned = s.run(k_max=4, tol=-1.0, graph=True)
    assert torch.equal(s.history(), h_eager)
    assert np.allclose(tuned["res"], eager["res"], rtol=1e-12, atol=0)
    s2 = _solver(cfg)
    assert s2.info.tuned == 1
    assert (s2.info.tx_tile, s2.info.wide_order, s2.info.depth_run) == \
        (t["tx_tile"], t["order"], t["depth"])
    s2.set_initial(c0)
    s2.run(k_max=4, tol=-1.0)
    assert torch.equal(s2.history(), h_eager)


def test_tuning_table_persists_through_a_file(tmp_path):
    """With SWR_TUNING_FILE set, swr_autotune writes its choice there and a
    new process's handle of the same problem starts from it (two child
    processes, one after the other)."""
    import os
    import subprocess
    import sys
    path = tmp_path / "tuning.txt"
    env = dict(os.environ, SWR_TUNING_FILE=str(path))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    prog = (
        "import sys; sys.path.insert(0, %r)\n"
        "import workloads\n"
        "from paper_1710_02401_amd import Solver\n"
        "base = {c['name']: c for c in workloads.tiny_configs()}['tiny-1d']\n"
        "cfg = dict(base, field=dict(base['field'], E0=0.03), factor='wide')\n"
        "s = Solver(cfg); s.assemble(); s.set_initial()\n"
        "if sys.argv[1] == 'tune':\n"
        "    t = s.autotune(k_iters=2); print('TUNED', t['tx_tile'], t['order'], s.info.tuned)\n"
        "else:\n"
        "    print('READ', s.info.tx_tile, s.info.wide_order, s.info.tuned)\n" % root)
    out1 = subprocess.run([sys.executable, "-c", prog, "tune"], env=env, capture_output=True,
                          text=True, timeout=240)
    assert out1.returncode == 0, out1.stderr[-2000:]
    tuned = next(l for l in out1.stdout.splitlines() if l.startswith("TUNED")).split()
    text = path.read_text()
    assert "wide" in text and "\t" in text
    out2 = subprocess.run([sys.executable, "-c", prog, "read"], env=env, capture_output=True,
                          text=True, timeout=240)
    assert out2.returncode == 0, out2.stderr[-2000:]
    read = next(l for l in out2.stdout.splitlines() if l.startswith("READ")).split()
    assert read[1:3] == tuned[1:3] and read[3] == "1"
