"""GPU parity of the learned warm start: the FP32 network kernels against
the FP64 oracle network, the interface-data plumbing against the oracle's
definitions, and the gain of the trained network over the plain guess.

Bars: network outputs and loss within 2e-5 of the oracle's scale, gradients
within 1e-4 of the largest gradient entry of each layer (FP32 sums of at
most a few thousand terms); Adam within 1e-6 relative; Robin data,
features, targets and interpolated guesses within 1e-9 relative (FP64, with
FP32 features and targets rounded once).
"""
import numpy as np
import pytest

import workloads
from oracle import learned as o_learned
from oracle import mlp as o_mlp
from oracle import swr as o_swr
from workloads import mlp_init

pytestmark = pytest.mark.gpu

TINY = {c["name"]: c for c in workloads.tiny_configs()}


def _np(t):
    return t.detach().cpu().numpy()


def _net(n_in, n_h, n_l, n_out, seed, max_batch=512):
    from paper_1710_02401_amd import Mlp
    p = mlp_init.initial_params(n_in, n_h, n_l, n_out, seed=seed)
    p = p + np.random.default_rng(seed + 1).normal(scale=0.05, size=p.size)
    p32 = p.astype(np.float32)
    return Mlp(n_in, n_h, n_l, n_out, p32, max_batch=max_batch), p32.astype(np.float64)


@pytest.mark.parametrize("sizes,batch", [((37, 48, 3, 70), 13), ((20, 64, 1, 8), 1),
                                         ((520, 256, 3, 4096), 64)])
def test_network_forward_loss_and_gradient(sizes, batch):
    import torch
    print(f"[gpu] mlp {sizes} batch {batch}", flush=True)
    net, p = _net(*sizes, seed=7)
    shapes = o_mlp.layer_shapes(*sizes)
    rng = np.random.default_rng(8)
    x = rng.normal(size=(batch, sizes[0])).astype(np.float32)
    t = rng.normal(size=(batch, sizes[3])).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    y = _np(net.forward(xd)).astype(np.float64)
    y_ref, _ = o_mlp.forward(p, x.astype(np.float64), shapes)
    assert np.max(np.abs(y - y_ref)) <= 2e-5 * np.max(np.abs(y_ref))
    loss, g = net.loss_grad(xd, td)
    loss_ref, g_ref = o_mlp.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64), shapes)
    assert float(loss.item()) == pytest.approx(loss_ref, rel=2e-5)
    g = _np(g).astype(np.float64)
    off = 0
    for o, i in shapes:
        for n in (o * i, o):
            ref = g_ref[off:off + n]
            assert np.max(np.abs(g[off:off + n] - ref)) <= 1e-4 * np.max(np.abs(ref)) + 1e-12
            off += n


def test_adam_matches_oracle():
    import torch
    net, p = _net(37, 48, 2, 70, seed=9)
    rng = np.random.default_rng(10)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 4):
        g = rng.normal(size=p.size).astype(np.float32)
        net.grad.copy_(torch.from_numpy(g))
        net.adam(1e-3)
        p, m, v = o_mlp.adam_step(p, g.astype(np.float64), m, v, step, 1e-3)
        got = _np(net.params).astype(np.float64)
        assert np.max(np.abs(got - p)) <= 1e-6 * np.max(np.abs(p))


def _tiny(n_steps=24, M=0):
    import torch
    from paper_1710_02401_amd import Solver
    # distinct time nodes need >= 11 steps for M = 8, >= 46 for M = 16
    cfg = dict(TINY["tiny-2d"], n_steps=n_steps, learned_nodes=M)
    print(f"[gpu] solver {cfg['name']}", flush=True)
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    torch.cuda.synchronize()
    return cfg, s, o_swr.Problem(cfg)


def _flat_nodes(prob, g_faces_per_item, rows):
    """(len(rows), n_face_nodes) in the library's node order."""
    return np.concatenate([np.concatenate(gf, axis=1)[rows] for gf in g_faces_per_item], axis=1)


def test_face_data_after_two_iterations():
    cfg, s, prob = _tiny()
    c0 = prob.initial_coeffs()
    hists, _ = o_swr.swr_window(prob, c0, iters=2)
    s.run(k_max=2)
    steps = [0, 3, prob.n_T]
    got = _np(s.face_data(steps))
    ref = _flat_nodes(prob, [o_swr.face_data(prob, i, lambda j: hists[j])
                             for i in range(prob.n_sub)], steps)
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("n_steps,M", [(24, 0), (60, 16)])
def test_features_targets_and_interpolated_guess(n_steps, M):
    import torch
    cfg, s, prob = _tiny(n_steps, M)
    c0 = prob.initial_coeffs()
    nodes = o_learned.time_nodes(prob.n_T, M or 8)
    assert s.time_nodes() == nodes
    # interface data of the oracle's iterate 2 at step 0 and at the time nodes
    hists, _ = o_swr.swr_window(prob, c0, iters=2)
    g_items = [o_swr.face_data(prob, i, lambda j: hists[j]) for i in range(prob.n_sub)]
    g_steps = [np.concatenate(gf, axis=1) for gf in g_items]         # per item (n_T+1, n_i)
    g0_items = [g[0] for g in g_steps]
    n_max = max(g.shape[1] for g in g_steps)
    M = len(nodes)
    n_in, n_out = 2 * n_max + M + 8 + 3, 2 * M * n_max + 5           # padded widths
    t0 = 0.37
    E = o_swr.field(cfg, t0 + np.array(nodes) * cfg["dt"])
    X_ref, sc_ref = o_learned.features(g0_items, E, n_in, o_learned.item_positions(prob),
                                       t0 / (prob.n_T * cfg["dt"]))
    g0_dev = torch.from_numpy(np.concatenate(g0_items)).cuda()
    x, sc = s.learned_features(g0_dev, t0, n_in)
    assert np.allclose(_np(sc), sc_ref, rtol=1e-12, atol=0)
    assert np.max(np.abs(_np(x) - X_ref)) <= 1e-6 * max(1.0, np.max(np.abs(X_ref)))
    # targets at the time nodes
    Y_ref = o_learned.targets([g[nodes] for g in g_steps], sc_ref, n_out)
    gn_dev = torch.from_numpy(np.ascontiguousarray(np.concatenate([g[nodes] for g in g_steps],
                                                                   axis=1))).cuda()
    y = s.learned_targets(gn_dev, sc, n_out)
    assert np.max(np.abs(_np(y) - Y_ref)) <= 1e-6 * max(1.0, np.max(np.abs(Y_ref)))
    # interpolated guess from seeded FP32 predictions
    yp = np.random.default_rng(12).normal(size=(prob.n_sub, n_out)).astype(np.float32)
    out = _np(s.learned_apply(torch.from_numpy(yp).cuda(), sc, g0_dev, n_out))
    out = out.reshape(prob.n_T + 1, -1)
    ref = np.concatenate(o_learned.apply(yp.astype(np.float64), sc_ref, g0_items, prob.n_T,
                                         cfg["dt"], M=len(nodes)), axis=1)
    assert np.max(np.abs(out - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_given_guess_from_apply_runs_and_matches_plain_answer():
    """A window started from an interpolated guess converges to the same
    answer as the plain start (the guess only moves the starting point)."""
    import torch
    cfg, s, prob = _tiny()
    c0 = s.initial().clone()
    st = s.run(k_max=40, tol=1e-12)
    h_plain = s.history().clone()
    n_max = int(max(s.n_nodes))
    g0 = s.face_data([0])[0].clone()
    s.set_initial(c0)
    M = len(s.time_nodes())
    x, sc = s.learned_features(s.face_data([0])[0].clone(), 0.0, 2 * n_max + M + 8)
    yp = torch.zeros((len(s.K), 2 * M * n_max), dtype=torch.float32, device="cuda")
    g_all = s.learned_apply(yp, sc, g0, 2 * M * n_max)
    st2 = s.run(k_max=40, tol=1e-12, warm=2, g=g_all)
    assert st["converged"] and st2["converged"]
    d = torch.linalg.norm(s.history() - h_plain) / torch.linalg.norm(h_plain)
    assert float(d) <= 1e-9


@pytest.mark.slow
def test_trained_network_saves_iterations():
    """Train on plain-SWR windows of the two-electron system (field
    amplitude and phase drawn with one seed), then start held-out windows
    (another seed) from the network's guess: fewer iterations to the same
    residual target, and the same converged answer."""
    from paper_1710_02401_amd import learned
    cfg = workloads.get_config("c4-2e-1d-learned", n_steps=200)
    out, _ = learned.experiment(cfg, n_traj=6, n_win=6, eval_traj=2, eval_win=3, steps=1500,
                                batch=256, lr=1e-3, k_max=cfg["iters"] * 2,
                                log=lambda m: print(m, flush=True))
    print({k: v for k, v in out.items() if k != "rows"}, flush=True)
    assert out["final_loss"] < 0.2 * out["first_loss"]
    assert out["all_converged"]
    assert out["max_rel_diff"] <= 1e-6
    assert out["learned_mean"] < out["plain_mean"]
