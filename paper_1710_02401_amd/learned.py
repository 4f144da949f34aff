"""Learned warm start of the SWR iteration.

The Schwarz initial guess of a window is free (Section 4.1, eq. (S1)).  The
plain guess holds the window's initial Robin data constant in time; the
learned guess adds a correction predicted by a small network from the
subdomain's own initial interface data and the field over the window.  The
network only changes where the iteration starts: every window is still
iterated by plain SWR to the same residual target, so the converged answer
is the plain one and the network can only save iterations.

Everything numerical runs in libswr.so kernels: Robin data at the face
nodes, features, targets, the network (FP32 forward/backward/Adam) and the
interpolation of the prediction to every time step.  This module only
orders the calls and keeps the training set.
"""
import math
import time

import numpy as np

from . import swr as S

def net_sizes(solver):
    """Input and output widths of the network for a solver's face nodes and
    M time nodes: (Re, Im) per node plus the M + 8 tail entries in, M
    corrections per node out."""
    n_max = int(max(solver.n_nodes))
    M = int(solver.info.learned_nodes)
    return 2 * n_max + M + 8, M * 2 * n_max


def window_length(cfg):
    return cfg["n_steps"] * cfg["dt"]


def _window_inputs(s, t0, n_in):
    g0 = s.face_data([0])[0].clone()          # current iterate = window initial state
    x, scale = s.learned_features(g0, t0, n_in)
    return g0, x, scale


def collect(s, cfg, n_traj, n_win, seed, k_max, tol, log=None):
    """Training pairs from plain SWR: for every window and subdomain, the
    features of its initial interface data and the converged correction.
    Field amplitude and phase of each trajectory are drawn from `seed`."""
    import torch
    rng = np.random.default_rng(seed)
    n_in, n_out = net_sizes(s)
    nodes = s.time_nodes()
    T = window_length(cfg)
    omega = cfg["field"]["omega"]
    X, Y, iters = [], [], []
    for tr in range(n_traj):
        E0 = float(rng.uniform(0.03, 0.07))
        phase = float(rng.uniform(0.0, 2.0 * math.pi))
        s.set_field(E0, omega, phase)
        s.set_initial()
        for w in range(n_win):
            t0 = w * T
            g0, x, scale = _window_inputs(s, t0, n_in)
            st = s.run(k_max=k_max, tol=tol, t0=t0, warm=S.SWR_WARM_PLAIN)
            y = s.learned_targets(s.face_data(nodes), scale, n_out)
            X.append(x)
            Y.append(y)
            iters.append(st["iters"])
            s.advance_window()
        if log:
            log(f"collect: trajectory {tr + 1}/{n_traj}, mean iterations {np.mean(iters):.1f}")
    X = torch.cat(X)
    Y = torch.cat(Y)
    keep = torch.isfinite(X).all(dim=1) & torch.isfinite(Y).all(dim=1)
    return X[keep], Y[keep], dict(samples=int(keep.sum()), dropped=int((~keep).sum()),
                                  plain_iters=iters)


def train(net, X, Y, steps, batch, lr, lr_min=1e-5, seed=0, log=None):
    """Adam on random mini-batches with a cosine learning-rate decay."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    batch = min(batch, n, net.max_batch)
    losses = []
    for k in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(X.device)
        loss, _ = net.loss_grad(X[idx], Y[idx])
        net.adam(lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * k / steps)))
        if k % max(1, steps // 20) == 0 or k == steps - 1:
            losses.append(float(loss.item()))
            if log:
                log(f"train: step {k + 1}/{steps} loss {losses[-1]:.4e}")
    return losses


def full_loss(net, X, Y):
    """Mean squared error over a whole sample set (the network's kernels)."""
    import torch
    tot = 0.0
    for a in range(0, X.shape[0], net.max_batch):
        y = net.forward(X[a:a + net.max_batch])
        tot += float(((y - Y[a:a + net.max_batch]) ** 2).sum().item())
    return tot / Y.numel()


def evaluate(s, net, cfg, n_traj, n_win, seed, k_max, tol, log=None):
    """Iterations to the residual target for the plain, learned and zero
    guesses on the same windows, for the guess built from the converged
    answer's own targets (the ceiling of the M-node representation),
    and the distance between the learned and plain answers."""
    import torch
    rng = np.random.default_rng(seed)
    n_in, n_out = net_sizes(s)
    nodes = s.time_nodes()
    T = window_length(cfg)
    omega = cfg["field"]["omega"]
    rows = []
    for tr in range(n_traj):
        E0 = float(rng.uniform(0.03, 0.07))
        phase = float(rng.uniform(0.0, 2.0 * math.pi))
        s.set_field(E0, omega, phase)
        s.set_initial()
        for w in range(n_win):
            t0 = w * T
            c0 = s.initial().clone()
            g0, x, scale = _window_inputs(s, t0, n_in)
            st_p = s.run(k_max=k_max, tol=tol, t0=t0, warm=S.SWR_WARM_PLAIN)
            h_p = s.history().clone()
            y_star = s.learned_targets(s.face_data(nodes), scale, n_out)
            runs = {}
            for name, y in (("learned", net.forward(x)), ("ideal", y_star)):
                s.set_initial(c0)
                g_all = s.learned_apply(y, scale, g0, n_out)
                runs[name] = s.run(k_max=k_max, tol=tol, t0=t0, warm=S.SWR_WARM_GIVEN, g=g_all)
                del g_all
                if name == "learned":
                    h_l = s.history().clone()
                    pred_err = float(((y - y_star) ** 2).mean().item())
            s.set_initial(c0)
            st_z = s.run(k_max=k_max, tol=tol, t0=t0, warm=S.SWR_WARM_ZERO)
            diff = float(torch.linalg.norm(h_l - h_p) / torch.linalg.norm(h_p))
            st_l, st_i = runs["learned"], runs["ideal"]
            rows.append(dict(traj=tr, window=w, plain=st_p["iters"], learned=st_l["iters"],
                             ideal=st_i["iters"], zero=st_z["iters"],
                             converged=bool(st_p["converged"] and st_l["converged"]),
                             prediction_mse=pred_err, rel_diff_learned_vs_plain=diff))
            if log:
                log(f"eval: traj {tr} window {w}: plain {st_p['iters']} learned {st_l['iters']} "
                    f"ideal {st_i['iters']} zero {st_z['iters']} mse {pred_err:.2e} "
                    f"diff {diff:.1e}")
            s.advance_window()   # from the zero-guess run: same converged answer
    return rows


def summarize(rows):
    col = lambda k: np.array([r[k] for r in rows], dtype=float)
    p, l, z, i = col("plain"), col("learned"), col("zero"), col("ideal")
    return dict(windows=len(rows), plain_mean=float(p.mean()), learned_mean=float(l.mean()),
                ideal_mean=float(i.mean()), zero_mean=float(z.mean()),
                plain_median=float(np.median(p)), learned_median=float(np.median(l)),
                iteration_reduction=float(1.0 - l.mean() / p.mean()),
                prediction_mse=float(col("prediction_mse").mean()),
                max_rel_diff=float(max(r["rel_diff_learned_vs_plain"] for r in rows)),
                all_converged=bool(all(r["converged"] for r in rows)))


def experiment(cfg, n_traj=8, n_win=8, eval_traj=2, eval_win=4, steps=4000, batch=256,
               lr=1e-3, k_max=120, tol=1e-8, collect_tol=1e-8, log=print):
    """Generate data with plain SWR, train the network on the GPU, and
    compare iterations to the residual target on held-out windows."""
    from workloads import mlp_init
    t = time.time()
    s = S.Solver(cfg)
    s.assemble()
    s.set_initial()
    n_in, n_out = net_sizes(s)
    X, Y, info = collect(s, cfg, n_traj, n_win, seed=2401, k_max=k_max, tol=collect_tol, log=log)
    t_collect = time.time() - t
    params = mlp_init.initial_params(n_in, mlp_init.N_HIDDEN, mlp_init.N_LAYERS, n_out)
    net = S.Mlp(n_in, mlp_init.N_HIDDEN, mlp_init.N_LAYERS, n_out, params)
    first = full_loss(net, X, Y)
    t = time.time()
    train(net, X, Y, steps, batch, lr, log=log)
    t_train = time.time() - t
    final = full_loss(net, X, Y)
    t = time.time()
    rows = evaluate(s, net, cfg, eval_traj, eval_win, seed=2402, k_max=k_max, tol=tol, log=log)
    t_eval = time.time() - t
    out = summarize(rows)
    out.update(train_samples=info["samples"], dropped_samples=info["dropped"],
               target_mean_square=float((Y ** 2).mean().item()),
               first_loss=first, final_loss=final, steps=steps,
               seconds=dict(collect=t_collect, train=t_train, evaluate=t_eval), rows=rows)
    return out, net
