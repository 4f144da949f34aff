"""Window-boundary checkpoints of a Solver.

A checkpoint holds what the next time window needs: the coefficients of the
current iterate at the window's last step (the next window's initial state,
Section 4.4 step 1 applied to the computed solution), the next window's time
origin, a hash of the workload description it belongs to, and optionally
the learned warm start's network (parameters, Adam moments and step count).

Resuming from it gives the next window the initial state that
swr_advance_window gives an uninterrupted run: bit for bit in real time on
the narrow and wide paths (both copy the same coefficients into the initial
state, and the run's plain warm start is formed from it); the block path
stores the state in its orthonormalised coordinates and resumes through the
coordinate change (agreement to rounding); imaginary time renormalises the
given state on entry (agreement to rounding).

Files are NumPy .npz archives of plain arrays, written and read without
pickles.
"""
import hashlib
import json

import numpy as np


def config_hash(cfg):
    """SHA-256 of the workload description (keys sorted, numbers as JSON)."""
    blob = json.dumps(cfg, sort_keys=True, default=lambda v: np.asarray(v).tolist())
    return hashlib.sha256(blob.encode()).hexdigest()


def save(path, solver, cfg, t_next, mlp=None):
    """Writes the checkpoint of `solver` (after a window's swr_run) to `path`:
    the current iterate's coefficients at the last step, t_next (the next
    window's origin), the description's hash, and `mlp`'s state if given."""
    import torch
    last = [h[-1] for h in solver.split_history(solver.history())]
    arrays = dict(c_end=torch.cat(last).cpu().numpy(), t_next=np.float64(t_next),
                  config=np.array(config_hash(cfg)))
    if mlp is not None:
        d = mlp.d
        arrays.update(mlp_shape=np.array([d.n_in, d.n_hidden, d.n_layers, d.n_out], dtype=np.int64),
                      mlp_params=mlp.params.cpu().numpy(), mlp_m=mlp.m.cpu().numpy(),
                      mlp_v=mlp.v.cpu().numpy(), mlp_step=np.int64(mlp.step))
    with open(path, "wb") as f:
        np.savez(f, **arrays)


def load(path, cfg):
    """The checkpoint's arrays, after checking that it belongs to `cfg`
    (ValueError otherwise).  Touches no GPU."""
    with np.load(path, allow_pickle=False) as z:
        data = {k: z[k] for k in z.files}
    if str(data["config"]) != config_hash(cfg):
        raise ValueError("checkpoint written for another workload description")
    return data


def resume(path, cfg, solver=None):
    """A Solver for `cfg` (assembled; `solver` if given) whose initial state is
    the checkpoint's, the next window's origin, and the network (an Mlp with
    the saved parameters and Adam state) or None."""
    import torch

    from .swr import Mlp, Solver
    data = load(path, cfg)
    s = solver
    if s is None:
        s = Solver(cfg)
        s.assemble()
    s.set_initial(torch.from_numpy(data["c_end"]).to(s.device))
    mlp = None
    if "mlp_params" in data:
        n_in, n_hidden, n_layers, n_out = (int(v) for v in data["mlp_shape"])
        mlp = Mlp(n_in, n_hidden, n_layers, n_out, data["mlp_params"], device=s.device)
        mlp.m.copy_(torch.from_numpy(data["mlp_m"]))
        mlp.v.copy_(torch.from_numpy(data["mlp_v"]))
        mlp.step = int(data["mlp_step"])
    return s, float(data["t_next"]), mlp
