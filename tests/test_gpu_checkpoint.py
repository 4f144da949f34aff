"""Window-boundary checkpoint and resume on the GPU: a second window
resumed from a checkpoint in a new Solver equals the uninterrupted run's
second window (swr_advance_window) bit for bit in real time, and the
learned warm start's network comes back with its parameters and Adam
state."""
import pytest

import workloads
from paper_1710_02401_amd import checkpoint

pytestmark = pytest.mark.gpu

TINY = {c["name"]: c for c in workloads.tiny_configs()}


def _solver(cfg):
    import torch
    from paper_1710_02401_amd import Solver
    print(f"[gpu] solver {cfg['name']}", flush=True)
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    torch.cuda.synchronize()
    return s


@pytest.mark.parametrize("name", ["tiny-2d", "c2-2e-1d"])
def test_resume_equals_uninterrupted_second_window(name, tmp_path):
    import torch
    from paper_1710_02401_amd import Mlp
    from workloads import mlp_init
    cfg = TINY[name] if name in TINY else workloads.get_config(name)
    T = cfg["n_steps"] * cfg["dt"]
    k = 5
    ref = _solver(cfg)
    ref.run(k_max=k, tol=-1.0)
    ref.advance_window()
    st_ref = ref.run(k_max=k, tol=-1.0, t0=T)
    h_ref = ref.history().clone()
    first = _solver(cfg)
    first.run(k_max=k, tol=-1.0)
    net = Mlp(16, 32, 2, 8, mlp_init.initial_params(16, 32, 2, 8, seed=5))
    net.step = 7
    net.m.fill_(0.25)
    path = tmp_path / "window.npz"
    checkpoint.save(path, first, cfg, T, mlp=net)
    del first
    s, t_next, net2 = checkpoint.resume(path, cfg)
    assert t_next == T
    st = s.run(k_max=k, tol=-1.0, t0=t_next)
    assert st["res"] == st_ref["res"]
    assert torch.equal(s.history(), h_ref)
    assert torch.equal(net2.params, net.params) and torch.equal(net2.m, net.m)
    assert net2.step == 7
