"""Failure handling of swr_run on the GPU, through the C ABI:

  * the iteration cap above the residual target returns SWR_E_NOCONV with
    the statistics and the state of a normal run (the binding reports it as
    converged=False);
  * the growth guard of a given warm start: consecutive increases of Res(k)
    make swr_run run the window again from the plain warm start, and the
    result is then the plain run's, bit for bit (one iterate at a time,
    pipelined, and replayed from a HIP graph)."""
import ctypes

import pytest

import workloads

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


def test_iteration_cap_above_target_returns_noconv():
    import torch
    from paper_1710_02401_amd import swr as S
    s = _solver(TINY["tiny-2d"])
    c0 = s.initial().clone()
    o = S.swr_run_opts(3, 1e-300, 0.0, S.SWR_WARM_PLAIN, None, 1, 0, 0, 0)
    st = S.swr_run_stats()
    rc = s.lib.swr_run(s.h, ctypes.byref(o), ctypes.byref(st), s._stream())
    assert rc == S.SWR_E_NOCONV
    assert "iteration cap" in s.lib.swr_last_error(s.h).decode()
    assert st.iters == 3 and st.converged == 0 and st.fallback == 0
    res_cap = [st.res[i] for i in range(3)]
    h_cap = s.history().clone()
    # the same iterations with tol <= 0 (exactly k_max) succeed, same state
    s.set_initial(c0)
    out = s.run(k_max=3, tol=-1.0, depth=1)
    assert out["res"] == res_cap
    assert torch.equal(s.history(), h_cap)
    # through the binding the cap is a result, not an exception
    s.set_initial(c0)
    out = s.run(k_max=3, tol=1e-300, depth=1)
    assert not out["converged"] and out["iters"] == 3
    # and a reachable target still converges with SWR_OK
    s.set_initial(c0)
    out = s.run(k_max=40, tol=1e-8)
    assert out["converged"]


def _given_plain_data(s):
    """Robin data at the face nodes that reproduce the plain warm start: the
    initial state's face data held constant over the window (the learned
    guess with a zero network output)."""
    import torch
    n_max = int(max(s.n_nodes))
    M = len(s.time_nodes())
    g0 = s.face_data([0])[0].clone()
    _, sc = s.learned_features(g0, 0.0, 2 * n_max + M + 8)
    y = torch.zeros((len(s.K), 2 * M * n_max), dtype=torch.float32, device="cuda")
    return s.learned_apply(y, sc, g0, 2 * M * n_max)


@pytest.mark.parametrize("depth,graph", [(1, False), (0, False), (0, True)])
def test_growth_guard_falls_back_to_plain(depth, graph):
    """The two-electron window's residual rises from iterate 1 to 2 (0.66 to
    2.24) from the plain start and from the equivalent given data: with the
    guard at one increase the given start is abandoned, without it kept."""
    import torch
    s = _solver(workloads.get_config("c2-2e-1d"))
    c0 = s.initial().clone()
    plain = s.run(k_max=4, tol=-1.0, depth=depth, graph=graph)
    h_plain = s.history().clone()
    assert plain["res"][1] > plain["res"][0] and not plain["fallback"]
    g = _given_plain_data(s)
    s.set_initial(c0)
    kept = s.run(k_max=4, tol=-1.0, depth=depth, graph=graph, warm=2, g=g, growth_guard=-1)
    assert not kept["fallback"]
    assert kept["res"][1] > kept["res"][0]
    assert kept["res"][0] == pytest.approx(plain["res"][0], rel=1e-9)
    s.set_initial(c0)
    back = s.run(k_max=4, tol=-1.0, depth=depth, graph=graph, warm=2, g=g, growth_guard=1)
    assert back["fallback"]
    assert back["res"] == plain["res"]
    assert torch.equal(s.history(), h_plain)
    # the default guard (two consecutive increases) leaves this window alone
    s.set_initial(c0)
    dflt = s.run(k_max=4, tol=-1.0, depth=depth, graph=graph, warm=2, g=g)
    assert not dflt["fallback"]
