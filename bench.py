"""Benchmark of the SWR hot path on one MI355X.

A step is one SWR time window of the two-electron workload (2 electrons in
one dimension each, 8x8 overlapping subdomains, 8x8 Gaussians per subdomain,
1000 Crank-Nicolson steps, 20 Schwarz iterations), run by swr_run: the
inverses of every local Crank-Nicolson matrix of the window (series in the
field around 128-step anchors, or one inversion per step where the series
bound does not hold), the plain warm start, then 20 Schwarz iterations of
local solves (recurrence), transmission and residual, with P iterates in
flight over chunks of the window (depth P and the transmission tile chosen
by the library's autotuner on this window before timing).  Inputs (assembled
matrices, initial coefficients) are resident in HBM before the timed region.

value = subdomain-solves per second = subdomains x Schwarz iterations x
steps / seconds, where a subdomain-solve is one subdomain's whole-window
local solve in one Schwarz iteration.  The timed windows run exactly 20
iterations each, their launches replayed from a HIP graph captured on the
first window (--no-graph: launched one by one); kernel durations come from
HIP events the library records around each launch on the run's stream, in a
second pass over as many windows launched one by one.

The same JSON line carries the other workloads as context objects (not the
headline value): the imaginary-time window, the batched wide-basis windows,
the two-electron two-dimension workload on the block path (256 subdomains of
1296 Gaussians, 30 Schwarz iterations in flight) and the learned warm start.
cpu_baseline is the oracle over the headline window on a process pool of the
host's cores (at most 16).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
# FP64 vector FMA issue: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
FP64_VALU_PEAK_TFS = 78.6

# HBM traffic of the dominant kernel from rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE, each scaled by the ratio of a plain device copy's known bytes
# to the counter's reading), per launch of that kernel in this benchmark's
# window.  Valid only for the kernel source it was measured on.
MEASURED_TRAFFIC = {
    # profiles/c2-2e-1d_traffic.md: FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000
    # (1 GiB copy calibration) over the first window at depth 4 with the
    # 16-step transmission tile (the autotuned default): 23 recurrence
    # launches (the series evaluated in the step), 27 transmissions, one
    # factorisation
    "k_cn_recur_series": {"kernels_sha256": "efa8b11e90fcd0d2", "bytes_per_launch": 0.22185e9},
    # per transmission tile (only the measured one)
    "k_tx_send+k_tx_recv": {"kernels_sha256": "efa8b11e90fcd0d2",
                            "bytes_per_launch_by_tile": {16: 0.45149e9}},
    # profiles/c3-1e-1d-batched_traffic.md: one sweep of the batched workload
    "k_cn_recur_wide": {"wide_sha256": "8b17b20586e217b0", "bytes_per_launch": 1350.81e9},
    # profiles/c5-2e-2d_traffic.md: median over the 529 step launches of one
    # window (FETCH_SIZE x 1.9999 + WRITE_SIZE x 1.000)
    "k_blk_solve": {"block_sha256": "b8fe3e9e4a331db2", "bytes_per_launch": 37.00e9},
}


def kernels_digest():
    import hashlib
    path = os.path.join(HERE, "paper_1710_02401_amd", "csrc", "kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def learned_summary(mode):
    """Iterations to Res <= 1e-8 from the plain, learned and zero guesses on
    held-out windows, after training the network on the GPU (quick: windows
    of 200 steps; full: the 1000-step windows of the two-electron workload)."""
    import workloads
    from paper_1710_02401_amd import learned
    if mode == "quick":
        cfg = workloads.get_config("c4-2e-1d-learned", n_steps=200)
        kw = dict(n_traj=10, n_win=8, eval_traj=2, eval_win=4, steps=3000)
    else:
        cfg = workloads.get_config("c4-2e-1d-learned")
        kw = dict(n_traj=64, n_win=6, eval_traj=2, eval_win=4, steps=8000)
    out, _ = learned.experiment(cfg, batch=256, lr=1e-3, k_max=150, log=lambda m: None, **kw)
    keep = ("windows", "plain_mean", "learned_mean", "zero_mean", "ideal_mean",
            "iteration_reduction", "prediction_mse", "max_rel_diff", "all_converged",
            "train_samples", "first_loss", "final_loss", "steps", "seconds")
    res = {k: out[k] for k in keep}
    # plain SWR with other Robin constants on the same held-out windows: the
    # optimised-mu baseline the learned guess is compared against
    from paper_1710_02401_amd import studies
    by_mu = studies.held_out_windows_by_mu(cfg, [-1j, -2.5j, -5j, -10j, -20j, -40j],
                                           kw["eval_traj"], kw["eval_win"], 2402, 150, 1e-8)
    res["plain_mean_by_mu"] = {f"{m['mu'][1]:g}i": m["mean_iters"] for m in by_mu}
    best = min(by_mu, key=lambda m: m["mean_iters"])
    res["best_mu"] = f"{best['mu'][1]:g}i"
    # the network trained and evaluated again at that mu
    out_b, _ = learned.experiment(dict(cfg, mu=best["mu"]), batch=256, lr=1e-3, k_max=150,
                                  log=lambda m: None, **kw)
    res["at_best_mu"] = {k: out_b[k] for k in ("plain_mean", "learned_mean", "zero_mean",
                                              "iteration_reduction", "all_converged")}
    res["workload"] = f"{cfg['name']}, {cfg['n_steps']}-step windows, tol 1e-8"
    if mode == "quick":
        # the default line's leg is a reduced configuration of the learned
        # workload, so that the whole benchmark stays within minutes
        res["reduced"] = ("200-step windows (the workload's are 1000 steps) and "
                          f"{res['train_samples']} training samples (the workload plans about "
                          "1e5); --learned full trains and evaluates on 1000-step windows")
    return res


def batched_cpu_baseline(cfg):
    """The oracle on a bounded sample of the batched workload: iteration 1
    (plain warm start) of every 16th subdomain of geometry 0 -- K from 32 to
    256 -- on one host thread, assembly and projection outside the timing."""
    from threadpoolctl import threadpool_limits

    from oracle import swr as o_swr
    prob = o_swr.Problem(dict(cfg, nuclei=cfg["geometries"][0], geometries=None))
    targets = list(range(0, prob.n_sub, 16))
    need = set(targets) | {j for i in targets for j in prob.neighbours(i)}
    with threadpool_limits(limits=1):
        c0 = {j: prob.initial_coeff(j) for j in need}
        for i in targets:
            prob.sys[i]
        t = time.perf_counter()
        o_swr.swr_sampled(prob, c0, targets, 1)
        dt = time.perf_counter() - t
    Ks = sorted(prob.sys[i].K for i in targets)
    return dict(value=len(targets) / dt, unit="subdomain-solves/s", cores=1, kind="oracle",
                sample=f"iteration 1 of {len(targets)} subdomains of geometry 0 (every 16th, K "
                       f"{Ks[0]}..{Ks[-1]}), {cfg['n_steps']} Crank-Nicolson steps each with "
                       f"Robin data, NumPy/LAPACK FP64 on one host thread: {dt:.1f} s")


def batched_summary(iters, cpu=True):
    """The batched uneven workload (64 geometries x 256 subdomains, 32..256
    Gaussians per subdomain, 200 steps) on the wide-basis path: the schedule
    autotuned on 2-iteration windows, then one window of `iters` Schwarz
    iterations replayed from a HIP graph captured on a first window (one
    iterate at a time: the items fill the GPU); kernel times from HIP events
    around every launch in a second, eager pass.  Recurrence bytes per sweep: per item and step the unique entries
    K(K+1)/2 of S2 (8 B) and of each series term the item applies (16 B),
    f^{n+1} read and c^{n+1} written (32 K B)."""
    import torch

    import workloads
    from paper_1710_02401_amd import Solver
    cfg = workloads.get_config("c3-1e-1d-batched")
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    torch.cuda.synchronize()
    c0 = s.initial().clone()
    # the schedule (transmission tile, recurrence order) by measurement on
    # short windows, then the window captured as a HIP graph and replayed
    tuning = s.autotune(k_iters=2)
    s.set_initial(c0)
    s.run(k_max=iters, tol=-1.0, graph=True)
    s.set_initial(c0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st_g = s.run(k_max=iters, tol=-1.0, graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    # kernel times: the same window launched one by one with HIP events
    s.set_initial(c0)
    st = s.run(k_max=iters, tol=-1.0, timing=True)
    torch.cuda.synchronize()
    Ks = [nb[0] for nb in cfg["nbasis"]] * len(cfg["geometries"])
    n, nT, terms = len(Ks), int(s.n_steps), s.factor_terms() + 1
    per_item = s.item_terms()
    rec_bytes = iters * nT * sum(k * (k + 1) / 2 * (8.0 + 16.0 * t) + 32.0 * k
                                 for k, t in zip(Ks, per_item))
    kern = st["kernels"]
    sec = kern["recur"]["ms"] * 1e-3
    achieved = rec_bytes / sec / 1e9
    m = MEASURED_TRAFFIC.get("k_cn_recur_wide")
    valid = m and m["wide_sha256"] == wide_digest()
    out = {
        "workload": f"{cfg['name']}: {len(cfg['geometries'])} geometries x {cfg['L'][0]} "
                    f"subdomains, K={min(Ks)}..{max(Ks)} Gaussians (1-D), {nT} steps per "
                    f"window, {iters} Schwarz iterations",
        "value": n * iters / wall, "unit": "subdomain-solves/s",
        "ms_per_window": 1e3 * wall, "ms_per_iteration": 1e3 * wall / iters,
        "series_terms": terms,
        "series_terms_largest_bases": int(per_item[Ks.index(max(Ks))]),
        "factor_ms": kern["factor"]["ms"],
        "recur_ms_per_sweep": kern["recur"]["ms"] / iters,
        "transmit_ms_per_sweep": kern["transmit"]["ms"] / iters,
        "roofline": {"kernel": "k_cn_recur_wide", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": m["bytes_per_launch"] / 1e9 if valid else None},
        "last_residual": st_g["res"][min(iters, 64) - 1],
        "schedule": {"tx_tile": tuning["tx_tile"], "order": "item order" if tuning["order"]
                     else "largest K first", "candidates": tuning["candidates"],
                     "windows_launched_as": "hip_graph"},
        # the paper's schedule: every matrix refactored in each sweep
        "paper_literal_sweep_ms": kern["factor"]["ms"] + (kern["recur"]["ms"] +
                                                          kern["transmit"]["ms"]) / iters,
    }
    if cpu:
        out["cpu_baseline"] = batched_cpu_baseline(cfg)
    return out


def slater_summary(iters=20):
    """The two-electron window in the Slater-like antisymmetric basis of
    Section 2 (eq. (LSD)): the same 8 x 8 decomposition and 1000 steps, 64
    antisymmetrised pairs per subdomain off the diagonal and 28 on it, from
    the antisymmetrised Gaussian pair; 20 Schwarz iterations after an
    untimed window, the schedule autotuned (the transmission is formed
    densely: the basis is not a tensor product)."""
    import torch

    import workloads
    from paper_1710_02401_amd import Solver
    cfg = workloads.get_config("c2-2e-1d-slater")
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    torch.cuda.synchronize()
    c0 = s.initial().clone()
    s.autotune(k_iters=2)
    s.set_initial(c0)
    s.run(k_max=iters, tol=-1.0, graph=True)
    s.set_initial(c0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = s.run(k_max=iters, tol=-1.0, graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    s.set_initial(c0)
    kern = s.run(k_max=iters, tol=-1.0, timing=True)["kernels"]
    n = int(s.info.n_items)
    return {
        "workload": f"{cfg['name']}: 2 electrons x 1-D, {n} subdomains, K={int(s.K.min())}.."
                    f"{int(s.K.max())} antisymmetrised Gaussian pairs, {int(s.n_steps)} steps, "
                    f"{iters} Schwarz iterations, depth {int(s.info.depth_run)}",
        "value": n * iters / wall, "unit": "subdomain-solves/s", "ms_per_window": 1e3 * wall,
        "kernels_ms_per_window": {k: kern[k]["ms"] for k in ("factor", "transmit", "recur",
                                                              "residual")},
        "last_residual": st["res"][iters - 1],
    }


def lsd_summary(name="paper-lsd-test-2a", iters=20):
    """The paper's determinant Tests in local Slater determinants of local
    orbitals (Section 3): 5 x 5 subdomains, imaginary time, 200
    implicit-Euler steps per window; Test 2.a with 8 orbitals per interval
    (64 determinants off the diagonal, 28 on it) and mu = 1, Test 2.b with 4
    orbitals and the two end Gaussians of each interval (Section 3.3; 36
    and 15) and mu = 10.  Assembly (orbital problems, tables, matrices, the
    determinants' condition check) timed once, then 20 Schwarz iterations
    after an untimed window."""
    import torch

    import workloads
    from paper_1710_02401_amd import Solver
    cfg = workloads.get_config(name)
    s = Solver(cfg)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.assemble()
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t
    s.set_initial()
    c0 = s.initial().clone()
    s.run(k_max=iters, tol=-1.0)
    s.set_initial(c0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = s.run(k_max=iters, tol=-1.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    n = int(s.info.n_items)
    return {
        "workload": f"{cfg['name']}: 2 electrons x 1-D, {n} subdomains, K={int(s.K.min())}.."
                    f"{int(s.K.max())} local Slater determinants, {int(s.n_steps)} "
                    f"imaginary-time steps, {iters} Schwarz iterations, depth {int(s.info.depth_run)}",
        "value": n * iters / wall, "unit": "subdomain-solves/s", "ms_per_window": 1e3 * wall,
        "assembly_ms": 1e3 * t_asm, "energy": st["energy"], "last_residual": st["res"][iters - 1],
    }


def lo_summary(iters=20):
    """Local orbitals of one electron in two dimensions (Section 3, d = 2):
    4 x 4 boxes, the 16 lowest orbitals of each box from its 8 x 8
    Gaussians, 200 real-time steps; assembly (the orbital problems with the
    mollified Coulomb attraction, the Gaussian matrices and their transforms,
    the transfer operators) timed once, then 20 Schwarz iterations after an
    untimed window."""
    import torch

    import workloads
    from paper_1710_02401_amd import Solver
    cfg = workloads.get_config("lo-1e-2d")
    s = Solver(cfg)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.assemble()
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t
    s.set_initial()
    c0 = s.initial().clone()
    s.run(k_max=iters, tol=-1.0)
    s.set_initial(c0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = s.run(k_max=iters, tol=-1.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    n = int(s.info.n_items)
    return {
        "workload": f"{cfg['name']}: 1 electron x 2-D, {n} subdomains, K={int(s.K.max())} local "
                    f"orbitals from 64 Gaussians each, {int(s.n_steps)} Crank-Nicolson steps, "
                    f"{iters} Schwarz iterations, depth {int(s.info.depth_run)}",
        "value": n * iters / wall, "unit": "subdomain-solves/s", "ms_per_window": 1e3 * wall,
        "assembly_ms": 1e3 * t_asm, "last_residual": st["res"][iters - 1],
    }


def tise_summary(iters=20):
    """Imaginary time on the two-electron workload (row a10): the ground
    state window (400 normalised implicit-Euler steps per Schwarz
    iteration, one launch per step: the normalisation couples every item at
    every step; the iterates in flight share each step launch) and the
    local generalised eigenproblems.  Bytes a step launch needs: per item A,
    the inverse (complex storage, real part used) and W, K^2 entries each
    (8 + 16 + 8 B), read once for all the iterates in it (they share them
    through L2), and per (item, step, iterate) the coefficients in and out
    (16 K B); the HIP-event time includes the gaps between the launches.
    The launches are latency-bound: the rate is far below the HBM peak.
    The window's time is that of its HIP-graph replay (captured by an untimed
    window); the kernel times come from a second, eager pass with events."""
    import torch

    import workloads
    from paper_1710_02401_amd import Solver
    cfg = workloads.get_config("c2-2e-1d-tise")
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    s.run(k_max=2, tol=-1.0)
    s.set_initial()
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = s.run(k_max=iters, tol=-1.0, timing=True)
    torch.cuda.synchronize()
    wall_events = time.perf_counter() - t
    # the same window replayed from its HIP graph (captured by an untimed run)
    s.set_initial()
    s.run(k_max=iters, tol=-1.0, graph=True)
    s.set_initial()
    torch.cuda.synchronize()
    t = time.perf_counter()
    st_g = s.run(k_max=iters, tol=-1.0, graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    assert st_g["energy"] == st["energy"]
    n, K, nT = int(s.info.n_items), int(s.info.K_max), int(s.n_steps)
    P = int(s.info.depth_run)
    S = -(-nT // P)
    launches = (iters + -(-nT // S) - 1) * S if P > 1 else iters * nT
    step_bytes = launches * n * 32.0 * K * K + iters * nT * n * 16.0 * K
    achieved = step_bytes / (st["kernels"]["recur"]["ms"] * 1e-3) / 1e9
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.local_eigen()
    torch.cuda.synchronize()
    eig_ms = 1e3 * (time.perf_counter() - t)
    return {
        "workload": f"{cfg['name']}: {n} subdomains, K={K}, {nT} imaginary-time steps of "
                    f"{cfg['dt']} per Schwarz iteration, mu = {cfg['mu'][0]:g}",
        "ms_per_iteration": 1e3 * wall / iters, "windows_launched_as": "hip_graph",
        "ms_per_iteration_eager_with_events": 1e3 * wall_events / iters, "energy": st["energy"],
        "last_residual": st["res"][iters - 1],
        "subdomain_solves_per_s": n * iters / wall,
        "depth": P, "step_launches_per_window": launches,
        "roofline": {"kernel": "k_ie_step", "bound": "latency", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None},
        "local_eigen_ms": eig_ms,
    }


def host_cpu():
    """Host core count and CPU model (the GPU machine's host when run there)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


_POOL = {}


def _pool_init(cfg):
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)
    from oracle import swr as o_swr
    p = o_swr.Problem(cfg)
    for i in range(p.n_sub):  # every system assembled before the timing
        p.sys[i]
    _POOL["prob"] = p


def _pool_view(name):
    a = _POOL[name]
    return np.frombuffer(a, dtype=np.complex128).reshape(_POOL["shape"])


def _pool_cn(args):
    """Iterate of subdomain i from its Robin data; its residual term."""
    from oracle import swr as o_swr
    i, cur = args
    p = _POOL["prob"]
    H = _pool_view(f"H{cur}")
    Hp = _pool_view(f"H{1 - cur}")
    F = _pool_view("F")
    c0 = _pool_view("C0")[i, 0]
    H[i] = o_swr.local_cn(p.sys[i], c0, F[i], _POOL["E"], p.dt)
    return o_swr.residual_terms(p, {i: H[i]}, {i: Hp[i]}, subs=[i])[i]


def _pool_tx(args):
    """Robin data of subdomain i from its neighbours' iterates."""
    from oracle import swr as o_swr
    i, cur = args
    H = _pool_view(f"H{cur}")
    F = _pool_view("F")
    F[i] = o_swr.forcing(_POOL["prob"], i, lambda j: H[j])
    return 0


def cpu_baseline_pool(cfg, iters, workers):
    """The oracle as it stands on every host core: a process pool over the
    subdomains runs, in each Schwarz iteration, their Crank-Nicolson windows
    with the residual terms, then their Robin data (one single-threaded
    LAPACK per process; the iterates live in shared memory).  The whole
    window of `iters` iterations is timed (assembly and projection
    outside)."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import swr as o_swr
    prob = o_swr.Problem(cfg)
    with threadpool_limits(limits=1):
        c0 = prob.initial_coeffs()
    K = max(len(c) for c in c0)
    assert all(len(c) == K for c in c0), "the pooled baseline takes uniform bases"
    shape = (prob.n_sub, prob.n_T + 1, K)
    n = int(np.prod(shape)) * 2
    for name in ("H0", "H1", "F", "C0"):
        _POOL[name] = mp.RawArray("d", n)
    _POOL["shape"] = shape
    _POOL["E"] = o_swr.field(cfg, prob.times(0.0))
    C0 = _pool_view("C0")
    for i in range(prob.n_sub):
        C0[i] = c0[i][None, :]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_pool_init, initargs=(cfg,)) as pool:
        pool.map(abs, range(workers))  # workers ready (systems assembled)
        t = time.perf_counter()
        # iterate 0: the initial state held constant; its Robin data
        _pool_view("H1")[:] = C0
        pool.map(_pool_tx, [(i, 1) for i in range(prob.n_sub)])
        cur = 0
        for _ in range(iters):
            terms = pool.map(_pool_cn, [(i, cur) for i in range(prob.n_sub)])
            float(np.sqrt(sum(terms)))
            pool.map(_pool_tx, [(i, cur) for i in range(prob.n_sub)])
            cur = 1 - cur
        dt = time.perf_counter() - t
    for name in ("H0", "H1", "F", "C0"):
        _POOL.pop(name)
    cores, model = host_cpu()
    return dict(value=prob.n_sub * iters / dt, unit="subdomain-solves/s", cores=workers,
                kind="oracle", host_cores=cores, cpu_model=model,
                sample=f"the whole window: {iters} Schwarz iterations x {prob.n_sub} subdomains x "
                       f"{cfg['n_steps']} Crank-Nicolson steps, Robin data and residual "
                       f"included; a pool of {workers} processes (NumPy/LAPACK FP64, one "
                       f"thread each) over the subdomains: {dt:.1f} s")


def four_dimensional_cpu_baseline(cfg, steps=10):
    """The oracle on a slice of the four-dimensional workload, extrapolated:
    one interior subdomain's Crank-Nicolson steps (K = 1296, LAPACK using
    every host core) and its Robin data for the window, scaled to 256
    subdomains x 500 steps per iteration.  The potential of the sampled
    subdomain is assembled with coarser panels outside the timing (its
    values do not change the cost of a solve)."""
    from oracle import swr as o_swr
    from oracle import assemble, gauss1d
    prob = o_swr.Problem(dict(cfg, quad_nodes=2))
    i = 85
    dec = prob.dec
    sy = prob.sys[i]
    need = prob.neighbours(i)
    c0 = {j: assemble.project_initial(dec, dec.subs[j], assemble.kron_all(
        [gauss1d.overlap(dec.subs[j].alpha[k], dec.subs[j].delta[k], dec.subs[j].lo[k],
                         dec.subs[j].hi[k]) for k in range(4)])).astype(complex)
          for j in need + [i]}
    E = o_swr.field(cfg, prob.times(0.0))
    t = time.perf_counter()
    f = o_swr.forcing(prob, i, lambda j: np.repeat(c0[j][None, :], prob.n_T + 1, axis=0))
    t_tx = time.perf_counter() - t
    t = time.perf_counter()
    o_swr.local_cn(sy, c0[i], f[:steps + 1], E[:steps + 1], prob.dt)
    t_cn = time.perf_counter() - t
    per_sub = t_cn * prob.n_T / steps + t_tx
    cores, model = host_cpu()
    return dict(value=1.0 / per_sub, unit="subdomain-solves/s", cores=cores, kind="oracle",
                host_cores=cores, cpu_model=model,
                sample=f"subdomain {i}: {steps} Crank-Nicolson steps with K = {sy.K} "
                       f"({t_cn:.1f} s, NumPy/LAPACK FP64 on {cores} threads) and its Robin "
                       f"data for the window ({t_tx:.1f} s), extrapolated to the window's "
                       f"{prob.n_T} steps: {per_sub:.0f} s per subdomain-solve")


def four_dimensional_summary(iters, cpu=True):
    """The two-electron, two-dimension workload (4^4 = 256 subdomains of 6^4
    = 1296 Gaussians, 500 steps) on the block path: one window of `iters`
    Schwarz iterations, all in flight, after an untimed window; kernel times
    from HIP events.  The step products' algorithmic work per window: per
    item, iterate and step, t_s series terms applied to a K-vector, 8 K^2
    real flops each (complex multiply-adds), on the FP64 matrix cores."""
    import torch

    import workloads
    from paper_1710_02401_amd import Solver
    cfg = workloads.get_config("c5-2e-2d")
    t = time.perf_counter()
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t
    s.run(k_max=iters, tol=-1.0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = s.run(k_max=iters, tol=-1.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    stt = s.run(k_max=iters, tol=-1.0, timing=True)
    torch.cuda.synchronize()
    n, K, nT = int(s.info.n_items), int(s.info.K_max), int(s.n_steps)
    terms = s.item_terms()
    flops = 8.0 * K * K * nT * iters * float(sum(terms))
    kern = stt["kernels"]
    sec = kern["recur"]["ms"] * 1e-3
    achieved = flops / sec / 1e12
    m = MEASURED_TRAFFIC["k_blk_solve"]
    traffic = m["bytes_per_launch"] / 1e9 if m["block_sha256"] == block_digest() else None
    lit = s.run(k_max=1, tol=-1.0, depth=1, timing=True)["kernels"]
    out = {
        "workload": f"{cfg['name']}: 2 electrons x 2-D, {n} subdomains, K={K} Gaussians, "
                    f"{nT} Crank-Nicolson steps per window, {iters} Schwarz iterations in "
                    f"flight, mu = {cfg['mu'][0]:g}{cfg['mu'][1]:+g}i",
        "value": n * iters / wall, "unit": "subdomain-solves/s",
        "ms_per_window": 1e3 * wall, "ms_per_iteration": 1e3 * wall / iters,
        "assembly_s": t_asm,
        "series_terms": [int(terms.min()), int(terms.max())],
        "factor_ms": kern["factor"]["ms"],
        "step_ms_per_window": kern["recur"]["ms"], "step_launches": kern["recur"]["launches"],
        "transmit_ms_per_window": kern["transmit"]["ms"],
        "residual_ms_per_window": kern["residual"]["ms"],
        "roofline": {"kernel": "k_blk_solve (+ k_blk_rhs)", "bound": "mfma",
                     "achieved": achieved, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFS, "traffic": traffic,
                     # the kernel forms each complex product from three real
                     # ones, so it issues 6 of the 8 flops counted above
                     "mfma_issued_tflops": 0.75 * achieved},
        "residuals": [st["res"][0], st["res"][min(iters, 64) - 1]],
        "converged": st["converged"],
        # the paper's schedule: the window's matrices refactored in each
        # sweep, one iterate at a time
        "paper_literal_sweep_ms": lit["factor"]["ms"] + lit["recur"]["ms"] + lit["transmit"]["ms"]
                                  + lit["residual"]["ms"],
    }
    if cpu:
        out["cpu_baseline"] = four_dimensional_cpu_baseline(cfg)
    return out


def block_digest():
    import hashlib
    path = os.path.join(HERE, "paper_1710_02401_amd", "csrc", "block.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def wide_digest():
    import hashlib
    path = os.path.join(HERE, "paper_1710_02401_amd", "csrc", "wide.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def copy_reference(mib):
    """A device copy of `mib` MiB (the known-size kernel that scales the
    HBM byte counters)."""
    if mib <= 0:
        return
    import torch
    a = torch.empty(mib * 2 ** 17, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2-2e-1d")
    ap.add_argument("--cpu-iters", type=int, default=3, help="Schwarz iterations the oracle times")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--depth", type=int, default=0, help="iterates in flight (0: library choice)")
    ap.add_argument("--tile", type=int, default=0,
                    help="with --depth: transmission steps per block (0: the library's default)")
    ap.add_argument("--learned", choices=("off", "quick", "full"), default="full")
    ap.add_argument("--batched-iters", type=int, default=30,
                    help="Schwarz iterations of the batched wide-basis window (0: skip it)")
    ap.add_argument("--c5-iters", type=int, default=30,
                    help="Schwarz iterations of the four-dimensional window (0: skip it)")
    ap.add_argument("--only-c5", action="store_true",
                    help="run the four-dimensional leg alone")
    ap.add_argument("--c5-single", action="store_true",
                    help="with --only-c5: assembly and one window only (profiling runs)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the oracle's pool (0: every host core, at most 16)")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the windows as eager launches instead of a replayed HIP graph")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="end with a device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_1710_02401_amd import Solver

    if args.only_c5:
        if args.c5_single:
            cfg = workloads.get_config("c5-2e-2d")
            s = Solver(cfg)
            s.assemble()
            s.set_initial()
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = s.run(k_max=max(1, args.c5_iters), tol=-1.0)
            torch.cuda.synchronize()
            print(json.dumps({"four_dimensional_single_window_ms": 1e3 * (time.perf_counter() - t),
                              "iters": st["iters"]}), flush=True)
            copy_reference(args.copy_ref_mib)
            return
        print(json.dumps({"four_dimensional": four_dimensional_summary(
            max(1, args.c5_iters), cpu=not args.no_cpu)}), flush=True)
        return

    cfg = workloads.get_config(args.config)
    iters = int(cfg["iters"])
    s = Solver(cfg)
    s.assemble()
    s.set_initial()
    torch.cuda.synchronize()
    n_sub = int(s.info.n_items)
    K = int(s.info.K_max)
    nT = int(s.n_steps)
    c0 = s.initial().clone()

    # exactly `iters` Schwarz iterations per window (tol < 0); the timed
    # windows replay the window captured as a HIP graph, a second pass over as
    # many windows records HIP events around every launch for the kernel times
    def window(graph):
        s.set_initial(c0)
        return s.run(k_max=iters, tol=-1.0, depth=args.depth, timing=not graph,
                     graph=graph and not args.no_graph)

    # the schedule (depth, transmission tile) by measurement, on this window,
    # or as given
    tuning = s.autotune(k_iters=iters) if args.depth == 0 else None
    if args.depth > 0 and args.tile > 0:
        s.set_schedule(args.depth, args.tile)
    for _ in range(args.warmup):
        window(True)
    torch.cuda.synchronize()
    runs = []
    t = time.perf_counter()
    for _ in range(args.steps):
        runs.append(window(True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    ms_step = 1e3 * wall / args.steps
    value = n_sub * iters * args.steps / wall
    truns = [window(False) for _ in range(args.steps)]
    torch.cuda.synchronize()

    kern = {k: dict(ms=sum(r["kernels"][k]["ms"] for r in truns) / args.steps,
                    launches=sum(r["kernels"][k]["launches"] for r in truns) / args.steps)
            for k in ("factor", "transmit", "recur", "residual")}
    # algorithmic work per window of each kernel class
    series = s.factor_terms() >= 0
    rec_series = s.rec_series()
    n_terms = s.factor_terms() + 1
    n_chunks = -(-nT // 128)
    inv_flops = n_sub * nT * 8.0 * K ** 3                    # complex Gauss-Jordan inverses
    inv_bytes = n_sub * nT * 16.0 * K * (K + 1) / 2          # symmetric inverses written
    # per (item, chunk): the anchor's inverse, its compensated residual and
    # refinement (8 K^3 each), G = i tau P_0 Q (4 K^3) and the further terms
    ser_flops = n_sub * n_chunks * (32.0 + 8.0 * (n_terms - 1)) * K ** 3
    # per (item, step): the symmetric inverse's K(K+1)/2 entries, f^{n+1}, c^{n+1}
    rec_bytes = iters * n_sub * nT * (16.0 * K * (K + 1) / 2 + 32.0 * K)
    # series evaluated in the step, per (item, step) and entry: S2 c (4
    # flops), Horner over the terms (4 per term after the first) and the
    # complex product (8)
    rec_flops = iters * n_sub * nT * (8.0 + 4.0 * n_terms) * K * K
    hist_bytes = n_sub * (nT + 1) * K * 16.0
    # Robin data (+ residual partials): read iterate and previous iterate, write f
    tx_bytes = (iters + 1) * 3.0 * hist_bytes
    if rec_series:
        factor_roof = dict(kernel="k_invert_mfma+k_series_residual+k_series_product",
                           bound="mfma", achieved=ser_flops / 1e12, peak=FP64_PEAK_TFS,
                           unit="TFLOP/s")
        recur_roof = dict(kernel="k_cn_recur_series", bound="alu", achieved=rec_flops / 1e12,
                          peak=FP64_VALU_PEAK_TFS, unit="TFLOP/s")
    else:
        factor_roof = (dict(kernel="k_series_assemble", bound="hbm", achieved=inv_bytes / 1e9,
                            peak=HBM_PEAK_GBS, unit="GB/s") if series else
                       dict(kernel="k_invert_mfma", bound="mfma", achieved=inv_flops / 1e12,
                            peak=FP64_PEAK_TFS, unit="TFLOP/s"))
        recur_roof = dict(kernel="k_cn_recur", bound="hbm", achieved=rec_bytes / 1e9,
                          peak=HBM_PEAK_GBS, unit="GB/s")
    roofs = {
        "factor": factor_roof,
        "recur": recur_roof,
        "transmit": dict(kernel="k_tx_send+k_tx_recv", bound="hbm", achieved=tx_bytes / 1e9,
                         peak=HBM_PEAK_GBS, unit="GB/s"),
        "residual": dict(kernel="k_res_reduce", bound="alu", achieved=None,
                         peak=None, unit=None),
    }
    digest = kernels_digest()
    for k, r in roofs.items():
        sec = kern[k]["ms"] * 1e-3
        r["achieved"] = r["achieved"] / sec if (sec > 0 and r["achieved"]) else None
        r["frac"] = r["achieved"] / r["peak"] if r["achieved"] else None
        r["ms_per_window"] = kern[k]["ms"]
        r["launches_per_window"] = kern[k]["launches"]
        m = MEASURED_TRAFFIC.get(r["kernel"])
        per = None
        if m and m["kernels_sha256"] == digest:
            per = m.get("bytes_per_launch_by_tile", {}).get(int(s.info.tx_tile),
                                                             m.get("bytes_per_launch"))
        r["traffic"] = per / 1e9 if per else None
    dom = max(roofs, key=lambda k: kern[k]["ms"])
    roofline = {k: v for k, v in roofs[dom].items() if k in
                ("kernel", "bound", "achieved", "peak", "unit", "frac", "traffic")}

    out = {
        "metric": "SWR sweep time & subdomain-solves/s; Schwarz iters to 1e-8, learned vs plain",
        "value": value,
        "unit": "subdomain-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: {cfg['n_elec']} electrons x {cfg['dim']}-D, "
                               f"{n_sub} subdomains, K={K} Gaussians each, {nT} Crank-Nicolson "
                               f"steps per window, {iters} Schwarz iterations per window",
                   "subdomains": n_sub, "K": K, "n_steps": nT, "schwarz_iters": iters,
                   "depth": int(s.info.depth_run) if args.depth == 0 else args.depth,
                   "tx_tile": int(s.info.tx_tile),
                   "autotuned": tuning is not None},
        "roofline": roofline,
        "factor_series_terms": s.factor_terms() + 1,
        "series_in_step": rec_series,
        "kernels_per_window": roofs,
        "windows_launched_as": "eager" if args.no_graph else "hip_graph",
        "sweep_ms_per_iteration": ms_step / iters,
        "last_residual": runs[-1]["res"][-1],
    }
    # the paper's own schedule: every Crank-Nicolson matrix refactored in
    # each sweep, one iterate at a time
    s.set_initial(c0)
    lit = s.run(k_max=3, tol=0.0, depth=1, timing=True)["kernels"]
    per_it = sum(lit[k]["ms"] for k in ("recur", "transmit", "residual")) / 3
    out["paper_literal_sweep_ms"] = lit["factor"]["ms"] + per_it
    out["wavefront_ms_per_iteration"] = ms_step / iters
    out["imaginary_time"] = tise_summary()
    out["slater_basis"] = slater_summary()
    out["local_slater_determinants"] = lsd_summary()
    out["local_slater_determinants_augmented"] = lsd_summary("paper-lsd-test-2b")
    out["local_orbitals_2d"] = lo_summary()
    if args.batched_iters > 0:
        del s
        torch.cuda.empty_cache()
        out["batched_wide_bases"] = batched_summary(args.batched_iters, cpu=not args.no_cpu)
    if args.c5_iters > 0:
        torch.cuda.empty_cache()
        out["four_dimensional"] = four_dimensional_summary(args.c5_iters, cpu=not args.no_cpu)
    if args.learned != "off":
        out["learned_warm_start"] = learned_summary(args.learned)
    if not args.no_cpu:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline_pool(cfg, iters, workers)
    copy_reference(args.copy_ref_mib)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
