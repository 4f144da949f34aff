"""Benchmark of the SWR hot path on one MI355X.

A step is one SWR time window of the two-electron workload (2 electrons in
one dimension each, 8x8 overlapping subdomains, 8x8 Gaussians per subdomain,
1000 Crank-Nicolson steps, 20 Schwarz iterations), run by swr_run: the
factorisation of every local Crank-Nicolson matrix of the window, the plain
warm start, then 20 Schwarz iterations of local solves (recurrence),
transmission and residual, with P iterates in flight over chunks of the
window (depth P, 4 here).  Inputs (assembled matrices, initial coefficients)
are resident in HBM before the timed region.

value = subdomain-solves per second = subdomains x Schwarz iterations x
steps / seconds, where a subdomain-solve is one subdomain's whole-window
local solve in one Schwarz iteration.  Kernel durations come from HIP events
the library records around each launch on the run's stream.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def cpu_baseline(cfg, n_sample):
    """The oracle as it stands, one thread, on a bounded sample: one Schwarz
    iteration (plain warm start) of n_sample subdomains, including the Robin
    data each of them needs."""
    from threadpoolctl import threadpool_limits

    from oracle import swr as o_swr
    with threadpool_limits(limits=1):
        prob = o_swr.Problem(cfg)
        c0 = prob.initial_coeffs()
        const = o_swr.constant_history(prob, c0)
        E = o_swr.field(cfg, prob.times())
        items = list(range(n_sample))
        t = time.perf_counter()
        for i in items:
            f = o_swr.forcing(prob, i, lambda j: const[j])
            o_swr.local_cn(prob.sys[i], c0[i], f, E, prob.dt)
        dt = time.perf_counter() - t
    return dict(value=n_sample / dt, unit="subdomain-solves/s", cores=1, kind="oracle",
                sample=f"one Schwarz iteration of {n_sample} of the {prob.n_sub} subdomains "
                       f"({cfg['n_steps']} Crank-Nicolson steps each, Robin data included), "
                       f"NumPy/LAPACK FP64 on one host thread: {dt:.2f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2-2e-1d")
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--depth", type=int, default=0, help="iterates in flight (0: library choice)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_1710_02401_amd import Solver

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

    def window():
        s.set_initial(c0)
        return s.run(k_max=iters, tol=0.0, depth=args.depth, timing=True)

    for _ in range(args.warmup):
        window()
    torch.cuda.synchronize()
    runs = []
    t = time.perf_counter()
    for _ in range(args.steps):
        runs.append(window())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    ms_step = 1e3 * wall / args.steps
    value = n_sub * iters * args.steps / wall

    kern = {k: dict(ms=sum(r["kernels"][k]["ms"] for r in runs) / args.steps,
                    launches=sum(r["kernels"][k]["launches"] for r in runs) / args.steps)
            for k in ("factor", "transmit", "recur", "residual")}
    # algorithmic work per window of each kernel class
    inv_flops = n_sub * nT * 8.0 * K ** 3                    # complex Gauss-Jordan inverses
    rec_bytes = iters * n_sub * nT * (16.0 * K * K + 32.0 * K)   # inverse + f^{n+1} + c^{n+1}
    hist_bytes = n_sub * (nT + 1) * K * 16.0
    tx_bytes = (iters + 1) * 2.0 * hist_bytes                # read iterate, write Robin data
    res_bytes = iters * 2.0 * hist_bytes                     # read two iterates
    roofs = {
        "factor": dict(kernel="k_invert", bound="alu", achieved=inv_flops / 1e12,
                       peak=FP64_PEAK_TFS, unit="TFLOP/s"),
        "recur": dict(kernel="k_cn_recur", bound="hbm", achieved=rec_bytes / 1e9,
                      peak=HBM_PEAK_GBS, unit="GB/s"),
        "transmit": dict(kernel="k_tx_send+k_tx_recv", bound="hbm", achieved=tx_bytes / 1e9,
                         peak=HBM_PEAK_GBS, unit="GB/s"),
        "residual": dict(kernel="k_residual", bound="hbm", achieved=res_bytes / 1e9,
                         peak=HBM_PEAK_GBS, unit="GB/s"),
    }
    for k, r in roofs.items():
        sec = kern[k]["ms"] * 1e-3
        r["achieved"] = r["achieved"] / sec if sec > 0 else None
        r["frac"] = r["achieved"] / r["peak"] if r["achieved"] else None
        r["ms_per_window"] = kern[k]["ms"]
        r["launches_per_window"] = kern[k]["launches"]
        r["traffic"] = None
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
                   "depth": int(s.info.depth) if args.depth == 0 else args.depth},
        "roofline": roofline,
        "kernels_per_window": roofs,
        "sweep_ms_per_iteration": ms_step / iters,
        "last_residual": runs[-1]["res"][-1],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
