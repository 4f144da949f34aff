"""Writes the stored oracle results of the two headline windows, computed by
the CPU oracle only:

  c2_window.json       the two-electron real-time window (64 subdomains of
                       8 x 8 Gaussians, 1000 Crank-Nicolson steps, plain warm
                       start, 20 Schwarz iterations): Res(k), k = 1..20
                       (Section 5 eq. (residueRT)), and the coefficients of
                       every subdomain at the last step of iterate 20
                       (Section 4.4 step 2).
  c2_tise_window.json  the imaginary-time window of the same decomposition
                       (400 normalised implicit-Euler steps per iteration,
                       Section 4.2 eq. (SIT)): Res(k), the energy after each
                       iteration, and the coefficients of every subdomain at
                       the last step of iterate 20.

Each takes about a minute or two on one host thread, which is why the values
are stored; the GPU tests run the benchmark's own launch path against them.

Run from the repository root:  python tests/golden/make_headline_fixtures.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import swr as o_swr  # noqa: E402
from oracle import tise as o_tise  # noqa: E402

ITERS = 20


def _pairs(v):
    v = np.asarray(v)
    if np.iscomplexobj(v):
        return [[float(z.real), float(z.imag)] for z in v]
    return [float(x) for x in v]


def real_time():
    cfg = workloads.get_config("c2-2e-1d")
    prob = o_swr.Problem(cfg)
    hists, res = o_swr.swr_window(prob, prob.initial_coeffs(), iters=ITERS)
    out = dict(workload="c2-2e-1d", iterations=ITERS, step=int(prob.n_T),
               residuals=[float(r) for r in res],
               final={str(i): _pairs(h[-1]) for i, h in enumerate(hists)},
               source="oracle.swr.swr_window (plain warm start, t0 = 0)")
    with open(os.path.join(HERE, "c2_window.json"), "w") as f:
        json.dump(out, f)
    print("real time", out["residuals"][:3], "...", out["residuals"][-1], flush=True)


def imaginary_time():
    cfg = workloads.get_config("c2-2e-1d-tise")
    prob = o_swr.Problem(cfg)
    hists, res, energies = o_tise.swr_tise(prob, iters=ITERS)
    out = dict(workload="c2-2e-1d-tise", iterations=ITERS, step=int(prob.n_T),
               residuals=[float(r) for r in res], energies=[float(e) for e in energies],
               final={str(i): _pairs(np.real(h[-1])) for i, h in enumerate(hists)},
               source="oracle.tise.swr_tise (plain warm start)")
    with open(os.path.join(HERE, "c2_tise_window.json"), "w") as f:
        json.dump(out, f)
    print("imaginary time", out["energies"][-1], out["residuals"][-1], flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["real", "imaginary"]
    if "real" in which:
        real_time()
    if "imaginary" in which:
        imaginary_time()
