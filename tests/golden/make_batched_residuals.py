"""Writes batched_geometry0_residuals.json: the residual sequence Res(k),
k = 1..6 (Section 5 eq. (residueRT)), of plain SWR on geometry 0 of the
batched one-electron workload (256 subdomains with 32..256 Gaussians, 200
steps), computed by the CPU oracle only.  It takes several minutes, which is
why the values are stored; the GPU test compares the whole geometry's
residuals with them.

Run from the repository root:  python tests/golden/make_batched_residuals.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import swr as o_swr  # noqa: E402

ITERS = 6


def main():
    cfg = workloads.get_config("c3-1e-1d-batched")
    prob = o_swr.Problem(dict(cfg, nuclei=cfg["geometries"][0], geometries=None))
    _, res = o_swr.swr_window(prob, prob.initial_coeffs(), iters=ITERS)
    out = dict(workload="c3-1e-1d-batched", geometry=0, iterations=ITERS,
               residuals=[float(r) for r in res],
               source="oracle.swr.swr_window (plain warm start, t0 = 0)")
    with open(os.path.join(HERE, "batched_geometry0_residuals.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out["residuals"])


if __name__ == "__main__":
    main()
