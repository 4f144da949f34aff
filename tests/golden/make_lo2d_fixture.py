"""Writes the stored oracle result of the two-dimensional local orbital
window, computed by the CPU oracle only:

  lo_1e_2d_window.json  one electron in two dimensions, 4 x 4 boxes with the
                        16 lowest local orbitals of each box from its 8 x 8
                        Gaussians (Section 3 with d = 2), 200
                        Crank-Nicolson steps, plain warm start, 20 Schwarz
                        iterations: Res(k), k = 1..20 (Section 5 eq.
                        (residueRT)), and the coefficients of every box at
                        the last step of iterate 20 (Section 4.4 step 2),
                        with every box's Gram matrix A for the A-norm.

Building the orbitals takes a few minutes on one host thread, which is why
the values are stored; the GPU test runs the library's window against them.

Run from the repository root:  python tests/golden/make_lo2d_fixture.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import swr as o_swr  # noqa: E402

ITERS = 20


def main():
    cfg = workloads.get_config("lo-1e-2d")
    prob = o_swr.Problem(cfg)
    hist, res = o_swr.swr_window(prob, prob.initial_coeffs(), iters=ITERS)
    last = [h[cfg["n_steps"]] for h in hist]
    out = {
        "workload": cfg["name"], "iters": ITERS, "res": [float(r) for r in res],
        "last": [[[float(z.real), float(z.imag)] for z in c] for c in last],
        "A": [sy.A.tolist() for sy in prob.sys],
    }
    with open(os.path.join(HERE, "lo_1e_2d_window.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
