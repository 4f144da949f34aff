"""Writes the oracle results the four-dimensional GPU tests compare with,
computed by the CPU oracle only (too slow to recompute inside the tests):

  c5_k16_window.json: plain SWR on the four-dimensional workload's 4^4
    decomposition with 2^4 Gaussians per subdomain (workload c5-k16, 10
    steps): Res(1..5) (Section 5 eq. residueRT) and the final iterate's
    coefficients at the last step of sampled subdomains;
  c5_iterate1.json: the full four-dimensional workload (c5-2e-2d, 6^4 =
    1296 Gaussians, 500 steps): iterate 1 (plain warm start) of sampled
    subdomains at selected steps (Section 4.4 step 2 Crank-Nicolson with the
    Robin data of Section 4.1), and sampled entries of their potential
    matrices (Section 5 eq. pseudo).

Run from the repository root:  python tests/golden/make_c5_fixtures.py [k16|full]
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import assemble, gauss1d  # noqa: E402
from oracle import swr as o_swr  # noqa: E402

K16_SAMPLES = [0, 85, 170, 255, 21, 106]   # corners and interior subdomains
FULL_TARGETS = [85, 0]                       # interior (1,1,1,1) and a corner
FULL_STEPS = [1, 250, 500]


def _c(v):
    return [[float(x.real), float(x.imag)] for x in np.asarray(v).ravel()]


def k16():
    cfg = workloads.get_config("c5-k16")
    prob = o_swr.Problem(cfg)
    h, res = o_swr.swr_window(prob, prob.initial_coeffs(), iters=cfg["iters"])
    out = dict(workload="c5-k16", iterations=cfg["iters"], residuals=[float(r) for r in res],
               samples={str(i): _c(h[i][-1]) for i in K16_SAMPLES},
               source="oracle.swr.swr_window (plain warm start, t0 = 0)")
    with open(os.path.join(HERE, "c5_k16_window.json"), "w") as f:
        json.dump(out, f)
    print(out["residuals"])


def _gram(s):
    return assemble.kron_all([gauss1d.overlap(s.alpha[k], s.delta[k], s.lo[k], s.hi[k])
                              for k in range(s.D)])


def full():
    cfg = workloads.get_config("c5-2e-2d")
    prob = o_swr.Problem(cfg)
    dec = prob.dec
    need = set(FULL_TARGETS)
    for i in FULL_TARGETS:
        need.update(prob.neighbours(i))
    # the neighbours' initial coefficients need only their Gram matrices
    c0 = {j: assemble.project_initial(dec, dec.subs[j], _gram(dec.subs[j])).astype(np.complex128)
          for j in sorted(need)}
    E = o_swr.field(cfg, prob.times(0.0))
    rng = np.random.default_rng(1296)
    out = dict(workload="c5-2e-2d", iterate=1, steps=FULL_STEPS, targets={},
               source="oracle.swr.local_cn with oracle.swr.forcing of the plain warm start")
    for i in FULL_TARGETS:
        sy = prob.sys[i]
        const = lambda j: np.repeat(c0[j][None, :], prob.n_T + 1, axis=0)
        f = o_swr.forcing(prob, i, const)
        hist = o_swr.local_cn(sy, c0[i], f, E, prob.dt)
        lm = rng.integers(0, sy.K, size=(64, 2))
        out["targets"][str(i)] = dict(
            c={str(n): _c(hist[n]) for n in FULL_STEPS},
            c0=_c(c0[i]),
            V=[[int(l), int(m), float(sy.V[l, m])] for l, m in lm])
        print("target", i, "done", flush=True)
    with open(os.path.join(HERE, "c5_iterate1.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "k16"
    (k16 if what == "k16" else full)()
