"""Writes config1_oracle.json, a stored record of the oracle on the config-1
workload (unit square, 32 x 32 cells x 2 triangles x 3 points = 6,144
points, 256 uniform targets, eps = 1e-2):

* dense J, gradient and per-point log-sum-exp at psi = 0 and at a seeded
  random psi (scale 0.01, seed 7);
* the geometric-cutoff evaluation (Eq. truncation_cutoff_geom, tau 1e-8)
  at the random psi.

The paper prints no per-instance values (its tables give times, iteration
counts and relative errors on its own meshes), so this file is a regression
record of the oracle and of the input generators, not a pin: the pins are
the closed forms, limits and library routines of tests/test_oracle_pins*.py.
Only the oracle and the generators are called here.

    python tests/golden/make_golden.py          (from the repository root)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2507_23602_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "config1_oracle.json")
L_STRIDE = 97   # stored per-point values: every 97th point


def compute():
    p = W.config1()
    rec = {"workload": p.name, "eps": p.eps, "n_quad": int(p.nq), "n_target": int(p.n),
           "psi_random": {"seed": 7, "scale": 0.01}, "L_stride": L_STRIDE}
    for tag, psi in (("zero", np.zeros(p.n)), ("random", W.random_psi(7, p.n, 0.01))):
        r = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps, want_L=True)
        rec[f"dense_{tag}"] = {"J": r.J, "grad": r.grad.tolist(),
                               "L": r.L[::L_STRIDE].tolist(), "kept": int(r.kept)}
    psi = W.random_psi(7, p.n, 0.01)
    absJ = abs(rec["dense_random"]["J"])
    C0 = oracle.covering_cost(p.x, p.y)
    C = oracle.cutoff_geom(C0, psi, p.nu, 1e-8, absJ, p.eps)
    r = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps, cutoff=C)
    rec["geom_random"] = {"tau": 1e-8, "C0": C0, "C": C, "J": r.J, "grad": r.grad.tolist(),
                          "kept": int(r.kept)}
    return rec


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(compute(), f, indent=1)
    print(f"wrote {OUT}")
