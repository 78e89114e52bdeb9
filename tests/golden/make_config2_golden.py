"""Writes config2_oracle.npz: the oracle's dense J and full gradient on the 3D
benchmark workload (unit cube, 64^3 cells x 6 tetrahedra x 4 points =
6,291,456 points, 65,536 mixture targets, eps = 1e-3) at the seeded potential
psi ~ N(0, eps^2) (seed 11), plus L_q at 4,096 seeded points.

A dense oracle pass at this size takes minutes on a many-core host, too long
for a GPU test, so its result is stored here; only the oracle and the input
generators are called. Like config1_oracle.json it is a record of the oracle
(which tests/test_oracle_pins*.py pin), not of the paper, which prints no
per-instance values.

    python tests/golden/make_config2_golden.py   (from the repository root)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2507_23602_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "config2_oracle.npz")
PSI_SEED = 11
L_SAMPLE_SEED, L_SAMPLE = 4, 4096


def compute():
    p = W.config2()
    psi = W.random_psi(PSI_SEED, p.n, p.eps)
    t0 = time.time()
    r = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps)
    idx = np.sort(np.random.default_rng(L_SAMPLE_SEED).choice(p.nq, L_SAMPLE, replace=False))
    rl = oracle.dual_eval(p.x[idx], p.mu[idx], p.y, p.nu, psi, p.eps, want_grad=False,
                          want_L=True)
    print(f"oracle pass {time.time() - t0:.0f} s", flush=True)
    return dict(workload=p.name, eps=p.eps, psi_seed=PSI_SEED, J=r.J, grad=r.grad,
                L_index=idx, L=rl.L, kept=r.kept)


if __name__ == "__main__":
    rec = compute()
    np.savez_compressed(OUT, **rec)
    print(f"wrote {OUT}")
