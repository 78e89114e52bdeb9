"""Blue-noise sampling on the unit sphere by Lloyd's algorithm with
Riemannian barycentres (Sec. 6.4, Algs. 4-5), ordered from library calls.

Each outer iteration solves the regularised problem for the current points
(Alg. 1, rsot_solve, warm-started from the previous potential) and then moves
every point to the Riemannian barycentre of its conditional measure by
repeated rsot_sphere_karcher_step calls (Alg. 5; the conditional measures of
that solve are held fixed). Python holds the loop and the stopping tests; all
arithmetic of the method runs in the library.
"""
from __future__ import annotations

import time

import numpy as np

from . import rsot


def _solve(prob, eps, psi0, tol):
    """rsot_solve from psi0; a line search that cannot improve the iterate
    at the pair loop's precision (RSOT_ERR_LINESEARCH) returns its best
    iterate, which the outer iteration uses like any other solution"""
    try:
        return prob.solve([eps], psi0=psi0, tol=tol)
    except rsot.RsotError as e:
        if e.code != rsot.ERR_LINESEARCH or e.psi is None:
            raise
        return e.psi, e.info


def lloyd(x, mu, y0, eps, *, nu=None, cost_scale=1.0, tol=1e-3, max_outer=200,
          inner_tol=1e-9, max_inner=50, alpha=0.5, solve_tol=1e-8, precision="fp64",
          truncation="dense", tau=1e-12):
    """Alg. 4 on the unit sphere with c = cost_scale d_g^2: returns (y, log),
    y the final points (n x 3), log a list of per-iteration records. Stops
    when ||y_{t+1} - y_t||_2 <= tol ||y_t||_2 (the algorithm's test) or after
    max_outer iterations. The inner Riemannian-barycentre loop (Alg. 5) stops
    when every step's Riemannian norm is below inner_tol."""
    import torch
    y = np.ascontiguousarray(y0, dtype=np.float64)
    n = y.shape[0]
    nu = np.full(n, 1.0 / n) if nu is None else np.asarray(nu, dtype=np.float64)
    psi = np.zeros(n)
    log = []
    t0 = time.perf_counter()
    for it in range(max_outer):
        prob = rsot.Problem(x, mu, y, nu, cost="sphere", cost_scale=cost_scale,
                            precision=precision, truncation=truncation, tau=tau)
        psi, info = _solve(prob, eps, psi, solve_tol)
        yc = torch.as_tensor(y, device="cuda")
        inner = 0
        for inner in range(1, max_inner + 1):
            yn, step, _, _ = prob.sphere_karcher_step(psi, eps, yc, alpha=alpha)
            yc = yn
            if float(step.max().item()) <= inner_tol:
                break
        prob.close()
        y_new = yc.cpu().numpy()
        dy = float(np.linalg.norm(y_new - y) / np.linalg.norm(y))
        log.append({"iteration": it + 1, "solve_iterations": info["iterations"],
                    "karcher_steps": inner, "rel_dy": dy, "J": info["J"],
                    "seconds": time.perf_counter() - t0})
        y = y_new
        if dy <= tol:
            break
    return y, log


def pairwise_angles(y):
    """Sorted great-circle distances between all pairs of points."""
    c = np.clip(y @ y.T, -1.0, 1.0)
    iu = np.triu_indices(y.shape[0], 1)
    return np.sort(np.arccos(c[iu]))
