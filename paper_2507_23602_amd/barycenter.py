"""Entropy-regularized Wasserstein barycentres of K source measures, ordered
from library calls: the damped Lloyd iteration (Sec. 6.2, Eqs.
barycenter_fixed_point and damped_lloyd) with uniform masses, and the
general algorithm that also moves the masses (Alg. 3).

The barycentre is sought as N_b points y_j with fixed uniform masses
nu_j = 1 / N_b. Each outer iteration solves the regularised problem from every
source mu_i to the current points (Alg. 1, rsot_solve, warm-started from that
source's previous potential), takes the conditional barycentres
T_ij = (1 / nu_j) sum_q mu_q p_qj x_q from rsot_plan_moments, and moves every
point to y_j <- (1 - theta) y_j + theta sum_i lambda_i T_ij. Python holds the
loop and the stopping test; all arithmetic of the method runs in the library.
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


def damped_lloyd(sources, y0, eps, *, lambdas=None, theta=0.5, tol=1e-3, max_outer=200,
                 solve_tol=1e-8, cost_scale=0.5, precision="fp64", truncation="dense",
                 tau=1e-12):
    """Eq. damped_lloyd for sources = [(x_i, mu_i), ...] (points n_i x d,
    masses summing to 1) and initial points y0 (N_b x d), weights lambdas
    (default uniform, summing to 1), damping theta in (0, 1]. Stops when
    ||y_{t+1} - y_t||_2 <= tol ||y_t||_2 or after max_outer iterations.
    Returns (y, log), log a list of per-iteration records (the weighted
    objective sum_i lambda_i J_i at the solved potentials, the relative
    step, solver iterations)."""
    import torch
    k = len(sources)
    lam = np.full(k, 1.0 / k) if lambdas is None else np.asarray(lambdas, dtype=np.float64)
    if lam.shape != (k,) or np.any(lam < 0) or abs(lam.sum() - 1.0) > 1e-12:
        raise ValueError("lambdas must be k non-negative weights summing to 1")
    if not 0.0 < theta <= 1.0:
        raise ValueError("theta must lie in (0, 1]")
    y = np.ascontiguousarray(y0, dtype=np.float64)
    n = y.shape[0]
    nu = np.full(n, 1.0 / n)
    psis = [np.zeros(n) for _ in range(k)]
    log = []
    t0 = time.perf_counter()
    for it in range(max_outer):
        target = np.zeros_like(y)
        J = 0.0
        iters = []
        for i, (x, mu) in enumerate(sources):
            prob = rsot.Problem(x, mu, y, nu, cost_scale=cost_scale, precision=precision,
                                truncation=truncation, tau=tau)
            psi, info = _solve(prob, eps, psis[i], solve_tol)
            _, first, _, _ = prob.plan_moments(torch.as_tensor(psi, device="cuda"), eps)
            prob.close()
            psis[i] = psi
            target += lam[i] * first.cpu().numpy() / nu[:, None]
            J += lam[i] * info["J"]
            iters.append(info["iterations"])
        y_new = (1.0 - theta) * y + theta * target
        dy = float(np.linalg.norm(y_new - y) / np.linalg.norm(y))
        log.append({"iteration": it + 1, "J": J, "rel_dy": dy, "solve_iterations": iters,
                    "seconds": time.perf_counter() - t0})
        y = y_new
        if dy <= tol:
            break
    return y, log


def wasserstein_barycenter(sources, y0, nu0, eps, *, lambdas=None, alpha=1.0, beta=1.0,
                           tol_nu=1e-4, tol_y=1e-4, max_outer=200, solve_tol=1e-8,
                           cost_scale=0.5, precision="fp64", truncation="dense", tau=1e-12):
    """Alg. 3 for sources = [(x_i, mu_i), ...], initial points y0 (N x d) and
    masses nu0 (N, positive). Each outer iteration solves every source to the
    current (nu, y), then
      delta_nu = sum_i lambda_i grad_nu W(mu_i, nu),
      nu <- nu * exp(-alpha nu * delta_nu), nu <- nu / ||nu||_1,
      delta_y  = sum_i lambda_i grad_y W(mu_i, nu),
      y <- y - beta delta_y,
    with grad_nu W the solved potential in the gauge sum_j nu_j psi_j = 0 and
    grad_{y_j} W = 2 cs (nu~_j y_j - sum_q mu_q p_qj x_q)
    (Danskin, Eq. barycenter_gradient_general). Both gradients are taken at
    the masses and points of the solve. Stops once ||delta_nu||_2 <=
    tol_nu ||nu||_2 and ||delta_y||_2 <= tol_y ||y||_2 (the algorithm's two
    tests), or after max_outer iterations. Returns (y, nu, log)."""
    import torch
    k = len(sources)
    lam = np.full(k, 1.0 / k) if lambdas is None else np.asarray(lambdas, dtype=np.float64)
    if lam.shape != (k,) or np.any(lam < 0) or abs(lam.sum() - 1.0) > 1e-12:
        raise ValueError("lambdas must be k non-negative weights summing to 1")
    y = np.ascontiguousarray(y0, dtype=np.float64)
    nu = np.asarray(nu0, dtype=np.float64).copy()
    if nu.shape != (y.shape[0],) or not np.all(nu > 0):
        raise ValueError("nu0 must hold one positive mass per point")
    nu /= nu.sum()
    psis = [np.zeros(y.shape[0]) for _ in range(k)]
    log = []
    t0 = time.perf_counter()
    for it in range(max_outer):
        dnu = np.zeros_like(nu)
        dy = np.zeros_like(y)
        J = 0.0
        for i, (x, mu) in enumerate(sources):
            prob = rsot.Problem(x, mu, y, nu, cost_scale=cost_scale, precision=precision,
                                truncation=truncation, tau=tau)
            psi, info = _solve(prob, eps, psis[i], solve_tol)
            mass, first, _, _ = prob.plan_moments(torch.as_tensor(psi, device="cuda"), eps)
            prob.close()
            psis[i] = psi
            dnu += lam[i] * (psi - nu.dot(psi))         # the gauge sum_j nu_j psi_j = 0
            dy += lam[i] * 2.0 * cost_scale * (mass.cpu().numpy()[:, None] * y
                                               - first.cpu().numpy())
            J += lam[i] * info["J"]
        rnu = float(np.linalg.norm(dnu) / np.linalg.norm(nu))
        ry = float(np.linalg.norm(dy) / np.linalg.norm(y))
        nu = nu * np.exp(-alpha * nu * dnu)
        nu /= nu.sum()
        y = y - beta * dy
        log.append({"iteration": it + 1, "J": J, "rel_dnu": rnu, "rel_dy": ry,
                    "seconds": time.perf_counter() - t0})
        if rnu <= tol_nu and ry <= tol_y:
            break
    return y, nu, log
