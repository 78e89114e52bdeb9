"""Wasserstein barycentres by the damped Lloyd iteration (Sec. 6.2, Eqs.
barycenter_fixed_point and damped_lloyd) through the library: step for step
against the same loop run on the oracle's solver and plan moments, and at
convergence the invariants the equations fix (the points' mean is the
lambda-weighted mean of the sources, every point is a fixed point of the
update)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2507_23602_amd import workloads as W


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sources():
    y = np.zeros((1, 2))
    a = W.gaussian_blob_square(12, (0.3, 0.35), 0.10, y, 1.0)
    b = W.gaussian_blob_square(12, (0.7, 0.6), 0.12, y, 1.0)
    return [(a.x, a.mu), (b.x, b.mu)]


@pytest.mark.gpu
def test_damped_lloyd_matches_the_oracle_loop():
    """Three damped Lloyd steps (theta = 1/2, lambda = (0.3, 0.7), eps = 2e-2,
    24 points) through the library and through the oracle (strong-Wolfe
    L-BFGS to ||g||_1 <= 1e-11, then its plan moments): the same points after
    every step."""
    from paper_2507_23602_amd import barycenter
    src = _sources()
    lam = np.array([0.3, 0.7])
    eps, theta = 2e-2, 0.5
    y0 = W.uniform_targets(31, 24, 2) * 0.6 + 0.2
    ys = []
    y = y0.copy()
    for t in range(3):
        y, _ = barycenter.damped_lloyd(src, y, eps, lambdas=lam, theta=theta, tol=0.0,
                                       max_outer=1, solve_tol=1e-11)
        ys.append(y)
    # the oracle's loop
    yo = y0.copy()
    n = yo.shape[0]
    nu = np.full(n, 1.0 / n)
    for t in range(3):
        target = np.zeros_like(yo)
        for lm, (x, mu) in zip(lam, src):
            def fun(psi, x=x, mu=mu, yy=yo):
                r = oracle.dual_eval(x, mu, yy, nu, psi, eps)
                return r.J, r.grad
            psi, _, g, _, _ = oracle.lbfgs_solve(fun, np.zeros(n), tol=1e-11, line_search="wolfe")
            _, first = oracle.plan_moments(x, mu, yo, nu, psi, eps)
            target += lm * first / nu[:, None]
        yo = (1.0 - theta) * yo + theta * target
        err = float(np.max(np.abs(ys[t] - yo)))
        _say(f"  step {t + 1}: max |y_gpu - y_oracle| {err:.1e}")
        assert err < 1e-9


@pytest.mark.gpu
def test_barycentre_mean_and_fixed_point():
    """Run to convergence: the points' mean equals sum_i lambda_i E_mu_i[x]
    (each step maps the mean to (1 - theta) m + theta M, since every row of
    the plan sums to one), and the final points are a fixed point of the
    damped update up to the stopping tolerance."""
    import torch
    from paper_2507_23602_amd import barycenter, rsot
    src = _sources()
    lam = np.array([0.5, 0.5])
    eps = 2e-2
    y0 = W.uniform_targets(32, 32, 2) * 0.6 + 0.2
    y, log = barycenter.damped_lloyd(src, y0, eps, lambdas=lam, theta=0.5, tol=1e-7,
                                     max_outer=200, solve_tol=1e-10)
    _say(f"  {len(log)} iterations, {log[-1]['seconds']:.2f} s, last rel_dy "
         f"{log[-1]['rel_dy']:.1e}, J {log[0]['J']:.6f} -> {log[-1]['J']:.6f}")
    assert log[-1]["rel_dy"] <= 1e-7
    M = sum(lm * (mu[:, None] * x).sum(0) for lm, (x, mu) in zip(lam, src))
    assert np.max(np.abs(y.mean(0) - M)) < 1e-9
    # the fixed point, checked with the oracle's moments at the final points
    n = y.shape[0]
    nu = np.full(n, 1.0 / n)
    target = np.zeros_like(y)
    for lm, (x, mu) in zip(lam, src):
        prob = rsot.Problem(x, mu, y, nu, precision="fp64")
        psi, _ = prob.solve([eps], tol=1e-11)
        prob.close()
        _, first = oracle.plan_moments(x, mu, y, nu, psi, eps)
        target += lm * first / nu[:, None]
    res = float(np.max(np.abs(target - y)))
    _say(f"  fixed-point residual {res:.1e}")
    assert res < 1e-5


def test_damped_lloyd_rejects_bad_weights_and_damping():
    from paper_2507_23602_amd import barycenter
    src = [(np.zeros((3, 2)), np.full(3, 1 / 3))] * 2
    y0 = np.zeros((2, 2))
    with pytest.raises(ValueError):
        barycenter.damped_lloyd(src, y0, 1e-2, lambdas=[0.5, 0.6])
    with pytest.raises(ValueError):
        barycenter.damped_lloyd(src, y0, 1e-2, lambdas=[1.0])
    with pytest.raises(ValueError):
        barycenter.damped_lloyd(src, y0, 1e-2, theta=0.0)
