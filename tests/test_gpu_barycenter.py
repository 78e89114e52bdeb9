"""Wasserstein barycentres through the library: the damped Lloyd iteration
(Sec. 6.2, Eqs. barycenter_fixed_point and damped_lloyd) and the general
algorithm with mass updates (Alg. 3), step for step against the same loops
run on the oracle's solver and plan moments; at convergence the invariants
the equations fix (the points' mean is the lambda-weighted mean of the
sources, every point is a fixed point of the update); Alg. 3 without mass
steps reduces to the damped Lloyd step."""
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


def _oracle_alg3_step(src, lam, y, nu, eps, alpha, beta, cs=0.5):
    n = y.shape[0]
    dnu = np.zeros(n)
    dy = np.zeros_like(y)
    for lm, (x, mu) in zip(lam, src):
        def fun(psi, x=x, mu=mu):
            r = oracle.dual_eval(x, mu, y, nu, psi, eps)
            return r.J, r.grad
        psi, _, _, _, _ = oracle.lbfgs_solve(fun, np.zeros(n), tol=1e-11, line_search="wolfe")
        psi = psi - nu.dot(psi)
        mass, first = oracle.plan_moments(x, mu, y, nu, psi, eps)
        dnu += lm * psi
        dy += lm * 2.0 * cs * (mass[:, None] * y - first)
    nu = nu * np.exp(-alpha * nu * dnu)
    return y - beta * dy, nu / nu.sum()


@pytest.mark.gpu
def test_alg3_matches_the_oracle_loop():
    """Three steps of Alg. 3 (mass step alpha = 40, point step beta = 4,
    lambda = (0.3, 0.7), eps = 2e-2, 24 points with uneven masses) through the
    library and through the oracle: the same points and masses after every
    step, masses positive and summing to one."""
    from paper_2507_23602_amd import barycenter
    src = _sources()
    lam = np.array([0.3, 0.7])
    eps, alpha, beta = 2e-2, 40.0, 4.0
    y = W.uniform_targets(34, 24, 2) * 0.6 + 0.2
    nu = np.random.default_rng(35).uniform(0.5, 1.5, 24)
    nu /= nu.sum()
    yo, nuo = y.copy(), nu.copy()
    for t in range(3):
        y, nu, _ = barycenter.wasserstein_barycenter(src, y, nu, eps, lambdas=lam, alpha=alpha,
                                                     beta=beta, tol_nu=0.0, tol_y=0.0,
                                                     max_outer=1, solve_tol=1e-11)
        yo, nuo = _oracle_alg3_step(src, lam, yo, nuo, eps, alpha, beta)
        ey, en = float(np.max(np.abs(y - yo))), float(np.max(np.abs(nu - nuo) / nuo))
        _say(f"  step {t + 1}: max |y - y_oracle| {ey:.1e}, max rel |nu - nu_oracle| {en:.1e}")
        assert ey < 1e-9 and en < 1e-9
        assert np.all(nu > 0) and abs(nu.sum() - 1.0) < 1e-14


@pytest.mark.gpu
def test_alg3_without_mass_steps_is_the_damped_lloyd_step():
    """With alpha = 0 the masses stay uniform, and with beta = theta N / (2 cs)
    the point step y - beta 2 cs (nu~ y - first) is the damped Lloyd step
    (1 - theta) y + theta first / nu (nu~ = nu at the solve's tolerance)."""
    from paper_2507_23602_amd import barycenter
    src = _sources()
    y0 = W.uniform_targets(36, 20, 2) * 0.6 + 0.2
    n = y0.shape[0]
    theta, eps = 0.5, 2e-2
    ya, nua, _ = barycenter.wasserstein_barycenter(src, y0, np.ones(n), eps, alpha=0.0,
                                                   beta=theta * n / (2 * 0.5), tol_nu=0.0,
                                                   tol_y=0.0, max_outer=1, solve_tol=1e-11)
    yb, _ = barycenter.damped_lloyd(src, y0, eps, theta=theta, tol=0.0, max_outer=1,
                                    solve_tol=1e-11)
    err = float(np.max(np.abs(ya - yb)))
    _say(f"  alg3 (alpha 0) vs damped Lloyd: {err:.1e}")
    assert np.allclose(nua, 1.0 / n, rtol=1e-14, atol=0.0)
    assert err < 1e-9


def test_alg3_rejects_bad_masses():
    from paper_2507_23602_amd import barycenter
    src = [(np.zeros((3, 2)), np.full(3, 1 / 3))]
    y0 = np.zeros((2, 2))
    with pytest.raises(ValueError):
        barycenter.wasserstein_barycenter(src, y0, np.array([1.0, 0.0]), 1e-2)
    with pytest.raises(ValueError):
        barycenter.wasserstein_barycenter(src, y0, np.ones(3), 1e-2)
