"""Pins of the oracle's squared-geodesic-cost functions on the unit sphere
(Sec. 6.4, Algs. 4-5) against closed forms, identities of the log and exp
maps, finite differences and brute force (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from paper_2507_23602_amd import workloads as W


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def test_cost_values_through_one_target():
    """One target (nu = 1, psi = 0): J = -sum_q mu_q c(x_q, y). Points at
    angles 0, pi/2 and pi from y give c = 0, (pi/2)^2, pi^2 (cost_scale 1);
    the chord |x - y|^2 would give 0, 2, 4."""
    y = _unit([0.2, -0.4, 0.9])
    o = _unit(np.cross(y, [1.0, 0.0, 0.0]))
    x = np.stack([y, o, -y])
    mu = np.full(3, 1.0 / 3.0)
    r = oracle.dual_eval_sphere(x, mu, y[None], np.ones(1), np.zeros(1), 0.05)
    assert r.J == pytest.approx(-(0.0 + (math.pi / 2) ** 2 + math.pi ** 2) / 3.0, rel=1e-14)
    r2 = oracle.dual_eval_sphere(x, mu, y[None], np.ones(1), np.zeros(1), 0.05, cost_scale=0.5)
    assert r2.J == pytest.approx(0.5 * r.J, rel=1e-14)


def test_uniform_sphere_closed_form_converges():
    """Uniform measure on the sphere, one target: -J = E[d_g^2] = (pi^2 - 4)/2
    for any target (the angle has density sin(theta)/2 on [0, pi]); the
    icosphere quadrature converges to it at O(h^2)."""
    exact = (math.pi ** 2 - 4.0) / 2.0
    y = _unit([0.3, 0.5, 0.8])[None]
    errs = []
    for k in (3, 4, 5):
        x, mu = W.sphere_quadrature(k, "uniform")
        r = oracle.dual_eval_sphere(x, mu, y, np.ones(1), np.zeros(1), 0.01)
        errs.append(abs(-r.J - exact))
    assert errs[-1] < 5e-7
    assert errs[2] < errs[1] < errs[0]
    assert errs[1] / errs[2] > 2.5                    # h halves: error / 4


def _small(seed=1, k=2, n=40, eps=0.05):
    x, mu = W.sphere_quadrature(k, "harmonic")
    y = W.sphere_points(seed, n)
    nu = np.random.default_rng(seed).uniform(0.5, 1.5, n)
    nu /= nu.sum()
    psi = np.random.default_rng(seed + 1).normal(0.0, eps, n)
    return x, mu, y, nu, psi, eps


def test_gradient_finite_differences_and_conservation():
    x, mu, y, nu, psi, eps = _small()
    r = oracle.dual_eval_sphere(x, mu, y, nu, psi, eps)
    assert abs(r.grad.sum() - (mu.sum() - nu.sum())) < 1e-14
    h = 1e-6
    for j in (0, 7, 23):
        e = np.zeros_like(psi)
        e[j] = h
        fd = (oracle.dual_eval_sphere(x, mu, y, nu, psi + e, eps).J -
              oracle.dual_eval_sphere(x, mu, y, nu, psi - e, eps).J) / (2 * h)
        assert abs(fd - r.grad[j]) < 1e-8


def test_small_angles_match_the_euclidean_cost():
    """Targets and points in a small cap: the geodesic and chord distances
    agree to O(theta^4), so J matches the squared Euclidean evaluation."""
    rng = np.random.default_rng(5)
    c = _unit([0.1, 0.2, 1.0])
    x = np.array([_unit(c + 1e-3 * rng.standard_normal(3)) for _ in range(200)])
    y = np.array([_unit(c + 1e-3 * rng.standard_normal(3)) for _ in range(20)])
    mu = np.full(200, 1 / 200)
    nu = np.full(20, 1 / 20)
    psi = rng.normal(0, 1e-7, 20)
    a = oracle.dual_eval_sphere(x, mu, y, nu, psi, 1e-6, cost_scale=0.5)
    b = oracle.dual_eval(x, mu, y, nu, psi, 1e-6, cost_scale=0.5)
    assert abs(a.J - b.J) < 1e-12


def test_karcher_step_lands_on_a_single_point():
    """One source point x0 and one target: the conditional measure is the
    Dirac at x0, delta = -2 log_y(x0), and with alpha = 1/2 the step goes
    exp_y(log_y(x0)) = x0 (sign, scale and the two maps together)."""
    x0 = _unit([0.6, -0.2, 0.3])
    for yc in (_unit([0.0, 0.0, 1.0]), _unit([-0.5, 0.8, 0.1]), _unit([0.6, -0.2, 0.31])):
        yn, step, mass = oracle.sphere_karcher_step(x0[None], np.ones(1), yc[None], np.ones(1),
                                                    np.zeros(1), 0.1, yc[None], alpha=0.5)
        np.testing.assert_allclose(yn[0], x0, atol=1e-13)
        th = math.acos(np.clip(x0 @ yc, -1, 1))
        assert step[0] == pytest.approx(2 * th, rel=1e-12) and mass[0] == pytest.approx(1.0)


def test_karcher_step_is_the_riemannian_gradient():
    """delta_j is the tangent gradient of the expected squared distance under
    the conditional measure: <delta, u> equals the derivative of
    sum_q w_q d_g(x_q, exp_y(t u))^2 / sum_q w_q at t = 0 along tangent
    directions u (finite differences)."""
    x, mu, _, _, _, _ = _small(k=2)
    y = _unit([0.3, 0.4, 0.5])
    yn, step, mass = oracle.sphere_karcher_step(x, mu, y[None], np.ones(1), np.zeros(1), 0.1,
                                                y[None], alpha=1e-3)
    # recover delta from the small step: y_next = exp_y(-alpha delta)
    alpha = 1e-3
    v = yn[0] - y * math.cos(alpha * step[0])
    delta = -v / math.sin(alpha * step[0]) * step[0]

    def F(yy):
        c = np.clip(x @ yy, -1, 1)
        return float((mu * np.arccos(c) ** 2).sum() / mu.sum())
    e1 = _unit(np.cross(y, [1.0, 0.0, 0.0]))
    e2 = np.cross(y, e1)
    h = 1e-6
    for u in (e1, e2):
        yp = math.cos(h) * y + math.sin(h) * u
        ym = math.cos(h) * y - math.sin(h) * u
        fd = (F(yp) - F(ym)) / (2 * h)
        assert abs(fd - delta @ u) < 1e-7


def test_karcher_iteration_finds_the_geodesic_midpoint():
    """Two source points of equal mass, one target: the Riemannian
    barycentre is the midpoint of the geodesic between them,
    (x1 + x2) / |x1 + x2|; steps with alpha = 1/2 reach it."""
    x1, x2 = _unit([1.0, 0.2, 0.1]), _unit([0.1, 1.0, -0.3])
    xs, mu = np.stack([x1, x2]), np.array([0.5, 0.5])
    y = _unit([0.0, 0.0, 1.0])
    for _ in range(60):
        yn, step, _ = oracle.sphere_karcher_step(xs, mu, y[None], np.ones(1), np.zeros(1), 0.1,
                                                 y[None], alpha=0.5)
        y = yn[0]
    np.testing.assert_allclose(y, _unit(x1 + x2), atol=1e-10)
    assert step[0] < 1e-9


def test_tile_rule_on_the_sphere_bounds_the_objective():
    """The geodesic tile rule: J_dense - J_trunc lies in [0, tau |J_ref|]
    (App. B's chain with the geodesic bounds of the boxes) and it drops
    pairs, at tau = 1e-6 and 1e-12."""
    x, mu = W.sphere_quadrature(3, "harmonic")
    y = W.sphere_points(9, 300)
    nu = np.full(300, 1 / 300)
    eps = 2e-3
    psi = np.random.default_rng(2).normal(0, eps, 300)
    order_x = np.argsort(np.floor((x[:, 2] + 1) * 8) * 64 + np.floor((np.arctan2(x[:, 1], x[:, 0]) + 4) * 8),
                         kind="stable")
    tile_of = np.empty(x.shape[0], dtype=np.int32)
    tile_of[order_x] = np.arange(x.shape[0]) // 64
    order_y = np.argsort(np.floor((y[:, 2] + 1) * 4) * 64 + np.floor((np.arctan2(y[:, 1], y[:, 0]) + 4) * 4),
                         kind="stable")
    block_of = np.empty(300, dtype=np.int32)
    block_of[order_y] = np.arange(300) // 16
    nt, nb = int(tile_of.max()) + 1, int(block_of.max()) + 1
    dense = oracle.dual_eval_sphere(x, mu, y, nu, psi, eps)
    for tau in (1e-6, 1e-12):
        r = oracle.dual_eval_tile_sphere(x, mu, y, nu, psi, eps, tile_of, nt, block_of, nb, tau,
                                         abs(dense.J), want_keep=True)
        assert 0 < r.kept < x.shape[0] * 300
        assert -1e-13 * abs(dense.J) <= dense.J - r.J <= tau * abs(dense.J)
