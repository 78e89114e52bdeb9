"""Pins of the oracle's plan moments and transport maps (Secs. 6.2, 6.3).

Each quantity is tied to something the oracle computes another way:
  * the target first moment sum_q mu_q p_qj x_q through Danskin's theorem
    (Eq. barycenter_gradient_general): at fixed psi, the derivative of -J in
    y_j is 2 cs (nu~_j y_j - first_j), checked by central differences of J;
  * the barycentric map through the derivative of the per-point log-sum-exp
    in x_q: T(x_q) = x_q + (eps / 2 cs) dL_q/dx_q, central differences of L_q;
  * both through the exchange of sums sum_q mu_q T(x_q) = sum_j nu~_j y_j and
    the totals sum_j first_j = sum_q mu_q x_q, sum_j nu~_j = sum_q mu_q;
  * the modal map through a brute-force argmax over the cost matrix, and the
    eps -> 0 limit in which the barycentric map collapses onto it;
  * the truncated versions through the tile rule's own gradient.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from paper_2507_23602_amd import workloads as W


def _problem(d, seed, n=9):
    rng = np.random.default_rng(seed)
    mesh = W.square_mesh(6) if d == 2 else W.cube_mesh(3)
    x, mu = W.quadrature(mesh, rng.uniform(0.5, 1.5, mesh.verts.shape[0]))
    y = rng.uniform(0.0, 1.0, (n, d))
    nu = rng.uniform(0.5, 1.5, n)
    nu /= nu.sum()
    psi = 0.02 * rng.standard_normal(n)
    return x, mu, y, nu, psi


@pytest.mark.parametrize("d,cs", [(2, 0.5), (3, 0.5), (2, 1.0)])
def test_first_moment_is_danskin_gradient(d, cs):
    x, mu, y, nu, psi = _problem(d, 50 + d)
    eps = 0.04
    mass, first = oracle.plan_moments(x, mu, y, nu, psi, eps, cost_scale=cs)
    h = 3e-6
    rng = np.random.default_rng(3)
    for j in range(y.shape[0]):
        e = rng.standard_normal(d)
        yp, ym = y.copy(), y.copy()
        yp[j] += h * e
        ym[j] -= h * e
        Jp = oracle.dual_eval(x, mu, yp, nu, psi, eps, cost_scale=cs, want_grad=False).J
        Jm = oracle.dual_eval(x, mu, ym, nu, psi, eps, cost_scale=cs, want_grad=False).J
        fd = -(Jp - Jm) / (2 * h)
        exact = 2 * cs * (mass[j] * y[j] - first[j]) @ e
        assert abs(fd - exact) <= 1e-8 * max(1e-3, abs(exact)), (j, fd, exact)


@pytest.mark.parametrize("d", [2, 3])
def test_barycentric_map_is_lse_derivative(d):
    x, mu, y, nu, psi = _problem(d, 60 + d)
    eps, cs = 0.05, 0.5
    bary, _, _ = oracle.transport_maps(x, y, nu, psi, eps)
    h = 1e-6
    for k in range(d):
        xp, xm = x.copy(), x.copy()
        xp[:, k] += h
        xm[:, k] -= h
        Lp = oracle.dual_eval(xp, mu, y, nu, psi, eps, want_grad=False, want_L=True).L
        Lm = oracle.dual_eval(xm, mu, y, nu, psi, eps, want_grad=False, want_L=True).L
        T = x[:, k] + eps / (2 * cs) * (Lp - Lm) / (2 * h)
        np.testing.assert_allclose(bary[:, k], T, rtol=0, atol=1e-7)


@pytest.mark.parametrize("d", [2, 3])
def test_moment_totals_and_exchange_of_sums(d):
    x, mu, y, nu, psi = _problem(d, 70 + d)
    eps = 0.03
    mass, first = oracle.plan_moments(x, mu, y, nu, psi, eps)
    bary, _, _ = oracle.transport_maps(x, y, nu, psi, eps)
    np.testing.assert_allclose(mass.sum(), mu.sum(), rtol=1e-14)
    np.testing.assert_allclose(first.sum(0), (mu[:, None] * x).sum(0), rtol=1e-13)
    np.testing.assert_allclose((mu[:, None] * bary).sum(0), (mass[:, None] * y).sum(0),
                               rtol=1e-13)
    # the target masses are the gradient plus nu (Eq. discretized_gradient)
    g = oracle.dual_eval(x, mu, y, nu, psi, eps).grad
    np.testing.assert_allclose(mass - nu, g, rtol=0, atol=1e-15)
    # one target: everything goes to it
    m1, f1 = oracle.plan_moments(x, mu, y[:1], np.ones(1), psi[:1], eps)
    np.testing.assert_allclose(f1[0], (mu[:, None] * x).sum(0), rtol=1e-14)
    b1, mo1, _ = oracle.transport_maps(x, y[:1], np.ones(1), psi[:1], eps)
    assert np.all(mo1 == 0) and np.allclose(b1, y[0], rtol=0, atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_modal_map_bruteforce_and_eps_limit(d):
    x, mu, y, nu, psi = _problem(d, 80 + d, n=13)
    eps = 1e-4
    bary, modal, val = oracle.transport_maps(x, y, nu, psi, eps)
    V = psi[None, :] - 0.5 * cdist(x, y, "sqeuclidean") + eps * np.log(nu)[None, :]
    np.testing.assert_array_equal(modal, np.argmax(V, axis=1))
    np.testing.assert_allclose(val, V.max(1), rtol=0, atol=1e-15)
    # eps -> 0: where the best target leads the second by >= 50 eps, the
    # barycentric map is that target to within e^-50
    Vs = np.sort(V, axis=1)
    clear = (Vs[:, -1] - Vs[:, -2]) >= 50 * eps
    assert clear.sum() > 0.8 * x.shape[0]
    np.testing.assert_allclose(bary[clear], y[modal[clear]], rtol=0, atol=1e-15)


def test_truncated_moments_follow_the_tile_rule():
    """With the keep matrix of the tile rule, the moments' masses are the tile
    rule's own gradient plus nu; an all-ones keep matrix is the dense plan."""
    x, mu, y, nu, psi = _problem(2, 90, n=40)
    eps = 1e-3
    # tiles and blocks: cells of a 3 x 3 and a 2 x 2 grid over the square
    tile_of = (np.minimum(2, (x[:, 0] * 3).astype(int)) * 3
               + np.minimum(2, (x[:, 1] * 3).astype(int))).astype(np.int32)
    block_of = (np.minimum(1, (y[:, 0] * 2).astype(int)) * 2
                + np.minimum(1, (y[:, 1] * 2).astype(int))).astype(np.int32)
    nt, nb = 9, 4
    J = oracle.dual_eval(x, mu, y, nu, psi, eps).J
    r = oracle.dual_eval_tile(x, mu, y, nu, psi, eps, tile_of, nt, block_of, nb, 1e-6, abs(J),
                              want_keep=True)
    assert 0 < r.keep.sum() < nt * nb
    mass, first = oracle.plan_moments(x, mu, y, nu, psi, eps, keep=(tile_of, block_of, r.keep))
    np.testing.assert_allclose(mass - nu, r.grad, rtol=0, atol=1e-15)
    ones = np.ones((nt, nb), dtype=np.uint8)
    m1, f1 = oracle.plan_moments(x, mu, y, nu, psi, eps, keep=(tile_of, block_of, ones))
    m0, f0 = oracle.plan_moments(x, mu, y, nu, psi, eps)
    np.testing.assert_array_equal(m1, m0)
    np.testing.assert_array_equal(f1, f0)
    b1, mo1, _ = oracle.transport_maps(x, y, nu, psi, eps, keep=(tile_of, block_of, ones))
    b0, mo0, _ = oracle.transport_maps(x, y, nu, psi, eps)
    np.testing.assert_array_equal(b1, b0)
    np.testing.assert_array_equal(mo1, mo0)


def test_cutoff_moments_follow_the_truncated_gradient():
    """With a cost cutoff C (Sec. 4.1) the moments' masses are the truncated
    evaluation's gradient plus nu, and the maps see only pairs with c < C."""
    x, mu, y, nu, psi = _problem(3, 91, n=30)
    eps, C = 0.01, 0.08
    r = oracle.dual_eval(x, mu, y, nu, psi, eps, cutoff=C)
    assert r.nempty == 0 and r.kept < x.shape[0] * y.shape[0]
    mass, _ = oracle.plan_moments(x, mu, y, nu, psi, eps, cutoff=C)
    np.testing.assert_allclose(mass - nu, r.grad, rtol=0, atol=1e-15)
    bary, modal, val = oracle.transport_maps(x, y, nu, psi, eps, cutoff=C)
    c = 0.5 * cdist(x, y, "sqeuclidean")
    V = np.where(c < C, psi[None, :] - c + eps * np.log(nu)[None, :], -np.inf)
    np.testing.assert_array_equal(modal, np.argmax(V, axis=1))
