"""Two-sided pins of the oracle's truncation quantities (Sec. 4.1, App. B).

The cutoffs of Eqs. truncation_cutoff_geom and truncation_cutoff_int are upper
bounds of the cost at which the neglected part of J reaches tau |J|. On a
configuration whose truncation error has a closed form the exact cutoff C*
is known without the paper's formulas, and App. B's chain loses only the
factor (1 - a) (targets outside the cut carry mass 1 - a, the bound uses 1)
and the step ln(1 + z) <= z. So the oracle's cutoff must lie in the window

    C* <= C <= C* + eps ln(1/(1 - a)) + tau |J|.

A cutoff that is too small (a dropped term, a sign error) fails the left
side; one that is too large (a missing eps factor, exp(+L) in D) fails the
right. D itself (the integrated inverse of the truncated sum) is pinned by
its shift rule and by an erfi closed form on the unit square.
"""
import math

import numpy as np
import pytest
from scipy.special import erfi

import oracle
from paper_2507_23602_amd import workloads as W


def _ring_problem(c_near, psi_near, a, c_ring, psi_ring, K=16):
    """One quadrature point at the origin (mu = 1) in 2D. Target 0 at cost
    c_near with mass a and potential psi_near; K targets on a circle at cost
    c_ring, each with mass (1 - a)/K and potential psi_ring."""
    x = np.zeros((1, 2))
    mu = np.ones(1)
    r0 = math.sqrt(2.0 * c_near)
    r1 = math.sqrt(2.0 * c_ring)
    ang = 2.0 * math.pi * (np.arange(K) + 0.25) / K
    y = np.vstack([[r0, 0.0], np.stack([r1 * np.cos(ang), r1 * np.sin(ang)], 1)])
    nu = np.concatenate([[a], np.full(K, (1.0 - a) / K)])
    psi = np.concatenate([[psi_near], np.full(K, psi_ring)])
    return x, mu, y, nu, psi


def _exact_cutoff(c_near, dpsi, a, tau_absJ, eps):
    """Cost c* of the ring at which the truncation error
    eps ln(1 + ((1 - a)/a) exp((dpsi + c_near - c*)/eps)) equals tau |J|
    (dpsi = psi_ring - psi_near): the exact cutoff of this configuration."""
    u = tau_absJ / eps
    return c_near + dpsi + eps * math.log((1.0 - a) / (a * math.expm1(u)))


CASES = [  # (eps, tau, a, c_near, psi_near, psi_ring)
    (1e-2, 1e-4, 1e-3, 0.02, 0.0, 0.0),
    (1e-3, 1e-8, 1e-3, 0.005, 0.01, 0.01),
    (5e-2, 1e-6, 2e-3, 0.1, -0.3, -0.3),
    (2e-3, 1e-12, 1e-3, 0.001, 0.0, 0.02),
    (1e-2, 1e-4, 1e-3, 0.02, -0.05, 0.03),
]


@pytest.mark.parametrize("eps,tau,a,c_near,psi_near,psi_ring", CASES)
def test_geometric_cutoff_window(eps, tau, a, c_near, psi_near, psi_ring):
    """Eq. truncation_cutoff_geom: the nearest target (mass a = nu_min,
    potential m) sits at the covering cost, the rest (potential M) outside
    the cut. C_geom must bracket the exact cutoff within the window."""
    M, m = max(psi_near, psi_ring), min(psi_near, psi_ring)
    if psi_near != m:
        pytest.skip("configuration needs the near target at the lowest potential")
    c_far = c_near + (M - m) + 40 * eps
    x, mu, y, nu, psi = _ring_problem(c_near, psi_near, a, c_far, psi_ring)
    dense = oracle.dual_eval(x, mu, y, nu, psi, eps)
    absJ = abs(dense.J)
    C0 = oracle.covering_cost(x, y)
    assert abs(C0 - c_near) <= 1e-15 + 1e-12 * c_near
    C = oracle.cutoff_geom(C0, psi, nu, tau, absJ, eps)
    Cs = _exact_cutoff(c_near, psi_ring - psi_near, a, tau * absJ, eps)
    assert Cs <= C <= Cs + eps * math.log(1.0 / (1.0 - a)) + tau * absJ, (C, Cs)
    # with the ring placed just outside the cut the truncation error is
    # nearly tau |J|, and never above it
    x, mu, y, nu, psi = _ring_problem(c_near, psi_near, a, C * (1 + 1e-9) + 1e-15, psi_ring)
    dense = oracle.dual_eval(x, mu, y, nu, psi, eps)
    tr = oracle.dual_eval(x, mu, y, nu, psi, eps, cutoff=C)
    assert tr.kept == 1
    E = dense.J - tr.J
    assert 0.9 * (1 - a) * tau * absJ <= E <= tau * absJ * (1 + 1e-6)


@pytest.mark.parametrize("eps,tau,a,c_near,psi_near,psi_ring", CASES)
def test_integral_cutoff_window(eps, tau, a, c_near, psi_near, psi_ring):
    """Eq. truncation_cutoff_int with D from a truncated evaluation that
    excludes the ring: C_int must bracket the exact cutoff (which only needs
    the ring's potential to be the maximum M)."""
    M = max(psi_near, psi_ring)
    if psi_ring != M:
        pytest.skip("configuration needs the ring at the highest potential")
    c_far = c_near + abs(psi_ring - psi_near) + 40 * eps
    x, mu, y, nu, psi = _ring_problem(c_near, psi_near, a, c_far, psi_ring)
    dense = oracle.dual_eval(x, mu, y, nu, psi, eps)
    absJ = abs(dense.J)
    C0 = oracle.covering_cost(x, y)
    tr = oracle.dual_eval(x, mu, y, nu, psi, eps, cutoff=0.5 * (c_near + c_far), want_L=True)
    assert tr.kept == 1
    D = oracle.integral_D(mu, tr.L)
    # one point, one kept target: D = 1 / (a exp((psi_near - c_near)/eps))
    assert abs(D * a * math.exp((psi_near - c_near) / eps) - 1.0) < 1e-13
    C = oracle.cutoff_int(C0, psi, D, tau, absJ, eps)
    Cs = _exact_cutoff(c_near, psi_ring - psi_near, a, tau * absJ, eps)
    assert Cs <= C <= Cs + eps * math.log(1.0 / (1.0 - a)) + tau * absJ, (C, Cs)
    x, mu, y, nu, psi = _ring_problem(c_near, psi_near, a, C * (1 + 1e-9) + 1e-15, psi_ring)
    dense = oracle.dual_eval(x, mu, y, nu, psi, eps)
    tr = oracle.dual_eval(x, mu, y, nu, psi, eps, cutoff=C)
    E = dense.J - tr.J
    assert 0.9 * (1 - a) * tau * absJ <= E <= tau * absJ * (1 + 1e-6)


def test_integral_D_shift_rule():
    """L_q(psi + t) = L_q(psi) + t/eps, so D(psi + t) = exp(-t/eps) D(psi):
    the sign of the exponent in D is fixed by the direction of the shift."""
    rng = np.random.default_rng(4)
    x, mu = W.quadrature(W.square_mesh(8), rng.uniform(0.5, 1.5, 81))
    y = rng.uniform(0, 1, (13, 2))
    nu = np.full(13, 1 / 13)
    psi = 0.01 * rng.standard_normal(13)
    eps = 0.02
    D0 = oracle.integral_D(mu, oracle.dual_eval(x, mu, y, nu, psi, eps, want_L=True).L)
    for t in [0.003, -0.01, 0.05]:
        Dt = oracle.integral_D(mu, oracle.dual_eval(x, mu, y, nu, psi + t, eps, want_L=True).L)
        assert abs(Dt / D0 - math.exp(-t / eps)) <= 1e-12 * math.exp(-t / eps)


def _D_one_target_exact(yk, psi, eps):
    """rho = 1 on the unit square, one target of mass 1: L(x) = (psi - c(x,y))/eps,
    D = exp(-psi/eps) prod_k int_0^1 exp((t - y_k)^2 / (2 eps)) dt
      = exp(-psi/eps) prod_k sqrt(pi eps/2) [erfi((1 - y_k)/sqrt(2 eps)) + erfi(y_k/sqrt(2 eps))]."""
    s = math.sqrt(2.0 * eps)
    f = [math.sqrt(math.pi * eps / 2) * (erfi((1 - v) / s) + erfi(v / s)) for v in yk]
    return math.exp(-psi / eps) * f[0] * f[1]


@pytest.mark.parametrize("eps,psi", [(0.5, 0.0), (0.2, 0.3), (1.0, -0.7)])
def test_integral_D_one_target_closed_form(eps, psi):
    """The quadrature sum converges to the erfi closed form at least at
    O(h^2) (the degree-2 rule on a smooth integrand; on this regular mesh the
    symmetric rule converges at fourth order)."""
    yk = np.array([0.3, 0.65])
    exact = _D_one_target_exact(yk, psi, eps)
    errs = []
    for cells in [4, 8, 16, 32]:
        x, mu = W.quadrature(W.square_mesh(cells))
        L = oracle.dual_eval(x, mu, yk[None, :], np.ones(1), np.array([psi]), eps, want_L=True).L
        errs.append(abs(oracle.integral_D(mu, L) - exact) / exact)
    for a, b in zip(errs, errs[1:]):
        assert a / b > 3.5, errs                 # at least second order
    assert errs[-1] < 1e-6


def test_integral_D_drops_empty_points():
    """Points with an empty kept set (L = -inf) are left out of D."""
    x, mu = W.quadrature(W.square_mesh(4))
    y = np.array([[0.1, 0.1]])
    r = oracle.dual_eval(x, mu, y, np.ones(1), np.zeros(1), 0.05, cutoff=0.05, want_L=True)
    keep = np.isfinite(r.L)
    assert 0 < keep.sum() < x.shape[0]
    c = 0.5 * ((x - y[0]) ** 2).sum(1)
    ref = np.sum(mu[keep] * np.exp(c[keep] / 0.05))
    assert abs(oracle.integral_D(mu, r.L) - ref) <= 1e-13 * ref


@pytest.mark.parametrize("d", [2, 3])
def test_kept_counts_bruteforce_and_totals(d):
    """|I_q| = #{j : c_qj < C} per point (Sec. 4.1): equal to a brute-force
    count from scipy's pairwise squared distances, summing to the kept-pair
    total and the empty-point count of the truncated evaluation, n at C = inf
    and 0 at C = 0."""
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(40 + d)
    x = rng.uniform(0, 1, (53, d))
    y = rng.uniform(-0.1, 1.1, (29, d))
    mu = np.full(53, 1 / 53)
    nu = np.full(29, 1 / 29)
    psi = 0.01 * rng.standard_normal(29)
    c = 0.5 * cdist(x, y, "sqeuclidean")
    for C in [0.004, 0.03, 0.2]:
        kept, near = oracle.kept_counts(x, y, C)
        assert np.array_equal(kept, (c < C).sum(1))
        ev = oracle.dual_eval(x, mu, y, nu, psi, 0.02, cutoff=C)
        assert int(kept.sum()) == ev.kept
        assert int((kept == 0).sum()) == ev.nempty
    assert np.all(oracle.kept_counts(x, y, math.inf)[0] == 29)
    assert np.all(oracle.kept_counts(x, y, 0.0)[0] == 0)


def test_kept_counts_near_band():
    """A target placed at cost exactly C from the point is outside I_q (the
    cut is strict) and inside the near-tie band; one slightly inside is kept."""
    C = 0.125
    x = np.zeros((1, 2))
    r = math.sqrt(2 * C)
    y = np.array([[r, 0.0], [0.0, r * (1 - 1e-9)], [0.9, 0.9]])
    kept, near = oracle.kept_counts(x, y, C, rel_band=1e-12)
    assert kept[0] == 1 and near[0] == 1
