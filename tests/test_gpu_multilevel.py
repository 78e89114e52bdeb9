"""GPU tests of the multilevel parts (Sec. 5): softmax refinement against the
oracle, k-means target hierarchy properties, combined multilevel solve."""
import sys

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_2507_23602_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("d", [2, 3])
def test_softmax_refine_parity(prec, d):
    """Eq. softmax_refinement_formula on the GPU against the oracle (log domain)."""
    import torch
    from paper_2507_23602_amd import rsot
    _say(f"refine parity d={d} prec={prec}")
    rng = np.random.default_rng(40 + d)
    if d == 2:
        x, mu = W.quadrature(W.square_mesh(30))
        eps = 2e-3
    else:
        p = W.cube_mixture(8, 10, 2e-3)
        x, mu, eps = p.x, p.mu, p.eps
    yc = rng.uniform(0.05, 0.95, size=(150, d))
    nuc = rng.uniform(0.5, 1.5, 150)
    nuc /= nuc.sum()
    yf = np.concatenate([yc + 0.01 * rng.standard_normal(yc.shape) for _ in range(4)])
    psic = 0.01 * rng.standard_normal(150)
    prob = rsot.Problem(x, mu, yc, nuc, precision=prec)
    out = prob.softmax_refine(torch.as_tensor(psic, device="cuda"), eps,
                              torch.as_tensor(yf, device="cuda")).cpu().numpy()
    L = oracle.dual_eval(x, mu, yc, nuc, psic, eps, want_L=True).L
    ref = oracle.softmax_refine(x, mu, L, yf, eps)
    err = np.max(np.abs(out - ref))
    _say(f"  max |dpsi| = {err:.3e} (eps {eps})")
    assert err <= (1e-6 if prec == "mixed" else 1e-12) * eps


def test_softmax_refine_matches_one_sinkhorn_step():
    """Fine targets = coarse targets: refinement equals psi - eps ln(nu~/nu)
    with nu~ from the GPU gradient (two GPU paths, one identity)."""
    import torch
    from paper_2507_23602_amd import rsot
    p = W.config1()
    prob = rsot.Problem(p.x, p.mu, p.y, p.nu, precision="fp64")
    psi = torch.as_tensor(W.random_psi(3, p.n, p.eps), device="cuda")
    r = prob.dual_eval(psi, p.eps)
    nut = r.grad.cpu().numpy() + p.nu
    out = prob.softmax_refine(psi, p.eps, torch.as_tensor(p.y, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(out, psi.cpu().numpy() - p.eps * np.log(nut / p.nu), rtol=0,
                               atol=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_target_hierarchy(d):
    import torch
    from paper_2507_23602_amd import rsot
    _say(f"hierarchy d={d}")
    y = W.blob_targets_disk(20000, seed=5) if d == 2 else W.cube_mixture(2, 20000, 1e-2).y
    nu = np.random.default_rng(1).uniform(0.5, 1.5, 20000)
    nu /= nu.sum()
    sizes = [300, 1200, 5000, 20000]
    levels, parents = rsot.target_hierarchy(torch.as_tensor(y, device="cuda"),
                                            torch.as_tensor(nu, device="cuda"), sizes,
                                            lloyd_iters=20, with_parents=True)
    prev_y, prev_nu = y, nu
    for l in range(len(sizes) - 2, -1, -1):
        yc = levels[l][0].cpu().numpy()
        nc = levels[l][1].cpu().numpy()
        par = parents[l + 1].cpu().numpy()
        _say(f"  level {l}: {len(nc)} of {sizes[l]} points")
        assert len(nc) <= sizes[l] and len(nc) >= 0.9 * sizes[l]
        assert abs(nc.sum() - 1.0) < 1e-12                      # mass conservation
        assert par.min() >= 0 and par.max() < len(nc)
        # every coarse point is the mean of its members and carries their mass
        cnt = np.bincount(par, minlength=len(nc))
        assert cnt.min() >= 1
        mean = np.stack([np.bincount(par, weights=prev_y[:, k], minlength=len(nc)) for k in range(d)], 1)
        np.testing.assert_allclose(yc, mean / cnt[:, None], rtol=0, atol=1e-12)
        np.testing.assert_allclose(nc, np.bincount(par, weights=prev_nu, minlength=len(nc)),
                                   rtol=0, atol=1e-15)
        # Lloyd after 20 iterations: members are (almost all) nearest to their centroid
        _, nearest = cKDTree(yc).query(prev_y)
        frac = np.mean(nearest == par)
        _say(f"    nearest-centroid agreement {frac:.4f}")
        assert frac > 0.97
        prev_y, prev_nu = yc, nc


def test_multilevel_solve_small():
    import torch
    from paper_2507_23602_amd import rsot
    _say("multilevel small")
    meshes = W.disk_hierarchy(rings=8, levels=3)
    sources = [W.quadrature(m) for m in meshes]
    yf = W.blob_targets_disk(4096, seed=5)
    nuf = np.full(4096, 1 / 4096)
    levels = rsot.target_hierarchy(torch.as_tensor(yf, device="cuda"),
                                   torch.as_tensor(nuf, device="cuda"), [256, 1024, 4096])
    targets = [(l[0], l[1]) for l in levels]
    ml = rsot.Multilevel(sources, targets, precision="mixed", truncation="tile", tau=1e-12)
    eps = [0.08, 0.04, 0.02, 0.01, 0.005]
    lev = [0, 0, 1, 2, 2]
    psi, info = ml.solve(eps, lev, tol=1e-6, level_tol=1e-5)
    _say(f"  {info}")
    assert info["status"] == rsot.OK
    assert info["source_level"] == [0, 1, 2] and info["target_level"] == [0, 1, 2]
    x, mu = sources[-1]
    r = oracle.dual_eval(x, mu, yf, nuf, psi, eps[-1])
    g1 = np.abs(r.grad).sum()
    _say(f"  oracle |g|_1 at multilevel psi = {g1:.3e}")
    assert g1 < 2e-6


def test_multilevel_stalled_levels_and_final_failure():
    """Failure handling across levels (host-side hook: the solver sees -grad,
    so no line search can decrease J): every non-final step stalls and hands
    its iterate on (counted in stalled_levels), and the final step's
    RSOT_ERR_LINESEARCH is the solve's status, with the info attached."""
    import torch
    from paper_2507_23602_amd import rsot
    meshes = W.disk_hierarchy(rings=6, levels=3)
    sources = [W.quadrature(m) for m in meshes]
    yf = W.blob_targets_disk(1024, seed=5)
    nuf = np.full(1024, 1 / 1024)
    levels = rsot.target_hierarchy(torch.as_tensor(yf, device="cuda"),
                                   torch.as_tensor(nuf, device="cuda"), [64, 256, 1024])
    ml = rsot.Multilevel(sources, [(l[0], l[1]) for l in levels], precision="fp64")
    with pytest.raises(rsot.RsotError) as e:
        ml.solve([0.04, 0.02, 0.01], [0, 1, 2], tol=1e-8, test_flip_gradient=True)
    err = e.value
    _say(f"  status {err.code}, info {err.info}")
    assert err.code == rsot.ERR_LINESEARCH
    assert err.info["stalled_levels"] == 2 and err.info["n_steps"] == 3
    assert err.info["iterations"] == [0, 0, 0]
    assert np.all(np.isfinite(err.psi))
