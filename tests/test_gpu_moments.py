"""GPU parity of the plan moments and transport maps (Secs. 6.2, 6.3)
against the oracle, through the C ABI.

Bounds. First moments: e_M = max_j |M_j - M_ref_j| / ((nu_j + nu~_ref_j) R)
with R the largest coordinate magnitude of the points, <= 1e-6 (mixed) or
1e-12 (FP64): the gradient's bound with the coordinates' scale. Barycentric
map: max |T - T_ref| / R <= 1e-6 / 1e-12. Modal map: equal index wherever the
best target leads the runner-up by more than 1e-12 of the value; where two
targets tie to FP64 rounding, the GPU's choice must attain the maximum.
"""
import math
import sys

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from paper_2507_23602_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"mixed": 1e-6, "fp64": 1e-12, "mixed_fp32": 1e-6}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(p, prec, rule, tau=1e-8):
    from paper_2507_23602_amd import rsot
    kw = dict(precision="mixed" if prec == "mixed_fp32" else prec, truncation=rule, tau=tau)
    if prec == "mixed_fp32":
        kw["fp64_below_points"] = 0
    return rsot.Problem(p.x, p.mu, p.y, p.nu, **kw)


def _keep_for(prob, p, rule, psi, r):
    """The oracle's restriction for the GPU evaluation that produced r."""
    if rule == "tile":
        # the kept (tile, 8-target chunk) set, whatever the culling group
        tile_of, block_of, nt, nb = prob.partition()
        bits = prob.tile_chunk_keep().cpu().numpy()
        chunk_of = (prob.target_slots().cpu().numpy() // 8).astype(np.int32)
        keep_c = np.unpackbits(bits[:, :, None], axis=2, bitorder="little").reshape(nt, nb * 8)
        return dict(keep=(tile_of.cpu().numpy(), chunk_of, keep_c > 0))
    if rule in ("geom", "pw"):
        return dict(cutoff=r.info["cutoff"])
    return {}


def _check_modal(modal, ref_modal, ref_val, x, y, nu, psi, eps, cs=0.5):
    diff = np.flatnonzero(modal != ref_modal)
    for q in diff:                      # a tie to FP64 rounding: must attain the max
        v = psi[modal[q]] - cs * np.sum((x[q] - y[modal[q]]) ** 2) + eps * math.log(nu[modal[q]])
        assert ref_val[q] - v <= 1e-12 * max(1.0, abs(ref_val[q])), (q, modal[q], ref_modal[q])
    return len(diff)


@pytest.mark.parametrize("prec", ["mixed", "fp64", "mixed_fp32"])
@pytest.mark.parametrize("rule", ["dense", "tile", "geom"])
@pytest.mark.parametrize("d", [2, 3])
def test_moments_and_maps_parity(d, rule, prec):
    import torch
    _say(f"moments/maps d={d} rule={rule} prec={prec}")
    p = W.cube_mixture(8, 1500, 2e-3) if d == 3 else W.square_uniform(24, 700, seed=21, eps=2e-3)
    prob = _problem(p, prec, rule, tau=1e-6)
    psi = W.random_psi(17, p.n, p.eps)
    pt = torch.as_tensor(psi, device="cuda")
    if rule != "dense":
        dense = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps)
        prob.set_reference(abs(dense.J))
    mass, first, info, ms = prob.plan_moments(pt, p.eps)
    r = prob.dual_eval(pt, p.eps)
    assert r.info["kept_pairs"] == info["kept_pairs"]
    if rule != "dense":
        assert 0 < info["kept_pairs"] < p.nq * p.n
    kw = _keep_for(prob, p, rule, psi, r)
    ref_mass, ref_first = oracle.plan_moments(p.x, p.mu, p.y, p.nu, psi, p.eps, **kw)
    R = float(np.abs(p.x).max())
    mass, first = mass.cpu().numpy(), first.cpu().numpy()
    scale = (p.nu + ref_mass)[:, None] * R
    em = float(np.max(np.abs(first - ref_first) / scale))
    eg = float(np.max(np.abs(mass - ref_mass) / (p.nu + ref_mass)))
    bary, modal, minfo, mms = prob.transport_maps(pt, p.eps)
    ref_bary, ref_modal, ref_val = oracle.transport_maps(p.x, p.y, p.nu, psi, p.eps, **kw)
    eb = float(np.nanmax(np.abs(bary.cpu().numpy() - ref_bary)) / R)
    nt = _check_modal(modal.cpu().numpy(), ref_modal, ref_val, p.x, p.y, p.nu, psi, p.eps)
    _say(f"  kept {info['kept_pairs'] / (p.nq * p.n):.3f}: e_M {em:.1e}, mass {eg:.1e}, "
         f"bary {eb:.1e}, modal ties {nt}; {ms:.3f} + {mms:.3f} ms")
    tol = TOL[prec]
    assert eg <= tol and em <= tol and eb <= tol
    assert np.array_equal(np.isnan(bary.cpu().numpy()), np.isnan(ref_bary))


def test_moments_totals_and_maps_at_full_size():
    """The 3D benchmark workload (6,291,456 points x 65,536 targets), dense:
    the first moments sum to the source's first moment, the masses to its
    mass, sum_q mu_q T(x_q) = sum_j nu~_j y_j, and the maps at 500 sampled
    points equal the oracle's (a point's maps depend on that point only)."""
    import torch
    from paper_2507_23602_amd import rsot
    _say("moments/maps at full size")
    p = W.config2()
    prob = rsot.Problem(*[torch.as_tensor(a, device="cuda") for a in (p.x, p.mu, p.y, p.nu)])
    psi = W.random_psi(11, p.n, p.eps)
    pt = torch.as_tensor(psi, device="cuda")
    mass, first, info, ms = prob.plan_moments(pt, p.eps)
    bary, modal, minfo, mms = prob.transport_maps(pt, p.eps)
    mass, first = mass.cpu().numpy(), first.cpu().numpy()
    src1 = (p.mu[:, None] * p.x).sum(0)
    assert abs(mass.sum() - p.mu.sum()) <= 1e-9
    np.testing.assert_allclose(first.sum(0), src1, rtol=0, atol=1e-8)
    b = bary.cpu().numpy()
    np.testing.assert_allclose((p.mu[:, None] * b).sum(0), (mass[:, None] * p.y).sum(0),
                               rtol=0, atol=1e-8)
    idx = np.random.default_rng(5).choice(p.nq, 500, replace=False)
    rb, rm, rv = oracle.transport_maps(p.x[idx], p.y, p.nu, psi, p.eps)
    eb = float(np.max(np.abs(b[idx] - rb)))
    nt = _check_modal(modal.cpu().numpy()[idx], rm, rv, p.x[idx], p.y, p.nu, psi, p.eps)
    _say(f"  moments {ms:.1f} ms, maps {mms:.1f} ms; sampled bary err {eb:.1e}, ties {nt}")
    assert eb <= 1e-6
