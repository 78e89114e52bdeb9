"""GPU tests of the batched evaluation (one launch per pass) and of the\nautotuner's work granularities."""
import sys

import numpy as np
import pytest

import oracle
from paper_2507_23602_amd import workloads as W


pytestmark = pytest.mark.gpu


def grad_err(g, gref, nu):
    return float(np.max(np.abs(g - gref) / (nu + (gref + nu))))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _instances(k, scale):
    return [W.config5_instance(i, scale=scale) for i in range(k)]


def test_batched_equals_single_calls():
    """Uneven instances in one batch give the same J and gradients as one call
    per instance (dense and tile rules, 2D and 3D, mixed and FP64 members)."""
    import torch
    from paper_2507_23602_amd import rsot
    _say("batched vs single")
    insts = _instances(6, 0.02)
    insts.append(W.config1())
    probs, psis, rules = [], [], []
    for i, p in enumerate(insts):
        rule = "tile" if i % 2 else "dense"
        prec = "fp64" if i == 3 else "mixed"
        # fp64_below_points = 0: these small members run the FP32-exponential
        # batched kernels, not the FP64 pair loop small problems default to
        pr = rsot.Problem(p.x, p.mu, p.y, p.nu, truncation=rule, tau=1e-10, precision=prec,
                          fp64_below_points=0)
        probs.append(pr)
        psis.append(torch.as_tensor(W.random_psi(i, p.n, p.eps), device="cuda"))
        rules.append(rule)
    # references: |J| for the tile rule, then one call per instance
    single = []
    for pr, p, ps in zip(probs, insts, psis):
        r0 = pr.dual_eval(ps, p.eps)                 # dense first call sets |J_ref|
        r = pr.dual_eval(ps, p.eps)
        single.append((r.J, r.grad.cpu().numpy(), r.info["kept_pairs"]))
    J, grads, infos, ms = rsot.dual_eval_batched(probs, [p.eps for p in insts], psis)
    _say(f"  batch {ms:.2f} ms, kept {[i['kept_pairs'] for i in infos]}")
    for k, (p, (Js, gs, ks)) in enumerate(zip(insts, single)):
        g = grads[k].cpu().numpy()
        assert infos[k]["kept_pairs"] == ks
        assert abs(J[k] - Js) <= 1e-14 * abs(Js)
        np.testing.assert_allclose(g, gs, rtol=0, atol=1e-16)


def test_batched_against_oracle():
    """Small members forced onto the FP32-exponential batched kernels
    (fp64_below_points = 0): gradient e_g <= 1e-6, and J within the per-term
    arithmetic bound 1.5e-7 eps sum(mu) (too few points to average the FP32
    errors below 1e-9 of J; by default such members run the FP64 loop)."""
    import torch
    from paper_2507_23602_amd import rsot
    _say("batched vs oracle")
    insts = _instances(4, 0.01)
    probs = [rsot.Problem(p.x, p.mu, p.y, p.nu, fp64_below_points=0) for p in insts]
    psis = [torch.as_tensor(W.random_psi(7 + i, p.n, p.eps), device="cuda")
            for i, p in enumerate(insts)]
    J, grads, infos, ms = rsot.dual_eval_batched(probs, [p.eps for p in insts], psis)
    for k, p in enumerate(insts):
        ref = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psis[k].cpu().numpy(), p.eps)
        g = grads[k].cpu().numpy()
        eg = np.max(np.abs(g - ref.grad) / (p.nu + ref.grad + p.nu))
        ej = abs(J[k] - ref.J) / abs(ref.J)
        _say(f"  instance {k}: nq={p.nq} n={p.n} eps={p.eps:.2e} ej={ej:.2e} eg={eg:.2e}")
        assert infos[k]["fp64_pairs"] == 0
        assert abs(J[k] - ref.J) <= 1.5e-7 * p.eps * p.mu.sum() and eg <= 1e-6


def test_autotune_choice_is_valid_and_equivalent():
    import torch
    from paper_2507_23602_amd import rsot
    _say("autotune")
    p = W.cube_mixture(16, 8192, 2e-3)
    pr = rsot.Problem(p.x, p.mu, p.y, p.nu, truncation="tile", tau=1e-10)
    psi = torch.as_tensor(W.random_psi(2, p.n, p.eps), device="cuda")
    r0 = pr.dual_eval(psi, p.eps)                     # dense, sets |J_ref|
    r1 = pr.dual_eval(psi, p.eps)
    res = pr.autotune(psi, p.eps, reps=2)
    _say(f"  {res}")
    assert res["seg_blocks"] in (0, 64, 128, 256, 512, 1024)
    assert res["seg_tiles"] in (0, 16, 32, 64, 128, 256, 512, 1024, 4096)
    assert res["best_ms"] <= res["default_ms"]
    assert res["tile_group"] in (0, 8, 16, 32, 64)
    r2 = pr.dual_eval(psi, p.eps)
    # Another objective-pass segmentation gives each work item another
    # reference exponent for its FP32 chunk sums, so the two evaluations
    # round differently; both must stay inside the mixed-precision bounds
    # (objective 1e-9 relative, gradient 1e-6), checked against each other.
    # Another culling group keeps another set of pairs: then the objectives
    # differ by at most the rule's bound tau |J| on top.
    same_group = res["tile_group"] in (0, 64)
    if same_group:
        assert r2.info["kept_pairs"] == r1.info["kept_pairs"]
    assert abs(r2.J - r1.J) <= (1e-9 + (0 if same_group else 1e-10)) * abs(r1.J)
    g1, g2 = r1.grad.cpu().numpy(), r2.grad.cpu().numpy()
    if same_group:
        assert np.max(np.abs(g1 - g2) / (p.nu + g1 + p.nu)) < 1e-6


@pytest.mark.parametrize("rule", ["dense", "tile"])
def test_autotune_candidates_against_oracle(rule):
    """Every granularity the autotuner may choose, on a 98,304 x 8,192
    problem: the evaluation under each (culling group x objective-pass
    segment x gradient-pass segment) equals the oracle's (J 1e-9, e_g 1e-6)
    with the oracle's kept-pair count (the tile rule's oracle cut into the
    same groups), and the tuner's own choice reproduces the evaluation the
    problem keeps, bit for bit."""
    import torch
    from paper_2507_23602_amd import rsot
    _say(f"autotune candidates vs oracle, {rule}")
    p = W.cube_mixture(16, 8192, 2e-3)
    assert p.nq == 98304 and p.n == 8192
    psi = W.random_psi(5, p.n, p.eps)
    pt = torch.as_tensor(psi, device="cuda")
    dense = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps)
    tau = 1e-10
    pr = rsot.Problem(p.x, p.mu, p.y, p.nu, truncation=rule, tau=tau)
    pr.set_reference(abs(dense.J))
    res = pr.autotune(pt, p.eps, reps=1)
    _say(f"  tuner: {res}")
    chosen = pr.dual_eval(pt, p.eps)
    groups = (0,) if rule == "dense" else (64, 32, 16, 8)
    refs = {0: dense}
    if rule == "tile":
        tile_of, _, nt, nb = pr.partition()
        tile_of = tile_of.cpu().numpy()
        slots = pr.target_slots().cpu().numpy()
        for gr in groups:
            refs[gr] = oracle.dual_eval_tile(p.x, p.mu, p.y, p.nu, psi, p.eps, tile_of, nt,
                                             (slots // gr).astype(np.int32), nb * 64 // gr, tau,
                                             abs(dense.J))
    tuned = (res["seg_blocks"], res["seg_tiles"],
             res["tile_group"] or (64 if rule == "tile" else 0))
    worst_j = worst_g = 0.0
    n_cfg = 0
    for gr in groups:
        ref = refs[gr]
        for sb in (0, 64, 128, 256, 512, 1024):
            for st in (0, 16, 32, 64, 128, 256, 512, 1024, 4096):
                pr.set_tuning(sb, st, gr)
                r = pr.dual_eval(pt, p.eps)
                assert r.info["kept_pairs"] == ref.kept, (gr, sb, st)
                ej = abs(r.J - ref.J) / abs(ref.J)
                eg = grad_err(r.grad.cpu().numpy(), ref.grad, p.nu)
                worst_j, worst_g = max(worst_j, ej), max(worst_g, eg)
                assert ej <= 1e-9 and eg <= 1e-6, (gr, sb, st, ej, eg)
                if (sb, st, gr) == tuned:
                    assert r.J == chosen.J
                    assert torch.equal(r.grad, chosen.grad)
                n_cfg += 1
    _say(f"  {n_cfg} configurations: worst J {worst_j:.2e}, worst e_g {worst_g:.2e}")


def test_batched_full_size_smallest_instances_against_oracle():
    """The eight smallest instances of the 64-instance batched workload at
    full size (1.4e9 to 4.2e9 pairs each), dense rule, mixed precision, in
    one batched call, each against the FP64 oracle."""
    import torch
    from paper_2507_23602_amd import rsot
    sizes = sorted((W.config5_sizes(i)[0] * W.config5_sizes(i)[1], i) for i in range(64))
    ids = [i for _, i in sizes[:8]]
    insts = [W.config5_instance(i) for i in ids]
    _say(f"full-size batch: instances {ids}")
    probs = [rsot.Problem(p.x, p.mu, p.y, p.nu) for p in insts]
    psis = [torch.as_tensor(W.random_psi(300 + i, p.n, p.eps), device="cuda")
            for i, p in zip(ids, insts)]
    J, grads, infos, ms = rsot.dual_eval_batched(probs, [p.eps for p in insts], psis)
    _say(f"  batch {ms:.1f} ms for {sum(p.nq * p.n for p in insts):.3e} pairs")
    for k, p in enumerate(insts):
        ref = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psis[k].cpu().numpy(), p.eps)
        g = grads[k].cpu().numpy()
        eg = np.max(np.abs(g - ref.grad) / (p.nu + ref.grad + p.nu))
        ej = abs(J[k] - ref.J) / abs(ref.J)
        _say(f"  instance {ids[k]}: nq={p.nq} n={p.n} eps={p.eps:.2e} ej={ej:.2e} eg={eg:.2e}")
        assert ej <= 1e-9 and eg <= 1e-6
        assert infos[k]["kept_pairs"] == p.nq * p.n
