"""GPU parity of rsot_dual_eval against the CPU oracle (through the C ABI).

Tolerances (from the precision targets): gradient
    e_g = max_j |g_j - g_ref_j| / (nu_j + nu~_ref_j) <= 1e-6 (mixed), 1e-12 (fp64)
objective |J - J_ref| / |J_ref| <= 1e-9 (both) at every size: the mixed
path's FP32 exponential errors average out over points, and problems with
too few (effective) points for that run the FP64 pair loop. Per-point L_q:
absolute error <= 1e-6 (mixed), 1e-10 (fp64) relative to max(1, |L_q|).

"mixed_fp32" forces the FP32-exponential kernels on these small problems
(fp64_below_points = 0), to test the kernels themselves on ragged and edge
shapes. Without averaging over points, J is then bounded by the per-term
arithmetic: every term of a point's sum carries at most 8.4e-8 (measured
instruction error) + 2^-24 |u| ln 2 (argument rounding, |u| <= 1 for the
terms that matter) < 1.5e-7 relative error, so |L_q - L_q^ref| < 1.5e-7 and
|J - J_ref| <= 1.5e-7 eps sum(mu).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2507_23602_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"mixed": (1e-6, 1e-9, 1e-6), "fp64": (1e-12, 1e-12, 1e-10),
       "mixed_fp32": (1e-6, None, 1e-6)}
PREC = ["mixed", "fp64", "mixed_fp32"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def grad_err(g, gref, nu):
    return float(np.max(np.abs(g - gref) / (nu + (gref + nu))))


def _problem(x, mu, y, nu, **kw):
    from paper_2507_23602_amd import rsot
    if kw.get("precision") == "mixed_fp32":
        kw.update(precision="mixed", fp64_below_points=0)
    return rsot.Problem(x, mu, y, nu, **kw)


def _n_eff(mu):
    return mu.sum() ** 2 / (mu ** 2).sum()


def _check(prob, x, mu, y, nu, psi, eps, prec, cutoff=math.inf, check_L=True, ref=None,
           r=None):
    import torch
    if r is None:
        r = prob.dual_eval(torch.as_tensor(psi, device="cuda"), eps)
    if ref is None:
        ref = oracle.dual_eval(x, mu, y, nu, psi, eps, cutoff=cutoff, want_L=check_L)
    tg, tj, tl = TOL[prec]
    g = r.grad.cpu().numpy()
    eg = grad_err(g, ref.grad, nu)
    ej = abs(r.J - ref.J) / abs(ref.J)
    _say(f"  J={r.J:.15e} ref={ref.J:.15e} ej={ej:.2e} eg={eg:.2e} "
         f"fp64 pairs {r.info['fp64_pairs']}")
    expect_fp64 = prec == "fp64" or (prec == "mixed" and _n_eff(mu) < 16384
                                     and x.shape[0] * y.shape[0] < 2 ** 27)
    assert r.info["fp64_pairs"] == int(expect_fp64)
    if tj is None:
        assert abs(r.J - ref.J) <= 1.5e-7 * eps * mu.sum(), (r.J, ref.J)
    else:
        assert ej <= tj, (ej, r.J, ref.J)
    assert eg <= tg, eg
    if check_L:
        L = prob.lse().cpu().numpy()
        fin = np.isfinite(ref.L)
        assert np.array_equal(np.isfinite(L), fin)
        el = np.max(np.abs(L[fin] - ref.L[fin]) / np.maximum(1.0, np.abs(ref.L[fin])))
        assert el <= tl, el
    return r, ref


def _rand_problem(d, cells, n, seed, ragged=True):
    rng = np.random.default_rng(seed)
    mesh = W.square_mesh(cells) if d == 2 else W.cube_mesh(cells)
    rho_v = rng.uniform(0.3, 1.7, size=mesh.verts.shape[0])
    x, mu = W.quadrature(mesh, rho_v)
    if ragged:                                   # drop a few points: ragged tail
        keep = x.shape[0] - 37
        x, mu = x[:keep], mu[:keep] / mu[:keep].sum()
    y = rng.uniform(-0.05, 1.05, size=(n, d))
    nu = rng.uniform(0.5, 1.5, size=n)
    nu /= nu.sum()
    return x, mu, y, nu


@pytest.mark.parametrize("prec", PREC)
@pytest.mark.parametrize("d,cells,n", [(2, 12, 77), (2, 20, 300), (3, 5, 130), (3, 7, 517)])
def test_dense_parity_random(prec, d, cells, n):
    _say(f"dense parity d={d} cells={cells} n={n} prec={prec}")
    x, mu, y, nu = _rand_problem(d, cells, n, seed=100 * d + n)
    eps = 0.01
    psi = 0.02 * np.random.default_rng(n).standard_normal(n)
    prob = _problem(x, mu, y, nu, precision=prec)
    _check(prob, x, mu, y, nu, psi, eps, prec)
    _check(prob, x, mu, y, nu, np.zeros(n), 0.003, prec)


@pytest.mark.parametrize("prec", PREC)
def test_config1_parity(prec):
    _say(f"config1 parity prec={prec}")
    p = W.config1()
    prob = _problem(p.x, p.mu, p.y, p.nu, precision=prec)
    _check(prob, p.x, p.mu, p.y, p.nu, np.zeros(p.n), p.eps, prec)
    psi = W.random_psi(9, p.n, p.eps)
    _check(prob, p.x, p.mu, p.y, p.nu, psi, p.eps, prec)


@pytest.mark.parametrize("prec", PREC)
def test_cube_mixture_parity(prec):
    """Config-2 family at a size the oracle finishes in seconds:
    cube 12^3 x 24 = 41,472 points, 2,048 mixture targets, eps = 1e-3."""
    _say(f"cube mixture parity prec={prec}")
    p = W.cube_mixture(12, 2048, 1e-3)
    prob = _problem(p.x, p.mu, p.y, p.nu, precision=prec)
    _check(prob, p.x, p.mu, p.y, p.nu, np.zeros(p.n), p.eps, prec)
    psi = W.random_psi(3, p.n, p.eps)
    _check(prob, p.x, p.mu, p.y, p.nu, psi, p.eps, prec)


def test_edge_cases():
    import torch
    from paper_2507_23602_amd import rsot
    _say("edge cases")
    # one target: closed form J = -(1/2|y - 1/2|^2 + d/24), grad = 0
    x, mu = W.quadrature(W.square_mesh(6))
    y = np.array([[0.3, 0.8]])
    prob = _problem(x, mu, y, np.ones(1))
    r = prob.dual_eval(torch.zeros(1, dtype=torch.float64, device="cuda"), 0.01)
    exact = -(0.5 * np.sum((y[0] - 0.5) ** 2) + 2 / 24.0)
    assert abs(r.J - exact) < 1e-9 * abs(exact)
    assert abs(float(r.grad[0])) < 2e-6          # e_g <= 1e-6 with nu = nu~ = 1
    # one point, many targets
    x1 = np.array([[0.4, 0.6, 0.5]])
    y3 = np.random.default_rng(1).uniform(0, 1, (70, 3))
    nu3 = np.full(70, 1 / 70)
    prob = _problem(x1, np.ones(1), y3, nu3)
    _check(prob, x1, np.ones(1), y3, nu3, np.zeros(70), 0.05, "mixed")
    # non-finite psi is reported, outputs untouched
    prob = _problem(x, mu, y, np.ones(1))
    bad = torch.tensor([float("nan")], dtype=torch.float64, device="cuda")
    out = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(rsot.RsotError) as e:
        prob.dual_eval(bad, 0.01, out=out)
    assert e.value.code == rsot.ERR_NONFINITE
    assert float(out[0]) == 7.0
    with pytest.raises(rsot.RsotError) as e:
        prob.dual_eval(torch.zeros(1, dtype=torch.float64, device="cuda"), -1.0)
    assert e.value.code == rsot.ERR_INVALID_ARG
    # invalid inputs at creation
    with pytest.raises(rsot.RsotError) as e:
        _problem(x, mu, y, -np.ones(1))
    assert e.value.code == rsot.ERR_INVALID_ARG
    xn = x.copy()
    xn[3, 0] = np.inf
    with pytest.raises(rsot.RsotError) as e:
        _problem(xn, mu, y, np.ones(1))
    assert e.value.code == rsot.ERR_NONFINITE
    # memory cap
    with pytest.raises(rsot.RsotError) as e:
        _problem(x, mu, y, np.ones(1), mem_limit_bytes=4096)
    assert e.value.code == rsot.ERR_OOM


def test_bitwise_repeatable():
    import torch
    _say("bitwise repeat")
    p = W.cube_mixture(8, 1000, 2e-3)
    prob = _problem(p.x, p.mu, p.y, p.nu)
    psi = torch.as_tensor(W.random_psi(5, p.n, 2e-3), device="cuda")
    a = prob.dual_eval(psi, p.eps)
    ga = a.grad.clone()
    b = prob.dual_eval(psi, p.eps)
    assert a.J == b.J
    assert torch.equal(ga, b.grad)


def test_objective_only_matches():
    import torch
    p = W.config1()
    prob = _problem(p.x, p.mu, p.y, p.nu)
    psi = torch.as_tensor(W.random_psi(2, p.n, p.eps), device="cuda")
    a = prob.dual_eval(psi, p.eps)
    b = prob.dual_eval(psi, p.eps, want_grad=False)
    assert a.J == b.J and b.grad is None


# -- truncated rules ---------------------------------------------------------
@pytest.mark.parametrize("rule", ["geom", "int", "pw"])
@pytest.mark.parametrize("prec", PREC)
def test_cutoff_rules_parity(rule, prec):
    """Paper's cutoff rules (Eqs. truncation_cutoff_geom/int, cost_cutoff_delta):
    the GPU's cutoff agrees with the oracle's formula, and the truncated J, grad
    and kept-pair count agree with the oracle at that cutoff."""
    import torch
    _say(f"cutoff rule {rule} prec={prec}")
    p = W.cube_mixture(10, 3000, 2e-3)
    tau = {"geom": 1e-6, "int": 1e-6, "pw": None}[rule]
    delta = 1e-8
    prob = _problem(p.x, p.mu, p.y, p.nu, precision=prec, truncation=rule,
                    tau=tau or 1e-12, delta_thr=delta)
    psi = W.random_psi(4, p.n, p.eps)
    dense = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps, want_L=True)
    absJ = abs(dense.J)
    C0 = oracle.covering_cost(p.x, p.y)
    assert abs(prob.covering_cost() - C0) <= 1e-14 * C0
    prob.set_reference(absJ)
    psi_d = torch.as_tensor(psi, device="cuda")
    if rule == "int":
        r0 = prob.dual_eval(psi_d, p.eps)          # first call: dense, stores D
        assert r0.info["dense_fallback"] == 1
        D = oracle.integral_D(p.mu, dense.L)
        # ln D is dominated by the points with the smallest sums, so it carries
        # a single point's error (mixed: FP32 exponentials, not averaged)
        assert abs(r0.info["log_D"] - math.log(D)) < (1e-12 if r0.info["fp64_pairs"] else 1e-8)
        C_ref = oracle.cutoff_int(C0, psi, D, tau, absJ, p.eps)
    elif rule == "geom":
        C_ref = oracle.cutoff_geom(C0, psi, p.nu, tau, absJ, p.eps)
    else:
        C_ref = oracle.cutoff_pw(psi, p.nu, delta, p.eps)
    r = prob.dual_eval(psi_d, p.eps)
    C = r.info["cutoff"]
    _say(f"  C={C:.15e} C_ref={C_ref:.15e} kept={r.info['kept_pairs']}")
    # the INT cutoff carries the (mixed-precision) D of the previous evaluation
    ctol = 1e-9 if (rule == "int" and not r.info["fp64_pairs"]) else 1e-12
    assert abs(C - C_ref) <= ctol * abs(C_ref)
    ref = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps, cutoff=C, want_L=True)
    assert r.info["kept_pairs"] == ref.kept
    assert r.info["kept_pairs"] < p.nq * p.n
    assert r.info["n_empty_qp"] == ref.nempty
    # the kept set itself, point by point: |I_q| = #{j : c_qj < C} (index
    # work, compared exactly; a difference is allowed only at a point whose
    # cost to some target lies within 1e-12 C of C, where two exact FP64
    # evaluation orders of the cost may round to different sides)
    cnt = prob.kept_counts().cpu().numpy()
    ref_cnt, near = oracle.kept_counts(p.x, p.y, C, rel_band=1e-12)
    diff = np.abs(cnt.astype(np.int64) - ref_cnt)
    _say(f"  kept sets: {int((diff > 0).sum())} points differ, {int(near.sum())} near-tie pairs")
    assert np.all(diff <= near), np.flatnonzero(diff > near)[:10]
    keep = prob.tile_keep().cpu().numpy()
    tile_of, block_of, nt, nb = prob.partition()
    tile_of, block_of = tile_of.cpu().numpy(), block_of.cpu().numpy()
    # the box culling is valid: a skipped (tile, block) holds no pair with
    # c < C and a block kept whole holds no pair with c >= C, so |I_q| lies
    # between the sizes of the point's whole blocks and of its non-skipped ones
    bsz = np.bincount(block_of, minlength=nb)
    lower = (keep[tile_of] == 2).astype(np.int64) @ bsz
    upper = (keep[tile_of] > 0).astype(np.int64) @ bsz
    assert np.all(lower <= ref_cnt) and np.all(ref_cnt <= upper)
    assert int((keep == 1).sum()) > 0
    _check(prob, p.x, p.mu, p.y, p.nu, psi, p.eps, prec, ref=ref, r=r)
    if rule != "pw":           # App. B bound, up to FP64 round-off of the two sums
        assert -1e-13 * absJ <= dense.J - ref.J <= tau * absJ


def _chunk_keep_from_groups(keep_g, slots, n_blocks, g, n):
    """The oracle's (tile, group) keep matrix as the library's per (tile,
    block) chunk bits, and the mask of chunks that hold a real target."""
    nt = keep_g.shape[0]
    bits = np.zeros((nt, n_blocks), dtype=np.uint8)
    real = np.zeros(n_blocks * 8, dtype=bool)
    real[slots // 8] = True
    for c in range(8):
        grp = (np.arange(n_blocks) * 64 + 8 * c) // g            # group of chunk c of each block
        ok = grp < keep_g.shape[1]
        col = np.zeros((nt, n_blocks), dtype=bool)
        col[:, ok] = keep_g[:, grp[ok]] > 0
        bits |= (col.astype(np.uint8) << c)
    return bits, real.reshape(n_blocks, 8)


@pytest.mark.parametrize("prec", PREC)
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("group", [64, 32, 16, 8])
def test_tile_rule_parity(prec, d, group):
    """Tile-local rule at every culling granularity (targets per group): the
    GPU's kept set, chunk by chunk, equals the oracle's rule applied to the
    GPU's own tiles and groups (the library's sorted target order cut into
    groups of g); per-point |I_q|, J and grad equal the oracle's; the
    truncation bound holds."""
    import torch
    _say(f"tile rule d={d} prec={prec} group={group}")
    if d == 3:
        p = W.cube_mixture(10, 3000, 1e-3)
    else:
        p = W.square_uniform(48, 4000, seed=6, eps=1e-3)
    tau = 1e-8
    prob = _problem(p.x, p.mu, p.y, p.nu, precision=prec, truncation="tile", tau=tau,
                    tile_group=group)
    psi = W.random_psi(8, p.n, p.eps)
    dense = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps)
    prob.set_reference(abs(dense.J))
    r = prob.dual_eval(torch.as_tensor(psi, device="cuda"), p.eps)
    tile_of, block_of, nt, nb = prob.partition()
    tile_of = tile_of.cpu().numpy()
    slots = prob.target_slots().cpu().numpy()
    assert np.array_equal(slots // 64, block_of.cpu().numpy())
    group_of = (slots // group).astype(np.int32)
    ng = nb * 64 // group
    ref = oracle.dual_eval_tile(p.x, p.mu, p.y, p.nu, psi, p.eps, tile_of, nt, group_of, ng, tau,
                                abs(dense.J), want_L=True, want_keep=True)
    _say(f"  kept gpu={r.info['kept_pairs']} oracle={ref.kept} of {p.nq * p.n}")
    assert r.info["kept_pairs"] == ref.kept
    assert ref.kept < p.nq * p.n
    # the kept (tile, chunk) set, bit for bit on the chunks holding targets
    bits = prob.tile_chunk_keep().cpu().numpy()
    ref_bits, real = _chunk_keep_from_groups(ref.keep, slots, nb, group, p.n)
    realbits = np.packbits(real[:, ::-1], axis=1, bitorder="big").reshape(-1)
    assert np.array_equal(bits & realbits[None, :], ref_bits & realbits[None, :])
    keep = prob.tile_keep().cpu().numpy()
    if group == 64:
        assert set(np.unique(keep)) <= {0, 2}
    assert np.array_equal(keep > 0, (ref_bits & realbits[None, :]) > 0)
    _say(f"  kept (tile, chunk) pairs: {int(np.unpackbits(bits & realbits[None, :]).sum())}")
    cnt = prob.kept_counts().cpu().numpy()
    ref_cnt = (ref.keep[tile_of] > 0).astype(np.int64) @ np.bincount(group_of, minlength=ng)
    assert np.array_equal(cnt, ref_cnt)
    _check(prob, p.x, p.mu, p.y, p.nu, psi, p.eps, prec, ref=ref, r=r)
    assert -1e-13 * abs(dense.J) <= dense.J - ref.J <= tau * abs(dense.J)


@pytest.mark.parametrize("rule,group", [("tile", 64), ("tile", 8), ("geom", 64)])
def test_culling_parity_many_tiles(rule, group):
    """Culling past one workgroup's prefix sums: 331,776 points (5,184 tiles,
    more than the 4,096 counts one scan workgroup takes) x 2,000 targets (a
    ragged last block). The kept set against the oracle's rule: (tile, chunk)
    bits and per-point |I_q| for the tile rule, the kept-pair count and per-
    point |I_q| (up to near ties) for GEOM. The column lists, built from the
    transposed row bits, carry the gradient: J and grad against the oracle."""
    import torch
    _say(f"culling with many tiles: {rule}, group {group}")
    p = W.cube_mixture(24, 2000, 1e-3)
    psi = W.random_psi(21, p.n, p.eps)
    dense = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps)
    tau = 1e-8
    prob = _problem(p.x, p.mu, p.y, p.nu, precision="mixed", truncation=rule, tau=tau,
                    tile_group=group)
    tile_of, block_of, nt, nb = prob.partition()
    assert nt > 4096 and p.n % 64 != 0
    prob.set_reference(abs(dense.J))
    r = prob.dual_eval(torch.as_tensor(psi, device="cuda"), p.eps)
    tile_of = tile_of.cpu().numpy()
    cnt = prob.kept_counts().cpu().numpy()
    if rule == "tile":
        slots = prob.target_slots().cpu().numpy()
        group_of = (slots // group).astype(np.int32)
        ng = nb * 64 // group
        ref = oracle.dual_eval_tile(p.x, p.mu, p.y, p.nu, psi, p.eps, tile_of, nt, group_of, ng,
                                    tau, abs(dense.J), want_L=True, want_keep=True)
        bits = prob.tile_chunk_keep().cpu().numpy()
        ref_bits, real = _chunk_keep_from_groups(ref.keep, slots, nb, group, p.n)
        realbits = np.packbits(real[:, ::-1], axis=1, bitorder="big").reshape(-1)
        assert np.array_equal(bits & realbits[None, :], ref_bits & realbits[None, :])
        ref_cnt = (ref.keep[tile_of] > 0).astype(np.int64) @ np.bincount(group_of, minlength=ng)
        assert np.array_equal(cnt, ref_cnt)
    else:
        C = r.info["cutoff"]
        ref = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps, cutoff=C, want_L=True)
        ref_cnt, near = oracle.kept_counts(p.x, p.y, C, rel_band=1e-12)
        assert np.all(np.abs(cnt.astype(np.int64) - ref_cnt) <= near)
    _say(f"  tiles {nt}, blocks {nb}: kept gpu {r.info['kept_pairs']} oracle {ref.kept} of "
         f"{p.nq * p.n}")
    assert r.info["kept_pairs"] == ref.kept
    assert 0 < ref.kept < p.nq * p.n
    _check(prob, p.x, p.mu, p.y, p.nu, psi, p.eps, "mixed", ref=ref, r=r)


def test_tile_rule_groups_keep_fewer_pairs():
    """Finer culling groups give a tighter rule: on the same problem groups
    of 8 targets keep fewer pairs than whole blocks, and every granularity
    stays within the tau |J| bound of the dense objective."""
    import torch
    p = W.cube_mixture(12, 6000, 1e-3)
    psi = W.random_psi(9, p.n, p.eps)
    dense = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps)
    kept = []
    for g in (64, 32, 16, 8):
        prob = _problem(p.x, p.mu, p.y, p.nu, precision="fp64", truncation="tile", tau=1e-8,
                        tile_group=g)
        prob.set_reference(abs(dense.J))
        r = prob.dual_eval(torch.as_tensor(psi, device="cuda"), p.eps)
        kept.append(r.info["kept_pairs"])
        assert -1e-13 * abs(dense.J) <= dense.J - r.J <= 1e-8 * abs(dense.J)
    _say(f"  kept pairs by group 64/32/16/8: {kept}")
    assert kept[-1] < kept[0]


def test_full_size_sampled_points():
    """Full-size 3D workload (6.29M points x 65,536 targets) in the launch
    configuration the benchmark times: the per-point L_q of 3,000 sampled
    points equal the oracle's (L_q depends on that point only), and the
    gradient sums to sum mu - sum nu."""
    import torch
    _say("full size sampled")
    p = W.config2()
    prob = _problem(torch.as_tensor(p.x, device="cuda"), torch.as_tensor(p.mu, device="cuda"),
                    torch.as_tensor(p.y, device="cuda"), torch.as_tensor(p.nu, device="cuda"))
    psi = W.random_psi(11, p.n, p.eps)
    r = prob.dual_eval(torch.as_tensor(psi, device="cuda"), p.eps)
    L = prob.lse().cpu().numpy()
    idx = np.random.default_rng(0).choice(p.nq, 3000, replace=False)
    ref = oracle.dual_eval(p.x[idx], p.mu[idx], p.y, p.nu, psi, p.eps, want_L=True)
    el = np.max(np.abs(L[idx] - ref.L) / np.maximum(1.0, np.abs(ref.L)))
    _say(f"  sampled L err {el:.2e}")
    assert el <= 1e-6
    g = r.grad.cpu().numpy()
    assert abs(g.sum() - (p.mu.sum() - p.nu.sum())) < 1e-9
    assert r.info["kept_pairs"] == p.nq * p.n


def test_full_size_disk_sampled_points():
    """Finest level of the 2D disk workload at full size (4,147,200 points x
    1,048,576 targets, eps 1e-4, psi ~ N(0, eps^2)), dense and then under the
    tile rule with tau = 1e-12 and the dense |J| as reference: per-point L_q
    of 512 sampled points equal the oracle's dense values (the tile rule's
    neglected mass is below eta = tau |J| / (eps sum mu) of the kept sum at
    every point, so its L_q moves by less than eta); both gradients sum to
    sum mu - sum nu within 1e-9 sum mu. On this uniform mesh at eps = 1e-4
    the dominant gradient-pass arguments would share one fractional part
    without the spread tile references, and the FP32 exponential's error at
    that one argument would not average to its (removed) mean."""
    import torch
    _say("full size disk, dense and tile rule")
    c3 = W.config3()
    x, mu = c3["sources"][-1]
    y, nu = c3["y"], c3["nu"]
    eps = 1e-4
    prob = _problem(*[torch.as_tensor(a, device="cuda") for a in (x, mu, y, nu)])
    psi = W.random_psi(11, y.shape[0], eps)
    pt = torch.as_tensor(psi, device="cuda")
    idx = np.random.default_rng(3).choice(x.shape[0], 512, replace=False)
    ref = oracle.dual_eval(x[idx], mu[idx], y, nu, psi, eps, want_L=True)
    r = prob.dual_eval(pt, eps)
    assert r.info["kept_pairs"] == x.shape[0] * y.shape[0]
    results = [("dense", r, prob.lse().cpu().numpy())]
    prob.set_truncation("tile", tau=1e-12)
    prob.set_reference(abs(r.J))
    rt = prob.dual_eval(pt, eps)
    assert rt.info["dense_fallback"] == 0
    assert 0 < rt.info["kept_pairs"] < x.shape[0] * y.shape[0]
    results.append(("tile", rt, prob.lse().cpu().numpy()))
    for name, res, L in results:
        el = np.max(np.abs(L[idx] - ref.L) / np.maximum(1.0, np.abs(ref.L)))
        gsum = float(res.grad.sum().item())
        _say(f"  {name}: kept {res.info['kept_pairs'] / (x.shape[0] * y.shape[0]):.4f}, "
             f"sampled L err {el:.2e}, sum g {gsum:.2e}, {res.info['kernel_ms']:.1f} ms")
        assert el <= 1e-6
        assert abs(gsum - (mu.sum() - nu.sum())) < 1e-9 * mu.sum()
    # truncation bound tau |J| plus the mixed path's 1e-9 on each of the two
    assert abs(rt.J - r.J) <= (1e-12 + 2e-9) * abs(r.J)


def test_full_size_disk_gradient_elementwise():
    """The disk's finest uniform mesh (4,147,200 points of nearly equal mass)
    against 8,192 of its targets at eps = 1e-4, mixed precision: the whole
    gradient element by element against the oracle's dense pass (run here,
    3.4e10 pairs), e_g <= 1e-6, and J within 1e-9. At
    this eps most of a point's mass sits in one target, so the gradient pass's
    dominant arguments sit near log2 mu_q, the same value at every point of a
    uniform mesh: a rounding of that argument that does not average out would
    show here as a systematic error."""
    import torch
    _say("full size disk, element-wise gradient, 8192 targets")
    c3 = W.config3()
    x, mu = c3["sources"][-1]
    sel = np.sort(np.random.default_rng(12).choice(c3["y"].shape[0], 8192, replace=False))
    y = np.ascontiguousarray(c3["y"][sel])
    nu = np.full(y.shape[0], mu.sum() / y.shape[0])
    eps = 1e-4
    psi = W.random_psi(13, y.shape[0], eps)
    prob = _problem(*[torch.as_tensor(a, device="cuda") for a in (x, mu, y, nu)])
    r = prob.dual_eval(torch.as_tensor(psi, device="cuda"), eps)
    assert r.info["fp64_pairs"] == 0          # the mixed path ran
    g = r.grad.cpu().numpy()
    ref = oracle.dual_eval(x, mu, y, nu, psi, eps)
    eg = grad_err(g, ref.grad, nu)
    ej = abs(r.J - ref.J) / abs(ref.J)
    _say(f"  e_g {eg:.2e}, J {ej:.2e}, sum g {g.sum():.2e}")
    assert eg <= 1e-6 and ej <= 1e-9
    assert abs(g.sum()) < 1e-9 * mu.sum()


@pytest.mark.parametrize("which", ["zero", "random", "lbfgs20"])
def test_full_size_error_table(which):
    """Full-size 3D workload at three potentials (zero, N(0, eps^2), the
    iterate after 20 L-BFGS iterations): sampled L_q against the oracle, and
    the mixed-precision objective and gradient against the FP64 path (which
    the oracle pins at smaller sizes) within the stated bounds (objective
    1e-9 relative, gradient 1e-6 against the local mass scale)."""
    import torch
    _say(f"full size error table: psi {which}")
    p = W.config2()
    dev = [torch.as_tensor(a, device="cuda") for a in (p.x, p.mu, p.y, p.nu)]
    prob = _problem(*dev)
    if which == "zero":
        psi = np.zeros(p.n)
    elif which == "random":
        psi = W.random_psi(11, p.n, p.eps)
    else:
        psi, info = prob.solve([p.eps], max_iter=20)
        _say(f"  20 iterations: |g|_1 {info['grad_l1']:.3e}")
    pt = torch.as_tensor(psi, device="cuda")
    r = prob.dual_eval(pt, p.eps)
    L = prob.lse().cpu().numpy()
    g = r.grad.cpu().numpy()
    prob.set_precision("fp64")
    r64 = prob.dual_eval(pt, p.eps)
    g64 = r64.grad.cpu().numpy()
    idx = np.random.default_rng(1).choice(p.nq, 2000, replace=False)
    ref = oracle.dual_eval(p.x[idx], p.mu[idx], p.y, p.nu, psi, p.eps, want_L=True)
    el = np.max(np.abs(L[idx] - ref.L) / np.maximum(1.0, np.abs(ref.L)))
    ej = abs(r.J - r64.J) / abs(r64.J)
    eg = np.max(np.abs(g - g64) / (p.nu + g64 + p.nu))
    _say(f"  sampled L err {el:.2e}, J mixed vs fp64 {ej:.2e}, grad {eg:.2e}")
    assert el <= 1e-6 and ej <= 1e-9 and eg <= 1e-6


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_size_gradient_against_stored_oracle(prec):
    """The 3D benchmark workload at full size (6,291,456 points x 65,536
    targets), dense, in the launch configuration the benchmark times: J and
    the whole gradient, element by element, against the oracle's stored dense
    pass at psi ~ N(0, eps^2) (seed 11; tests/golden/make_config2_golden.py),
    and L_q at its 4,096 stored points. Bounds: mixed e_g <= 1e-6, J <= 1e-9
    relative; FP64 e_g <= 1e-11, J <= 1e-12 (sums over 4e11 pairs in another
    order)."""
    import os
    import torch
    rec_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                            "config2_oracle.npz")
    rec = np.load(rec_path)
    _say(f"full size vs stored oracle, {prec}")
    p = W.config2()
    assert p.name == str(rec["workload"])
    prob = _problem(*[torch.as_tensor(a, device="cuda") for a in (p.x, p.mu, p.y, p.nu)],
                    precision=prec)
    psi = W.random_psi(int(rec["psi_seed"]), p.n, p.eps)
    r = prob.dual_eval(torch.as_tensor(psi, device="cuda"), p.eps)
    g = r.grad.cpu().numpy()
    gref = rec["grad"]
    eg = grad_err(g, gref, p.nu)
    ej = abs(r.J - float(rec["J"])) / abs(float(rec["J"]))
    L = prob.lse().cpu().numpy()[rec["L_index"]]
    el = float(np.max(np.abs(L - rec["L"]) / np.maximum(1.0, np.abs(rec["L"]))))
    _say(f"  J {r.J:.15e} vs {float(rec['J']):.15e}: {ej:.1e}; e_g {eg:.1e}; L {el:.1e}")
    tg, tj, tl = (1e-6, 1e-9, 1e-6) if prec == "mixed" else (1e-11, 1e-12, 1e-10)
    assert eg <= tg and ej <= tj and el <= tl
