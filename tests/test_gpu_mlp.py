"""GPU parity of the warm-start network kernels (include/rsot_mlp.h) against
the FP64 reference oracle/mlp.py.

Tolerances. The reference run with ``emulate_bf16=True`` rounds at the same
points as the device, so what is left is FP32 against FP64 accumulation
(about 1e-6 relative per sum) and the bfloat16 roundings this flips (one
unit of 2^-8 on a few activations per row). Redoing the reference with
FP32 sums on the CPU at these sizes moves the output by 8e-5 normwise (1e-3
of max|o| at worst) and the gradients by 5e-4 normwise; the bounds below
allow 4-5 times that. Against the unrounded FP64 network the gap is the
bfloat16 arithmetic itself (2e-3 on outputs, 5e-3 on gradients); bound 2e-2.
"""
import sys

import numpy as np
import pytest

from oracle import mlp as M
from paper_2507_23602_amd import workloads as W

pytestmark = pytest.mark.gpu

OM, OS = 0.01, 0.2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _feats(seed, R):
    rng = np.random.default_rng(seed)
    f = np.empty((R, 6))
    f[:, :2] = rng.uniform(0, 1, (R, 2))
    f[:, 2:4] = rng.uniform(0.2, 0.8, (R, 2))
    f[:, 4] = rng.uniform(0.05, 0.2, R)
    f[:, 5] = np.log(rng.uniform(1e-3, 1e-1, R))
    return f.astype(np.float32)


def _norm(f):
    fm = f.astype(np.float64).mean(0).astype(np.float32)
    fs = f.astype(np.float64).std(0).astype(np.float32)
    return fm, fs


def _model(seed=0, f=None):
    from paper_2507_23602_amd import rsot
    th = W.mlp_init_params(seed)
    m = rsot.MLP(th)
    fm, fs = _norm(f if f is not None else _feats(99, 4096))
    m.set_normalization(fm, fs, OM, OS)
    norm = (fm.astype(np.float64), fs.astype(np.float64), float(np.float32(OM)),
            float(np.float32(OS)))
    return m, th.astype(np.float64), norm


def _abs_backward(cache, dout):
    """The backward recursion of oracle.mlp with every factor replaced by its
    magnitude: for each gradient element the sum of the magnitudes of the
    terms it adds up, the scale of the rounding error it can carry."""
    W, hs, zs = cache["W"], cache["h"], cache["z"]
    NH = M.N_HIDDEN
    d = np.abs(np.asarray(dout, dtype=np.float64))
    G = {f"W{NH}": np.abs(hs[-1]).T @ d, f"b{NH}": np.array([d.sum()])}
    dz = np.outer(d, np.abs(W[NH])) * np.abs(M.gelu_prime(zs[-1]))
    for l in range(NH - 1, 0, -1):
        G[f"W{l}"] = np.abs(hs[l - 1]).T @ dz
        G[f"b{l}"] = dz.sum(axis=0)
        dz = (dz @ np.abs(W[l]).T) * np.abs(M.gelu_prime(zs[l - 1]))
    G["W0"] = np.abs(cache["F"]).T @ dz
    G["b0"] = dz.sum(axis=0)
    return M.pack(G)


def _blocks():
    off, out = 0, {}
    for name, shape in M.layout():
        k = int(np.prod(shape))
        out[name] = slice(off, off + k)
        off += k
    return out


def test_device_weights_are_rne_bf16_of_masters():
    m, th, _ = _model(1)
    used = m.params(1).astype(np.float64)
    B = _blocks()
    for name, sl in B.items():
        ref = M.bf16_round(th[sl]) if name.startswith("W") else th[sl].astype(np.float32)
        np.testing.assert_array_equal(used[sl], ref, err_msg=name)
    np.testing.assert_array_equal(m.params(0), th.astype(np.float32))


@pytest.mark.parametrize("R", [1, 1000, 1024, 1025, 3000])
def test_forward_matches_reference(R):
    import torch
    _say(f"forward R={R}")
    m, th, norm = _model(2)
    f = _feats(3 + R, R)
    out = m.forward(torch.as_tensor(f, device="cuda")).cpu().numpy().astype(np.float64)
    o_dev = (out - norm[2]) / norm[3]
    _, c = M.forward(th, f.astype(np.float64), norm, emulate_bf16=True)
    o = c["o"]
    err = np.abs(o_dev - o)
    _say(f"  max {err.max():.2e} norm {np.linalg.norm(o_dev - o) / np.linalg.norm(o):.2e} "
         f"max|o| {np.abs(o).max():.2e}")
    assert np.linalg.norm(o_dev - o) <= 5e-4 * np.linalg.norm(o)
    assert err.max() <= 5e-3 * np.abs(o).max()
    _, cf = M.forward(th, f.astype(np.float64), norm, emulate_bf16=False)
    assert np.linalg.norm(o_dev - cf["o"]) <= 2e-2 * np.linalg.norm(cf["o"])


@pytest.mark.parametrize("R", [700, 3000])
def test_backward_matches_reference(R):
    import torch
    _say(f"backward R={R}")
    m, th, norm = _model(4)
    f = _feats(5, R)
    dout = np.random.default_rng(6).standard_normal(R).astype(np.float32)
    g = m.backward(torch.as_tensor(f, device="cuda"),
                   torch.as_tensor(dout, device="cuda")).cpu().numpy().astype(np.float64)
    _, c = M.forward(th, f.astype(np.float64), norm, emulate_bf16=True)
    ref = M.backward(th, c, dout.astype(np.float64) * norm[3])
    _, cf = M.forward(th, f.astype(np.float64), norm)
    ref64 = M.backward(th, cf, dout.astype(np.float64) * norm[3])
    # element by element: each gradient entry within 5e-4 of the magnitude
    # sum of its terms (FP32 sums: ~1e-6 of it; an activation whose bf16
    # rounding flips moves its terms by 2^-8; measured worst 5e-5)
    S = _abs_backward(c, dout.astype(np.float64) * norm[3])
    for name, sl in _blocks().items():
        e = np.linalg.norm(g[sl] - ref[sl]) / np.linalg.norm(ref[sl])
        e64 = np.linalg.norm(g[sl] - ref64[sl]) / np.linalg.norm(ref64[sl])
        ratio = float(np.max(np.abs(g[sl] - ref[sl]) / (S[sl] + 1e-30)))
        _say(f"  {name}: {e:.2e} (fp64 {e64:.2e}), worst element {ratio:.2e} of its term sum")
        assert e <= 2e-3, name
        assert e64 <= 2e-2, name
        assert ratio <= 5e-4, name


def test_adam_matches_reference_and_remakes_copies():
    import torch
    m, th, _ = _model(7)
    rng = np.random.default_rng(8)
    mm, vv, p = np.zeros_like(th), np.zeros_like(th), th.copy()
    for step in (1, 2, 3):
        g = (rng.standard_normal(th.size) * 10.0 ** rng.integers(-4, 1, th.size)).astype(np.float32)
        m.adam_step(torch.as_tensor(g, device="cuda"), lr=1e-3, b1=0.9, b2=0.999, eps=1e-8)
        p, mm, vv = M.adam(p, mm, vv, g.astype(np.float64), 1e-3, 0.9, 0.999, 1e-8, step)
    got = m.params(0).astype(np.float64)
    np.testing.assert_allclose(got, p, rtol=2e-6, atol=1e-8)
    used = m.params(1).astype(np.float64)
    for name, sl in _blocks().items():
        if name.startswith("W"):
            np.testing.assert_array_equal(used[sl], M.bf16_round(got[sl]), err_msg=name)


def test_train_step_matches_reference():
    """Forward, MSE, backward and Adam fused, on a gathered batch. With Adam's
    eps = 1 the first step is lr g / (|g| + 1), close to lr g, so the update
    carries the gradient itself rather than its sign."""
    import torch
    m, th, norm = _model(9)
    N, R = 3000, 2500
    f = _feats(10, N)
    t = (np.sin(3 * f[:, 0]) * 0.05 + 0.02 * f[:, 1]).astype(np.float32)
    idx = np.random.default_rng(11).permutation(N)[:R].astype(np.int64)
    ft, tt = torch.as_tensor(f, device="cuda"), torch.as_tensor(t, device="cuda")
    it = torch.as_tensor(idx, device="cuda")
    loss = m.train_step(ft, tt, it, lr=1e-3, b1=0.9, b2=0.999, eps=1.0)
    fb = f[idx].astype(np.float64)
    _, c = M.forward(th, fb, norm, emulate_bf16=True)
    L, dL = M.mse(c["o"], t[idx].astype(np.float64), norm)
    g = M.backward(th, c, dL)
    p, _, _ = M.adam(th, np.zeros_like(th), np.zeros_like(th), g, 1e-3, 0.9, 0.999, 1.0, 1)
    _say(f"train step: loss {loss:.6e} ref {L:.6e}")
    assert abs(loss - L) <= 1e-4 * L
    got = m.params(0).astype(np.float64)
    for name, sl in _blocks().items():
        d, dr = got[sl] - th[sl], p[sl] - th[sl]
        # the update is below one FP32 ulp of some masters: compare it where
        # it is resolved, i.e. against the master's own spacing
        tol = 3e-3 * np.linalg.norm(dr) + np.linalg.norm(np.spacing(th[sl].astype(np.float32)))
        assert np.linalg.norm(d - dr) <= tol, name


def test_train_step_is_deterministic_and_reduces_loss():
    import torch
    N = 4096
    f = _feats(12, N)
    t = (0.05 * np.sin(4 * f[:, 0]) * np.cos(3 * f[:, 1]) + 0.1 * f[:, 4]).astype(np.float32)
    ft, tt = torch.as_tensor(f, device="cuda"), torch.as_tensor(t, device="cuda")
    runs = []
    for _ in range(2):
        m, _, _ = _model(13, f)
        m.fit_normalization(ft, tt)
        losses = [m.train_step(ft, tt, None, lr=2e-3) for _ in range(60)]
        runs.append((m.params(0), losses))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    assert runs[0][1] == runs[1][1]
    _say(f"loss {runs[0][1][0]:.3e} -> {runs[0][1][-1]:.3e}")
    assert runs[0][1][-1] < 0.1 * runs[0][1][0]


def test_fit_normalization_matches_moments():
    import torch
    m, _, _ = _model(14)
    f = _feats(15, 5000)
    t = np.random.default_rng(16).standard_normal(5000).astype(np.float32) * 0.3 + 0.1
    m.fit_normalization(torch.as_tensor(f, device="cuda"), torch.as_tensor(t, device="cuda"))
    fm, fs, om, osd = m.normalization()
    f64 = f.astype(np.float64)
    np.testing.assert_allclose(fm, f64.mean(0), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(fs, f64.std(0), rtol=1e-5)
    assert abs(om - t.astype(np.float64).mean()) < 1e-6
    assert abs(osd - t.astype(np.float64).std()) < 1e-6 * t.std()


def test_features_and_centred_prediction():
    import torch
    from paper_2507_23602_amd import rsot
    m, th, norm = _model(17)
    rng = np.random.default_rng(18)
    n = 1537
    y = rng.uniform(0, 1, (n, 2))
    nu = rng.uniform(0.5, 1.5, n)
    cond = (0.4, 0.6, 0.11, 3e-3)
    fd = rsot.mlp_features(torch.as_tensor(y, device="cuda"), cond).cpu().numpy()
    np.testing.assert_array_equal(fd, M.features(y, cond[:2], cond[2], cond[3]).astype(np.float32))
    psi = m.predict_psi(torch.as_tensor(y, device="cuda"), torch.as_tensor(nu, device="cuda"),
                        cond).cpu().numpy()
    assert abs(np.dot(nu, psi)) <= 1e-12 * np.dot(nu, np.abs(psi))
    ref, _ = M.forward(th, fd.astype(np.float64), norm, emulate_bf16=True)
    ref = M.centre(ref, nu)
    assert np.linalg.norm(psi - ref) <= 5e-4 * norm[3] * np.sqrt(n) + 5e-4 * np.linalg.norm(ref)


def test_invalid_arguments_are_rejected():
    import torch
    from paper_2507_23602_amd import rsot
    m, _, _ = _model(19)
    with pytest.raises(rsot.RsotError):
        m.set_normalization(np.zeros(6), np.zeros(6), 0.0, 1.0)      # std 0
    with pytest.raises(rsot.RsotError):
        m.set_normalization(np.zeros(6), np.ones(6), 0.0, -1.0)
    bad = W.mlp_init_params(0)
    bad[5] = np.nan
    with pytest.raises(rsot.RsotError):
        rsot.MLP(bad)
    with pytest.raises(rsot.RsotError):
        m.adam_step(torch.zeros(rsot.MLP_NPARAMS, device="cuda"), lr=0.0)
    with pytest.raises(rsot.RsotError):
        rsot.mlp_features(torch.zeros((3, 2), dtype=torch.float64, device="cuda"),
                          (0.5, 0.5, 0.1, 0.0))                         # eps = 0
    assert m.forward(torch.zeros((0, 6), device="cuda")).numel() == 0


def _small_instance(i):
    return W.config4_instance(i, n_cells=16, n_targets=512)


def test_learned_start_on_held_out_instances():
    """The learned warm start generalises: trained on the solutions of 128
    blob instances (16 x 16 mesh, 512 targets), it starts 8 other instances
    with fewer L-BFGS iterations to ||grad||_1 < 1e-6 than the zero start with
    the eps schedule and than the combined multilevel start (Sec. 5.3), on
    average, and its solutions pass the oracle's gradient check."""
    import torch
    from paper_2507_23602_amd import rsot, warmstart
    train_ids, test_ids = list(range(3000, 3128)), list(range(3200, 3208))
    feats, target, recs = warmstart.build_dataset(train_ids, n_cells=16, n_targets=512,
                                                  every=64)
    assert all(r["status"] == rsot.OK for r in recs)
    m, log = warmstart.train(feats, target, epochs=60, batch=4096, lr=2e-3)
    _say(f"  trained: final batch loss {log[-1]['train_batch_loss']:.3e}")
    res = warmstart.compare(m, test_ids, n_cells=16, n_targets=512, coarse_cells=(4, 8),
                            target_levels=(32, 128), keep_psi=len(test_ids))
    s = warmstart.summarize(res)
    _say(f"  {s}")
    it = {k: s[k]["mean_iterations"] for k in ("zero_sched", "learned", "multilevel")}
    assert s["learned_used"] >= 6
    assert it["learned"] < it["zero_sched"] and it["learned"] < it["multilevel"]
    for r in res:
        assert r["learned"]["status"] == rsot.OK
        p = W.config4_instance(r["id"], n_cells=16, n_targets=512)
        g = oracle_grad_l1(p, r["learned"]["psi"])
        assert g <= 1.5e-6, (r["id"], g)


def oracle_grad_l1(p, psi):
    import oracle
    return float(np.abs(oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps).grad).sum())


def test_solve_learned_uses_a_good_start_and_falls_back_on_a_bad_one():
    """After fitting one instance's solution, the solve from the learned start
    is taken (lower J than zero) and needs fewer iterations than the eps
    schedule from zero; an untrained model's start is rejected when it is
    worse than zero. Either way the result equals the zero-start solution."""
    import torch
    from paper_2507_23602_amd import rsot
    p = _small_instance(3)
    cond = (p.meta["c"][0], p.meta["c"][1], p.meta["s"], p.eps)
    sched = [p.eps * 2.0 ** k for k in range(6, 0, -1) if p.eps * 2.0 ** k < 0.5] + [p.eps]
    pr = rsot.Problem(p.x, p.mu, p.y, p.nu)
    psi0, i0 = pr.solve(sched)
    _say(f"zero start: {i0['iterations']} it, status {i0['status']}")
    assert i0["status"] == rsot.OK
    # fit the network to this solution
    f = rsot.mlp_features(torch.as_tensor(p.y, device="cuda"), cond)
    t = torch.as_tensor(psi0.astype(np.float32), device="cuda")
    m, _, _ = _model(20)
    m.fit_normalization(f, t)
    for _ in range(400):
        m.train_step(f, t, None, lr=1e-3, want_loss=False)
    psi1, i1, l1 = pr.solve_learned(m, cond, sched)
    _say(f"learned: used {l1['used_learned']}, J_pred {l1['J_pred']:.6e} J_zero {l1['J_zero']:.6e}, "
         f"{i1['iterations']} it")
    assert l1["used_learned"] == 1 and l1["J_pred"] < l1["J_zero"]
    assert i1["status"] == rsot.OK and i1["iterations"] < i0["iterations"]
    scale = np.max(np.abs(psi0))
    assert np.max(np.abs(psi1 - psi0)) <= 1e-4 * scale
    # an untrained network with a shifted, scaled output: worse than zero
    m2, _, _ = _model(21)
    m2.set_normalization(np.full(6, 0.5), np.full(6, 0.3), 0.0, 5.0)
    psi2, i2, l2 = pr.solve_learned(m2, cond, sched)
    _say(f"untrained: used {l2['used_learned']}, J_pred {l2['J_pred']:.6e} J_zero {l2['J_zero']:.6e}")
    assert l2["used_learned"] == (1 if l2["J_pred"] < l2["J_zero"] else 0)
    assert i2["status"] == rsot.OK
    assert np.max(np.abs(psi2 - psi0)) <= 1e-4 * scale
