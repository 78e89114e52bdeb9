"""Pins of the FP64 warm-start network reference (oracle/mlp.py) against facts
that do not come from the reference itself."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def _net(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shape in M.layout():
        fan_in = shape[0] if len(shape) == 2 else M.WIDTH
        parts[name] = rng.uniform(-1, 1, size=shape) * scale / math.sqrt(fan_in)
        if name.startswith("b"):
            parts[name] = rng.uniform(-0.3, 0.3, size=shape)
    return M.pack(parts)


NORM = (np.array([0.5, 0.5, 0.5, 0.5, 0.12, -4.6]), np.array([0.29, 0.29, 0.17, 0.17, 0.04, 1.3]),
        0.01, 0.2)


def _feats(seed, n):
    rng = np.random.default_rng(seed)
    f = np.empty((n, 6))
    f[:, :4] = rng.uniform(0, 1, size=(n, 4))
    f[:, 4] = rng.uniform(0.05, 0.2, size=n)
    f[:, 5] = np.log(rng.uniform(1e-3, 1e-1, size=n))
    return f


def test_parameter_count_matches_architecture():
    # 6*256+256 + 3*(256*256+256) + 256+1
    assert M.n_params() == 1792 + 3 * 65792 + 257 == 199425


def test_gelu_closed_forms():
    phi1 = 0.8413447460685429  # standard normal CDF at 1 (tables)
    assert M.gelu(np.array(0.0)) == 0.0
    assert abs(M.gelu(np.array(1.0)) - phi1) < 1e-15
    assert abs(M.gelu(np.array(-1.0)) + (1.0 - phi1)) < 1e-15
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(M.gelu(x) - M.gelu(-x), x, atol=1e-14)   # x Phi(x) + x Phi(-x) = x
    assert M.gelu_prime(np.array(0.0)) == 0.5
    h = 1e-5
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_prime(x), fd, atol=1e-9)


def test_zero_hidden_weights_give_constant_output():
    """With W1..W3 = 0 every row sees h3 = GELU(b3), so o = W4 . GELU(b3) + b4."""
    P = M.unpack(_net(3))
    for l in (1, 2, 3):
        P[f"W{l}"] = np.zeros_like(P[f"W{l}"])
    th = M.pack(P)
    psi, cache = M.forward(th, _feats(4, 9), NORM)
    o = float(np.dot(P["W4"], 0.5 * P["b3"] * (1 + np.vectorize(math.erf)(P["b3"] / math.sqrt(2))))
              + P["b4"][0])
    np.testing.assert_allclose(cache["o"], o, rtol=1e-13)
    np.testing.assert_allclose(psi, o * NORM[3] + NORM[2], rtol=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_finite_differences(seed):
    th = _net(seed, scale=1.5)
    F = _feats(10 + seed, 5)
    d = np.random.default_rng(20 + seed).standard_normal(5)

    def loss(t):
        return float(np.dot(d, M.forward(t, F, NORM)[1]["o"]))

    _, cache = M.forward(th, F, NORM)
    g = M.backward(th, cache, d)
    rng = np.random.default_rng(30 + seed)
    # every block: W0, b0 and the output layer in full, samples of the rest
    idx = list(range(0, 1792, 7)) + list(rng.integers(1792, M.n_params() - 257, 300)) + \
        list(range(M.n_params() - 257, M.n_params(), 3))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (loss(th + e) - loss(th - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_mse_derivative_matches_finite_differences():
    rng = np.random.default_rng(5)
    o, t = rng.standard_normal(7), rng.standard_normal(7)
    L, dL = M.mse(o, t, NORM)
    tt = (t - NORM[2]) / NORM[3]
    assert abs(L - np.mean((o - tt) ** 2)) < 1e-14
    h = 1e-6
    for i in range(7):
        e = np.zeros(7)
        e[i] = h
        fd = (M.mse(o + e, t, NORM)[0] - M.mse(o - e, t, NORM)[0]) / (2 * h)
        assert abs(fd - dL[i]) < 1e-8


def test_adam_constant_gradient_moves_linearly():
    """Under a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each step moves by lr g / (|g| + eps); with eps = 0 the
    first step is exactly lr sign(g)."""
    rng = np.random.default_rng(6)
    g = rng.standard_normal(50)
    th0 = rng.standard_normal(50)
    th, m, v = th0.copy(), np.zeros(50), np.zeros(50)
    th1, _, _ = M.adam(th0, m, v, g, 1e-3, 0.9, 0.999, 0.0, 1)
    np.testing.assert_allclose(th1, th0 - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    for t in range(1, 31):
        th, m, v = M.adam(th, m, v, g, 1e-3, 0.9, 0.999, 1e-8, t)
    np.testing.assert_allclose(th, th0 - 30 * 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_bf16_round_matches_library_conversion():
    import torch
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 8, 2000),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, 2 ** -130]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16_round(x), ref)
    # ties go to the even mantissa
    assert M.bf16_round(np.array(1 + 2 ** -8)) == 1.0
    assert M.bf16_round(np.array(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def test_bf16_emulation_stays_close_to_fp64():
    """Rounding weights and activations to 8 significant bits moves the output
    by a few parts in a thousand of its spread, not more."""
    th = _net(8)
    F = _feats(9, 200)
    a = M.forward(th, F, NORM)[1]["o"]
    b = M.forward(th, F, NORM, emulate_bf16=True)[1]["o"]
    assert np.max(np.abs(a - b)) < 2e-2 * (np.std(a) + np.max(np.abs(a)))
    assert np.max(np.abs(a - b)) > 0.0


def test_centre_fixes_gauge():
    rng = np.random.default_rng(11)
    psi, nu = rng.standard_normal(40), rng.uniform(0.5, 1.5, 40)
    c = M.centre(psi, nu)
    assert abs(np.dot(nu, c)) < 1e-13
    np.testing.assert_allclose(M.centre(psi + 3.0, nu), c, atol=1e-13)


def test_features_layout():
    y = np.array([[0.1, 0.2], [0.3, 0.4]])
    f = M.features(y, (0.5, 0.6), 0.07, 1e-2)
    np.testing.assert_array_equal(f[:, :2], y)
    np.testing.assert_array_equal(f[:, 2:5], [[0.5, 0.6, 0.07]] * 2)
    assert np.all(f[:, 5] == math.log(1e-2))
