"""FP64 reference of the learned warm-start network (TEST INFRASTRUCTURE ONLY).

Plain numpy, used by the tests, the smoke check and the benchmark's CPU leg
and by nothing else; it shares no code with the HIP library.

The network is not in the paper: it predicts the dual potential psi_j of
target j from six features (y_j in R^2, the source blob's centre c in R^2,
its width s, log eps), to warm-start the solver of Alg. 1. Reading used here:
six inputs, four hidden layers of width 256 with the exact (erf) GELU, one
linear output; 199,425 parameters.

Functions:
  layout / unpack      -- flat parameter order shared with the library's ABI
  gelu / gelu_prime    -- x Phi(x) and Phi(x) + x phi(x)
  bf16_round           -- round to nearest even to bfloat16, value kept in float
  features             -- (y0, y1, c0, c1, s, log eps) per target
  forward              -- standardise inputs, 4 x (affine, GELU), affine out
  backward             -- gradient of sum_r dout_r * out_r w.r.t. all params
  mse                  -- mean squared error in standardised output units
  adam                 -- one Adam step (Kingma & Ba, Algorithm 1)
  centre               -- shift so that sum_j nu_j psi_j = 0 (the solver's gauge)

``emulate_bf16=True`` rounds to bfloat16 at the points where the device
stores bfloat16: the weight matrices (not the biases), every hidden
activation, and every pre-activation gradient that feeds a matrix product.
Everything else stays FP64 here (FP32 on the device).

Parity pins: tests/test_oracle_pins_mlp.py (finite differences, GELU closed
forms, zero-weight network, Adam's first-step identity, RNE rounding against
the library conversion).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_IN = 6
WIDTH = 256
N_HIDDEN = 4


def layout():
    """(name, shape) of every parameter block in flat order. Weight matrices
    are [fan_in][fan_out] row-major."""
    out = [("W0", (N_IN, WIDTH)), ("b0", (WIDTH,))]
    for l in range(1, N_HIDDEN):
        out += [(f"W{l}", (WIDTH, WIDTH)), (f"b{l}", (WIDTH,))]
    out += [(f"W{N_HIDDEN}", (WIDTH,)), (f"b{N_HIDDEN}", (1,))]
    return out


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in layout()))


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (n_params(),)
    out, off = {}, 0
    for name, shape in layout():
        k = int(np.prod(shape))
        out[name] = theta[off:off + k].reshape(shape)
        off += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1)
                           for name, _ in layout()])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_prime(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def bf16_round(x):
    """Nearest bfloat16 (ties to even) of the float32 value of x, returned as
    float64. Finite inputs only."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def features(y, c, s, eps):
    """Per-target input rows (y0, y1, c0, c1, s, log eps)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    f = np.empty((n, N_IN))
    f[:, 0:2] = y
    f[:, 2] = c[0]
    f[:, 3] = c[1]
    f[:, 4] = s
    f[:, 5] = math.log(eps)
    return f


def _weights(P, emulate):
    W = {}
    for l in range(N_HIDDEN + 1):
        w = P[f"W{l}"]
        W[l] = bf16_round(w) if emulate else w
    return W


def forward(theta, feats, norm, emulate_bf16=False):
    """Returns (psi, cache): psi = o * out_std + out_mean with o the
    standardised output. ``norm`` = (feat_mean[6], feat_std[6], out_mean,
    out_std)."""
    P = unpack(theta)
    W = _weights(P, emulate_bf16)
    fm, fs, om, osd = norm
    F = (np.asarray(feats, dtype=np.float64) - np.asarray(fm)) / np.asarray(fs)
    rnd = bf16_round if emulate_bf16 else (lambda a: a)
    zs, hs = [], []
    h = F
    for l in range(N_HIDDEN):
        z = h @ W[l] + P[f"b{l}"]
        h = rnd(gelu(z))
        zs.append(z)
        hs.append(h)
    o = h @ W[N_HIDDEN] + P[f"b{N_HIDDEN}"][0]
    cache = dict(F=F, z=zs, h=hs, o=o, W=W, emulate=emulate_bf16)
    return o * osd + om, cache


def backward(theta, cache, dout_std):
    """Gradient (flat, FP64) of sum_r dout_std[r] * o_r with respect to every
    parameter, o the standardised output of ``forward``."""
    P = unpack(theta)
    W = cache["W"]
    rnd = bf16_round if cache["emulate"] else (lambda a: a)
    d = np.asarray(dout_std, dtype=np.float64)
    hs, zs = cache["h"], cache["z"]
    G = {f"W{N_HIDDEN}": hs[-1].T @ d, f"b{N_HIDDEN}": np.array([d.sum()])}
    dz = rnd(np.outer(d, W[N_HIDDEN]) * gelu_prime(zs[-1]))
    for l in range(N_HIDDEN - 1, 0, -1):
        G[f"W{l}"] = hs[l - 1].T @ dz
        G[f"b{l}"] = dz.sum(axis=0)
        dz = rnd((dz @ W[l].T) * gelu_prime(zs[l - 1]))
    G["W0"] = cache["F"].T @ dz
    G["b0"] = dz.sum(axis=0)
    del P
    return pack(G)


def mse(o_std, target, norm):
    """Loss mean_r (o_r - t_r)^2 with t standardised by the output mean/std,
    and its derivative with respect to o."""
    om, osd = norm[2], norm[3]
    t = (np.asarray(target, dtype=np.float64) - om) / osd
    r = np.asarray(o_std, dtype=np.float64) - t
    n = r.shape[0]
    return float(np.mean(r * r)), 2.0 * r / n


def adam(theta, m, v, g, lr, b1, b2, eps, step):
    """One Adam step; ``step`` counts from 1. Returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def centre(psi, nu):
    psi = np.asarray(psi, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    return psi - np.dot(nu, psi) / nu.sum()
