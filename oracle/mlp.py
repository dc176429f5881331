"""FP64 reference of the constitutive surrogate network (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the test-suite is the
only caller.  Nothing here is used by the HIP library or its binding.

The surrogate replaces the intralaminar update of Section 2.3.1 (Algorithm 4)
by a multilayer perceptron 10 -> 64 -> 64 -> 64 -> 10 with SiLU hidden
activations:

  inputs   x = (eps_k * E_k / X_k for the six material-frame strain
               components, s_N = 1 - 1/r_N for the four damage thresholds);
  outputs  y = (sigma_k / X_k for the six stresses, then the four new s_N
               through a logistic sigmoid).

(E_k, X_k) = (E1, XT), (E2, YT), (E2, YT), (G23, SL), (G12, SL), (G12, SL).
The loss is the mean square error over samples and the ten outputs.

Parameters are one flat float vector in this order (W stored [in][out]):
W1[10][64], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[64][10], b4[10].

``quant="bf16"`` rounds the inputs, weights, activations and (in the
gradient) the SiLU derivatives and back-propagated errors to bfloat16 (round to nearest even)
before the FP64 arithmetic: the operands the matrix cores receive.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 10, 64, 10
SHAPES = [(N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, N_OUT), (N_OUT,)]
N_PARAMS = int(sum(np.prod(s) for s in SHAPES))          # 9674
N_LINEAR = 6                                               # stress outputs (no sigmoid)


def unpack(w: np.ndarray):
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    assert w.size == N_PARAMS
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(w[o:o + n].reshape(s))
        o += n
    return out


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s + z * s * (1.0 - s)


def forward(w, x, quant: str | None = None, keep: bool = False):
    """y = f(x) for x of shape (n, 10); with keep=True also the layer values."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(w)
    x = np.asarray(x, dtype=np.float64)
    if quant == "bf16":
        W1, b1, W2, W3, W4 = (bf16_round(a) for a in (W1, b1, W2, W3, W4))
        x = bf16_round(x)
    z1 = x @ W1 + b1
    h1 = silu(z1)
    if quant == "bf16":
        h1 = bf16_round(h1)
    z2 = h1 @ W2 + b2
    h2 = silu(z2)
    if quant == "bf16":
        h2 = bf16_round(h2)
    z3 = h2 @ W3 + b3
    h3 = silu(z3)
    if quant == "bf16":
        h3 = bf16_round(h3)
    z4 = h3 @ W4 + b4
    y = z4.copy()
    y[:, N_LINEAR:] = sigmoid(z4[:, N_LINEAR:])
    if keep:
        return y, (x, z1, h1, z2, h2, z3, h3, z4)
    return y


def loss(w, x, t, quant: str | None = None) -> float:
    y = forward(w, x, quant)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(w, x, t, quant: str | None = None):
    """(loss, d loss / d w) by back-propagation through the layers above."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(w)
    if quant == "bf16":
        W2, W3, W4 = bf16_round(W2), bf16_round(W3), bf16_round(W4)
    y, (x0, z1, h1, z2, h2, z3, h3, z4) = forward(w, x, quant, keep=True)
    t = np.asarray(t, dtype=np.float64)
    n = y.shape[0]
    L = float(np.mean((y - t) ** 2))
    # with quant="bf16" the back-propagated errors are bf16 operands too
    q = bf16_round if quant == "bf16" else (lambda a: a)
    dy = 2.0 * (y - t) / (n * N_OUT)
    dz4 = dy.copy()
    dz4[:, N_LINEAR:] *= y[:, N_LINEAR:] * (1.0 - y[:, N_LINEAR:])
    dz4 = q(dz4)
    gW4, gb4 = h3.T @ dz4, dz4.sum(0)
    dz3 = q((dz4 @ W4.T) * q(dsilu(z3)))
    gW3, gb3 = h2.T @ dz3, dz3.sum(0)
    dz2 = q((dz3 @ W3.T) * q(dsilu(z2)))
    gW2, gb2 = h1.T @ dz2, dz2.sum(0)
    dz1 = q((dz2 @ W2.T) * q(dsilu(z1)))
    gW1, gb1 = x0.T @ dz1, dz1.sum(0)
    g = np.concatenate([a.reshape(-1) for a in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])
    return L, g


def init(seed: int = 1) -> np.ndarray:
    """Glorot-uniform weights, zero biases (a seeded starting point)."""
    rs = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            a = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rs.uniform(-a, a, size=s).reshape(-1))
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)
