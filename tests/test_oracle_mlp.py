"""Pins of the FP64 surrogate network reference (oracle/mlp.py) and of the
training-path recipe: finite differences, closed forms, an affine regime in
which the network reduces to a product of its matrices."""
import numpy as np

import workloads as W
from oracle import mlp


def _rand_problem(seed=3, n=37):
    rs = np.random.default_rng(seed)
    w = mlp.init(seed)
    w += 0.05 * rs.standard_normal(w.size)            # non-zero biases too
    x = rs.uniform(-2, 2, size=(n, mlp.N_IN))
    t = rs.uniform(-1, 1, size=(n, mlp.N_OUT))
    return w, x, t


def test_gradient_matches_central_differences():
    w, x, t = _rand_problem()
    L, g = mlp.grad(w, x, t)
    assert abs(L - mlp.loss(w, x, t)) <= 1e-15 * L
    rs = np.random.default_rng(0)
    idx = np.concatenate([rs.choice(mlp.N_PARAMS, 150, replace=False),
                          [0, 639, 640, 703, 704, 4800, 8900, 9663, 9664, 9673]])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss(wp, x, t) - mlp.loss(wm, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(abs(g).max(), 1e-30), (i, fd, g[i])


def test_affine_regime_is_the_matrix_product():
    """With large positive hidden biases every SiLU is the identity to 1e-17,
    so the stress outputs are x W1 W2 W3 W4 plus the propagated biases."""
    rs = np.random.default_rng(5)
    W1, W2, W3, W4 = (0.01 * rs.standard_normal(s) for s in ((10, 64), (64, 64), (64, 64), (64, 10)))
    b1, b2, b3 = 40.0 + rs.uniform(size=64), 40.0 + rs.uniform(size=64), 40.0 + rs.uniform(size=64)
    b4 = rs.uniform(-1, 1, size=10)
    w = np.concatenate([a.reshape(-1) for a in (W1, b1, W2, b2, W3, b3, W4, b4)])
    x = rs.uniform(-3, 3, size=(9, 10))
    y = mlp.forward(w, x)
    lin = (((x @ W1 + b1) @ W2 + b2) @ W3 + b3) @ W4 + b4
    assert np.allclose(y[:, :6], lin[:, :6], rtol=1e-12, atol=1e-12)
    assert np.allclose(y[:, 6:], 1.0 / (1.0 + np.exp(-lin[:, 6:])), rtol=1e-12, atol=1e-12)
    # a transposed weight would not reproduce it
    wt = np.concatenate([a.reshape(-1) for a in (W1, b1, W2.T, b2, W3, b3, W4, b4)])
    assert not np.allclose(mlp.forward(wt, x)[:, :6], lin[:, :6], rtol=1e-6)


def test_closed_forms():
    assert mlp.silu(0.0) == 0.0 and mlp.dsilu(0.0) == 0.5 and mlp.sigmoid(0.0) == 0.5
    assert abs(mlp.silu(1.0) - 1.0 / (1.0 + np.exp(-1.0))) < 1e-16
    w = np.zeros(mlp.N_PARAMS)
    b4 = np.arange(10) * 0.1 - 0.3
    w[-10:] = b4
    y = mlp.forward(w, np.ones((3, 10)))
    assert np.array_equal(y[:, :6], np.tile(b4[:6], (3, 1)))
    assert np.allclose(y[:, 6:], 1.0 / (1.0 + np.exp(-b4[6:])), rtol=1e-15)
    assert mlp.N_PARAMS == 9674


def test_bf16_rounding_ties_to_even():
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 3.14159, -2.0 ** -130, 65504.0])
    r = mlp.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                                  # halfway: even mantissa kept
    assert r[2] == 1.0 + 2.0 ** -6                      # halfway: rounds up to even
    assert r[3] == 3.140625
    assert r[4] == -2.0 ** -130                         # subnormal kept exactly (high half only)
    assert r[5] == 65536.0


def test_path_recipe():
    for p in range(40):
        x = W.sur_path(p)
        assert x.shape == (32, 6)
        assert np.abs(x).max() <= 3.0
        # every increment lies on one line through the origin
        d = x[np.argmax(np.linalg.norm(x, axis=1))]
        d = d / np.linalg.norm(d)
        assert np.allclose(x - np.outer(x @ d, d), 0.0, atol=1e-15)
        s = x @ d
        turns = int(np.sum(np.diff(np.sign(np.diff(np.concatenate([[0.0], s])))) != 0))
        if p % 2 == 0:
            assert turns == 0 and np.all(np.diff(np.abs(s)) >= 0)
        else:
            assert 2 <= turns <= 4, (p, turns)
    assert np.array_equal(W.sur_path(7), W.sur_path(7))
