"""Pins of the float64 reference of the learned cost model (CPU)."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, n=40):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.NPARAM) * 0.3
    X = rng.standard_normal((n, mlp.IN))
    t = rng.standard_normal(n)
    return p, X, t


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    p, X, t = _data(seed)
    g = mlp.gradient(p, X, t)
    rng = np.random.default_rng(100 + seed)
    idx = rng.choice(mlp.NPARAM, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_linear_regime_closed_form():
    # With every pre-activation positive the model is linear, y = x W1 W2 w3 + const,
    # and the gradient of the bias b3 is the mean residual times 2.
    rng = np.random.default_rng(7)
    W1 = np.abs(rng.standard_normal((mlp.IN, mlp.H))) * 0.1
    b1 = np.ones(mlp.H)
    W2 = np.abs(rng.standard_normal((mlp.H, mlp.H))) * 0.1
    b2 = np.ones(mlp.H)
    w3 = rng.standard_normal(mlp.H)
    b3 = 0.5
    p = mlp.pack(W1, b1, W2, b2, w3, b3)
    X = np.abs(rng.standard_normal((25, mlp.IN)))
    t = rng.standard_normal(25)
    y, _ = mlp.forward(p, X)
    want = ((X @ W1 + b1) @ W2 + b2) @ w3 + b3
    assert np.allclose(y, want, rtol=1e-14, atol=1e-14)
    g = mlp.gradient(p, X, t)
    assert np.isclose(g[-1], 2.0 * np.mean(want - t), rtol=1e-13)
    # d/dw3 = 2/N sum (y - t) a2 with a2 = z2
    a2 = (X @ W1 + b1) @ W2 + b2
    assert np.allclose(g[-1 - mlp.H:-1], 2.0 / 25 * a2.T @ (want - t), rtol=1e-12)


def test_dead_units_have_zero_gradient():
    p, X, t = _data(3)
    W1, b1, W2, b2, w3, b3 = [np.array(x, copy=True) for x in mlp.unpack(p)]
    b1[:5] = -1e6  # these first-layer units never fire
    p2 = mlp.pack(W1, b1, W2, b2, w3, float(b3))
    g = mlp.gradient(p2, X, t)
    gW1 = g[:mlp.IN * mlp.H].reshape(mlp.IN, mlp.H)
    assert np.all(gW1[:, :5] == 0.0)
    assert np.all(g[mlp.IN * mlp.H:mlp.IN * mlp.H + 5] == 0.0)


def test_adam_first_step_is_signed_lr():
    # At step 1 the bias-corrected moments are g and g^2, so the update is lr * g / (|g| + eps).
    rng = np.random.default_rng(4)
    p = rng.standard_normal(mlp.NPARAM)
    g = rng.standard_normal(mlp.NPARAM)
    p1, m, v = mlp.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-2, eps=1e-12)
    assert np.allclose(p - p1, 1e-2 * np.sign(g), rtol=1e-9)


def test_training_fits_a_smooth_function():
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (200, mlp.IN))
    t = X[:, 0] ** 2 + 0.5 * X[:, 1] - X[:, 2] * X[:, 3]
    p = rng.standard_normal(mlp.NPARAM) * 0.1
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = mlp.loss(p, X, t)
    for k in range(1, 301):
        p, m, v = mlp.adam_step(p, mlp.gradient(p, X, t), m, v, k, lr=3e-3)
    assert mlp.loss(p, X, t) < 0.05 * l0
