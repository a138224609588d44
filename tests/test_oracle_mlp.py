"""Pins for the FP64 reference network: back-propagated gradients against central finite
differences, and the parameter layout against a hand-built two-layer case."""
import numpy as np

from oracle import mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    dims = [4, 7, 5, 3]
    n = sum(i * o + o for i, o in zip(dims[:-1], dims[1:]))
    p = rng.normal(0, 0.5, n)
    x = rng.normal(0, 1, (6, 4))
    t = rng.normal(0, 1, (6, 3))
    g = mlp.mse_gradient(p, dims, x, t)
    h = 1e-6
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        fd = (mlp.mse(p + e, dims, x, t) - mlp.mse(p - e, dims, x, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-6 * abs(fd)


def test_layout_and_forward_by_hand():
    dims = [2, 2, 1]
    W0 = np.array([[0.5, -1.0], [2.0, 0.25]])
    b0 = np.array([0.1, -0.2])
    W1 = np.array([[1.5, -0.5]])
    b1 = np.array([0.3])
    p = np.concatenate([W0.ravel(), b0, W1.ravel(), b1])
    x = np.array([[0.3, -0.7]])
    h = np.tanh(W0 @ x[0] + b0)
    y = W1 @ h + b1
    assert np.allclose(mlp.forward(p, dims, x)[-1][0], y, rtol=0, atol=1e-15)
