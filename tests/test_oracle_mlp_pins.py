"""Pins of the FP64 cost-model MLP oracle: finite differences, Adam's first step, a hand net."""
import numpy as np

from oracle import mlp


def rand_problem(seed, n=7):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.N_PARAMS)
    X = rng.normal(0, 1, (n, mlp.IN))
    T = rng.normal(0, 1, (n, mlp.OUT))
    M = (rng.random((n, mlp.OUT)) < 0.7).astype(float)
    M[0, 0] = 1.0
    return p, X, T, M


def test_parameter_count():
    assert mlp.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3 == 5187


def test_gradient_matches_central_differences():
    p, X, T, M = rand_problem(1)
    g = mlp.grad(p, X, T, M)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, T, M) - mlp.loss(p - e, X, T, M)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_closed_form():
    # with zero moments, the bias-corrected first step moves each parameter by
    # -lr * g / (|g| + eps)
    rng = np.random.default_rng(3)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = mlp.adam(p, g, np.zeros(50), np.zeros(50), step=1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_hand_built_network():
    # W1 copies x0 into unit 0 (and -x0 into unit 1), W2 sums units 0 and 1, W3 reads it:
    # y0 = relu(x0) + relu(-x0) = |x0|; other outputs are their biases
    P = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    P["W1"][0, 0], P["W1"][1, 0] = 1.0, -1.0
    P["W2"][0, 0], P["W2"][0, 1] = 1.0, 1.0
    P["W3"][0, 0] = 1.0
    P["b3"][:] = [0.0, 2.0, -3.0]
    p = np.concatenate([P[name].reshape(-1) for name, _ in mlp.SHAPES])
    X = np.zeros((3, 12))
    X[:, 0] = [-2.5, 0.0, 4.0]
    y, _ = mlp.forward(p, X)
    assert np.allclose(y[:, 0], [2.5, 0.0, 4.0]) and np.allclose(y[:, 1:], [[2.0, -3.0]] * 3)
