"""Pins of the float64 tile-scoring network reference: the analytic gradient
agrees with central finite differences; the loss is the textbook binary
cross-entropy of sigmoid(z); a step against the gradient lowers the loss."""
import numpy as np

from oracle import mlp


def _data(n=64, seed=1):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.normal(size=(n, mlp.D_IN))
    y = (rng.random(n) < 0.3).astype(np.float64)
    return X, y


def test_param_count():
    assert mlp.N_PARAMS == 6337
    assert len(mlp.flatten(mlp.init(0))) == 6337


def test_loss_is_bce_of_sigmoid():
    p = mlp.init(3)
    X, y = _data()
    z, _ = mlp.forward(p, X)
    s = 1 / (1 + np.exp(-z))
    ref = -np.mean(y * np.log(s) + (1 - y) * np.log(1 - s))
    assert abs(mlp.loss(p, X, y) - ref) < 1e-12


def test_gradient_matches_finite_differences():
    p = mlp.init(5)
    X, y = _data()
    g = mlp.flatten(mlp.grad(p, X, y))
    rng = np.random.Generator(np.random.PCG64(9))
    idx = list(rng.choice(mlp.N_PARAMS, 60, replace=False)) + [mlp.N_PARAMS - 1]
    num = mlp.numeric_grad(p, X, y, idx)
    ana = g[idx]
    assert np.allclose(ana, num, rtol=1e-5, atol=1e-8)


def test_descent_step_lowers_loss():
    p = mlp.init(7)
    X, y = _data(256)
    l0 = mlp.loss(p, X, y)
    g = mlp.grad(p, X, y)
    q = {k: p[k] - 0.05 * g[k] for k in p}
    assert mlp.loss(q, X, y) < l0
