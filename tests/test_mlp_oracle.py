"""Pins of the float64 tile-scoring network reference: forward, loss and
gradient agree with torch float64 autograd; the analytic gradient
agrees with central finite differences; the loss is the textbook binary
cross-entropy of sigmoid(z); a step against the gradient lowers the loss."""
import numpy as np
import pytest

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


def _torch_loss(p, X, y):
    """The same network written with torch's own layers and loss, float64:
    F.linear(x, W, b) = x W^T + b (output-major W), relu, and
    binary_cross_entropy_with_logits (mean)."""
    import torch
    import torch.nn.functional as Fn
    t = {k: torch.tensor(np.atleast_1d(v), dtype=torch.float64,
                         requires_grad=True) for k, v in p.items()}
    Xt = torch.tensor(X, dtype=torch.float64)
    yt = torch.tensor(y, dtype=torch.float64)
    h1 = torch.relu(Fn.linear(Xt, t["W1"], t["b1"]))
    h2 = torch.relu(Fn.linear(h1, t["W2"], t["b2"]))
    z = Fn.linear(h2, t["w3"].reshape(1, -1), t["b3"]).reshape(-1)
    loss = Fn.binary_cross_entropy_with_logits(z, yt)
    loss.backward()
    return z.detach().numpy(), float(loss), {k: v.grad.numpy() for k, v in t.items()}


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_matches_torch_autograd(seed):
    """forward, loss and every gradient against torch float64 autograd (an
    implementation of the same textbook network that shares nothing with the
    reference)."""
    pytest.importorskip("torch")
    p = mlp.init(seed)
    # non-zero biases so that their layout and broadcast are exercised
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    X, y = _data(96, seed)
    z_t, l_t, g_t = _torch_loss(p, X, y)
    z, _ = mlp.forward(p, X)
    assert np.allclose(z, z_t, rtol=1e-10, atol=1e-12)
    assert abs(mlp.loss(p, X, y) - l_t) <= 1e-10 * max(1.0, abs(l_t))
    g = mlp.grad(p, X, y)
    for k in g:
        assert np.allclose(np.atleast_1d(g[k]), g_t[k].reshape(np.shape(np.atleast_1d(g[k]))),
                           rtol=1e-10, atol=1e-12), k
