"""Float64 reference of the tile-scoring network (test infrastructure).

The network scores block-pair tiles: 32 input features -> 64 -> 64 -> 1 with
ReLU between layers, trained with binary cross-entropy on logits.  The paper
has no learned component; this is the plain textbook definition used to check
the GPU's forward and backward kernels:

  h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = w3 . h2 + b3
  loss = mean over samples of  max(z, 0) - z y + log(1 + exp(-|z|))
  (the numerically stable form of -[y log s(z) + (1 - y) log(1 - s(z))])

Parameters are float64 numpy arrays.  Layouts match the library's: W1 is
64 x 32 row-major (output-major), W2 64 x 64, w3 64.
"""
import numpy as np

D_IN, D_H = 32, 64
N_PARAMS = D_H * D_IN + D_H + D_H * D_H + D_H + D_H + 1  # 6337


def init(seed=0):
    """He-style initialisation (deterministic in the seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return {"W1": rng.normal(0, np.sqrt(2.0 / D_IN), (D_H, D_IN)),
            "b1": np.zeros(D_H),
            "W2": rng.normal(0, np.sqrt(2.0 / D_H), (D_H, D_H)),
            "b2": np.zeros(D_H),
            "w3": rng.normal(0, np.sqrt(1.0 / D_H), D_H),
            "b3": np.zeros(1)}


def flatten(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"],
                           p["w3"], p["b3"]])


def unflatten(v):
    v = np.asarray(v, dtype=np.float64)
    o = 0
    out = {}
    for k, shape in (("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)),
                     ("b2", (D_H,)), ("w3", (D_H,)), ("b3", (1,))):
        n = int(np.prod(shape))
        out[k] = v[o:o + n].reshape(shape)
        o += n
    return out


def forward(p, X):
    """Logits for samples X (n x 32); also the activations."""
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0)
    z = h2 @ p["w3"] + p["b3"][0]
    return z, (X, a1, h1, a2, h2)


def loss(p, X, y):
    z, _ = forward(p, X)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def grad(p, X, y):
    """Analytic gradient of loss() by the chain rule."""
    z, (X, a1, h1, a2, h2) = forward(p, X)
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n          # d loss / d z
    g = {"w3": h2.T @ dz, "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, p["w3"])
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(0)
    return g


def numeric_grad(p, X, y, idx, eps=1e-6):
    """Central finite differences of loss() at flat parameter indices."""
    v = flatten(p)
    out = []
    for i in idx:
        vp, vm = v.copy(), v.copy()
        vp[i] += eps
        vm[i] -= eps
        out.append((loss(unflatten(vp), X, y) - loss(unflatten(vm), X, y)) / (2 * eps))
    return np.array(out)
