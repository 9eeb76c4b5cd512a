"""FP64 reference of the (k, q) predictor network (test infrastructure).

Network: x (128) -> h1 = tanh(W1 x + b1) (64) -> h2 = tanh(W2 h1 + b2) (64)
-> y = W3 h2 + b3 (4). Parameters are one flat vector in the order W1 (64 x 128,
row-major), b1, W2 (64 x 64), b2, W3 (4 x 64), b3 (12676 values).
Loss of a minibatch: mean over its B x 4 outputs of (y - t)^2.
Adam: Kingma & Ba, "Adam: a method for stochastic optimization" (2015),
Algorithm 1, with bias-corrected moments.

Probe features (the network's input): for the probe sketch Y0 = A Omega[:, :l],
l = min(128, m, n), with s_j its singular values (descending),
f_j = clamp(log10(s_j / s_1) / 8, -1, 0) for j < l and -1 beyond.
"""
import numpy as np

N_IN, N_H, N_OUT = 128, 64, 4
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    """Views of the flat parameter vector as the named arrays."""
    theta = np.asarray(theta, dtype=np.float64)
    out, off = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = theta[off:off + size].reshape(shape)
        off += size
    return out


def init_params(seed, scale=None):
    """Glorot-uniform weights, zero biases (FP64; the caller casts)."""
    gen = np.random.default_rng(seed)
    parts = []
    for name, shape in SIZES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(gen.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape).ravel())
    return np.concatenate(parts)


def forward(theta, X):
    """Outputs Y (B x 4) and the activations (H1, H2) of a batch X (B x 128)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.tanh(X @ p["W1"].T + p["b1"])
    H2 = np.tanh(H1 @ p["W2"].T + p["b2"])
    Y = H2 @ p["W3"].T + p["b3"]
    return Y, H1, H2


def loss(theta, X, T):
    Y, _, _ = forward(theta, X)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def backward(theta, X, T):
    """(loss, gradient as a flat vector) by the chain rule, layer by layer."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    Y, H1, H2 = forward(theta, X)
    B = X.shape[0]
    R = Y - T
    dY = 2.0 * R / (B * N_OUT)                    # d loss / d y
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dH2 = dY @ p["W3"]
    dZ2 = dH2 * (1.0 - H2 ** 2)                   # tanh' = 1 - tanh^2
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dH1 = dZ2 @ p["W2"]
    dZ1 = dH1 * (1.0 - H1 ** 2)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    grad = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return float(np.mean(R ** 2)), grad


def adam_step(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1). Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def features_from_singular_values(s, n_feat=N_IN):
    s = np.asarray(s, dtype=np.float64)
    f = -np.ones(n_feat)
    if s.size and s[0] > 0:
        r = s[:n_feat] / s[0]
        val = np.where(r > 1e-8, np.log10(np.maximum(r, 1e-300)) / 8.0, -1.0)
        f[:val.size] = val
    return f


def probe_features(A, seed):
    """Features of A from the probe sketch with the method's Omega of that seed."""
    from . import sorsvd as osvd
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = min(128, m, n)
    Y0 = A @ osvd.omega(seed, n, l)
    return features_from_singular_values(np.linalg.svd(Y0, compute_uv=False))
