"""Pins of the FP64 oracle of the (k, q) network against something other than
itself: central finite differences of the loss, the closed form of Adam's
first step, convergence on a problem with a known minimiser, and the feature
definition on spectra with known singular values."""
import numpy as np

import workloads as W
from oracle import mlp


def _batch(seed, B=7):
    gen = np.random.default_rng(seed)
    X = gen.uniform(-1.0, 0.0, size=(B, mlp.N_IN))
    T = gen.uniform(2.0, 8.0, size=(B, mlp.N_OUT))
    return X, T


def test_parameter_count():
    assert mlp.N_PARAMS == 12676
    assert mlp.init_params(0).size == 12676


def test_gradient_matches_central_differences():
    theta = mlp.init_params(3) + 0.05 * np.random.default_rng(4).standard_normal(mlp.N_PARAMS)
    X, T = _batch(5)
    _, g = mlp.backward(theta, X, T)
    gen = np.random.default_rng(6)
    # every bias and output weight, and a sample of the first two layers' weights
    idx = np.concatenate([np.arange(8192, 8256), np.arange(12352, 12676), gen.choice(8192, 150, replace=False),
                          8256 + gen.choice(4096, 150, replace=False)])
    h = 1e-5
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss(theta + e, X, T) - mlp.loss(theta - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_loss_value_is_the_mean_squared_error():
    theta = mlp.init_params(1)
    X, T = _batch(2)
    Y, _, _ = mlp.forward(theta, X)
    L, _ = mlp.backward(theta, X, T)
    assert abs(L - np.sum((Y - T) ** 2) / Y.size) < 1e-14


def test_adam_first_step_closed_form():
    # from zero moments the bias-corrected moments are g and g^2, so the step is lr g / (|g| + eps)
    g = np.array([3.0, -0.25, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_minimises_a_quadratic():
    target = np.array([1.0, -2.0, 0.5])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        th, m, v = mlp.adam_step(th, 2 * (th - target), m, v, t, lr=0.01)
    assert np.abs(th - target).max() < 1e-3


def test_training_fits_a_smooth_target():
    gen = np.random.default_rng(11)
    X = gen.uniform(-1.0, 0.0, size=(256, mlp.N_IN))
    T = np.stack([X[:, :8].sum(1), X[:, 8:16].mean(1), np.tanh(X[:, 0]), X[:, 1] ** 2], axis=1)
    th = mlp.init_params(12)
    m, v = np.zeros_like(th), np.zeros_like(th)
    L0, _ = mlp.backward(th, X, T)
    for t in range(1, 301):
        _, g = mlp.backward(th, X, T)
        th, m, v = mlp.adam_step(th, g, m, v, t, lr=3e-3)
    L1, _ = mlp.backward(th, X, T)
    assert L1 < 0.02 * L0


def test_features_of_known_spectra():
    s = np.array([4.0, 0.4, 4e-3, 4e-9, 0.0])
    f = mlp.features_from_singular_values(s)
    assert np.allclose(f[:3], [0.0, -1 / 8, -3 / 8], atol=1e-15)
    assert f[3] == -1.0 and f[4] == -1.0 and np.all(f[5:] == -1.0)


def test_probe_features_of_diagonal_and_rotated_inputs_share_a_distribution():
    # Omega is rotation-invariant: the probe of U diag(s) V^T is the probe of
    # diag(s) with V^T Omega; with an exactly known spectrum, both feature
    # vectors fall in the same band (median over draws within 0.05)
    n = 300
    sigma = 0.93 ** np.arange(n)
    A, _, _ = W.spectral(n, n, sigma, 7)
    fa = np.median([mlp.probe_features(A, s) for s in range(12)], axis=0)
    fd = np.median([mlp.probe_features(np.diag(sigma), s) for s in range(12)], axis=0)
    assert np.abs(fa - fd)[:100].max() < 0.05
