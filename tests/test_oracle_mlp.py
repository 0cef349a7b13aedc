"""Pins of the float64 MLP oracle (the learned selector's reference): central
finite differences for the back-propagation, closed values for a zero
network, and the closed form of Adam's first step."""
import numpy as np
import pytest

from oracle import mlp


def batch(seed, B=9):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 2, (B, mlp.NIN))
    y = rng.integers(0, mlp.NCLS, B)
    t = rng.normal(0, 1, B)
    mu, sd = rng.normal(0, 1, mlp.NIN), rng.uniform(0.5, 2, mlp.NIN)
    return X, y, t, mu, sd


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_central_differences(seed):
    X, y, t, mu, sd = batch(seed)
    theta = mlp.init(seed) + np.random.default_rng(seed + 9).normal(0, 0.05, mlp.NPARAMS)
    lam = 0.7
    g = mlp.grad(theta, mu, sd, X, y, t, lam)
    idx = np.random.default_rng(seed).choice(mlp.NPARAMS, 400, replace=False)
    idx = np.concatenate([idx, np.arange(mlp.NPARAMS - 5 - 5 * mlp.NH, mlp.NPARAMS)])  # every head weight
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAMS)
        e[i] = h
        fd = (mlp.loss(theta + e, mu, sd, X, y, t, lam) - mlp.loss(theta - e, mu, sd, X, y, t, lam)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, i


def test_zero_network_closed_values():
    X, y, t, mu, sd = batch(3, 40)
    theta = np.zeros(mlp.NPARAMS)
    p = mlp.unpack(theta)
    p["b3"][mlp.NCLS] = 0.25                 # predictor head outputs 0.25 for every input
    theta = mlp.pack(p)
    lam = 2.0
    assert mlp.loss(theta, mu, sd, X, y, t, lam) == pytest.approx(np.log(4) + lam * np.mean((0.25 - t) ** 2), rel=1e-12)
    g = mlp.unpack(mlp.grad(theta, mu, sd, X, y, t, lam))
    frac = np.bincount(y, minlength=mlp.NCLS) / len(y)
    np.testing.assert_allclose(g["b3"][:mlp.NCLS], 0.25 - frac, rtol=0, atol=1e-15)
    assert g["b3"][mlp.NCLS] == pytest.approx(2 * lam * np.mean(0.25 - t), rel=1e-12)
    assert not g["W1"].any() and not g["W2"].any()   # no signal reaches the hidden layers


def test_standardization_is_applied():
    X, y, t, mu, sd = batch(4)
    theta = mlp.init(4)
    z1, _ = mlp.forward(theta, mu, sd, X)
    z2, _ = mlp.forward(theta, np.zeros(mlp.NIN), np.ones(mlp.NIN), (X - mu) / sd)
    np.testing.assert_allclose(z1, z2, rtol=1e-12, atol=1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    theta, g = rng.normal(size=50), rng.normal(size=50)
    new, m, v = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    np.testing.assert_allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_training_reduces_the_loss_on_a_learnable_rule():
    # labels from a rule of the first two features; full-batch Adam must fit it
    rng = np.random.default_rng(6)
    X = rng.normal(size=(256, mlp.NIN))
    y = (X[:, 0] > 0).astype(int) + 2 * (X[:, 1] > 0).astype(int)
    t = 0.5 * X[:, 2]
    mu, sd = np.zeros(mlp.NIN), np.ones(mlp.NIN)
    theta = mlp.init(1)
    m = v = np.zeros(mlp.NPARAMS)
    l0 = mlp.loss(theta, mu, sd, X, y, t, 1.0)
    for s in range(1, 301):
        theta, m, v = mlp.adam_step(theta, mlp.grad(theta, mu, sd, X, y, t, 1.0), m, v, s, lr=3e-3)
    z, _ = mlp.forward(theta, mu, sd, X)
    assert mlp.loss(theta, mu, sd, X, y, t, 1.0) < 0.2 * l0
    assert np.mean(z[:, :4].argmax(1) == y) > 0.9
