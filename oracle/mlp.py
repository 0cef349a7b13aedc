"""CPU ORACLE (test infrastructure only) for the learned path selector and
nnz predictor: a small multilayer perceptron in float64, written out step by
step so that every formula can be checked by eye.

The paper leaves learning the choice of reordering and clustering to future
work (Sec. "Conclusion and Future Work") and fixes no model, so the model is
this library's reading:

    x_n = (x - mu) / sd                      (32 structure features, standardized)
    h1  = relu(W1 x_n + b1)                  (64)
    h2  = relu(W2 h1 + b2)                   (64)
    z   = W3 h2 + b3                         (5): z[0:4] path logits, z[4] log compression ratio

    loss = mean_b [ -log softmax(z_b[0:4])[y_b] ] + lam * mean_b [ (z_b[4] - t_b)^2 ]

with y the fastest path and t = log(nnz(C) / products).  Parameters are one
flat vector: W1 (64x32, row-major), b1 (64), W2 (64x64), b2 (64), W3 (5x64),
b3 (5).  Training uses Adam (Kingma and Ba) with bias correction.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT, NCLS = 32, 64, 5, 4
SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def forward(theta, mu, sd, X):
    """Returns (z, cache) for inputs X [B x 32]."""
    p = unpack(np.asarray(theta, np.float64))
    xn = (np.asarray(X, np.float64) - mu) / sd
    a1 = xn @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"].T + p["b3"]
    return z, (xn, a1, h1, a2, h2, p)


def loss(theta, mu, sd, X, y, t, lam):
    z, _ = forward(theta, mu, sd, X)
    logits = z[:, :NCLS]
    m = logits.max(axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(logits - m).sum(axis=1))
    ce = lse - logits[np.arange(len(y)), y]
    return float(ce.mean() + lam * np.mean((z[:, NCLS] - t) ** 2))


def grad(theta, mu, sd, X, y, t, lam):
    """Gradient of ``loss`` with respect to theta (back-propagation, layer by layer)."""
    z, (xn, a1, h1, a2, h2, p) = forward(theta, mu, sd, X)
    B = len(y)
    logits = z[:, :NCLS]
    e = np.exp(logits - logits.max(axis=1, keepdims=True))
    sm = e / e.sum(axis=1, keepdims=True)
    dz = np.zeros_like(z)
    dz[:, :NCLS] = sm
    dz[np.arange(B), y] -= 1.0
    dz[:, :NCLS] /= B
    dz[:, NCLS] = 2.0 * lam * (z[:, NCLS] - t) / B
    g = {"W3": dz.T @ h2, "b3": dz.sum(axis=0)}
    dh2 = dz @ p["W3"]
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ xn
    g["b1"] = da1.sum(axis=0)
    return pack(g)


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init(seed: int) -> np.ndarray:
    """He-style initial weights from a seeded generator, zero biases."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0, np.sqrt(2 / NIN), (NH, NIN)), "b1": np.zeros(NH),
         "W2": rng.normal(0, np.sqrt(2 / NH), (NH, NH)), "b2": np.zeros(NH),
         "W3": rng.normal(0, np.sqrt(1 / NH), (NOUT, NH)), "b3": np.zeros(NOUT)}
    return pack(p)
