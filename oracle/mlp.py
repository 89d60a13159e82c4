"""Plain float64 reference of the refinement classifier (test infrastructure).

The network reads 64 features of a leaf (the last four rows of its 16 x 16
Chebyshev coefficient array) and returns one logit for "refine": two hidden
layers of 64 units with the exact GELU, x Phi(x) = x (1 + erf(x / sqrt 2)) / 2,
and a linear output; the training loss is the mean binary cross-entropy of
the logits.  Parameters are one flat vector in the order
W1 (64 x 64, [out][in]), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1).
Forward and backward passes are written out layer by layer (no autodiff) so
they can be checked against finite differences; Adam follows Kingma & Ba
(2015) with bias correction.
"""
import math

import numpy as np

D = 64
SIZES = (("W1", (D, D)), ("b1", (D,)), ("W2", (D, D)), ("b2", (D,)), ("w3", (D,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init(seed):
    """He-style initialisation (normal, std sqrt(2/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0, math.sqrt(2 / D), (D, D)), "b1": np.zeros(D),
         "W2": rng.normal(0, math.sqrt(2 / D), (D, D)), "b2": np.zeros(D),
         "w3": rng.normal(0, math.sqrt(1 / D), D), "b3": np.zeros(1)}
    return pack(p)


_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    # d/dz [z Phi(z)] = Phi(z) + z phi(z)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X):
    """Logits (B,) and the intermediate values (z1, a1, z2, a2)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    a1 = gelu(z1)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = gelu(z2)
    logit = a2 @ p["w3"] + p["b3"][0]
    return logit, (z1, a1, z2, a2)


def loss(theta, X, y):
    """Mean binary cross-entropy with logits, in the stable form
    max(s, 0) - s y + log(1 + exp(-|s|))."""
    s, _ = forward(theta, X)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.maximum(s, 0) - s * y + np.log1p(np.exp(-np.abs(s)))))


def backward(theta, X, y):
    """Gradient of loss() with respect to the flat parameter vector."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    B = X.shape[0]
    s, (z1, a1, z2, a2) = forward(theta, X)
    ds = (1.0 / (1.0 + np.exp(-s)) - y) / B          # dL/ds
    g = {"w3": a2.T @ ds, "b3": np.array([ds.sum()])}
    dz2 = np.outer(ds, p["w3"]) * gelu_prime(z2)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * gelu_prime(z1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns the new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
