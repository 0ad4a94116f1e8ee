"""Plain FP64 reference of the warm-start perceptron (test infrastructure only:
imported by tests/, smoke() and the benchmark's CPU baseline, never by the
library path).

The model is in0 -> h -> h -> out with GELU after the two hidden layers,
GELU(z) = z Phi(z) with Phi the standard normal CDF (the erf form), plus a
linear skip path from the input to the output: Y = H2 W2 + b2 + X Ws.  It is
trained on the mean-squared error mean((Y - T)^2) with Adam (Kingma & Ba;
beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments).  Parameters are one
flat vector: W0 (in0 x h, row-major), b0, W1 (h x h), b1, W2 (h x out), b2,
Ws (in0 x out).
Everything is written from the definitions, in float64, one layer at a time.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def shapes(dims):
    return [(dims[0], dims[1]), (dims[1],), (dims[1], dims[2]), (dims[2],), (dims[2], dims[3]),
            (dims[3],), (dims[0], dims[3])]


def n_params(dims):
    return sum(int(np.prod(s)) for s in shapes(dims))


def unpack(params, dims):
    out, o = [], 0
    for s in shapes(dims):
        k = int(np.prod(s))
        out.append(np.asarray(params[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def init_params(dims, seed):
    """He-style normal weights (std sqrt(2/fan_in)), zero biases, zero skip."""
    rng = np.random.default_rng(np.random.SeedSequence([55, seed]))
    parts = []
    for q, s in enumerate(shapes(dims)):
        if len(s) == 2 and q < 6:
            parts.append(rng.standard_normal(s) * np.sqrt(2.0 / s[0]))
        else:
            parts.append(np.zeros(s))
    return np.concatenate([p.ravel() for p in parts])


def forward(params, dims, X):
    W0, b0, W1, b1, W2, b2, Ws = unpack(params, dims)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W0 + b0
    H1 = gelu(Z1)
    Z2 = H1 @ W1 + b1
    H2 = gelu(Z2)
    Y = H2 @ W2 + b2 + X @ Ws
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grad(params, dims, X, T):
    """Mean-squared error and its gradient by the chain rule, layer by layer."""
    W0, b0, W1, b1, W2, b2, Ws = unpack(params, dims)
    Y, (X, Z1, H1, Z2, H2) = forward(params, dims, X)
    D = Y - np.asarray(T, dtype=np.float64)
    L = float(np.mean(D * D))
    dY = 2.0 * D / D.size
    gW2 = H2.T @ dY
    gb2 = dY.sum(axis=0)
    dZ2 = (dY @ W2.T) * gelu_grad(Z2)
    gW1 = H1.T @ dZ2
    gb1 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W1.T) * gelu_grad(Z1)
    gW0 = X.T @ dZ1
    gb0 = dZ1.sum(axis=0)
    gWs = X.T @ dY
    g = np.concatenate([a.ravel() for a in (gW0, gb0, gW1, gb1, gW2, gb2, gWs)])
    return L, g


def adam_step(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
