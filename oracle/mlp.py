"""Plain FP64 reference of the warm-start network (test infrastructure).

A multilayer perceptron y = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3 maps the
(normalised) parameter x = (mu - x_mean) / x_scale to the normalised reduced
coordinates y; z0 = y_mean + y_scale * y.  gelu(t) = t Phi(t) with Phi the
standard normal CDF (the erf form).  The training loss is the mean squared
error over samples and outputs, L = sum (y - t)^2 / (N * n_out).

Forward and backward are written out layer by layer, in the plain order of
the chain rule, so that a reader can check them by eye; the tests pin the
gradient to central finite differences.
"""
from __future__ import annotations

import math

import numpy as np

_SQRT2 = math.sqrt(2.0)
_INV_SQRT2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(t):
    from scipy.special import erf
    return 0.5 * t * (1.0 + erf(t / _SQRT2))


def gelu_prime(t):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(t / _SQRT2)) + t * _INV_SQRT2PI * np.exp(-0.5 * t * t)


def init_params(n_in: int, hidden: int, n_out: int, seed: int):
    """W_l [out, in] ~ U(-1/sqrt(in), 1/sqrt(in)), b_l = 0 (layer order 1, 2, 3)."""
    rng = np.random.default_rng(seed)
    dims = [(hidden, n_in), (hidden, hidden), (n_out, hidden)]
    out = []
    for o, i in dims:
        lim = 1.0 / math.sqrt(i)
        out.append((rng.uniform(-lim, lim, size=(o, i)), np.zeros(o)))
    return out


def forward(params, X):
    """Outputs [N, n_out] and the per-layer (input, pre-activation) pairs."""
    cache = []
    h = np.asarray(X, dtype=np.float64)
    for li, (W, b) in enumerate(params):
        a = h @ W.T + b
        cache.append((h, a))
        h = gelu(a) if li < len(params) - 1 else a
    return h, cache


def loss_and_grad(params, X, T):
    """MSE loss and its gradient [(dW, db)] per layer."""
    Y, cache = forward(params, X)
    N, n_out = Y.shape
    L = float(np.sum((Y - T) ** 2) / (N * n_out))
    d = 2.0 * (Y - T) / (N * n_out)                 # dL/dY
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h_in, a = cache[li]
        if li < len(params) - 1:
            d = d * gelu_prime(a)                   # through the activation
        grads[li] = (d.T @ h_in, d.sum(axis=0))
        d = d @ W                                   # to the layer input
    return L, grads


def flatten(params):
    """Flat vector in the library's layout: for each layer W (row-major) then b."""
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def unflatten(v, n_in: int, hidden: int, n_out: int):
    dims = [(hidden, n_in), (hidden, hidden), (n_out, hidden)]
    out, o = [], 0
    for r, c in dims:
        W = v[o:o + r * c].reshape(r, c)
        o += r * c
        b = v[o:o + r]
        o += r
        out.append((W.copy(), b.copy()))
    return out
