"""Pins of the warm-start network oracle: the GELU closed forms and the
gradient against central finite differences."""
import math

import numpy as np

from oracle import mlp


def test_gelu_special_values():
    # gelu(0) = 0, gelu(t) -> t for large t, -> 0 for very negative t,
    # gelu(1) = Phi(1) = (1 + erf(1/sqrt2)) / 2
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) < 1e-12
    assert abs(mlp.gelu(np.array([-10.0]))[0]) < 1e-12
    phi1 = 0.5 * (1.0 + math.erf(1.0 / math.sqrt(2.0)))
    assert abs(mlp.gelu(np.array([1.0]))[0] - phi1) < 1e-15
    # derivative against a central difference
    t = np.linspace(-3, 3, 13)
    h = 1e-6
    fd = (mlp.gelu(t + h) - mlp.gelu(t - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_prime(t))) < 1e-8


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    params = mlp.init_params(2, 7, 3, seed=9)
    params = [(W, rng.normal(size=b.shape) * 0.1) for W, b in params]
    X = rng.normal(size=(11, 2))
    T = rng.normal(size=(11, 3))
    L, grads = mlp.loss_and_grad(params, X, T)
    g = mlp.flatten(grads)
    v = mlp.flatten(params)
    h = 1e-6
    for idx in rng.choice(v.size, size=40, replace=False):
        vp, vm = v.copy(), v.copy()
        vp[idx] += h
        vm[idx] -= h
        Lp, _ = mlp.loss_and_grad(mlp.unflatten(vp, 2, 7, 3), X, T)
        Lm, _ = mlp.loss_and_grad(mlp.unflatten(vm, 2, 7, 3), X, T)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(fd)), idx


def test_flatten_roundtrip_and_layout():
    params = mlp.init_params(2, 4, 3, seed=1)
    v = mlp.flatten(params)
    assert v.size == 4 * 2 + 4 + 4 * 4 + 4 + 3 * 4 + 3
    back = mlp.unflatten(v, 2, 4, 3)
    for (W, b), (W2, b2) in zip(params, back):
        assert np.array_equal(W, W2) and np.array_equal(b, b2)
    # W1 row-major first, then b1
    assert np.array_equal(v[:8], params[0][0].ravel())
