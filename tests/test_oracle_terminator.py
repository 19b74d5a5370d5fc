"""CPU pins of the oracle's learned-terminator pieces: the constant-chain closure of
the continued fraction and the network (dense layers, GELU, MSE, Adam)."""

from __future__ import annotations

import math

import numpy as np

import oracle as O
from oracle import mlp


# ---- constant-chain closure -------------------------------------------------------
def test_constant_chain_density_is_the_semicircle():
    """-Im g / pi of a constant chain tends to the semicircle sqrt(4 b^2 - x^2) / (2 pi b^2)."""
    a, b = 0.7, 1.3
    x = np.linspace(a - 2 * b + 0.05, a + 2 * b - 0.05, 101)
    dos = -O.constant_chain_g(x + 1e-9j, a, b).imag / math.pi
    ref = np.sqrt(4 * b * b - (x - a) ** 2) / (2 * math.pi * b * b)
    assert np.abs(dos - ref).max() < 1e-6
    # outside the band: no weight, and g ~ 1/z far away
    assert abs(O.constant_chain_g(a + 2 * b + 1.0 + 1e-9j, a, b).imag) < 1e-6
    z = 1e4 + 0.3j
    assert abs(O.constant_chain_g(z, a, b) * (z - a) - 1.0) < 1e-6


def test_constant_chain_weight_is_one():
    a, b, eta = 0.0, 1.0, 0.05
    w = np.linspace(-40.0, 40.0, 400001)
    dos = -O.constant_chain_g(w + 1j * eta, a, b).imag / math.pi
    assert abs(np.trapezoid(dos, w) - 1.0) < 2e-3


def test_terminated_fraction_equals_a_long_explicit_chain():
    """m computed coefficients closed by (a_inf, b_inf) = the same head followed by
    thousands of explicit constant coefficients (truncated far away)."""
    rng = np.random.default_rng(3)
    m, a_inf, b_inf = 5, 2.0, 0.8
    a_head = rng.uniform(1.0, 3.0, m)
    b_head = np.concatenate([[0.0], rng.uniform(0.5, 1.0, m - 1), [b_inf]])   # b_1..b_{m+1}
    om = np.linspace(0.0, 4.0, 41)
    eta = 0.3
    term = O.continued_fraction_terminated(a_head[None], b_head[None], [1.0], 1.0, om, eta, a_inf, b_inf)
    n_long = 4000
    a_long = np.concatenate([a_head, np.full(n_long, a_inf)])
    b_long = np.concatenate([b_head[:m + 1], np.full(n_long, b_inf)])
    plain = O.continued_fraction(a_long[None], b_long[None], [1.0], 1.0, om, eta)
    assert np.abs(term - plain).max() < 1e-10


# ---- network ------------------------------------------------------------------------
def test_gelu_values_and_derivative():
    # GELU(1) = Phi(1), the standard normal distribution function at 1
    assert abs(mlp.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert abs(mlp.gelu(np.array(-40.0))) < 1e-300 and abs(mlp.gelu(np.array(40.0)) - 40.0) < 1e-12
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(z)).max() < 1e-8


def test_backward_matches_central_differences():
    rng = np.random.default_rng(7)
    sizes = [6, 5, 5, 4]
    params = mlp.init_params(sizes, seed=1)
    params = [(W, rng.normal(size=b.shape) * 0.1) for W, b in params]
    x = rng.normal(size=(9, sizes[0]))
    t = rng.normal(size=(9, sizes[-1]))

    def loss(ps):
        y, _ = mlp.forward(ps, x)
        return mlp.mse(y, t)[0]

    y, cache = mlp.forward(params, x)
    _, dy = mlp.mse(y, t)
    grads = mlp.backward(params, cache, dy)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat, gf = arr.reshape(-1), g.reshape(-1)
            for k in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[k]
                flat[k] = old + h
                lp = loss(params)
                flat[k] = old - h
                lm = loss(params)
                flat[k] = old
                assert abs((lp - lm) / (2 * h) - gf[k]) < 1e-7 * max(1.0, abs(gf[k]))


def test_single_linear_layer_gradient_closed_form():
    """One identity layer: dL/dW = 2/n (X W^T + b - T)^T X, dL/db = 2/n column sums."""
    rng = np.random.default_rng(8)
    X, T = rng.normal(size=(11, 4)), rng.normal(size=(11, 3))
    W, b = rng.normal(size=(3, 4)), rng.normal(size=3)
    y, cache = mlp.forward([(W, b)], X)
    _, dy = mlp.mse(y, T)
    (dW, db), = mlp.backward([(W, b)], cache, dy)
    R = X @ W.T + b - T
    assert np.allclose(dW, 2.0 / R.size * R.T @ X, rtol=1e-13, atol=1e-15)
    assert np.allclose(db, 2.0 / R.size * R.sum(axis=0), rtol=1e-13, atol=1e-15)


def test_adam_first_step_is_a_signed_step_of_lr():
    """With zero moments, the bias-corrected first step is lr * g / (|g| + eps)."""
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-16)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_minimises_a_quadratic():
    p = np.array([3.0, -1.0])
    m = v = np.zeros(2)
    for t in range(1, 3001):
        p, m, v = mlp.adam_step(p, p, m, v, t, lr=0.01)   # gradient of |p|^2 / 2
    assert np.abs(p).max() < 1e-3
