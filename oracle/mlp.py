"""TEST INFRASTRUCTURE -- plain FP64 reference of the learned continued-fraction
terminator's network (a multilayer perceptron), for checking the HIP kernels.

The network is a stack of dense layers y = act(x W^T + b) with act = GELU on the
hidden layers and the identity on the last one; the loss is the mean squared error.
Everything is written out directly in NumPy FP64: the forward pass, the backward
pass by the chain rule (no automatic differentiation), and one Adam update
(Kingma and Ba, "Adam: a method for stochastic optimization", ICLR 2015, Alg. 1).
The paper has no learned part; these are the textbook definitions.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
SQRT2PI = math.sqrt(2.0 * math.pi)


def gelu(z):
    """GELU(z) = z Phi(z) with Phi the standard normal distribution function."""
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    """d GELU / dz = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / SQRT2PI


def init_params(sizes, seed):
    """[(W [out, in], b [out]), ...] with W ~ U(-1/sqrt(in), 1/sqrt(in)), b = 0."""
    rng = np.random.default_rng(seed)
    params = []
    for n_in, n_out in zip(sizes[:-1], sizes[1:]):
        lim = 1.0 / math.sqrt(n_in)
        params.append((rng.uniform(-lim, lim, size=(n_out, n_in)), np.zeros(n_out)))
    return params


def forward(params, x):
    """Returns the output and the cache (inputs and pre-activations of every layer)."""
    cache = []
    h = np.asarray(x, dtype=np.float64)
    for i, (W, b) in enumerate(params):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if i < len(params) - 1 else z
    return h, cache


def mse(y, t):
    """L = mean over all entries of (y - t)^2, and dL/dy."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dy):
    """Gradients [(dW, db), ...] of a scalar loss with dL/dy = dy."""
    grads = [None] * len(params)
    g = dy
    for i in range(len(params) - 1, -1, -1):
        W, b = params[i]
        h, z = cache[i]
        dz = g if i == len(params) - 1 else g * gelu_grad(z)
        grads[i] = (dz.T @ h, dz.sum(axis=0))
        g = dz @ W
    return grads


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of p (returns new p, m, v); t counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
