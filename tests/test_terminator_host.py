"""Host-side pieces of the learned terminator (no GPU): normalisation round trip."""

import numpy as np

from paper_1602_01863_amd import terminator as T


def test_normalise_targets_denormalise_round_trip():
    rng = np.random.default_rng(1)
    n = 6
    a = rng.uniform(1.0, 6.0, size=(n, T.CHAIN_LEN))
    b = np.concatenate([np.zeros((n, 1)), rng.uniform(0.2, 2.0, size=(n, T.CHAIN_LEN))], axis=1)
    x, c, s = T.normalise(a, b)
    assert x.shape == (n, T.N_IN)
    assert np.allclose(x[:, :T.M_IN].mean(axis=1), 0.0, atol=1e-12)
    assert np.allclose(x[:, T.M_IN:].mean(axis=1), 0.5)          # b / (2 mean b)
    y = T.targets(a, b, c, s, smooth=1)
    assert y.shape == (n, T.N_OUT)
    # the training targets are the same residuals, moving-averaged along the tail
    ys = T.targets(a, b, c, s)
    assert np.allclose(ys[:, :T.M_OUT], T.moving_average(y[:, :T.M_OUT], T.SMOOTH))
    assert np.allclose(ys[:, T.M_OUT:2 * T.M_OUT], T.moving_average(y[:, T.M_OUT:2 * T.M_OUT], T.SMOOTH))
    assert np.array_equal(ys[:, 2 * T.M_OUT:], y[:, 2 * T.M_OUT:])
    const = np.full((2, 40), 3.0)
    assert np.allclose(T.moving_average(const, 8), 3.0)
    at, bt, ainf, binf = T.denormalise(y, a, b, s)
    assert np.allclose(at, a[:, T.M_IN:T.M_IN + T.M_OUT], rtol=1e-13)
    assert np.allclose(bt, b[:, T.M_IN + 1:T.M_IN + T.M_OUT + 1], rtol=1e-13)
    assert np.allclose(ainf, a[:, T.M_IN + T.M_OUT:].mean(axis=1), rtol=1e-13)
    assert np.allclose(binf, b[:, T.M_IN + T.M_OUT + 1:].mean(axis=1), rtol=1e-13)
    # a network that predicts zero reproduces the method's own closure
    z = T.denormalise(np.zeros_like(y), a, b, s)
    ha, hb = T.head_closure(a, b)
    assert np.allclose(z[0], ha[:, None]) and np.allclose(z[3], hb)
