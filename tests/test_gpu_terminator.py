"""GPU parity of the learned terminator's kernels against the FP64 oracle: dense layer
forward and backward (the gradients), mean squared error, Adam, BF16 inference, and
the continued fraction closed by a constant tail."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from oracle import mlp

from _cases import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bse():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_01863_amd import bse as mod
    return mod


def _dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()


def _net(sizes, seed):
    rng = np.random.default_rng(seed)
    params = mlp.init_params(sizes, seed)
    return [(W, rng.normal(size=b.shape) * 0.1) for W, b in params]


@pytest.mark.parametrize("batch", [1, 37, 256])
def test_network_forward_and_gradients_match_oracle(bse, batch):
    from paper_1602_01863_amd.terminator import TerminatorMLP
    sizes = (128, 128, 128, 128, 386)
    params = _net(sizes, 3)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(batch, sizes[0]))
    t = rng.normal(size=(batch, sizes[-1]))
    # the oracle sees the FP32-rounded parameters and inputs the device uses
    params32 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in params]
    x32 = x.astype(np.float32).astype(np.float64)
    t32 = t.astype(np.float32).astype(np.float64)
    y_ref, cache = mlp.forward(params32, x32)
    loss_ref, dy_ref = mlp.mse(y_ref, t32)
    g_ref = mlp.backward(params32, cache, dy_ref)

    net = TerminatorMLP(sizes=sizes)
    net.W = [_dev(W) for W, _ in params32]
    net.b = [_dev(b) for _, b in params32]
    y = net.forward(_dev(x32)).cpu().numpy()
    assert rel_l2(y, y_ref) < 1e-5
    loss, grads = net.loss_and_grads(_dev(x32), _dev(t32))
    assert abs(loss.item() - loss_ref) < 1e-5 * loss_ref
    for (dW, db), (rW, rb) in zip(grads, g_ref):
        assert rel_l2(dW.cpu().numpy(), rW) < 1e-4
        assert rel_l2(db.cpu().numpy(), rb) < 1e-4


def test_adam_step_matches_oracle(bse):
    rng = np.random.default_rng(5)
    p, g = rng.normal(size=1000), rng.normal(size=1000)
    m, v = rng.normal(size=1000) * 0.1, np.abs(rng.normal(size=1000)) * 0.01
    r32 = lambda a: a.astype(np.float32).astype(np.float64)
    pr, mr, vr = mlp.adam_step(r32(p), r32(g), r32(m), r32(v), 7, lr=1e-3)
    P, G, M, V = _dev(r32(p)), _dev(r32(g)), _dev(r32(m)), _dev(r32(v))
    bse.bse_adam_step(P, G, M, V, 1000, 1e-3, 0.9, 0.999, 1e-8, 7)
    # FP32 arithmetic with the FP32 forms of the constants: 1 - beta2 = 0.001 in FP32
    # is 0.00099998713 (relative error 1.3e-5), so the second moment differs at 1e-5
    assert np.abs(P.cpu().numpy() - pr).max() < 1e-6
    assert rel_l2(M.cpu().numpy(), mr) < 1e-6 and rel_l2(V.cpu().numpy(), vr) < 2e-5


def test_bf16_inference_within_format_error(bse):
    from paper_1602_01863_amd.terminator import TerminatorMLP
    net = TerminatorMLP(seed=9)
    x = _dev(np.random.default_rng(6).normal(size=(50, 128)))
    y32 = net.forward(x).cpu().numpy()
    y16 = net.infer_bf16(x).cpu().numpy()
    # BF16 inputs and weights (unit roundoff 2^-8) through 4 layers, FP32 accumulation
    assert rel_l2(y16, y32) < 4 * 4 * 2.0 ** -8


def test_training_kernels_fit_a_smooth_map(bse):
    """Adam with the library's gradients drives the loss of a smooth regression down."""
    from paper_1602_01863_amd.terminator import TerminatorMLP, train
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, size=(2048, 8))
    t = np.stack([np.sin(2 * x[:, 0]) * x[:, 1], x[:, 2] ** 2 - x[:, 3], np.cos(x[:, 4] + x[:, 5])], axis=1)
    net = TerminatorMLP(seed=1, sizes=(8, 64, 64, 3))
    hist = train(net, x, t, epochs=60, batch=128, lr=3e-3)
    assert hist[-1] < 0.05 * hist[0]


def test_terminated_continued_fraction_matches_oracle(bse):
    from paper_1602_01863_amd.terminator import closed_spectrum
    rng = np.random.default_rng(8)
    n, m = 5, 40
    a = rng.uniform(1.0, 5.0, size=(n, m))
    b = np.concatenate([np.zeros((n, 1)), rng.uniform(0.3, 1.5, size=(n, m))], axis=1)
    pn = rng.uniform(0.5, 2.0, size=n)
    ainf, binf = rng.uniform(2, 4, size=n), rng.uniform(0.5, 1.2, size=n)
    om = np.linspace(0.0, 8.0, 301)
    for eta in (0.05, 0.3):
        got = closed_spectrum(a, b, pn, ainf, binf, 0.7, om, eta)
        ref = O.continued_fraction_terminated(a, b, pn, 0.7, om, eta, ainf, binf)
        assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_trained_network_gains_over_the_method_without_it(bse):
    """Held-out C1-size chains (8 seeded problems x 3 polarisations) against 600-step
    plain chains.  From the first 64 steps, the committed network's closure is far
    better than the truncated fraction (the method without a terminator) and better
    than closing with the constant chain of the last computed coefficients."""
    from paper_1602_01863_amd import terminator as T
    net = T.TerminatorMLP.load(T.default_weights_path())
    rows = T.evaluate(net, n_problems=8, etas=(0.05, 0.1, 0.2))
    for eta, r in rows.items():
        assert r["network_64"] < 0.5 * r["truncated_64"], eta
        assert r["network_64"] < r["head_closure_64"], eta
        assert r["plain_300"] < r["network_64"], eta


def test_error_estimate_admits_no_chain_beyond_the_rule(bse):
    """The fallback rule on held-out C1-size chains (8 seeded problems x 3 polarisations)
    against 600-step plain chains: no chain whose estimate (the move of the closed
    spectrum when 32 computed coefficients replace predicted ones) is <= 1e-3 has a true
    eps2 error above 1e-3, at eta = 0.1, 0.2 and 0.5 eV."""
    from paper_1602_01863_amd import terminator as T
    net = T.TerminatorMLP.load(T.default_weights_path())
    rows = T.evaluate(net, n_problems=8, etas=(0.1, 0.2, 0.5))
    for eta, r in rows.items():
        assert r["false_accepts"] == 0, (eta, r)
        if r["accepted"]:
            assert r["worst_accepted_error"] <= 1e-3, (eta, r)


def test_fallback_hands_chains_to_the_plain_run(bse):
    """With a zero threshold every chain of a C0 problem at eta = 0.1 falls back and the
    spectrum is the plain chain's; with a loose threshold none does and the spectrum is
    the network's checked closure."""
    import tbinputs as ti
    from _cases import bands
    from paper_1602_01863_amd import terminator as T
    cfg = ti.get_config("c0")
    bs = bands(cfg)
    prob = bse.problem_from_bands(bs, cfg, dtype="f64", max_rhs=1)
    net = T.TerminatorMLP.load(T.default_weights_path())
    P = bs.P_flat()
    om, C = cfg.omega(), cfg.prefactor()
    eps, fb = T.run_with_fallback(prob, P, net, cfg.steps, C, om, 0.1, threshold=0.0)
    plain = prob.continued_fraction(prob.haydock(P, cfg.steps), C, om, 0.1).cpu().numpy()
    assert fb.all() and np.array_equal(eps, plain)
    eps2, fb2 = T.run_with_fallback(prob, P, net, cfg.steps, C, om, 0.1, threshold=10.0)
    ch = prob.haydock(P, T.M_IN + T.K_CHECK)
    a, b = ch["a"].cpu().numpy(), ch["b"].cpu().numpy()
    e_net, _, _ = T.terminated_eps(net, a, b, ch["pnorm2"].cpu().numpy(), C, om, 0.1, threshold=10.0)
    assert not fb2.any() and np.array_equal(eps2, e_net)
    prob.close()
