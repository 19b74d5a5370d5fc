"""Chains run to a converged spectrum (bse_haydock_converge): the stop rule of Sec. 2
(after Eq. fraccont) on the device, against the oracle and against the fixed-length run."""

import numpy as np
import pytest

import oracle as O
import tbinputs as ti

from _cases import bands, oracle_operator, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bse():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_01863_amd import bse as mod
    return mod


def _host(ch):
    return {k: v.cpu().numpy().copy() for k, v in ch.items()}


def test_converged_chain_stops_by_the_rule_and_matches_the_oracle(bse):
    """C0 in FP64 at eta = 0.3 eV: the chain stops at the first check where eps2 moved by
    at most tol of its peak since the previous check; its coefficients are the
    fixed-length run's up to that step (same kernels) and zero after it; the returned
    spectrum is Eq. (fraccont) of those coefficients and lies within 10 tol of the
    oracle's converged spectrum."""
    cfg = ti.get_config("c0")
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f64", max_rhs=1)
    P = bands(cfg).P_flat()[:1]
    om = cfg.omega()
    eta, tol, every, cap = 0.3, 1e-5, 10, 400
    ch, eps = prob.haydock_converge(P, cap, om, eta, cfg.prefactor(), tol, check_every=every)
    ch = _host(ch)
    eps = eps.cpu().numpy()
    m = int(ch["steps"][0])
    assert ch["status"][0] == bse.BSE_OK
    assert m % every == 0 and every < m < cap
    assert np.all(ch["a"][0, m:] == 0) and np.all(ch["b"][0, m + 1:] == 0)
    full = _host(prob.haydock(P, m))
    assert np.array_equal(full["a"][0], ch["a"][0, :m]) and np.array_equal(full["b"][0], ch["b"][0, :m + 1])
    # the returned spectrum and the stop rule, recomputed from the coefficients
    e_m = O.continued_fraction(ch["a"][:, :m], ch["b"][:, :m + 1], ch["pnorm2"], cfg.prefactor(), om, eta)
    e_prev = O.continued_fraction(ch["a"][:, :m - every], ch["b"][:, :m - every + 1], ch["pnorm2"],
                                  cfg.prefactor(), om, eta)
    e_prev2 = O.continued_fraction(ch["a"][:, :m - 2 * every], ch["b"][:, :m - 2 * every + 1], ch["pnorm2"],
                                   cfg.prefactor(), om, eta)
    assert rel_l2(eps.imag, e_m.imag) < 1e-12 and rel_l2(eps.real - 1, e_m.real - 1) < 1e-12
    peak = np.abs(e_m.imag).max()
    assert np.abs(e_m.imag - e_prev.imag).max() <= tol * peak
    assert np.abs(e_prev.imag - e_prev2.imag).max() > tol * np.abs(e_prev.imag).max()
    # against the oracle's converged spectrum (400 steps): the spectrum converges
    # geometrically in the chain length, so what remains after the last change of at
    # most tol of the peak is of that order; held to 10 tol
    op = oracle_operator(cfg)
    och = O.haydock(op.apply, P, cap)
    oeps = O.continued_fraction(och["a"], och["b"], och["pnorm2"], cfg.prefactor(), om, eta)
    assert rel_l2(eps.imag, oeps.imag) < 10 * tol
    prob.close()


def test_chains_stop_independently(bse):
    """Three polarisations at FP32 storage stop at their own checks; a zero start vector
    ends its chain at once (eps_M = 1, Eq. fraccont with ||P|| = 0)."""
    cfg = ti.tiny_config(n_coarse=3, n_div=3, nv=3, nc=6, n_orb=9, seed=11, n_pol=3)
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f32", max_rhs=3)
    P = bands(cfg).P_flat().copy()
    P[1] = 0.0
    om = np.linspace(0.0, 16.0, 801)
    ch, eps = prob.haydock_converge(P, 300, om, 0.5, cfg.prefactor(), 1e-4, check_every=8)
    ch = _host(ch)
    eps = eps.cpu().numpy()
    assert ch["status"][1] == bse.BSE_INFO_ZERO_START and ch["steps"][1] == 0
    assert np.all(eps[1].real == 1.0) and np.all(eps[1].imag == 0.0)
    for r in (0, 2):
        m = int(ch["steps"][r])
        assert ch["status"][r] == bse.BSE_OK and m % 8 == 0 and m < 300
        e_m = O.continued_fraction(ch["a"][r:r + 1, :m], ch["b"][r:r + 1, :m + 1], ch["pnorm2"][r:r + 1],
                                   cfg.prefactor(), om, 0.5)
        assert rel_l2(eps[r].imag, e_m[0].imag) < 1e-12
    prob.close()


def test_closed_convergence_matches_the_oracle_and_stops_no_later(bse):
    """The same C0 chain with each checked fraction closed by the constant chain of its last
    16 coefficients (bse_plan_set_converge_closure): the returned spectrum is the oracle's
    closed fraction of the device's own coefficients (1e-12), the stop rule holds on the
    closed spectra, it lies within 10 tol of the oracle's converged spectrum, and it stops
    no later than the truncated run."""
    cfg = ti.get_config("c0")
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f64", max_rhs=1)
    P = bands(cfg).P_flat()[:1]
    om = cfg.omega()
    C = cfg.prefactor()
    eta, tol, every, cap, k = 0.3, 1e-5, 10, 400, 16
    ch0, _ = prob.haydock_converge(P, cap, om, eta, C, tol, check_every=every)
    m0 = int(ch0["steps"][0])
    ch, eps = prob.haydock_converge(P, cap, om, eta, C, tol, check_every=every, closure=k)
    ch = _host(ch)
    eps = eps.cpu().numpy()
    m = int(ch["steps"][0])
    assert ch["status"][0] == bse.BSE_OK and m % every == 0 and k <= m <= m0

    def closed(mm):   # a check with fewer than k steps uses the truncated fraction
        a, b = ch["a"][:, :mm], ch["b"][:, :mm + 1]
        if mm < k:
            return O.continued_fraction(a, b, ch["pnorm2"], C, om, eta)
        return O.continued_fraction_terminated(a, b, ch["pnorm2"], C, om, eta, a[:, mm - k:mm].mean(axis=1),
                                               b[:, mm - k + 1:mm + 1].mean(axis=1))

    e_m, e_prev, e_prev2 = closed(m), closed(m - every), closed(m - 2 * every)
    assert rel_l2(eps.imag, e_m.imag) < 1e-12 and rel_l2(eps.real - 1, e_m.real - 1) < 1e-12
    assert np.abs(e_m.imag - e_prev.imag).max() <= tol * np.abs(e_m.imag).max()
    assert np.abs(e_prev.imag - e_prev2.imag).max() > tol * np.abs(e_prev.imag).max()
    op = oracle_operator(cfg)
    och = O.haydock(op.apply, P, cap)
    oeps = O.continued_fraction(och["a"], och["b"], och["pnorm2"], C, om, eta)
    assert rel_l2(eps.imag, oeps.imag) < 10 * tol
    prob.close()


@pytest.mark.parametrize("every", [1, 3, 5, 40])
def test_unconverged_run_is_the_fixed_length_chain(bse, every):
    """tol = 0 never stops a chain, so it runs to max_steps (37, not a multiple of the check
    interval: the last chunk is short; the interval 1 checks after every step, 40 exceeds
    the whole run): the coefficients, norms and status are the fixed-length run's bit for
    bit, whatever steps were enqueued ahead of each check, and the spectrum is Eq.
    (fraccont) of all 37 coefficients."""
    cfg = ti.get_config("c0")
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f64", max_rhs=1)
    P = bands(cfg).P_flat()[:1]
    om = cfg.omega()
    n = 37
    ch, eps = prob.haydock_converge(P, n, om, 0.3, cfg.prefactor(), 0.0, check_every=every)
    ch = _host(ch)
    full = _host(prob.haydock(P, n))
    for k in ("a", "b", "pnorm2", "steps", "status"):
        assert np.array_equal(ch[k], full[k]), k
    assert ch["steps"][0] == n
    e_n = O.continued_fraction(ch["a"], ch["b"], ch["pnorm2"], cfg.prefactor(), om, 0.3)
    assert rel_l2(eps.cpu().numpy().imag, e_n.imag) < 1e-12
    prob.close()
