"""CPU pins of the oracle's Method 3 (Sec. 4): the divergent part of Eq. (diverg)
for the model kernel, the band of offsets, the explicit M3 kernel and its sparse
correction form."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import tbinputs as ti

from _cases import bands, oracle_operator


def _shape_params(cfg):
    k2 = O.screening_kappa2(cfg.eps_inf, cfg.lam)
    s0 = O.s_q0_average(cfg.n_coarse, cfg.n_div, k2, cfg.q0_quad)
    return k2, s0


def _identity_vectors(nk, nb):
    v = np.zeros((nk, nb, nb), dtype=np.complex128)
    v[:, np.arange(nb), np.arange(nb)] = 1.0
    return v


def test_screened_shape_is_w_up_to_its_prefactor():
    """W(Q) = s(Q) / (pi eps_inf), at q != 0 and as mini-cell means at q = 0."""
    cfg = ti.get_config("c0")
    k2, s0 = _shape_params(cfg)
    q = np.random.default_rng(0).uniform(-0.5, 0.5, size=(50, 3))
    np.testing.assert_allclose(O.w_model(q, cfg.eps_inf, cfg.lam),
                               O.s_shape(q, k2) / (np.pi * cfg.eps_inf), rtol=1e-14)
    wq0 = O.w_q0_average(cfg.n_coarse, cfg.n_div, cfg.eps_inf, cfg.lam, cfg.q0_quad)
    assert abs(wq0 - s0 / (np.pi * cfg.eps_inf)) < 1e-14 * wq0


@pytest.mark.parametrize("seed", [0, 5])
def test_divergence_coefficient_is_the_g0_direct_term(seed):
    """With only G = 0 in the model (no exchange, one direct term) the coarse kernel is
    exactly a_c S_c: sign, prefactor, conjugate placement and the q = 0 mean."""
    cfg = ti.tiny_config(n_coarse=3, n_div=2, nv=2, nc=3, n_orb=6, seed=seed).with_(g2_max=0)
    bs = bands(cfg)
    K = O.coarse_kernel(bs.vecs_coarse, bs.tau, 2, 3, 3, 2, cfg)
    a = O.divergence_coefficient(bs.vecs_coarse, bs.tau, 2, 3, 3, 2, cfg)
    k2, s0 = _shape_params(cfg)
    S = np.kron(O.coarse_shape(3, k2, s0), np.ones((6, 6)))
    np.testing.assert_allclose(a * S, K, rtol=0, atol=1e-13 * np.abs(K).max())
    assert np.abs(a - a.conj().T).max() == 0.0


def test_band_offsets_are_the_lattice_points_of_the_ball():
    # lattice points with |o|^2 <= 1, 4, 16: 7, 33, 257
    assert [len(O.m3.band_offsets(n, 1.0)) for n in (1, 2, 4)] == [7, 33, 257]
    assert len(O.m3.band_offsets(4, 0.5)) == 33 and len(O.m3.band_offsets(2, 0.4)) == 1
    off = O.m3.band_offsets(3, 1.0)
    assert set(map(tuple, off)) == set(map(tuple, -off))
    assert [tuple(o) for o in off] == sorted(tuple(o) for o in off)


def test_m3_reproduces_the_dense_mesh_kernel_inside_the_band():
    """One site, orbital-diagonal bands, G = 0 only: the dense-mesh kernel is
    a s(q_dense) with a constant a.  Method 3 gives it exactly inside the band (and
    keeps Method 1 outside), while Method 1 alone does not."""
    n_c, n_div, w = 4, 2, 1.0
    cfg = ti.tiny_config(n_coarse=n_c, n_div=n_div, nv=1, nc=1, n_orb=2).with_(g2_max=0)
    nd = n_c * n_div
    vc, vd = _identity_vectors(n_c ** 3, 2), _identity_vectors(nd ** 3, 2)
    tau = np.zeros((2, 3))
    Dv, Dc = O.overlaps(vc, vd, n_c, n_div, 1, 1)
    Kc = O.coarse_kernel(vc, tau, 1, 1, n_c, n_div, cfg)
    op = O.InterpOperator(Dv, Dc, O.trilinear_weights(n_div), Kc, np.zeros(nd ** 3), n_c, n_div, 1, 1)
    a = O.divergence_coefficient(vc, tau, 1, 1, n_c, n_div, cfg)
    k2, s0 = _shape_params(cfg)
    K3 = O.m3.explicit_kernel(op, a, O.coarse_shape(n_c, k2, s0), w, k2, s0)
    K1 = op.explicit_kernel()
    # the kernel built directly on the dense mesh, put in cell-major order
    Kd = O.coarse_kernel(vd, tau, 1, 1, nd, 1, cfg)
    x = O.m3.dense_coords(n_c, n_div)
    lex = (x[:, 0] * nd + x[:, 1]) * nd + x[:, 2]
    Kd = Kd[np.ix_(lex, lex)]
    o = O.fold_int(x[:, None, :] - x[None, :, :], nd)
    band = np.sum(o * o, axis=-1) <= (w * n_div) ** 2
    scale = np.abs(Kd).max()
    assert np.abs(K3 - Kd)[band].max() < 1e-13 * scale
    assert np.abs(K1 - Kd)[band].max() > 0.1 * scale
    np.testing.assert_array_equal(K3[~band], K1[~band])


def test_m3_with_one_division_is_the_coarse_kernel():
    cfg = ti.tiny_config(n_coarse=3, n_div=1, nv=2, nc=2)
    bs = bands(cfg)
    op = oracle_operator(cfg)
    a = O.divergence_coefficient(bs.vecs_coarse, bs.tau, 2, 2, 3, 1, cfg)
    k2, s0 = _shape_params(cfg)
    K3 = O.m3.explicit_kernel(op, a, O.coarse_shape(3, k2, s0), 1.0, k2, s0)
    assert np.abs(K3 - op.Kc).max() < 1e-14 * np.abs(op.Kc).max()


@pytest.mark.parametrize("weights", ["trilinear", "nearest"])
def test_sparse_correction_equals_the_explicit_kernel(weights):
    """M1 product + sum_o Delta(k, k + o) x_{k+o} = (diag + K^{M3}) x, brute force."""
    cfg = ti.tiny_config(n_coarse=3, n_div=2, nv=2, nc=2, n_orb=5, seed=4)
    bs = bands(cfg)
    op = oracle_operator(cfg, weights)
    a = O.divergence_coefficient(bs.vecs_coarse, bs.tau, 2, 2, 3, 2, cfg)
    k2, s0 = _shape_params(cfg)
    Sc = O.coarse_shape(3, k2, s0)
    w = 1.0
    K3 = O.m3.explicit_kernel(op, a, Sc, w, k2, s0)
    assert np.abs(K3 - K3.conj().T).max() < 1e-15 * np.abs(K3).max()
    off = O.m3.band_offsets(2, w)
    sd = O.m3.dense_shape(off, 3, 2, k2, s0)
    blocks = O.m3.band_blocks(op, a, Sc, off, sd)
    x = np.random.default_rng(1).normal(size=(2, op.N)) + 1j * np.random.default_rng(2).normal(size=(2, op.N))
    ref = (op.delta[:, None] * x.T + K3 @ x.T).T
    got = O.m3.apply(op, blocks, off, x)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # the band changes the operator (it is not a no-op on this case)
    assert np.abs(K3 - op.explicit_kernel()).max() > 1e-3 * np.abs(K3).max()


def test_m3_is_closer_than_m1_to_the_dense_mesh_spectrum():
    """Sec. 5 finds Method 3 closest to the dense-mesh result.  Against the BSE
    built directly on the dense mesh (no interpolation), eps2 from M3 (w = 1) is
    clearly closer than from M1 on a small crystal (eigendecomposition, eta = 0.1)."""
    cfg = ti.tiny_config(n_coarse=3, n_div=2, nv=2, nc=2, n_orb=5, seed=4)
    bs = bands(cfg)
    op = oracle_operator(cfg)
    nd = 6
    x = O.m3.dense_coords(3, 2)
    lex = (x[:, 0] * nd + x[:, 1]) * nd + x[:, 2]
    inv = np.empty_like(lex)
    inv[lex] = np.arange(len(lex))
    Kd = O.coarse_kernel(bs.vecs_dense[inv], bs.tau, 2, 2, nd, 1, cfg)
    Kd = Kd.reshape(nd ** 3, 4, nd ** 3, 4)[lex][:, :, lex].reshape(nd ** 3 * 4, -1)
    a = O.divergence_coefficient(bs.vecs_coarse, bs.tau, 2, 2, 3, 2, cfg)
    k2, s0 = _shape_params(cfg)
    K3 = O.m3.explicit_kernel(op, a, O.coarse_shape(3, k2, s0), 1.0, k2, s0)
    D = np.diag(op.delta).astype(complex)
    P, om, C = bs.P_flat(), cfg.omega(), cfg.prefactor()
    ref = O.eigh_spectrum(D + Kd, P, C, om, 0.1).imag
    err = lambda K: np.linalg.norm(O.eigh_spectrum(D + K, P, C, om, 0.1).imag - ref) / np.linalg.norm(ref)
    e1, e3 = err(op.explicit_kernel()), err(K3)
    assert e3 < 0.7 * e1, (e1, e3)
