"""Pins for the oracle's interpolated Hamiltonian and its on-the-fly product
(Eqs. bse1, interp1, matmul1-matmul3)."""

import numpy as np
import pytest

import oracle as O
import tbinputs as ti

from _cases import bands, oracle_operator, oracle_parts, rel_l2

SMALL = [
    ti.tiny_config(n_coarse=2, n_div=2, nv=2, nc=2),
    ti.tiny_config(n_coarse=3, n_div=2, nv=2, nc=3, n_orb=6, seed=4),
    ti.tiny_config(n_coarse=2, n_div=3, nv=1, nc=2, n_orb=4, seed=9),
]


@pytest.mark.parametrize("cfg", SMALL + [ti.get_config("c0")], ids=lambda c: c.name)
def test_fast_matvec_equals_explicit_interpolated_matrix(cfg):
    op = oracle_operator(cfg)
    H = op.explicit_hamiltonian()
    x = ti.random_vectors(op.N, 2, 21)
    y_fast = op.apply(x)
    y_ref = (H @ x.T).T
    assert rel_l2(y_fast, y_ref) < 1e-13
    # and the kernel alone (the diagonal cannot hide an error in the small part)
    assert rel_l2(op.apply_kernel(x), (op.explicit_kernel() @ x.T).T) < 1e-13


@pytest.mark.parametrize("cfg", SMALL + [ti.get_config("c0")], ids=lambda c: c.name)
def test_collapsed_corner_sum_equals_literal_eq_matmul2(cfg):
    op = oracle_operator(cfg)
    x = ti.random_vectors(op.N, 1, 5)
    assert rel_l2(op.apply(x), op.apply_literal(x)) < 1e-13


@pytest.mark.parametrize("cfg", SMALL, ids=lambda c: c.name)
def test_interpolated_hamiltonian_hermitian_and_restrict_prolong_adjoint(cfg):
    op = oracle_operator(cfg)
    H = op.explicit_hamiltonian()
    assert np.abs(H - H.conj().T).max() < 1e-14 * np.abs(H).max()
    x = ti.random_vectors(op.N, 1, 1)
    y = ti.random_vectors(op.N, 1, 2)
    lhs = np.vdot(x, op.apply(y))
    rhs = np.vdot(op.apply(x), y)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    r = ti.random_vectors(op.Nc, 1, 3)
    a = np.vdot(op.restrict(x), r)
    b = np.vdot(x, op.prolong(r))
    assert abs(a - b) < 1e-13 * abs(a)


@pytest.mark.parametrize("n_c,nv,nc", [(2, 2, 2), (3, 1, 3)])
def test_single_division_reproduces_coarse_bse(n_c, nv, nc):
    """n_div = 1: the dense mesh is the coarse one and H^i = diag(delta) + K_c."""
    cfg = ti.tiny_config(n_coarse=n_c, n_div=1, nv=nv, nc=nc, n_orb=nv + nc + 1, seed=n_c)
    bs, Dv, Dc, f, Kc, delta = oracle_parts(cfg)
    op = oracle_operator(cfg)
    x = ti.random_vectors(op.N, 2, 8)
    ref = delta[None] * x + (Kc @ x.T).T
    assert rel_l2(op.apply(x), ref) < 1e-14


def test_zero_kernel_is_the_diagonal():
    cfg = SMALL[1]
    op = oracle_operator(cfg, Kc=np.zeros((SMALL[1].n_trans_coarse,) * 2, complex))
    x = ti.random_vectors(op.N, 1, 4)
    np.testing.assert_array_equal(op.apply(x), op.delta[None] * x)


@pytest.mark.parametrize("n_div", [2, 3, 4])
def test_linear_in_k_separable_kernel_is_interpolated_exactly(n_div):
    """d = I (k-independent bands) and K_c(k~, k~') = g(k~) g(k~')^H with g affine in
    k~: on cells away from the periodic wrap the interpolated kernel equals
    g(k) g(k')^H at the dense points (trilinear interpolation of an affine g)."""
    n_c, nv, nc = 4, 1, 2
    npair = nv * nc
    nk = n_c ** 3 * n_div ** 3
    rng = np.random.default_rng(2)
    alpha = rng.normal(size=(npair, 3)) + 1j * rng.normal(size=(npair, 3))
    beta = rng.normal(size=npair) + 1j * rng.normal(size=npair)
    kc = ti.coarse_kpoints(n_c)
    g = (kc @ alpha.T + beta).reshape(-1)                      # [(k~, pair)]
    Kc = np.outer(g, g.conj())
    Dv = np.broadcast_to(np.eye(nv), (nk, 8, nv, nv)).astype(complex)
    Dc = np.broadcast_to(np.eye(nc), (nk, 8, nc, nc)).astype(complex)
    op = O.InterpOperator(Dv, Dc, O.trilinear_weights(n_div), Kc, np.zeros(nk * npair),
                          n_c, n_div, nv, nc)
    kd = ti.dense_kpoints(n_c, n_div)
    interior = np.all(kd < (n_c - 1) / n_c, axis=1)          # cells with i < n_c - 1
    mask = np.repeat(interior, npair)
    x = ti.random_vectors(op.N, 1, 6)
    x[:, ~mask] = 0
    gd = (kd @ alpha.T + beta).reshape(-1)
    ref = gd * np.vdot(gd[mask], x[0, mask])
    y = op.apply_kernel(x)[0]
    np.testing.assert_allclose(y[mask], ref[mask], rtol=0, atol=1e-12 * np.abs(ref).max())


def test_gauge_invariance_of_the_matvec():
    """Random phases on every dense and coarse band transform H^i as U^H H^i U."""
    cfg = SMALL[1]
    bs = bands(cfg)
    rng = np.random.default_rng(12)
    th = np.exp(1j * rng.uniform(0, 2 * np.pi, size=bs.vecs_dense.shape[:2]))
    vd = bs.vecs_dense * th[..., None]
    vc = vd[::cfg.n_div3].copy()
    Dv, Dc = O.overlaps(vc, vd, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    Kc = O.coarse_kernel(vc, bs.tau, cfg.nv, cfg.nc, cfg.n_coarse, cfg.n_div, cfg)
    delta = O.transition_energies(bs.eps_dense, cfg.nv, cfg.nc)
    op2 = O.InterpOperator(Dv, Dc, O.trilinear_weights(cfg.n_div), Kc, delta, cfg.n_coarse,
                           cfg.n_div, cfg.nv, cfg.nc)
    op1 = oracle_operator(cfg)
    u = (np.conj(th[:, :cfg.nv, None]) * th[:, None, cfg.nv:cfg.nv + cfg.nc]).reshape(-1)
    x = ti.random_vectors(op1.N, 1, 13)
    # H2 = U^H H1 U  with U = diag(u)
    np.testing.assert_allclose(op2.apply(x)[0], np.conj(u) * op1.apply(u * x)[0], atol=1e-12)
