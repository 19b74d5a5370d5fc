"""Pins for the overlaps d (Eq. completeness) and the coarse kernel (Eqs. bse2-bse3b)."""

import numpy as np
import pytest
from scipy import integrate

import oracle as O
import tbinputs as ti

from _cases import bands, oracle_parts


def test_overlaps_identity_at_shared_points():
    """At j = 0 the dense point is the coarse corner 000 with the same vectors: d = I."""
    cfg = ti.tiny_config(n_coarse=3, n_div=2, nv=2, nc=3, n_orb=6)
    bs = bands(cfg)
    Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    sub0 = np.arange(cfg.nk_coarse) * cfg.n_div3
    np.testing.assert_allclose(Dv[sub0, 0], np.broadcast_to(np.eye(2), (len(sub0), 2, 2)), atol=1e-14)
    np.testing.assert_allclose(Dc[sub0, 0], np.broadcast_to(np.eye(3), (len(sub0), 3, 3)), atol=1e-14)


def test_overlaps_gauge_covariance():
    """A phase on dense band n multiplies row n of d; a phase on coarse band n'
    multiplies column n' by its conjugate (d = <u_{n'k~}|u_{nk}>)."""
    cfg = ti.tiny_config(n_coarse=2, n_div=2, nv=2, nc=2)
    bs = bands(cfg)
    rng = np.random.default_rng(3)
    th_d = np.exp(1j * rng.uniform(0, 2 * np.pi, size=bs.vecs_dense.shape[:2]))
    th_c = np.exp(1j * rng.uniform(0, 2 * np.pi, size=bs.vecs_coarse.shape[:2]))
    Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, 2, 2, 2, 2)
    Dv2, Dc2 = O.overlaps(bs.vecs_coarse * th_c[..., None], bs.vecs_dense * th_d[..., None],
                          2, 2, 2, 2)
    nbr = O.neighbour_table(2)
    cell = np.arange(bs.vecs_dense.shape[0]) // 8
    for z in range(8):
        kc = nbr[cell, z]
        exp_v = th_d[:, :2, None] * np.conj(th_c[kc, None, :2]) * Dv[:, z]
        exp_c = th_d[:, 2:, None] * np.conj(th_c[kc, None, 2:]) * Dc[:, z]
        np.testing.assert_allclose(Dv2[:, z], exp_v, atol=1e-14)
        np.testing.assert_allclose(Dc2[:, z], exp_c, atol=1e-14)


def test_overlaps_unitary_for_decoupled_manifolds():
    """If H(k) never mixes valence and conduction orbitals, both blocks are unitary."""
    cfg = ti.tiny_config(n_coarse=2, n_div=3, nv=2, nc=2)
    model = ti.make_model(cfg)
    model.HR[:, :2, 2:] = 0
    model.HR[:, 2:, :2] = 0
    bs = ti.band_structure(cfg, model)
    Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, 2, 3, 2, 2)
    eye = np.eye(2)
    np.testing.assert_allclose(np.einsum("kzvn,kzvm->kznm", Dv.conj(), Dv),
                               np.broadcast_to(eye, Dv.shape), atol=1e-13)
    np.testing.assert_allclose(np.einsum("kzvn,kzvm->kznm", Dc.conj(), Dc),
                               np.broadcast_to(eye, Dc.shape), atol=1e-13)


def test_g_vectors_sphere():
    G = O.g_vectors(4)
    assert len(G) == 33
    assert {tuple(g) for g in G} == {tuple(-g) for g in G}
    assert np.all((G ** 2).sum(1) <= 4)


@pytest.mark.parametrize("n_c,n_div", [(2, 1), (4, 2)])
def test_w_q0_average_matches_adaptive_quadrature(n_c, n_div):
    eps, lam = 12.0, 0.3
    h = 0.5 / (n_c * n_div)
    val, _ = integrate.tplquad(lambda z, y, x: O.w_model(np.array([x, y, z]), eps, lam),
                               -h, h, -h, h, -h, h, epsabs=1e-10, epsrel=1e-10)
    exact = val / (2 * h) ** 3
    # the midpoint rule converges to the adaptive value (peaked integrand at q = 0)
    assert abs(O.w_q0_average(n_c, n_div, eps, lam, 16) - exact) / exact < 1e-2
    assert abs(O.w_q0_average(n_c, n_div, eps, lam, 128) - exact) / exact < 5e-5


def _identity_vectors(nk, nb, n_orb):
    v = np.zeros((nk, nb, n_orb), dtype=np.complex128)
    v[:, np.arange(nb), np.arange(nb)] = 1.0
    return v


def test_kernel_direct_term_lattice_sum_special_case():
    """Orbital-diagonal bands on one site: no exchange, and the direct term of each
    pair reduces to the scalar lattice sum sum_G W(q + G) (W averaged at q = G = 0)."""
    cfg = ti.tiny_config(n_coarse=3, n_div=2, nv=1, nc=2, n_orb=3)
    vecs = _identity_vectors(cfg.nk_coarse, 3, 3)
    tau = np.zeros((3, 3))
    K = O.coarse_kernel(vecs, tau, 1, 2, 3, 2, cfg).reshape(27, 2, 27, 2)
    G = O.g_vectors(cfg.g2_max)
    ijk = np.stack(np.meshgrid(*[np.arange(3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    wq0 = O.w_q0_average(3, 2, cfg.eps_inf, cfg.lam, cfg.q0_quad)
    for k in (0, 5, 13):
        for kp in (0, 7, 13, 26):
            q = O.fold_int(ijk[k] - ijk[kp], 3) / 3.0
            s = 0.0
            for g in G:
                if k == kp and not g.any():
                    s += wq0
                else:
                    s += O.w_model(q + g, cfg.eps_inf, cfg.lam)
            expect = -(cfg.kernel_energy / cfg.nk_dense) * s
            np.testing.assert_allclose(K[k, :, kp, :], expect * np.eye(2), rtol=1e-13, atol=1e-15)


def test_kernel_exchange_only_is_psd_low_rank():
    """Without screening (W -> 0) K_c = 2 X: a Gram matrix over the 32 G != 0."""
    cfg = ti.tiny_config(n_coarse=3, n_div=1, nv=2, nc=2).with_(eps_inf=1e30, lam=1e15)
    bs = bands(ti.tiny_config(n_coarse=3, n_div=1, nv=2, nc=2))
    K = O.coarse_kernel(bs.vecs_coarse, bs.tau, 2, 2, 3, 1, cfg)
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-12 * ev.max()
    assert np.sum(ev > 1e-10 * ev.max()) <= 32
    assert ev.max() > 0


def test_kernel_same_site_has_no_exchange_and_attractive_diagonal():
    cfg = ti.tiny_config(n_coarse=2, n_div=2, nv=2, nc=2)
    bs = bands(cfg)
    K = O.coarse_kernel(bs.vecs_coarse, np.zeros_like(bs.tau), 2, 2, 2, 2, cfg)
    # with every tau equal, M_cv(k,k;G) = <c|v> = 0: only -W remains; its diagonal is
    # -sum_G W |<c|c>|^2 |<v|v>|^2 < 0 at q = 0
    assert np.all(np.real(np.diag(K)) < 0)


def test_kernel_hermitian_and_block_rows():
    cfg = ti.get_config("c0")
    bs, Dv, Dc, f, Kc, delta = oracle_parts(cfg)
    assert np.abs(Kc - Kc.conj().T).max() == 0.0
    rows = O.coarse_kernel_block_rows(bs.vecs_coarse, bs.tau, 3, 3, 4, 2, cfg, np.array([0, 21, 63]))
    ref = Kc.reshape(64, 9, -1)[[0, 21, 63]]
    np.testing.assert_allclose(rows, ref, rtol=0, atol=1e-15)


def test_kernel_gauge_covariance():
    """Phases on coarse bands transform K_c as U^H K_c U (pair phase conj(t_v) t_c)."""
    cfg = ti.tiny_config(n_coarse=2, n_div=2, nv=2, nc=2)
    bs = bands(cfg)
    rng = np.random.default_rng(11)
    th = np.exp(1j * rng.uniform(0, 2 * np.pi, size=bs.vecs_coarse.shape[:2]))
    K1 = O.coarse_kernel(bs.vecs_coarse, bs.tau, 2, 2, 2, 2, cfg)
    K2 = O.coarse_kernel(bs.vecs_coarse * th[..., None], bs.tau, 2, 2, 2, 2, cfg)
    # pair (v, c, k): u*_v u_c picks up conj(t_v) t_c
    u = (np.conj(th[:, :2, None]) * th[:, None, 2:]).reshape(-1)
    np.testing.assert_allclose(K2, np.conj(u)[:, None] * K1 * u[None, :], atol=1e-15)


# ---- closed-form pins of the kernel's scales (Eq. bse2, Eq. bse3a, Eq. bse3b / Wcoul) ----
PI = np.pi


def test_w_model_literal_values():
    """W(Q) = 4 pi / (eps_inf |Q|^2 + lambda^2) with Cartesian |Q| = 2 pi |q + G| of the
    cubic cell (lattice constant 1): literal values at eps_inf = 12, lambda = 0.3."""
    eps, lam = 12.0, 0.3
    cases = [((0.5, 0.0, 0.0), 4 * PI / (12 * PI ** 2 + 0.09)),          # |2 pi Q|^2 = pi^2
             ((0.0, 0.0, 0.0), 4 * PI / 0.09),
             ((1.0, 1.0, 0.0), 4 * PI / (96 * PI ** 2 + 0.09)),          # 8 pi^2
             ((0.25, -0.5, 1.0), 4 * PI / (12 * 4 * PI ** 2 * 1.3125 + 0.09))]
    for Q, expect in cases:
        assert O.w_model(np.array(Q), eps, lam) == pytest.approx(expect, rel=1e-15)
    got = O.w_model(np.array([c[0] for c in cases]), eps, lam)
    np.testing.assert_allclose(got, [c[1] for c in cases], rtol=1e-15)


def _two_site_hybrid(nk):
    """One orbital on each of two sites, tau_A = 0 and tau_B = (1/4, 1/4, 1/4), and the
    same bonding / antibonding pair at every k: v = (A + B)/sqrt 2, c = (A - B)/sqrt 2."""
    s = 1.0 / np.sqrt(2.0)
    vecs = np.empty((nk, 2, 2), dtype=np.complex128)
    vecs[:, 0] = (s, s)
    vecs[:, 1] = (s, -s)
    tau = np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.25]])
    return vecs, tau


def test_kernel_exchange_closed_form_two_sites():
    """Exchange scale: with W switched off, K_c = (E_K / N_k) 2 X (Eq. bse2) and
    X = sum_{G != 0} v(G) |M_cv(G)|^2 with v(G) = 4 pi / |2 pi G|^2 (Eq. bse3a).
    For the hybridised pair M_cv(k,k;G) = (1 - exp(i 2 pi G.tau_B)) / 2, so
    |M_cv|^2 = sin^2(pi (G1 + G2 + G3) / 4), the same for every (k, k').
    Shell by shell over |G|^2 <= 4 (6, 12, 8 and 6 vectors):
      |G|^2 = 1: 6 (1/pi) (1/2)    = 3/pi
      |G|^2 = 2: 6 of 12 with s = +-2, each 1/(2 pi)  = 3/pi
      |G|^2 = 3: 8 (1/(3 pi)) (1/2) = 4/(3 pi)
      |G|^2 = 4: 6 (1/(4 pi)) 1     = 3/(2 pi)
    X = 53/(6 pi), so every element is (E_K / N_k) 53/(3 pi).  A dropped factor 2,
    a reduced |G| in v, or a wrong sign of the exchange fails this."""
    cfg = ti.tiny_config(n_coarse=2, n_div=3, nv=1, nc=1, n_orb=2).with_(eps_inf=1e30, lam=1e15)
    vecs, tau = _two_site_hybrid(cfg.nk_coarse)
    K = O.coarse_kernel(vecs, tau, 1, 1, cfg.n_coarse, cfg.n_div, cfg)
    expect = cfg.kernel_energy / cfg.nk_dense * 53.0 / (3.0 * PI)
    np.testing.assert_allclose(K, np.full(K.shape, expect), rtol=1e-13, atol=0)


def test_kernel_direct_closed_form_two_sites_q0():
    """Direct scale and sign at q = 0 (Eq. bse3b with the model W): for the same pair,
    M_cc(k,k;Q) conj(M_vv(k,k;Q)) = cos^2(pi (Q1 + Q2 + Q3) / 4), which is 1 at G = 0,
    1/2 on |G|^2 = 1 and 3, 1 on the six |G|^2 = 2 vectors with G1 + G2 + G3 = 0 and 0
    on the rest.  So on the diagonal blocks
      D = <W>_0 + 3 W_1 + 6 W_2 + 4 W_3,  W_n = 4 pi / (12 (2 pi)^2 n + 0.09),
    <W>_0 the mini-cell mean of W at q = 0, and K_c = (E_K / N_k) (2 X - D) with X of
    the exchange pin.  W in reduced |Q| (12 n + 0.09) or +D fails this."""
    cfg = ti.tiny_config(n_coarse=2, n_div=2, nv=1, nc=1, n_orb=2)
    vecs, tau = _two_site_hybrid(cfg.nk_coarse)
    K = O.coarse_kernel(vecs, tau, 1, 1, cfg.n_coarse, cfg.n_div, cfg)
    Wn = [4 * PI / (12.0 * 4 * PI ** 2 * n + 0.09) for n in (1, 2, 3)]
    w0 = O.w_q0_average(cfg.n_coarse, cfg.n_div, 12.0, 0.3, cfg.q0_quad)
    D = w0 + 3 * Wn[0] + 6 * Wn[1] + 4 * Wn[2]
    expect = cfg.kernel_energy / cfg.nk_dense * (2 * 53.0 / (6.0 * PI) - D)
    np.testing.assert_allclose(np.diag(K), np.full(cfg.nk_coarse, expect), rtol=1e-13, atol=0)
