"""Coarse-mesh BSE kernel K_c for the synthetic crystal.

Eq. (bse2): K = 2 <v c k | v_bar | v' c' k'> - <v c k | W | v' c' k'>, with the
exchange integral of Eq. (bse3a) (bare Coulomb, G = 0 removed) and the direct
integral of Eq. (bse3b) (screened W, Eq. Wcoul).  In the plane-wave form of
these integrals, with pair densities
    M_nm(k, k'; Q) = <n k| e^{i Q.r} |m k'>
                   ~ sum_a conj(c_{nk,a}) c_{mk',a} exp(i 2 pi Q.tau_a)
for point-like orbitals at reduced positions tau_a:

  exchange  X = sum_{G != 0} v(G) M_cv(k,k;G) conj(M_c'v'(k',k';G)),
  direct    D = sum_G W(q+G) M_cc'(k,k';q+G) conj(M_vv'(k,k';q+G)),
            q = k - k' folded into [-1/2, 1/2)^3,

with v(G) = 4 pi / |G|^2 and the model screened interaction
W(Q) = 4 pi / (eps_inf |Q|^2 + lambda^2), diagonal in G.  Wavevector lengths
are Cartesian, |Q| = 2 pi |q + G| for a cubic lattice of lattice constant 1,
and the integer G run over |G|^2 <= g2_max.  For q = 0 and G = 0 the direct
term uses W averaged over the dense mini-cell around q = 0 (midpoint rule)
instead of W(0).

Readings taken where the paper is silent:
* K_c carries 1 / N_k(dense): the interpolated kernel then has the
  normalisation of a kernel built directly on the dense mesh, and n_div = 1
  gives back the coarse-mesh BSE.  K_c = kernel_energy / N_k(dense) (2X - D).
* With an even mesh, q = +-1/2 both fold to -1/2, which breaks W(q) = W(-q)
  between (k, k') and (k', k).  K_c is made Hermitian by construction: the
  block (k, k') is evaluated for k <= k', the block (k', k) is its conjugate
  transpose, and diagonal blocks are replaced by (A + A^H) / 2.

Transition index on the coarse mesh: T = (k~ * nv + n1) * nc + n2.

Divergent part (Eq. diverg, used by Method 3 of Sec. 4).  The paper splits
each kernel element into a/q^2 + b/q + c.  For this model the only term that
varies sharply as q -> 0 is the G = 0 direct term, and since
W(q) = s(q) / (pi eps_inf) with s(q) = 1 / (|q|^2 + kappa^2) and
kappa^2 = lambda^2 / (4 pi^2 eps_inf) (q reduced), the split reads
    K_c = a_c s(q) + c_c,   b = 0,
    a_c = -(kernel_energy / N_k(dense)) / (pi eps_inf) M_cc'(k,k';q) conj(M_vv'(k,k';q)),
with s(q) in place of 1/q^2 (the two agree as lambda -> 0: the model's
Coulomb tail is screened).  Where K_c uses the mini-cell mean of W at q = 0,
the split uses the mini-cell mean of s.  b = 0 because W is diagonal in G
(no head-wing terms).
"""

from __future__ import annotations

import itertools

import numpy as np

from .grids import cell_coords, fold_int

TWO_PI = 2.0 * np.pi


def g_vectors(g2_max: int = 4) -> np.ndarray:
    """Integer reciprocal vectors with |G|^2 <= g2_max (33 for g2_max = 4)."""
    r = int(np.floor(np.sqrt(g2_max)))
    gs = [g for g in itertools.product(range(-r, r + 1), repeat=3)
          if g[0] ** 2 + g[1] ** 2 + g[2] ** 2 <= g2_max]
    return np.array(gs, dtype=np.int64)


def w_model(Q: np.ndarray, eps_inf: float, lam: float) -> np.ndarray:
    """W(Q) = 4 pi / (eps_inf |2 pi Q|^2 + lam^2) for reduced Q[..., 3]."""
    q2 = np.sum((TWO_PI * np.asarray(Q, dtype=np.float64)) ** 2, axis=-1)
    return 4.0 * np.pi / (eps_inf * q2 + lam * lam)


def w_q0_average(n_c: int, n_div: int, eps_inf: float, lam: float, n_quad: int = 16) -> float:
    """Mean of W(q) over q in [-1/2, 1/2)^3 / (n_c n_div), midpoint rule n_quad^3."""
    t = ((np.arange(n_quad) + 0.5) / n_quad - 0.5) / (n_c * n_div)
    q = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    return float(np.mean(w_model(q, eps_inf, lam)))


def _pair_density(ca: np.ndarray, cb: np.ndarray, phase: np.ndarray) -> np.ndarray:
    """M[p, i, j] = sum_a conj(ca[p, i, a]) phase[p, a] cb[p, j, a]."""
    return np.matmul(ca.conj() * phase[:, None, :], cb.swapaxes(-1, -2))


def _direct_formula_blocks(vecs_coarse, tau, nv, nc, n_c, n_div, ks, kps, *, eps_inf, lam,
                           g2_max, kernel_energy, q0_quad):
    """Unsymmetrised blocks B[p, v, c, v', c'] of K_c for pairs (ks[p], kps[p])."""
    ks = np.asarray(ks)
    kps = np.asarray(kps)
    npairs = ks.shape[0]
    nkd = n_c ** 3 * n_div ** 3
    G = g_vectors(g2_max)
    ijk = cell_coords(n_c)
    q = fold_int(ijk[ks] - ijk[kps], n_c).astype(np.float64) / n_c      # [p, 3]
    A = vecs_coarse[ks]
    B = vecs_coarse[kps]
    Av, Ac = A[:, :nv], A[:, nv:nv + nc]
    Bv, Bc = B[:, :nv], B[:, nv:nv + nc]
    same = ks == kps
    wq0 = w_q0_average(n_c, n_div, eps_inf, lam, q0_quad)
    X = np.zeros((npairs, nv, nc, nv, nc), dtype=np.complex128)
    D = np.zeros((npairs, nv, nc, nv, nc), dtype=np.complex128)
    for g in G:
        g = g.astype(np.float64)
        g2 = float(g @ g)
        # exchange: pair densities at zero momentum transfer plus G
        if g2 > 0.0:
            ph = np.exp(2j * np.pi * (tau @ g))                  # [n_orb]
            phs = np.broadcast_to(ph, (npairs, ph.shape[0]))
            mk = _pair_density(Ac, Av, phs)                      # M_cv(k,k;G)  [p, c, v]
            mkp = _pair_density(Bc, Bv, phs)                     # M_c'v'(k',k';G)
            vg = 4.0 * np.pi / (TWO_PI * TWO_PI * g2)
            # X[p, v, c, v', c'] += v(G) M_cv(k,k;G) conj(M_c'v'(k',k';G))
            X += vg * (mk.transpose(0, 2, 1)[:, :, :, None, None]
                       * mkp.conj().transpose(0, 2, 1)[:, None, None, :, :])
        # direct: momentum transfer q + G
        Q = q + g
        wq = w_model(Q, eps_inf, lam)
        if g2 == 0.0:
            wq = np.where(same, wq0, wq)
        ph = np.exp(2j * np.pi * (Q @ tau.T))                    # [p, n_orb]
        mcc = _pair_density(Ac, Bc, ph)                          # M_cc'(k,k';Q)  [p, c, c']
        mvv = _pair_density(Av, Bv, ph)                          # M_vv'(k,k';Q)  [p, v, v']
        # D[p, v, c, v', c'] += W(q+G) M_cc'(k,k';q+G) conj(M_vv'(k,k';q+G))
        D += wq[:, None, None, None, None] * (mcc[:, None, :, None, :]
                                              * mvv.conj()[:, :, None, :, None])
    return (kernel_energy / nkd) * (2.0 * X - D)


def _params(cfg_like):
    return dict(eps_inf=cfg_like.eps_inf, lam=cfg_like.lam, g2_max=cfg_like.g2_max,
                kernel_energy=cfg_like.kernel_energy, q0_quad=cfg_like.q0_quad)


def coarse_kernel(vecs_coarse: np.ndarray, tau: np.ndarray, nv: int, nc: int, n_c: int,
                  n_div: int, cfg_like, chunk: int = 4096) -> np.ndarray:
    """Full Hermitian K_c [N_coarse, N_coarse] (complex128).

    cfg_like supplies eps_inf, lam, g2_max, kernel_energy and q0_quad.
    """
    prm = _params(cfg_like)
    return _assemble_hermitian(
        lambda ks, kps: _direct_formula_blocks(vecs_coarse, tau, nv, nc, n_c, n_div, ks, kps, **prm),
        n_c ** 3, nv * nc, chunk)


def _assemble_hermitian(blocks, nk: int, npair: int, chunk: int) -> np.ndarray:
    """[nk npair, nk npair] matrix from blocks(ks, kps) evaluated for k <= k': the block
    (k', k) is the conjugate transpose of (k, k'), diagonal blocks are (A + A^H) / 2."""
    iu, ju = np.triu_indices(nk)
    K = np.zeros((nk, npair, nk, npair), dtype=np.complex128)
    for s in range(0, iu.shape[0], chunk):
        ks, kps = iu[s:s + chunk], ju[s:s + chunk]
        blk = blocks(ks, kps).reshape(-1, npair, npair)
        diag = ks == kps
        blk[diag] = 0.5 * (blk[diag] + blk[diag].conj().transpose(0, 2, 1))
        K[ks, :, kps, :] = blk
        off = ~diag
        K[kps[off], :, ks[off], :] = blk[off].conj().transpose(0, 2, 1)
    return K.reshape(nk * npair, nk * npair)


# ---- Eq. (diverg): the divergent part of the kernel ----------------------------------
def screening_kappa2(eps_inf: float, lam: float) -> float:
    """kappa^2 of s(q) = 1 / (|q|^2 + kappa^2), W(q) = s(q) / (pi eps_inf), q reduced."""
    return lam * lam / (4.0 * np.pi * np.pi * eps_inf)


def s_shape(q: np.ndarray, kappa2: float) -> np.ndarray:
    """s(q) = 1 / (|q|^2 + kappa^2) for reduced q[..., 3]."""
    q = np.asarray(q, dtype=np.float64)
    return 1.0 / (np.sum(q * q, axis=-1) + kappa2)


def s_q0_average(n_c: int, n_div: int, kappa2: float, n_quad: int = 16) -> float:
    """Mean of s(q) over the dense mini-cell q in [-1/2, 1/2)^3 / (n_c n_div), midpoint rule."""
    t = ((np.arange(n_quad) + 0.5) / n_quad - 0.5) / (n_c * n_div)
    q = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    return float(np.mean(s_shape(q, kappa2)))


def coarse_shape(n_c: int, kappa2: float, s0: float) -> np.ndarray:
    """S_c[k~, k~'] = s(q) with q = k~ - k~' folded (reduced), and s0 at q = 0."""
    ijk = cell_coords(n_c)
    q = fold_int(ijk[:, None, :] - ijk[None, :, :], n_c).astype(np.float64) / n_c
    S = s_shape(q, kappa2)
    np.fill_diagonal(S, s0)
    return S


def _divergence_blocks(vecs_coarse, tau, nv, nc, n_c, n_div, ks, kps, *, eps_inf, kernel_energy):
    """Unsymmetrised blocks a[p, v, c, v', c'] of the coefficient of s(q) for pairs (ks[p], kps[p])."""
    ks = np.asarray(ks)
    kps = np.asarray(kps)
    nkd = n_c ** 3 * n_div ** 3
    ijk = cell_coords(n_c)
    q = fold_int(ijk[ks] - ijk[kps], n_c).astype(np.float64) / n_c
    A = vecs_coarse[ks]
    B = vecs_coarse[kps]
    ph = np.exp(2j * np.pi * (q @ tau.T))
    mcc = _pair_density(A[:, nv:nv + nc], B[:, nv:nv + nc], ph)      # M_cc'(k,k';q)
    mvv = _pair_density(A[:, :nv], B[:, :nv], ph)                    # M_vv'(k,k';q)
    coef = -(kernel_energy / nkd) / (np.pi * eps_inf)
    return coef * (mcc[:, None, :, None, :] * mvv.conj()[:, :, None, :, None])


def divergence_coefficient(vecs_coarse: np.ndarray, tau: np.ndarray, nv: int, nc: int, n_c: int,
                           n_div: int, cfg_like, chunk: int = 4096) -> np.ndarray:
    """a_c [N_coarse, N_coarse] of Eq. (diverg) for the model kernel (see the module
    notes): the G = 0 direct term of K_c equals a_c s(q); Hermitian by the same
    construction as K_c."""
    prm = dict(eps_inf=cfg_like.eps_inf, kernel_energy=cfg_like.kernel_energy)
    return _assemble_hermitian(
        lambda ks, kps: _divergence_blocks(vecs_coarse, tau, nv, nc, n_c, n_div, ks, kps, **prm),
        n_c ** 3, nv * nc, chunk)


def coarse_kernel_block_rows(vecs_coarse: np.ndarray, tau: np.ndarray, nv: int, nc: int,
                             n_c: int, n_div: int, cfg_like, rows_k: np.ndarray) -> np.ndarray:
    """Rows of K_c for the coarse points rows_k: [len(rows_k), npair, N_coarse].

    Same values as coarse_kernel(...) restricted to those block rows; used to
    check large meshes where the full matrix is too costly for the oracle.
    """
    nk = n_c ** 3
    npair = nv * nc
    prm = _params(cfg_like)
    out = np.zeros((len(rows_k), npair, nk, npair), dtype=np.complex128)
    kp_all = np.arange(nk)
    for i, k in enumerate(rows_k):
        up = kp_all[kp_all >= k]
        lo = kp_all[kp_all < k]
        blk = _direct_formula_blocks(vecs_coarse, tau, nv, nc, n_c, n_div,
                                     np.full(up.shape, k), up, **prm).reshape(-1, npair, npair)
        blk[0] = 0.5 * (blk[0] + blk[0].conj().T)        # up[0] == k
        out[i, :, up, :] = blk
        if lo.size:
            blo = _direct_formula_blocks(vecs_coarse, tau, nv, nc, n_c, n_div,
                                         lo, np.full(lo.shape, k), **prm).reshape(-1, npair, npair)
            out[i, :, lo, :] = blo.conj().transpose(0, 2, 1)
    return out.reshape(len(rows_k), npair, nk * npair)
