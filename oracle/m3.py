"""Method 3 of Sec. 4: the divergence treated in a band along the diagonal.

TEST INFRASTRUCTURE: only the tests, the smoke check of the entry module and the
CPU-baseline leg of the benchmark use this module.

Sec. 4 (the width paragraph and the band figure): pairs of dense points with
||k - k'|| > w d are interpolated as in Method 1 (Eq. interp1 applied to K_c);
for the pairs with ||k - k'|| <= w d, the coefficients of Eq. (diverg) are
interpolated with the same scheme and combined with the dense-mesh q.  With the
model's split K_c = a_c s(q) + c_c (see ``kernel``):

    K^{M3}(k, k') = a^i(k, k') s(q_dense) + c^i(k, k')      inside the band
    K^{M3}(k, k') = K^i(k, k')                               outside,

where X^i is Eq. (interp1) applied to X and s(q_dense) is s at the folded
dense difference q = k - k' (the mini-cell mean at q = 0).  d is the smallest
distance between two coarse points, 1 / n_c in reduced units, and distances
are taken between periodic images (the minimum image).

Because Eq. (interp1) is linear, K^{M3} = K^i + Delta inside the band with

    Delta(k, k') = sum_{z z'} f(k,z) f(k',z') [s(q_dense) - S_c(k~z, k~'z')]
                   L_{kz} a_c(k~z, k~'z') L_{k'z'}^H,
    L_{kz}[(v c), (n1 n2)] = d_{vk}^{n1 k~z} conj(d_{ck}^{n2 k~z}),

so the band is a sparse correction added to the on-the-fly product: for every
dense k and every offset o of the band, one block Delta(k, k + o) (Table
tab:scalings: O(N~_k N_div^2) extra work for a sparse implementation).

Band offsets: integer offsets o of the dense mesh with |o|^2 <= (w n_div)^2
(||o|| / (n_c n_div) <= w / n_c), in lexicographic order of (o1, o2, o3).  The
band must not reach round the periodic mesh: 2 floor(w n_div) < n_c n_div.
"""

from __future__ import annotations

import math

import numpy as np

from .grids import cell_coords, fold_int
from .kernel import s_shape


def band_offsets(n_div: int, w: float) -> np.ndarray:
    """[n_off, 3] integer offsets o with |o|^2 <= (w n_div)^2, lexicographic."""
    R2 = (w * n_div) ** 2
    r = int(math.floor(w * n_div + 1e-9))
    out = []
    for a in range(-r, r + 1):
        for b in range(-r, r + 1):
            for c in range(-r, r + 1):
                if a * a + b * b + c * c <= R2 * (1.0 + 1e-12) + 1e-12:
                    out.append((a, b, c))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def dense_coords(n_c: int, n_div: int) -> np.ndarray:
    """[N_k, 3] integer dense coordinates i n_div + j of dense point kd (cell-major)."""
    ijk = cell_coords(n_c)
    jjj = cell_coords(n_div)
    kd = np.arange(n_c ** 3 * n_div ** 3)
    return ijk[kd // n_div ** 3] * n_div + jjj[kd % n_div ** 3]


def dense_index(coords: np.ndarray, n_c: int, n_div: int) -> np.ndarray:
    """Cell-major dense index of integer dense coordinates (wrapped periodically)."""
    n = n_c * n_div
    c = np.mod(coords, n)
    cell = ((c[..., 0] // n_div) * n_c + c[..., 1] // n_div) * n_c + c[..., 2] // n_div
    sub = ((c[..., 0] % n_div) * n_div + c[..., 1] % n_div) * n_div + c[..., 2] % n_div
    return cell * n_div ** 3 + sub


def band_neighbours(n_c: int, n_div: int, offsets: np.ndarray) -> np.ndarray:
    """[N_k, n_off]: dense index of k + o."""
    return dense_index(dense_coords(n_c, n_div)[:, None, :] + offsets[None, :, :], n_c, n_div)


def dense_shape(offsets: np.ndarray, n_c: int, n_div: int, kappa2: float, s0: float) -> np.ndarray:
    """s(q_dense) per offset, q = o / (n_c n_div); s0 (the mini-cell mean) at o = 0."""
    q = np.asarray(offsets, dtype=np.float64) / (n_c * n_div)
    s = s_shape(q, kappa2)
    s[~np.asarray(offsets).any(axis=1)] = s0
    return s


def explicit_kernel(op, a_c: np.ndarray, S_c: np.ndarray, w: float, kappa2: float, s0: float) -> np.ndarray:
    """K^{M3} [N, N] written out as defined (small meshes only): interpolate a_c and
    c_c = K_c - a_c S_c with Eq. (interp1); inside the band a^i s(q_dense) + c^i,
    outside the Method 1 kernel K^i."""
    npair = op.nv * op.nc
    E = op.expansion_matrix()
    K1 = E @ op.Kc @ E.conj().T
    Sc_full = np.kron(S_c, np.ones((npair, npair)))
    a_i = E @ a_c @ E.conj().T
    c_i = E @ (op.Kc - a_c * Sc_full) @ E.conj().T
    # folded dense differences and the band between every pair of dense points
    x = dense_coords(op.n_c, op.n_div)
    n = op.n_c * op.n_div
    o = fold_int(x[:, None, :] - x[None, :, :], n)
    in_band = np.sum(o * o, axis=-1) <= (w * op.n_div) ** 2 * (1.0 + 1e-12) + 1e-12
    s_d = s_shape(o.astype(np.float64) / n, kappa2)
    s_d[~o.any(axis=-1)] = s0
    one = np.ones((npair, npair))
    band = np.kron(in_band, one).astype(bool)
    return np.where(band, a_i * np.kron(s_d, one) + c_i, K1)


def band_blocks(op, a_c: np.ndarray, S_c: np.ndarray, offsets: np.ndarray, s_d: np.ndarray,
                ks=None, absolute: bool = False) -> np.ndarray:
    """Delta(k, k + o) [len(ks), n_off, npair, npair] from its definition (module notes).

    absolute=True takes the modulus of the scalar weights as well (with op and a_c
    given as moduli, the result bounds the sum of |terms| of each entry)."""
    nv, nc = op.nv, op.nc
    npair = nv * nc
    ks = np.arange(op.nk) if ks is None else np.asarray(ks)
    nbr = band_neighbours(op.n_c, op.n_div, offsets)
    ablk = a_c.reshape(op.nkc, npair, op.nkc, npair)
    # L[k, z][(v c), (n1 n2)] = d_v^{n1} conj(d_c^{n2})
    def L(k):
        return np.einsum("zab,zcd->zacbd", op.Dv[k], np.conj(op.Dc[k])).reshape(8, npair, npair)
    out = np.zeros((len(ks), len(offsets), npair, npair), dtype=np.complex128)
    for i, k in enumerate(ks):
        Lk = L(k)
        ck = op.corner_k[k]
        for j in range(len(offsets)):
            kp = nbr[k, j]
            Lp = L(kp)
            cp = op.corner_k[kp]
            g = op.fk[k][:, None] * op.fk[kp][None, :] * (s_d[j] - S_c[ck[:, None], cp[None, :]])
            if absolute:
                g = np.abs(g)
            blk = np.zeros((npair, npair), dtype=np.complex128)
            for z in range(8):
                for zp in range(8):
                    if g[z, zp] != 0.0:
                        blk += g[z, zp] * (Lk[z] @ ablk[ck[z], :, cp[zp], :] @ Lp[zp].conj().T)
            out[i, j] = blk
    return out


def band_product(blocks: np.ndarray, offsets: np.ndarray, x: np.ndarray, n_c: int, n_div: int,
                 ks=None) -> np.ndarray:
    """y_k = sum_o Delta(k, k + o) x_{k+o} for the dense points ks (all by default);
    blocks [len(ks), n_off, npair, npair], x [n_rhs, N] -> y [n_rhs, len(ks), npair]."""
    x = np.atleast_2d(x)
    npair = blocks.shape[-1]
    nk = n_c ** 3 * n_div ** 3
    ks = np.arange(nk) if ks is None else np.asarray(ks)
    nbr = band_neighbours(n_c, n_div, offsets)[ks]
    xb = x.reshape(x.shape[0], nk, npair)
    return np.einsum("kopq,rkoq->rkp", blocks, xb[:, nbr, :])


def apply(op, blocks: np.ndarray, offsets: np.ndarray, x: np.ndarray) -> np.ndarray:
    """H^{M3} x = H^i x + sum_o Delta(k, k + o) x_{k+o} (blocks for every dense k)."""
    x = np.atleast_2d(x)
    y = band_product(blocks, offsets, x, op.n_c, op.n_div)
    return op.apply(x) + y.reshape(x.shape[0], -1)
