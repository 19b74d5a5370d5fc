"""Sampled-output checks of a full-size matvec against the oracle.

At the larger meshes the oracle cannot form the whole coarse kernel in seconds, so
the check takes a few cells: the oracle computes the K_c block rows of their corners
one by one and the restriction of the whole input vector, and every dense output of
those cells is compared with the library's, componentwise against the sum of
|terms| of its product and in relative L2.
"""

from __future__ import annotations

import numpy as np

import oracle as O
import tbinputs as ti

from _cases import rel_l2


def oracle_pieces(cfg, bs):
    """(Dv, Dc, delta) of the oracle for cfg."""
    Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    delta = O.transition_energies(bs.eps_dense, cfg.nv, cfg.nc)
    return Dv, Dc, delta


def check_sampled_cells(cfg, bs, prob, pieces, cells, seed, unit, factors, rel, n_rhs=3):
    """y = H^i x of `prob` on the dense points of `cells` against the oracle, within
    `factors` units `unit` of the sum of |terms| of each output (or (diagonal, kernel)
    units for the two kinds of terms), and `rel` in relative L2."""
    Dv, Dc, delta = pieces
    f = O.trilinear_weights(cfg.n_div)
    x = prob.vector(ti.random_vectors(cfg.n_trans, n_rhs, seed))
    y = prob.matvec(x).cpu().numpy().astype(complex)
    xh = x.cpu().numpy().astype(complex)
    nbr = O.neighbour_table(cfg.n_coarse)
    need = np.unique(nbr[np.asarray(cells)].ravel())
    rows = O.coarse_kernel_block_rows(bs.vecs_coarse, bs.tau, cfg.nv, cfg.nc, cfg.n_coarse, cfg.n_div, cfg, need)
    np_ = cfg.n_pair
    op = O.InterpOperator(Dv, Dc, f, None, delta, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    aop = O.InterpOperator(np.abs(Dv).astype(complex), np.abs(Dc).astype(complex), f, None, np.abs(delta),
                           cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    qbar = op.restrict(xh)
    qabs = aop.restrict(np.abs(xh))
    r = np.zeros((n_rhs, cfg.n_trans_coarse), dtype=complex)
    rabs = np.zeros((n_rhs, cfg.n_trans_coarse), dtype=complex)
    for i, k in enumerate(need):
        r[:, k * np_:(k + 1) * np_] = (rows[i] @ qbar.T).T
        rabs[:, k * np_:(k + 1) * np_] = (np.abs(rows[i]) @ np.abs(qabs).T).T
    ref = delta[None] * xh + op.prolong(r)
    fd, fk = factors if isinstance(factors, tuple) else (factors, factors)
    bound = unit * (fd * np.abs(delta)[None] * np.abs(xh) + fk * np.abs(aop.prolong(rabs)))
    ndiv3 = cfg.n_div3
    for cell in cells:
        sl = slice(cell * ndiv3 * np_, (cell + 1) * ndiv3 * np_)
        assert np.all(np.abs(y[:, sl] - ref[:, sl]) <= bound[:, sl]), f"cell {cell}"
        assert rel_l2(y[:, sl], ref[:, sl]) < rel
