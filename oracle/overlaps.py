"""Wavefunction overlaps between dense points and their coarse neighbours.

Eq. (completeness): u_{nk} = sum_{n'} d_{nk}^{n'k~} u_{n'k~} with
d_{nk}^{n'k~} = <u_{n'k~} | u_{nk}>.  Only the valence-valence and
conduction-conduction blocks enter the pair expansion (Eq. expansion); the
valence/conduction mixing is dropped, as the paper does in Sec. 5.
"""

from __future__ import annotations

import numpy as np

from .grids import neighbour_table


def overlaps(vecs_coarse: np.ndarray, vecs_dense: np.ndarray, n_c: int, n_div: int,
             nv: int, nc: int):
    """Return (Dv, Dc).

    vecs_*[k, n, a] = coefficient a of band n at point k (orbital basis).
    Dv[kd, z, v, n1] = <u_{n1, k~z} | u_{v, kd}>            v, n1 < nv
    Dc[kd, z, c, n2] = <u_{nv+n2, k~z} | u_{nv+c, kd}>      c, n2 < nc
    where k~z is corner z of the cell holding kd.
    """
    ndiv3 = n_div ** 3
    nkd = vecs_dense.shape[0]
    nbr = neighbour_table(n_c)
    cell = np.arange(nkd) // ndiv3
    Dv = np.empty((nkd, 8, nv, nv), dtype=np.complex128)
    Dc = np.empty((nkd, 8, nc, nc), dtype=np.complex128)
    for z in range(8):
        kc = nbr[cell, z]
        cv = vecs_coarse[kc]          # [nkd, nb, n_orb]
        # <u_{n' k~}|u_{n k}> = sum_a conj(c_{n' k~, a}) c_{n k, a}
        ov = np.einsum("kpa,kna->knp", cv.conj(), vecs_dense)   # [kd, n, n']
        Dv[:, z] = ov[:, :nv, :nv]
        Dc[:, z] = ov[:, nv:nv + nc, nv:nv + nc]
    return Dv, Dc
