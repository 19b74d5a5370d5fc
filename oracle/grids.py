"""Meshes, neighbourhoods and interpolation prefactors (Sec. 3).

Coarse point k~_(i1,i2,i3) and dense point k_(i,j) = (i + j/n_div)/n_c in
reduced coordinates.  Index conventions used throughout:

* coarse / cell index   cell = (i1*n_c + i2)*n_c + i3
* subpoint index        sub  = (j1*n_div + j2)*n_div + j3
* dense index           kd   = cell * n_div^3 + sub
* corner index          z    = 4*l + 2*m + n for the neighbour k~^{lmn}

The neighbourhood N(k) of Eq. (neighborhood) is the set of the 8 corners
k~_(i1+l, i2+m, i3+n) of the cell that holds k.  The paper gives no rule for
indices past the last coarse point; they wrap periodically (the crystal is
periodic in k).
"""

from __future__ import annotations

import numpy as np


def corner_offsets() -> np.ndarray:
    """[8, 3] offsets (l, m, n) of corner z = 4l + 2m + n."""
    z = np.arange(8)
    return np.stack([(z >> 2) & 1, (z >> 1) & 1, z & 1], axis=1)


def cell_coords(n_c: int) -> np.ndarray:
    """[n_c^3, 3] integer coordinates (i1, i2, i3) of each coarse point."""
    i = np.arange(n_c)
    return np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1).reshape(-1, 3)


def neighbour_table(n_c: int) -> np.ndarray:
    """[n_c^3, 8]: coarse index of corner z of each cell, Eq. (neighborhood)."""
    ijk = cell_coords(n_c)
    out = np.empty((n_c ** 3, 8), dtype=np.int64)
    for z, (l, m, n) in enumerate(corner_offsets()):
        c = (ijk + np.array([l, m, n])) % n_c
        out[:, z] = (c[:, 0] * n_c + c[:, 1]) * n_c + c[:, 2]
    return out


def _axis_weights(n_div: int) -> np.ndarray:
    """[n_div, 2]: f^l_j, l = 0, 1 (1 - j/n and j/n)."""
    j = np.arange(n_div, dtype=np.float64)
    return np.stack([1.0 - j / n_div, j / n_div], axis=1)


def trilinear_weights(n_div: int) -> np.ndarray:
    """[n_div^3, 8]: f^{lmn}(sub) = f^l_{j1} f^m_{j2} f^n_{j3} (Sec. 3)."""
    w = _axis_weights(n_div)
    f = np.empty((n_div ** 3, 8))
    for j1 in range(n_div):
        for j2 in range(n_div):
            for j3 in range(n_div):
                sub = (j1 * n_div + j2) * n_div + j3
                for z, (l, m, n) in enumerate(corner_offsets()):
                    f[sub, z] = w[j1, l] * w[j2, m] * w[j3, n]
    return f


def nearest_corner_weights(n_div: int) -> np.ndarray:
    """[n_div^3, 8]: one-hot prefactor of the one-neighbour scheme (Eq. eqRL).

    The paper sets f = 1 for "a chosen neighbour".  The chosen one here is the
    nearest corner; on each axis j/n_div <= 1/2 picks l = 0, else l = 1.
    """
    f = np.zeros((n_div ** 3, 8))
    for j1 in range(n_div):
        for j2 in range(n_div):
            for j3 in range(n_div):
                sub = (j1 * n_div + j2) * n_div + j3
                l, m, n = (int(2 * j > n_div) for j in (j1, j2, j3))
                f[sub, 4 * l + 2 * m + n] = 1.0
    return f


def dense_index_map(n_c: int, n_div: int) -> np.ndarray:
    """[n_c^3 n_div^3, 3] reduced coordinates of dense point kd (Sec. 3)."""
    out = np.empty((n_c ** 3 * n_div ** 3, 3))
    ijk = cell_coords(n_c)
    jjj = cell_coords(n_div)
    for cell in range(n_c ** 3):
        for sub in range(n_div ** 3):
            out[cell * n_div ** 3 + sub] = (ijk[cell] + jjj[sub] / n_div) / n_c
    return out


def fold_int(d: np.ndarray, n: int) -> np.ndarray:
    """Fold integer differences d (in units of 1/n) into [-n//2, n - n//2).

    For even n the half-way point maps to -n/2, i.e. q = -1/2.
    """
    h = n // 2
    return np.mod(d + h, n) - h
