"""Pins for the oracle's meshes, neighbourhoods and prefactors (Sec. 3)."""

import os

import numpy as np
import pytest

import oracle as O
import tbinputs as ti

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_trilinear_table_matches_hand_derived_ndiv2():
    ref = np.loadtxt(os.path.join(GOLDEN, "trilinear_ndiv2.txt"))
    assert np.array_equal(O.trilinear_weights(2), ref)


@pytest.mark.parametrize("n_div", [1, 2, 3, 4, 5])
def test_trilinear_partition_of_unity_and_origin(n_div):
    f = O.trilinear_weights(n_div)
    assert f.shape == (n_div ** 3, 8)
    assert np.all(f >= 0)
    np.testing.assert_allclose(f.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    e0 = np.zeros(8)
    e0[0] = 1.0
    assert np.array_equal(f[0], e0)          # j = 0: the point is the coarse corner itself


@pytest.mark.parametrize("n_div", [2, 3, 4])
def test_trilinear_reproduces_affine_functions(n_div):
    """Trilinear interpolation is exact for g(x) = alpha.x + beta on a cell."""
    rng = np.random.default_rng(5)
    alpha, beta = rng.normal(size=3), rng.normal()
    f = O.trilinear_weights(n_div)
    corners = O.corner_offsets().astype(float)           # corner positions in the unit cell
    j = np.stack(np.meshgrid(*[np.arange(n_div)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pts = j / n_div
    interp = f @ (corners @ alpha + beta)
    np.testing.assert_allclose(interp, pts @ alpha + beta, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n_div", [1, 2, 3, 4, 5])
def test_nearest_corner_is_one_hot_and_nearest(n_div):
    f = O.nearest_corner_weights(n_div)
    assert np.all(f.sum(axis=1) == 1.0)
    assert np.all((f == 0) | (f == 1))
    corners = O.corner_offsets().astype(float)
    j = np.stack(np.meshgrid(*[np.arange(n_div)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pts = j / n_div
    dist = np.linalg.norm(pts[:, None, :] - corners[None], axis=-1)
    chosen = np.argmax(f, axis=1)
    assert np.all(dist[np.arange(len(pts)), chosen] <= dist.min(axis=1) + 1e-15)


@pytest.mark.parametrize("n_c", [1, 2, 3, 4, 5])
def test_neighbour_table_counts_and_offsets(n_c):
    nbr = O.neighbour_table(n_c)
    # every coarse point is the corner z of exactly one cell, for each z
    for z in range(8):
        assert sorted(nbr[:, z].tolist()) == list(range(n_c ** 3))
    counts = np.bincount(nbr.ravel(), minlength=n_c ** 3)
    assert np.all(counts == 8)
    # corner z of cell (i1,i2,i3) sits at (i1+l, i2+m, i3+n) mod n_c
    i = np.arange(n_c)
    ijk = np.stack(np.meshgrid(i, i, i, indexing="ij"), -1).reshape(-1, 3)
    for z, off in enumerate(O.corner_offsets()):
        c = ijk[nbr[:, z]]
        assert np.all((c - ijk - off) % n_c == 0)


@pytest.mark.parametrize("n_c,n_div", [(2, 2), (3, 2), (4, 3)])
def test_dense_index_map_agrees_with_input_generator(n_c, n_div):
    np.testing.assert_array_equal(O.dense_index_map(n_c, n_div), ti.dense_kpoints(n_c, n_div))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8])
def test_fold_range_and_antisymmetry(n):
    d = np.arange(-3 * n, 3 * n)
    q = O.fold_int(d, n)
    assert np.all(q >= -(n // 2)) and np.all(q < n - n // 2)
    assert np.all((q - d) % n == 0)
    mq = O.fold_int(-d, n)
    tie = (2 * q == -n)                      # only the half-way point breaks q(-d) = -q(d)
    assert np.all((mq == -q) | tie)
