"""Host-side checks of the batching workload's definition (no GPU)."""

import numpy as np

import tbinputs as ti


def test_batch_has_48_uneven_members():
    b = ti.batch_configs()
    assert len(b) == 48 and len({c.name for c in b}) == 48
    shapes = {(c.n_coarse, c.n_div, c.nc) for c in b}
    assert shapes == {(g, d, nc) for g, d in ti.configs.BATCH_GRIDS for nc in (3, 6)}
    sizes = sorted({c.n_coarse ** 3 * c.n_div ** 3 * c.nv * c.nc for c in b})
    assert sizes[0] == 4608 and sizes[-1] == 589824          # 4^3 x 2 3v3c ... 8^3 x 4 3v6c
    assert all(c.n_pol == 3 and c.steps == 200 and c.n_orb == 9 for c in b)


def test_displacements_come_in_plus_minus_pairs():
    b = ti.batch_configs()
    for c in b:
        delta, dseed = c.perturb
        assert abs(abs(delta) - 0.01) < 1e-15
        partner = [o for o in b if o.perturb == (-delta, dseed) and o.n_coarse == c.n_coarse]
        assert len(partner) == 1


def test_displacement_moves_the_bands_linearly():
    """+delta and -delta shift the band energies by opposite first-order amounts."""
    c = [x for x in ti.batch_configs() if x.n_coarse == 4][0]
    base = c.with_(perturb=None)
    e0 = ti.band_structure(base).eps_dense
    ep = ti.band_structure(c.with_(nc=3)).eps_dense
    em = ti.band_structure(c.with_(nc=3, perturb=(-c.perturb[0], c.perturb[1]))).eps_dense
    d1, d2 = ep - e0, em - e0
    assert np.abs(d1).max() > 1e-4
    # the odd (first-order) part dominates the even (second-order) part
    assert np.linalg.norm(d1 + d2) < 0.2 * np.linalg.norm(d1 - d2)
