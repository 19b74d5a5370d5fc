"""Batching form on the GPU: many chains of uneven Hamiltonians recorded into one
HIP graph (bse_batch_*), and the autotuner of the plan tunables."""

from __future__ import annotations

import numpy as np
import pytest

import tbinputs as ti

from _cases import bands, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MEMBERS = [
    (ti.get_config("c0"), "f64"),
    (ti.tiny_config(n_coarse=3, n_div=3, nv=3, nc=6, n_orb=9, seed=11, n_pol=3), "f32"),
    (ti.tiny_config(n_coarse=2, n_div=4, nv=4, nc=6, n_orb=10, seed=14, n_pol=2), "bf16"),
    (ti.tiny_config(n_coarse=2, n_div=5, nv=2, nc=3, n_orb=5, seed=12, n_pol=4), "f32v64"),
    (ti.tiny_config(n_coarse=4, n_div=2, nv=3, nc=3, n_orb=9, seed=3, n_pol=3, perturb=(0.01, 1000)), "f32"),
]


@pytest.fixture(scope="module")
def bse():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_01863_amd import bse as mod
    return mod


def _host(ch):
    return {k: v.cpu().numpy().copy() for k, v in ch.items()}


def test_batch_graph_matches_eager_chains(bse):
    """Every replay of the graph gives the eager chains bit for bit, with eager work
    on the same plans between the replays."""
    steps = 30
    probs = [bse.problem_from_bands(bands(c), c, dtype=dt, max_rhs=c.n_pol) for c, dt in MEMBERS]
    Ps = [bands(c).P_flat() for c, _ in MEMBERS]
    eager = [_host(p.haydock(P, steps)) for p, P in zip(probs, Ps)]
    batch = bse.BSEBatch(probs, Ps, steps, n_branches=3)
    rng = np.random.default_rng(5)
    for rep in range(3):
        chains = batch.run()
        torch.cuda.synchronize()
        for i, (ch, ref) in enumerate(zip(chains, eager)):
            got = _host(ch)
            for k in ("a", "b", "pnorm2", "steps", "status"):
                assert np.array_equal(got[k], ref[k]), (rep, i, k)
        # eager work on the plans between replays (overwrites their workspaces)
        for p in probs[:2]:
            x = rng.standard_normal((1, p.N)) + 1j * rng.standard_normal((1, p.N))
            p.matvec(p.vector(x))
        torch.cuda.synchronize()
    batch.close()
    for p in probs:
        p.close()


def test_batch_rejects_a_plan_twice(bse):
    c, dt = MEMBERS[1]
    p = bse.problem_from_bands(bands(c), c, dtype=dt, max_rhs=c.n_pol)
    P = bands(c).P_flat()
    with pytest.raises(bse.BSEError):
        bse.BSEBatch([p, p], [P, P], 5)
    p.close()


def test_autotune_picks_a_setting_and_keeps_results(bse, tmp_path):
    from paper_1602_01863_amd.autotune import autotune
    c = MEMBERS[1][0]
    p = bse.problem_from_bands(bands(c), c, dtype="f32", max_rhs=3)
    P = bands(c).P_flat()
    ref = _host(p.haydock(P, 20))
    cache = str(tmp_path / "tuning.json")
    res = autotune(p, P, steps=4, repeats=1, splits=(0, 4, 16), cache=cache)
    assert res["group"] in (1, 3) and res["splits"] in (0, 4, 16) and not res["cached"]
    assert len(res["trials"]) == 6 and res["ms_per_step"] > 0
    got = _host(p.haydock(P, 20))
    assert rel_l2(got["a"][:, :12], ref["a"][:, :12]) < 1e-6
    again = autotune(p, P, cache=cache)
    assert again["cached"] and (again["splits"], again["group"]) == (res["splits"], res["group"])
    p.close()
