"""Batching form on the GPU: many chains of uneven Hamiltonians recorded into one
HIP graph (bse_batch_*), and the autotuner of the plan tunables."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import tbinputs as ti

from _cases import bands, oracle_operator, oracle_parts, rel_l2
from _gpu import U32, fp32_kernel_factors
from _sampled import check_sampled_cells, oracle_pieces

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MEMBERS = [
    (ti.get_config("c0"), "f64"),
    (ti.tiny_config(n_coarse=3, n_div=3, nv=3, nc=6, n_orb=9, seed=11, n_pol=3), "f32"),
    (ti.tiny_config(n_coarse=2, n_div=4, nv=4, nc=6, n_orb=10, seed=14, n_pol=2), "bf16"),
    (ti.tiny_config(n_coarse=2, n_div=5, nv=2, nc=3, n_orb=5, seed=12, n_pol=4), "f32v64"),
    (ti.tiny_config(n_coarse=4, n_div=2, nv=3, nc=3, n_orb=9, seed=3, n_pol=3, perturb=(0.01, 1000)), "f32"),
    # a band pair without a compiled form: the run-time restrict and prolong in the graphs
    (ti.tiny_config(n_coarse=3, n_div=2, nv=2, nc=5, n_orb=7, seed=21, n_pol=3), "f32"),
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


def _window(ref, other, tol):
    """Leading coefficients where `other` agrees with `ref` to tol (relative), min over chains."""
    out = []
    for key, lo in (("a", 0), ("b", 1)):
        x, y = other[key][:, lo:], ref[key][:, lo:]
        bad = np.abs(x - y) > tol * np.abs(y)
        out += [int(np.argmax(row)) if row.any() else row.size for row in bad]
    return min(out)


def _fp32_storage(cfg):
    """The oracle's operator with its overlaps and K_c rounded to complex64 (the storage
    of the FP32 forms), still applied in FP64."""
    bs, Dv, Dc, f, Kc, delta = oracle_parts(cfg)
    c64 = lambda a: a.astype(np.complex64).astype(np.complex128)
    return O.InterpOperator(c64(Dv), c64(Dc), f, c64(Kc), delta, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)


def test_batch_chains_match_the_oracle(bse):
    """Every member's batched chains (Eqs. ai-ci; 200 steps, the batching workload's
    length) against the oracle's FP64 chains of the same Hamiltonian: the ±delta
    displaced member, the FP32-vector and FP64-vector members and the BF16 member.

    * head: the oracle against its own rounding-perturbed run (the FP64 member against
      a one-ulp change of the diagonal; the FP32 members with their overlaps and K_c
      rounded to complex64, and the vectors too where they are stored in FP32) stays at
      the rounding floor and then departs, growing 17-50x per step, once converged
      states re-enter.  Two steps before the emulated departure the batched
      coefficients agree with the oracle to 1e-10 (FP64) or, for the FP32 forms, 1e-5:
      their FP32 arithmetic (restrict, prolong, packed coarse product) perturbs each
      matvec by up to 115 FP32 units of the sum of |terms| of its kernel part, a few
      times the storage rounding (about 3e-6 of a_1 here); that window must hold at
      least 10 coefficients.  The BF16 member: a_1 within the
      format bound 2^-8 <|qbar_1|, |K_c| |qbar_1|> (K_c entries rounded to 8 significant
      bits, block scales are powers of two).
    * eps2 at eta = 0.5 eV, where 200 steps have converged (the oracle's FP32-storage
      emulation moves it by < 1e-7 there): 1e-10 (FP64), 1e-6 (FP32 storage), 1e-3
      (BF16 coarse kernel)."""
    steps = 200
    probs = [bse.problem_from_bands(bands(c), c, dtype=dt, max_rhs=c.n_pol) for c, dt in MEMBERS]
    Ps = [bands(c).P_flat() for c, _ in MEMBERS]
    batch = bse.BSEBatch(probs, Ps, steps, n_branches=3)
    chains = [_host(ch) for ch in batch.run()]
    torch.cuda.synchronize()
    om = np.linspace(0.0, 16.0, 800)
    for (cfg, dt), got, P in zip(MEMBERS, chains, Ps):
        assert np.all(got["status"] == bse.BSE_OK) and np.all(got["steps"] == steps), cfg.name
        op = oracle_operator(cfg)
        ref = O.haydock(op.apply, P, steps)
        np.testing.assert_allclose(got["pnorm2"], ref["pnorm2"], rtol=1e-12)
        if dt == "bf16":
            bs, Dv, Dc, f, Kc, delta = oracle_parts(cfg)
            psi = P / np.sqrt(ref["pnorm2"])[:, None]
            aop = O.InterpOperator(np.abs(Dv).astype(complex), np.abs(Dc).astype(complex), f,
                                   np.abs(Kc).astype(complex), delta, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
            qa = aop.restrict(np.abs(psi))
            bound = 2.0 ** -8 * np.real(np.sum(np.abs(qa) * (np.abs(Kc) @ np.abs(qa).T).T, axis=1))
            assert np.all(np.abs(got["a"][:, 0] - ref["a"][:, 0]) <= bound + 1e-12), cfg.name
            tol_eps = 1e-3
        else:
            tol = 1e-10 if dt == "f64" else 1e-5
            if dt == "f64":
                op2 = oracle_operator(cfg)
                op2.delta = np.nextafter(op.delta, np.inf)
                pert = O.haydock(op2.apply, P, 40)
            else:
                pert = O.haydock(_fp32_storage(cfg).apply, P, 40,
                                 round_dtype=np.complex64 if dt == "f32" else None)
            head = dict(a=ref["a"][:, :40], b=ref["b"][:, :41])
            w = _window(head, pert, 1e-10 if dt == "f64" else 1e-6) - 2
            assert w >= 10, (cfg.name, w)
            for r in range(P.shape[0]):
                assert np.all(np.abs(got["a"][r, :w] - ref["a"][r, :w]) <= tol * np.abs(ref["a"][r, :w])), (cfg.name, r)
                assert np.all(np.abs(got["b"][r, 1:w + 1] - ref["b"][r, 1:w + 1])
                              <= tol * np.abs(ref["b"][r, 1:w + 1])), (cfg.name, r)
            tol_eps = 1e-10 if dt == "f64" else 1e-6
        eps = O.continued_fraction(got["a"], got["b"], got["pnorm2"], cfg.prefactor(), om, 0.5)
        oeps = O.continued_fraction(ref["a"], ref["b"], ref["pnorm2"], cfg.prefactor(), om, 0.5)
        for r in range(P.shape[0]):
            assert rel_l2(eps[r].imag, oeps[r].imag) < tol_eps, (cfg.name, r)
    batch.close()
    for p in probs:
        p.close()


C3_SHAPES = [next(c for c in ti.batch_configs() if (c.n_coarse, c.n_div, c.nc) == shape)
             for shape in ((6, 3, 3), (8, 4, 6))]


@pytest.mark.parametrize("cfg", C3_SHAPES, ids=lambda c: c.name)
def test_batch_workload_shapes_against_the_oracle(bse, cfg):
    """The two larger grid shapes of the 48-member batching workload, one member each
    (6^3 x 3 displaced by +delta with 3v3c; 8^3 x 4 displaced by -delta with 3v6c), in
    FP32 storage as the workload runs them:
    * sampled matvec cells against the oracle, within the FP32 bound of each output's
      sum of |terms| (storage rounding, and the packed coarse product's arithmetic on the
      kernel terms) and 2e-6 in relative L2;
    * the member's chains run in a batch (200 steps, 3 polarisations) against the
      oracle's FP64 chain head to 1e-5, up to two steps before the oracle with every
      stored array in complex64 (overlaps, K_c, vectors) first departs from FP64 by more
      than 1e-6 (at least 8 coefficients; the tolerance as in the test above)."""
    bs = bands(cfg)
    prob = bse.problem_from_bands(bs, cfg, dtype="f32", max_rhs=3)
    cells = np.array([0, cfg.nk_coarse // 3, cfg.nk_coarse - 1])
    check_sampled_cells(cfg, bs, prob, oracle_pieces(cfg, bs), cells, 301, U32, (10, fp32_kernel_factors(True)),
                        2e-6)
    P = bs.P_flat()
    batch = bse.BSEBatch([prob], [P], 200, n_branches=1)
    got = _host(batch.run()[0])
    torch.cuda.synchronize()
    assert np.all(got["status"] == bse.BSE_OK)
    op = oracle_operator(cfg)
    n = 16
    ref = O.haydock(op.apply, P, n)
    emu = O.haydock(_fp32_storage(cfg).apply, P, n, round_dtype=np.complex64)
    w = _window(ref, emu, 1e-6) - 2
    assert w >= 8, w
    np.testing.assert_allclose(got["pnorm2"], ref["pnorm2"], rtol=1e-12)
    for r in range(3):
        assert np.all(np.abs(got["a"][r, :w] - ref["a"][r, :w]) <= 1e-5 * np.abs(ref["a"][r, :w])), r
        assert np.all(np.abs(got["b"][r, 1:w + 1] - ref["b"][r, 1:w + 1]) <= 1e-5 * np.abs(ref["b"][r, 1:w + 1])), r
    batch.close()
    prob.close()
