"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Sizes here keep the oracle within seconds while spanning several blocks, ragged
subpoint counts (n_div^3 = 27, not a multiple of the 64-lane wavefront; 125,
more than one subpoint per lane) and every compiled band pair used by the
workloads.  Full-size (32^3 dense) checks live in test_gpu_c1.py.
"""

import numpy as np
import pytest

import oracle as O
import tbinputs as ti

from _cases import bands, oracle_operator, oracle_parts, rel_l2
from _gpu import U32, U64, fp32_kernel_factors, gpu_overlaps_to_oracle, product_bound

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bse():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_01863_amd import bse as mod
    return mod


CASES = [
    ti.get_config("c0"),                                                        # 4^3 x 2, 3v3c
    ti.tiny_config(n_coarse=3, n_div=3, nv=3, nc=6, n_orb=9, seed=11, n_pol=3),  # 27 subpoints
    ti.tiny_config(n_coarse=2, n_div=5, nv=2, nc=3, n_orb=5, seed=12, n_pol=2),  # 125 subpoints
    ti.tiny_config(n_coarse=5, n_div=1, nv=1, nc=2, n_orb=3, seed=13, n_pol=4),  # single division
    ti.tiny_config(n_coarse=2, n_div=4, nv=4, nc=6, n_orb=10, seed=14, n_pol=1),
]
IDS = [c.name for c in CASES]


def _problem(bse, cfg, dtype, **kw):
    return bse.problem_from_bands(bands(cfg), cfg, dtype=dtype, max_rhs=max(cfg.n_pol, 1), **kw)


@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_overlaps_and_energies_match_oracle(bse, cfg):
    bs, Dv, Dc, f, Kc, delta = oracle_parts(cfg)
    prob = _problem(bse, cfg, "f64")
    torch.cuda.synchronize()
    gDv, gDc = gpu_overlaps_to_oracle(prob.d.cpu().numpy(), cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    assert np.abs(gDv - Dv).max() < 1e-14
    assert np.abs(gDc - Dc).max() < 1e-14
    assert np.array_equal(prob.delta.cpu().numpy(), delta)
    prob32 = _problem(bse, cfg, "f32")
    gDv32, gDc32 = gpu_overlaps_to_oracle(prob32.d.cpu().numpy(), cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    assert np.all(np.abs(gDv32 - Dv) <= U32 * np.abs(Dv) * 1.01 + 1e-15)
    assert np.all(np.abs(gDc32 - Dc) <= U32 * np.abs(Dc) * 1.01 + 1e-15)
    prob.close()
    prob32.close()


@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_coarse_kernel_matches_oracle(bse, cfg):
    bs, Dv, Dc, f, Kc, delta = oracle_parts(cfg)
    prob = _problem(bse, cfg, "f64")
    K = prob.Kc.cpu().numpy()
    scale = np.abs(Kc).max()
    assert np.abs(K - Kc).max() < 1e-13 * scale
    assert np.array_equal(K, K.conj().T)          # Hermitian by construction, exactly
    prob32 = _problem(bse, cfg, "f32")
    K32 = prob32.Kc.cpu().numpy().astype(complex)
    assert np.abs(K32 - Kc).max() <= 2 * U32 * scale
    prob.close()
    prob32.close()


@pytest.mark.parametrize("form", [0, 1], ids=["packed", "full"])
@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_matvec_fp64_matches_oracle(bse, cfg, form):
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, "f64")
    bse.bse_plan_set_coarse_product(prob.plan, form)
    x = ti.random_vectors(op.N, cfg.n_pol, 101)
    y = prob.matvec(x).cpu().numpy()
    ref = op.apply(x)
    assert rel_l2(y, ref) < 1e-13
    # componentwise: rounding of a few FP64 operations per term
    assert np.all(np.abs(y - ref) <= product_bound(op, x, U64, factors=64) + 1e-300)
    prob.close()


@pytest.mark.parametrize("form", [0, 1], ids=["packed", "full"])
@pytest.mark.parametrize("dtype", ["f32", "f32v64"])
@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_matvec_fp32_storage_within_rounding_bound(bse, cfg, dtype, form):
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, dtype)
    bse.bse_plan_set_coarse_product(prob.plan, form)
    x = ti.random_vectors(op.N, cfg.n_pol, 102)
    xs = prob.vector(x)                       # rounded to the vector storage
    y = prob.matvec(xs).cpu().numpy().astype(complex)
    ref = op.apply(xs.cpu().numpy().astype(complex))
    bound = product_bound(op, x, U32, 10, fp32_kernel_factors(form == 0))
    assert np.all(np.abs(y - ref) <= bound)
    assert rel_l2(y, ref) < 2e-6
    prob.close()


def test_matvec_nearest_corner_variant(bse):
    cfg = CASES[1]
    op = oracle_operator(cfg, weights="nearest")
    prob = _problem(bse, cfg, "f64", neighbours=1)
    x = ti.random_vectors(op.N, cfg.n_pol, 103)
    assert rel_l2(prob.matvec(x).cpu().numpy(), op.apply(x)) < 1e-13
    prob.close()


def test_matvec_multiple_rhs_are_independent(bse):
    cfg = CASES[1]
    prob = _problem(bse, cfg, "f64")
    x = ti.random_vectors(prob.N, 3, 104)
    y3 = prob.matvec(x).cpu().numpy()
    for r in range(3):
        y1 = prob.matvec(x[r:r + 1]).cpu().numpy()
        assert np.array_equal(y1[0], y3[r])
    prob.close()


@pytest.mark.parametrize("splits", [1, 3, 7, 64])
def test_matvec_independent_of_product_splits(bse, splits):
    cfg = ti.get_config("c0")
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, "f64")
    bse.bse_plan_set_coarse_product(prob.plan, 1)
    bse.bse_plan_set_gemv_splits(prob.plan, splits)
    x = ti.random_vectors(op.N, 1, 105)
    assert rel_l2(prob.matvec(x).cpu().numpy(), op.apply(x)) < 1e-13
    prob.close()


# the coarse product's other code paths: a column split longer than one LDS stage of
# qbar (2048 / n_rhs entries) stages qbar in pieces; an odd N_c in FP32 storage leaves the
# rows of K_c off 16-byte alignment, so every load is an element load
ODD_NC = ti.tiny_config(n_coarse=5, n_div=2, nv=3, nc=3, n_orb=7, seed=15, n_pol=4)  # N_c = 1125
PATH_CASES = [(ODD_NC, "f32"), (ODD_NC, "f64"), (ti.get_config("c0").with_(n_pol=4), "f32")]


@pytest.mark.parametrize("cfg,dtype", PATH_CASES, ids=[f"{c.name}-{d}" for c, d in PATH_CASES])
@pytest.mark.parametrize("splits", [1, 2, 0])
@pytest.mark.parametrize("n_rhs", [3, 4])
def test_matvec_product_paths_match_oracle(bse, cfg, dtype, splits, n_rhs):
    """The full-stream coarse product (its split and staging paths)."""
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, dtype)
    bse.bse_plan_set_coarse_product(prob.plan, 1)
    bse.bse_plan_set_gemv_splits(prob.plan, splits)
    x = ti.random_vectors(op.N, n_rhs, 108)
    xs = prob.vector(x)
    y = prob.matvec(xs).cpu().numpy().astype(complex)
    ref = op.apply(xs.cpu().numpy().astype(complex))
    if dtype == "f64":
        assert rel_l2(y, ref) < 1e-13
    else:
        assert np.all(np.abs(y - ref) <= product_bound(op, x, U32))
        assert rel_l2(y, ref) < 2e-6
    prob.close()


# the packed Hermitian coarse product: coarse spaces that are not whole 128-row tiles
# (576 = 4.5 tiles, 1125 = 8.8 tiles, 486 = 3.8 tiles), a single tile row (72 < 128), and
# every compiled right-hand-side count
PACKED_CASES = [ti.get_config("c0").with_(n_pol=4), ODD_NC,
                ti.tiny_config(n_coarse=3, n_div=2, nv=3, nc=6, n_orb=9, seed=17, n_pol=4),
                ti.tiny_config(n_coarse=2, n_div=3, nv=3, nc=3, n_orb=6, seed=18, n_pol=4)]


@pytest.mark.parametrize("cfg", PACKED_CASES, ids=[c.name for c in PACKED_CASES])
@pytest.mark.parametrize("n_rhs", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_matvec_packed_product_matches_oracle(bse, cfg, n_rhs, dtype):
    """K_c read once per Hermitian pair of tiles (Eqs. bse1-bse2).  FP32 coarse kernel:
    within storage rounding plus the bound of the product's FP32 arithmetic, and 2e-6 in
    relative L2; FP64: the bound of a few FP64 operations per term and 1e-13.  Results are
    reproducible bit for bit."""
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, dtype)
    x = ti.random_vectors(op.N, n_rhs, 110)
    xs = prob.vector(x)
    y = prob.matvec(xs)
    y2 = prob.matvec(xs)
    assert torch.equal(y, y2)
    y = y.cpu().numpy().astype(complex)
    ref = op.apply(xs.cpu().numpy().astype(complex))
    if dtype == "f64":
        assert np.all(np.abs(y - ref) <= product_bound(op, x, U64, factors=64) + 1e-300)
        assert rel_l2(y, ref) < 1e-13
    else:
        assert np.all(np.abs(y - ref) <= product_bound(op, x, U32, 10, fp32_kernel_factors(True)))
        assert rel_l2(y, ref) < 2e-6
    prob.close()


# 216 subpoints per cell with FP64 vectors: a cell's vector slice no longer fits the
# restrict's LDS tiles, and the restrict falls back to reading the overlaps in their
# input layout (k_restrict2); the prolong runs its one-block-per-cell form
WIDE_CELL = ti.tiny_config(n_coarse=2, n_div=6, nv=3, nc=6, n_orb=9, seed=16, n_pol=3, steps=20)


@pytest.mark.parametrize("dtype", ["f64", "f32v64"])
def test_wide_cell_matvec_and_chain_match_oracle(bse, dtype):
    cfg = WIDE_CELL
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, dtype)
    x = ti.random_vectors(op.N, 3, 109)
    xs = prob.vector(x)
    y = prob.matvec(xs).cpu().numpy().astype(complex)
    ref = op.apply(xs.cpu().numpy().astype(complex))
    if dtype == "f64":
        assert rel_l2(y, ref) < 1e-13
    else:
        assert np.all(np.abs(y - ref) <= product_bound(op, x, U32, 10, fp32_kernel_factors(True)))
    # chain start and update forms of the same restrict: the head of the chain
    P = bands(cfg).P_flat()
    och = O.haydock(op.apply, P, cfg.steps)
    ch = prob.haydock(P, cfg.steps)
    a, b = ch["a"].cpu().numpy(), ch["b"].cpu().numpy()
    tol = 1e-10 if dtype == "f64" else 1e-5
    assert np.all(ch["status"].cpu().numpy() == bse.BSE_OK)
    assert rel_l2(a[:, :10], och["a"][:, :10]) < tol
    assert rel_l2(b[:, 1:11], och["b"][:, 1:11]) < tol
    prob.close()


# 4v6c with three right-hand sides: the prolong splits the conduction index over three
# wavefronts per right-hand side
WIDE_BANDS = ti.tiny_config(n_coarse=2, n_div=4, nv=4, nc=6, n_orb=10, seed=26, n_pol=3, steps=20)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_wide_band_pair_three_rhs_matches_oracle(bse, dtype):
    cfg = WIDE_BANDS
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, dtype)
    x = ti.random_vectors(op.N, 3, 112)
    xs = prob.vector(x)
    y = prob.matvec(xs).cpu().numpy().astype(complex)
    ref = op.apply(xs.cpu().numpy().astype(complex))
    if dtype == "f64":
        assert rel_l2(y, ref) < 1e-13
    else:
        assert np.all(np.abs(y - ref) <= product_bound(op, x, U32, 10, fp32_kernel_factors(True)))
    P = bands(cfg).P_flat()
    och = O.haydock(op.apply, P, cfg.steps)
    ch = prob.haydock(P, cfg.steps)
    a, b = ch["a"].cpu().numpy(), ch["b"].cpu().numpy()
    tol = 1e-10 if dtype == "f64" else 1e-5
    assert np.all(ch["status"].cpu().numpy() == bse.BSE_OK)
    assert rel_l2(a[:, :10], och["a"][:, :10]) < tol
    assert rel_l2(b[:, 1:11], och["b"][:, 1:11]) < tol
    prob.close()


# band pairs without a compiled form: the run-time kernels (restrict and prolong take nv, nc
# as arguments); 8, 27 and 64 subpoints per cell, up to nv nc = 32 and nv + nc = 16
ANY_BANDS = [
    ti.tiny_config(n_coarse=3, n_div=2, nv=2, nc=5, n_orb=7, seed=21, n_pol=3, steps=20),
    ti.tiny_config(n_coarse=2, n_div=3, nv=5, nc=1, n_orb=6, seed=22, n_pol=2, steps=20),
    ti.tiny_config(n_coarse=2, n_div=4, nv=4, nc=8, n_orb=12, seed=23, n_pol=1, steps=20),
    ti.tiny_config(n_coarse=2, n_div=2, nv=2, nc=14, n_orb=16, seed=24, n_pol=2, steps=20),
    # the other ends of the range: eight valence bands, and a single one with 15 conduction
    ti.tiny_config(n_coarse=2, n_div=2, nv=8, nc=4, n_orb=12, seed=25, n_pol=1, steps=20),
    ti.tiny_config(n_coarse=2, n_div=3, nv=1, nc=15, n_orb=16, seed=26, n_pol=2, steps=20),
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("cfg", ANY_BANDS, ids=[c.name for c in ANY_BANDS])
def test_any_band_counts_match_oracle(bse, cfg, dtype):
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, dtype)
    x = ti.random_vectors(op.N, cfg.n_pol, 111)
    xs = prob.vector(x)
    y = prob.matvec(xs).cpu().numpy().astype(complex)
    ref = op.apply(xs.cpu().numpy().astype(complex))
    if dtype == "f64":
        assert rel_l2(y, ref) < 1e-13
    else:
        assert np.all(np.abs(y - ref) <= product_bound(op, x, U32, 10, fp32_kernel_factors(True)))
    # chain start and update forms: the head of the chain
    P = bands(cfg).P_flat()
    och = O.haydock(op.apply, P, cfg.steps)
    ch = prob.haydock(P, cfg.steps)
    a, b = ch["a"].cpu().numpy(), ch["b"].cpu().numpy()
    tol = 1e-10 if dtype == "f64" else 1e-5
    assert np.all(ch["status"].cpu().numpy() == bse.BSE_OK)
    assert rel_l2(a[:, :10], och["a"][:, :10]) < tol
    assert rel_l2(b[:, 1:11], och["b"][:, 1:11]) < tol
    prob.close()


@pytest.mark.parametrize("dtype,form", [("f32", 0), ("f64", 0), ("bf16", 0), ("f16", 0), ("f32", 1), ("bf16", 1)],
                         ids=["f32", "f64", "bf16", "f16", "f32-full", "bf16-full"])
def test_kernel_timing_modes(bse, dtype, form):
    """Plan timing: one event pair per coarse product of a chain step, around the whole
    product (mode 1) or carried by the launch of its streaming kernel alone (mode 3, which
    cannot take longer than the whole product); timing does not change the chain's
    coefficients."""
    cfg = ti.get_config("c0")
    prob = _problem(bse, cfg, dtype)
    bse.bse_plan_set_coarse_product(prob.plan, form)   # 1: the full-stream product
    P = bands(cfg).P_flat()
    ref = prob.haydock(P, 12)
    per_launch = {}
    for mode in (1, 3):
        prob.set_timing(mode)
        ch = prob.haydock(P, 12)
        ms, n = prob.timing()
        prob.set_timing(0)
        assert n == 12 and ms > 0.0
        per_launch[mode] = ms / n
        assert np.array_equal(ch["a"].cpu().numpy(), ref["a"].cpu().numpy())
        assert np.array_equal(ch["b"].cpu().numpy(), ref["b"].cpu().numpy())
    assert per_launch[3] < per_launch[1]
    prob.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_restrict_group_gives_same_matvec(bse, dtype):
    # one block per right-hand side, or one block for all three: same arithmetic per
    # output, so the same bits
    cfg = CASES[1]
    prob = _problem(bse, cfg, dtype)
    x = prob.vector(ti.random_vectors(prob.N, 3, 107))
    y1 = prob.matvec(x).cpu().numpy()
    bse.bse_plan_set_restrict_group(prob.plan, 3)
    y3 = prob.matvec(x).cpu().numpy()
    assert np.array_equal(y1, y3)
    prob.close()


def test_matvec_is_deterministic(bse):
    cfg = CASES[1]
    prob = _problem(bse, cfg, "f32")
    x = prob.vector(ti.random_vectors(prob.N, 3, 106))
    y1 = prob.matvec(x)
    y2 = prob.matvec(x)
    assert torch.equal(y1, y2)
    prob.close()


def _oracle_sensitivity(op, P, steps, omega, eta, prefactor):
    """Change of the oracle's own eps2 when the transition energies move by one ulp:
    the rounding sensitivity of a finite chain at this broadening."""
    rng = np.random.default_rng(0)
    op2 = O.InterpOperator(op.Dv, op.Dc, op.f, op.Kc,
                           op.delta * (1 + 2.0 ** -52 * rng.choice([-1.0, 0.0, 1.0], size=op.delta.shape)),
                           op.n_c, op.n_div, op.nv, op.nc)
    c1 = O.haydock(op.apply, P, steps)
    c2 = O.haydock(op2.apply, P, steps)
    e1 = O.continued_fraction(c1["a"], c1["b"], c1["pnorm2"], prefactor, omega, eta)
    e2 = O.continued_fraction(c2["a"], c2["b"], c2["pnorm2"], prefactor, omega, eta)
    return c1, rel_l2(e2.imag, e1.imag)


def test_haydock_c0_fp64_matches_oracle(bse):
    """C0 chain (FP64).  Coefficients are compared over the head of the chain that
    is well conditioned (the oracle against itself with one-ulp perturbed input
    agrees to 1e-12 for 20 steps; later, rounding decides when converged states
    re-enter).  eps2 is compared at a broadening where the 200-step chain has
    converged, and at the workload's eta against ten times the oracle's own
    one-ulp sensitivity."""
    cfg = ti.get_config("c0")
    op = oracle_operator(cfg)
    P = bands(cfg).P_flat()
    om = cfg.omega()
    och, sens = _oracle_sensitivity(op, P, cfg.steps, om, cfg.eta, cfg.prefactor())
    prob = _problem(bse, cfg, "f64")
    ch = prob.haydock(P, cfg.steps)
    a, b = ch["a"].cpu().numpy(), ch["b"].cpu().numpy()
    assert int(ch["steps"][0]) == cfg.steps and int(ch["status"][0]) == bse.BSE_OK
    assert abs(ch["pnorm2"][0].item() - och["pnorm2"][0]) < 1e-13 * och["pnorm2"][0]
    assert rel_l2(a[0, :20], och["a"][0, :20]) < 1e-10
    assert rel_l2(b[0, 1:21], och["b"][0, 1:21]) < 1e-10
    for eta in (0.3, 0.5):
        eps = prob.continued_fraction(ch, cfg.prefactor(), om, eta).cpu().numpy()
        oeps = O.continued_fraction(och["a"], och["b"], och["pnorm2"], cfg.prefactor(), om, eta)
        assert rel_l2(eps.imag, oeps.imag) < 1e-10, eta
    eps = prob.continued_fraction(ch, cfg.prefactor(), om, cfg.eta).cpu().numpy()
    oeps = O.continued_fraction(och["a"], och["b"], och["pnorm2"], cfg.prefactor(), om, cfg.eta)
    assert rel_l2(eps.imag, oeps.imag) < max(1e-10, 10 * sens)
    prob.close()


def test_continued_fraction_kernel_matches_oracle(bse):
    rng = np.random.default_rng(4)
    m, n_chains = 57, 3
    a = rng.uniform(1, 9, size=(n_chains, m))
    b = np.zeros((n_chains, m + 1))
    b[:, 1:] = rng.uniform(0.2, 2, size=(n_chains, m))
    pn = rng.uniform(0.5, 3, size=n_chains)
    steps = np.array([m, 20, 1], dtype=np.int32)
    om = np.linspace(0, 12, 777)
    dev = "cuda"
    chain = dict(a=torch.tensor(a, device=dev), b=torch.tensor(b, device=dev),
                 pnorm2=torch.tensor(pn, device=dev), steps=torch.tensor(steps, device=dev))
    eps = bse.BSEProblem.continued_fraction(chain, 0.37, om, 0.08).cpu().numpy()
    ref = O.continued_fraction(a, b, pn, 0.37, om, 0.08, steps)
    assert np.abs(eps - ref).max() < 1e-12 * np.abs(ref).max()


def test_haydock_breakdown_and_zero_start(bse):
    cfg = ti.tiny_config(n_coarse=2, n_div=2, nv=2, nc=2, n_pol=3)
    op = oracle_operator(cfg)
    H = op.explicit_hamiltonian()
    E, V = np.linalg.eigh(H)
    P = np.stack([2.0 * V[:, 5], np.zeros(op.N), bands(cfg).P_flat()[0]])
    prob = _problem(bse, cfg, "f64")
    ch = prob.haydock(P, 12)
    steps = ch["steps"].cpu().numpy()
    status = ch["status"].cpu().numpy()
    a = ch["a"].cpu().numpy()
    assert steps[0] == 1 and status[0] == bse.BSE_INFO_INVARIANT_SUBSPACE
    assert abs(a[0, 0] - E[5]) < 1e-12 and np.all(a[0, 1:] == 0)
    assert steps[1] == 0 and status[1] == bse.BSE_INFO_ZERO_START and np.all(a[1] == 0)
    assert steps[2] == 12 and status[2] == bse.BSE_OK
    och = O.haydock(op.apply, P[2:], 12)
    assert rel_l2(a[2], och["a"][0]) < 1e-12
    eps = prob.continued_fraction(ch, 1.0, np.linspace(0, 10, 11), 0.1).cpu().numpy()
    np.testing.assert_allclose(eps[0], 1.0 - 4.0 / (np.linspace(0, 10, 11) + 0.1j - E[5]), rtol=1e-11)
    assert np.all(eps[1] == 1.0)
    prob.close()


def test_haydock_is_deterministic_and_matches_matvec_chain(bse):
    """Chain on the device equals a host-driven chain built from bse_interp_matvec."""
    cfg = CASES[1]
    prob = _problem(bse, cfg, "f64")
    P = bands(cfg).P_flat()
    c1 = prob.haydock(P, 30)
    c2 = prob.haydock(P, 30)
    assert torch.equal(c1["a"], c2["a"]) and torch.equal(c1["b"], c2["b"])
    och = O.haydock(lambda x: prob.matvec(x).cpu().numpy(), P, 30)
    assert rel_l2(c1["a"].cpu().numpy()[:, :15], och["a"][:, :15]) < 1e-11
    prob.close()
