"""GPU parity of the low-precision forms: the coarse kernel of Eq. (matmul2) kept as
block-scaled BF16 or FP16 and multiplied on the matrix cores (FP32 accumulation
inside a 64-column block, FP64 across blocks), checked against the FP64 oracle.

The matvec is bounded componentwise from the arithmetic of the format (see
`lowp_bound`); the chain is compared on eps2 at broadenings where the chain has
converged, against the relative tolerance 1e-3 set for the low-precision form."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import tbinputs as ti

from _cases import bands, oracle_operator, rel_l2
from _gpu import FP32_INNER_UNITS, U32, abs_operator, product_bound

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# unit roundoff of the kernel's storage format (8 and 11 significant bits)
UNIT = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}

CASES = [
    ti.get_config("c0"),                                                        # 4^3 x 2, 3v3c
    ti.tiny_config(n_coarse=3, n_div=3, nv=3, nc=6, n_orb=9, seed=11, n_pol=3),  # Nc 486, ragged blocks
    ti.tiny_config(n_coarse=2, n_div=4, nv=4, nc=6, n_orb=10, seed=14, n_pol=2),
    ti.tiny_config(n_coarse=2, n_div=5, nv=2, nc=3, n_orb=5, seed=12, n_pol=4),  # 125 subpoints, 4 rhs
]
IDS = [c.name for c in CASES]


@pytest.fixture(scope="module")
def bse():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_01863_amd import bse as mod
    return mod


def _problem(bse, cfg, dtype):
    return bse.problem_from_bands(bands(cfg), cfg, dtype=dtype, max_rhs=max(cfg.n_pol, 1))


def lowp_bound(op, x, dtype):
    """Componentwise bound on |y_gpu - y| for the low-precision forms.

    - FP32 storage of x, the overlaps, K_c and the output: as for BSE_F32
      (`product_bound` with the FP32 unit).
    - K_c in the format: |dK| <= u |K| per entry, plus for FP16 an absolute floor
      of half the subnormal spacing, 2^-25 s_B <= 2^-24 max|K| (s_B < 2 max|K_B|).
    - qbar as leading part + remainder in the format: relative u^2, plus for FP16 an
      absolute floor of half the subnormal spacing over the group's scale: each 64-entry
      group of qbar is scaled by the power of two that puts its largest entry in
      [2^14, 2^15), so the floor is at most 2^-25 2^-14 max|qbar| <= 2^-39 max(|C||x|).
    - FP32 accumulation of the 64 products of one block: 64 u32 per |term|, plus 2 for the
      packed Hermitian form's column products (the two conjugation terms are subtracted and
      the leading and remainder parts added in FP32): 66.
    - the restrict's and prolong's FP32 contractions: FP32_INNER_UNITS u32.
    The kernel terms are bounded by |C|^H |K| |C| |x|.
    """
    aop = abs_operator(op)
    ax = np.abs(x)
    u = UNIT[dtype]
    bound = product_bound(op, x, U32) + (u + 4 * u * u + (66 + FP32_INNER_UNITS) * U32) * np.abs(aop.apply_kernel(ax))
    if dtype == "f16":
        kmax = np.abs(op.Kc).max()
        colsum = np.abs(aop.restrict(ax)).sum(axis=1)                # 1^T |C||x| per rhs
        w = np.abs(aop.prolong(np.ones((1, op.Nc))))                  # |C|^H 1
        rowk = np.abs(aop.prolong(np.abs(op.Kc).sum(axis=1)[None]))   # |C|^H |K| 1
        qmax = np.abs(aop.restrict(ax)).max(axis=1)                  # >= max|qbar| per rhs
        bound = bound + 2.0 ** -24 * kmax * colsum[:, None] * w + 2.0 ** -39 * qmax[:, None] * rowk
    return bound


@pytest.mark.parametrize("form", [0, 1], ids=["packed", "full"])
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_matvec_lowp_within_format_bound(bse, cfg, dtype, form):
    """Both coarse-product forms of the block-scaled kernel: the blocks on and above the
    diagonal with the column products on the matrix cores too (0, the default), or every
    block (1).  The packed form is reproducible bit for bit."""
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, dtype)
    bse.bse_plan_set_coarse_product(prob.plan, form)
    x = ti.random_vectors(op.N, cfg.n_pol, 301)
    x = x / np.linalg.norm(x, axis=1, keepdims=True)          # unit vectors, as in the chain
    xs = prob.vector(x)
    y = prob.matvec(xs)
    assert torch.equal(y, prob.matvec(xs))
    y = y.cpu().numpy().astype(complex)
    xr = xs.cpu().numpy().astype(complex)
    ref = op.apply(xr)
    assert np.all(np.isfinite(y))
    assert np.all(np.abs(y - ref) <= lowp_bound(op, xr, dtype))
    # the kernel part carries the format's rounding: far below one unit overall
    assert rel_l2(y - op.delta[None] * xr, ref - op.delta[None] * xr) < 2 * UNIT[dtype]
    prob.close()


@pytest.mark.parametrize("norm", [1e4, 1e-6])
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_matvec_lowp_any_input_norm(bse, dtype, norm):
    """A plain matvec of a vector far from unit norm: with norm 1e4 the entries of qbar
    reach about 800, past the 128 that FP16 held at the former fixed scale of 2^9, and
    with 1e-6 they would fall into its subnormals.  Each group of qbar carries its own power-of-two scale, so
    the product stays finite and within the same componentwise bound at any norm."""
    cfg = CASES[1]
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, dtype)
    x = ti.random_vectors(op.N, cfg.n_pol, 303)
    x = norm * x / np.linalg.norm(x, axis=1, keepdims=True)
    xs = prob.vector(x)
    y = prob.matvec(xs).cpu().numpy().astype(complex)
    xr = xs.cpu().numpy().astype(complex)
    ref = op.apply(xr)
    assert np.all(np.isfinite(y))
    if norm > 1:
        assert np.abs(op.restrict(xr)).max() > 65504 / 512       # past the former fixed scale
    assert np.all(np.abs(y - ref) <= lowp_bound(op, xr, dtype))
    assert rel_l2(y - op.delta[None] * xr, ref - op.delta[None] * xr) < 2 * UNIT[dtype]
    prob.close()


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_lowp_padding_columns_stay_clean(bse, dtype):
    """Two calls with different right-hand-side counts: the second's results do not
    depend on what the first left in the unused fragment columns."""
    cfg = CASES[3]
    op = oracle_operator(cfg)
    prob = _problem(bse, cfg, dtype)
    x = ti.random_vectors(op.N, 4, 302)
    x = x / np.linalg.norm(x, axis=1, keepdims=True)
    y4 = prob.matvec(prob.vector(x)).cpu().numpy()
    y1 = prob.matvec(prob.vector(x[1:2])).cpu().numpy()
    assert np.array_equal(y1[0], y4[1])
    prob.close()


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_haydock_c0_lowp_eps2_within_tolerance(bse, dtype):
    """C0 chain with the low-precision kernel against the FP64 oracle chain: eps2
    at broadenings where the 200-step chain has converged, relative L2 <= 1e-3."""
    cfg = ti.get_config("c0")
    op = oracle_operator(cfg)
    P = bands(cfg).P_flat()
    om = cfg.omega()
    och = O.haydock(op.apply, P, cfg.steps)
    prob = _problem(bse, cfg, dtype)
    ch = prob.haydock(P, cfg.steps)
    assert int(ch["status"][0]) == bse.BSE_OK and int(ch["steps"][0]) == cfg.steps
    for eta in (0.3, 0.5):
        eps = prob.continued_fraction(ch, cfg.prefactor(), om, eta).cpu().numpy()
        oeps = O.continued_fraction(och["a"], och["b"], och["pnorm2"], cfg.prefactor(), om, eta)
        assert rel_l2(eps.imag, oeps.imag) < 1e-3, eta
    prob.close()
