"""Full-size parity on the precision form's workload (10^3 coarse x 4 divisions,
4v6c: N = 1 536 000, K_c 24 000^2 block-scaled BF16), in the launch configuration
the benchmark times: sampled cells of the matvec against the FP64 oracle, computed
one by one (the K_c rows of the cells' corners and the restriction of the whole
vector), within the format's componentwise bound; adjointness of the applied
operator at full size.  The same cells in FP32 storage, where the coarse product
stages qbar in pieces."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import tbinputs as ti

from _cases import bands, rel_l2
from _gpu import FP32_INNER_UNITS, U32, fp32_kernel_factors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CFG = ti.get_config("c2")
SAMPLE_CELLS = np.array([0, 377, 999])
U_BF16 = 2.0 ** -8


@pytest.fixture(scope="module")
def bse():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_01863_amd import bse as mod
    return mod


@pytest.fixture(scope="module")
def c2(bse):
    bs = bands(CFG)
    prob = bse.problem_from_bands(bs, CFG, dtype="bf16", max_rhs=3)
    yield bs, prob
    prob.close()


def test_c2_bf16_matvec_sampled_cells(c2):
    """Bound per output: 10 FP32 units of the sum of |terms| (FP32 storage of x, the
    overlaps, K_c and the output), plus the format's rounding of K_c and qbar and the
    FP32 accumulation inside a 64-column block on the kernel terms, with the packed
    form's two FP32 combinations of its column products (u + 4u^2 + 66 u32) |C|^H |K| |C| |x|."""
    bs, prob = c2
    Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, CFG.n_coarse, CFG.n_div, CFG.nv, CFG.nc)
    delta = O.transition_energies(bs.eps_dense, CFG.nv, CFG.nc)
    f = O.trilinear_weights(CFG.n_div)
    x = ti.random_vectors(CFG.n_trans, 3, 401)
    x = x / np.linalg.norm(x, axis=1, keepdims=True)          # unit vectors, as in the chain
    xs = prob.vector(x)
    y = prob.matvec(xs).cpu().numpy().astype(complex)
    xh = xs.cpu().numpy().astype(complex)
    nbr = O.neighbour_table(CFG.n_coarse)
    need = np.unique(nbr[SAMPLE_CELLS].ravel())
    rows = O.coarse_kernel_block_rows(bs.vecs_coarse, bs.tau, CFG.nv, CFG.nc, CFG.n_coarse, CFG.n_div, CFG, need)
    np_ = CFG.n_pair
    op = O.InterpOperator(Dv, Dc, f, None, delta, CFG.n_coarse, CFG.n_div, CFG.nv, CFG.nc)
    aop = O.InterpOperator(np.abs(Dv).astype(complex), np.abs(Dc).astype(complex), f, None, np.abs(delta),
                           CFG.n_coarse, CFG.n_div, CFG.nv, CFG.nc)
    qbar = op.restrict(xh)
    qabs = aop.restrict(np.abs(xh))
    r = np.zeros((3, CFG.n_trans_coarse), dtype=complex)
    rabs = np.zeros((3, CFG.n_trans_coarse), dtype=complex)
    for i, k in enumerate(need):
        r[:, k * np_:(k + 1) * np_] = (rows[i] @ qbar.T).T
        rabs[:, k * np_:(k + 1) * np_] = (np.abs(rows[i]) @ np.abs(qabs).T).T
    ref = delta[None] * xh + op.prolong(r)
    kern_abs = np.abs(aop.prolong(rabs))
    bound = 10 * U32 * (np.abs(delta)[None] * np.abs(xh) + kern_abs) \
        + (U_BF16 + 4 * U_BF16 ** 2 + (66 + FP32_INNER_UNITS) * U32) * kern_abs
    ndiv3 = CFG.n_div3
    for cell in SAMPLE_CELLS:
        sl = slice(cell * ndiv3 * np_, (cell + 1) * ndiv3 * np_)
        assert np.all(np.abs(y[:, sl] - ref[:, sl]) <= bound[:, sl]), f"cell {cell}"
        # the kernel part carries the format's rounding: well below one BF16 unit overall
        kd, kr = y[:, sl] - delta[None, sl] * xh[:, sl], ref[:, sl] - delta[None, sl] * xh[:, sl]
        assert rel_l2(kd, kr) < 2 * U_BF16


def test_c2_fp32_matvec_sampled_cells(bse):
    """FP32 storage at C2 (the packed Hermitian coarse product at 24 000 coarse
    transitions): the same sampled cells within 10 FP32 units of the sum of |terms|, plus
    the packed product's arithmetic on the kernel terms."""
    bs = bands(CFG)
    prob = bse.problem_from_bands(bs, CFG, dtype="f32", max_rhs=3)
    Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, CFG.n_coarse, CFG.n_div, CFG.nv, CFG.nc)
    delta = O.transition_energies(bs.eps_dense, CFG.nv, CFG.nc)
    f = O.trilinear_weights(CFG.n_div)
    x = ti.random_vectors(CFG.n_trans, 3, 404)
    xs = prob.vector(x)
    y = prob.matvec(xs).cpu().numpy().astype(complex)
    xh = xs.cpu().numpy().astype(complex)
    nbr = O.neighbour_table(CFG.n_coarse)
    need = np.unique(nbr[SAMPLE_CELLS].ravel())
    rows = O.coarse_kernel_block_rows(bs.vecs_coarse, bs.tau, CFG.nv, CFG.nc, CFG.n_coarse, CFG.n_div, CFG, need)
    np_ = CFG.n_pair
    op = O.InterpOperator(Dv, Dc, f, None, delta, CFG.n_coarse, CFG.n_div, CFG.nv, CFG.nc)
    aop = O.InterpOperator(np.abs(Dv).astype(complex), np.abs(Dc).astype(complex), f, None, np.abs(delta),
                           CFG.n_coarse, CFG.n_div, CFG.nv, CFG.nc)
    qbar = op.restrict(xh)
    qabs = aop.restrict(np.abs(xh))
    r = np.zeros((3, CFG.n_trans_coarse), dtype=complex)
    rabs = np.zeros((3, CFG.n_trans_coarse), dtype=complex)
    for i, k in enumerate(need):
        r[:, k * np_:(k + 1) * np_] = (rows[i] @ qbar.T).T
        rabs[:, k * np_:(k + 1) * np_] = (np.abs(rows[i]) @ np.abs(qabs).T).T
    ref = delta[None] * xh + op.prolong(r)
    bound = U32 * (10 * np.abs(delta)[None] * np.abs(xh) + fp32_kernel_factors(True) * np.abs(aop.prolong(rabs)))
    ndiv3 = CFG.n_div3
    for cell in SAMPLE_CELLS:
        sl = slice(cell * ndiv3 * np_, (cell + 1) * ndiv3 * np_)
        assert np.all(np.abs(y[:, sl] - ref[:, sl]) <= bound[:, sl]), f"cell {cell}"
        assert rel_l2(y[:, sl], ref[:, sl]) < 2e-6
    prob.close()


def test_c2_bf16_operator_adjoint_at_full_size(c2):
    """The block-scaled kernel is exactly Hermitian (a block and its mirror share their
    scale, and rounding commutes with conjugation); the applied operator is
    self-adjoint to the accuracy of the format's product."""
    bs, prob = c2
    x = ti.random_vectors(CFG.n_trans, 3, 402)
    z = ti.random_vectors(CFG.n_trans, 3, 403)
    x, z = (v / np.linalg.norm(v, axis=1, keepdims=True) for v in (x, z))
    xs, zs = prob.vector(x), prob.vector(z)
    hx = prob.matvec(xs).to(torch.complex128)
    hz = prob.matvec(zs).to(torch.complex128)
    x64, z64 = xs.to(torch.complex128), zs.to(torch.complex128)
    lhs = (x64.conj() * hz).sum(dim=1)
    rhs = (hx.conj() * z64).sum(dim=1)
    scale = (x64.abs() * hz.abs()).sum(dim=1)
    assert torch.all((lhs - rhs).abs() <= 4 * U_BF16 ** 2 * scale + 64 * U32 * scale)
