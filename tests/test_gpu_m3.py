"""GPU parity of Method 3 (Sec. 4; the divergence of Eq. (diverg) treated in a band
||k - k'|| <= w d): the coarse coefficient a_c, the band blocks Delta(k, k + o), the
M3 matvec and the M3 Haydock chain, against the FP64 oracle."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import tbinputs as ti

from _cases import bands, oracle_operator, oracle_parts, rel_l2
from _gpu import FP32_INNER_UNITS, PACKED_PRODUCT_UNITS, U32, U64, abs_operator

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CHUNK = 16   # offsets per chunk of the library's band layout


@pytest.fixture(scope="module")
def bse():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_01863_amd import bse as mod
    return mod


def _shape(cfg):
    k2 = O.screening_kappa2(cfg.eps_inf, cfg.lam)
    return k2, O.s_q0_average(cfg.n_coarse, cfg.n_div, k2, cfg.q0_quad)


def _oracle_m3(cfg, weights="trilinear"):
    bs = bands(cfg)
    op = oracle_operator(cfg, weights)
    a = O.divergence_coefficient(bs.vecs_coarse, bs.tau, cfg.nv, cfg.nc, cfg.n_coarse, cfg.n_div, cfg)
    k2, s0 = _shape(cfg)
    return op, a, O.coarse_shape(cfg.n_coarse, k2, s0), k2, s0


def _gpu_blocks(prob, n_off):
    """Library band buffer -> [N_k, n_off, np, np] complex128.  Layout: per k, chunks
    of CHUNK offsets (the last one narrower; offsets padded to an even count), and
    inside a chunk of width W, row n holds its W np entries (o_local, m)."""
    npair = prob.dims.nv * prob.dims.nc
    n_pad = (n_off + 1) // 2 * 2
    start = (n_pad * 16 + 255) // 256 * 256
    esz = 16 if prob.mat_dtype == torch.complex128 else 8
    nbytes = prob.nk * n_pad * npair * npair * esz
    raw = prob.band[start:start + nbytes].cpu().numpy()
    arr = raw.view(np.complex128 if esz == 16 else np.complex64).astype(np.complex128)
    arr = arr.reshape(prob.nk, n_pad * npair * npair)
    out = np.empty((prob.nk, n_pad, npair, npair), dtype=np.complex128)
    for c0 in range(0, n_pad, CHUNK):
        W = min(CHUNK, n_pad - c0)
        chunk = arr[:, c0 * npair * npair:(c0 + W) * npair * npair].reshape(prob.nk, npair, W, npair)
        out[:, c0:c0 + W] = chunk.transpose(0, 2, 1, 3)
    return out[:, :n_off]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_divergence_coefficient_matches_oracle(bse, dtype):
    cfg = ti.get_config("c0")
    op, a, *_ = _oracle_m3(cfg)
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype=dtype, max_rhs=1)
    prob.set_m3(1.0)
    g = prob.a_coef.cpu().numpy().astype(np.complex128)
    scale = np.abs(a).max()
    if dtype == "f64":
        assert np.abs(g - a).max() <= 1e-14 * scale
    else:
        assert np.all(np.abs(g - a) <= U32 * np.abs(a) * 1.01 + 1e-14 * scale)
    assert np.abs(g - g.conj().T).max() == 0.0
    prob.close()


@pytest.mark.parametrize("w", [1.0, 0.5])
def test_band_blocks_match_oracle(bse, w):
    """Every block Delta(k, k + o) of sampled dense points (C0, FP64)."""
    cfg = ti.get_config("c0")
    op, a, Sc, k2, s0 = _oracle_m3(cfg)
    off = O.m3.band_offsets(cfg.n_div, w)
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f64", max_rhs=1)
    prob.set_m3(w)
    assert prob.m3_offsets == len(off)
    gb = _gpu_blocks(prob, len(off))
    ks = np.random.default_rng(3).choice(op.nk, 24, replace=False)
    ref = O.m3.band_blocks(op, a, Sc, off, O.m3.dense_shape(off, cfg.n_coarse, cfg.n_div, k2, s0), ks)
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(gb[ks] - ref).max() <= 1e-13 * scale
    prob.close()


@pytest.mark.parametrize("weights", ["trilinear", "nearest"])
def test_m3_matvec_fp64_matches_explicit_kernel(bse, weights):
    """C0 (N = 4 608): library matvec with the band = (diag + K^{M3}) x, K^{M3} written
    out by the oracle as defined."""
    cfg = ti.get_config("c0")
    op, a, Sc, k2, s0 = _oracle_m3(cfg, weights)
    K3 = O.m3.explicit_kernel(op, a, Sc, 1.0, k2, s0)
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f64", max_rhs=2,
                                  neighbours=8 if weights == "trilinear" else 1)
    prob.set_m3(1.0)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(2, op.N)) + 1j * rng.normal(size=(2, op.N))
    y = prob.matvec(x).cpu().numpy()
    ref = op.delta[None, :] * x + (K3 @ x.T).T
    assert rel_l2(y, ref) < 1e-13
    assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()
    # the band is not a no-op, and detaching it gives Method 1 back
    y1 = op.apply(x)
    assert rel_l2(y1, ref) > 1e-3
    prob.set_m3(None)
    assert rel_l2(prob.matvec(x).cpu().numpy(), y1) < 1e-13
    prob.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_m3_any_band_counts(bse, dtype):
    """A band pair without a compiled form (2v5c): the run-time band product.  FP64: the
    library matvec against (diag + K^{M3}) x with K^{M3} written out by the oracle; FP32
    storage: within the rounding bound of the test below."""
    cfg = ti.tiny_config(n_coarse=3, n_div=2, nv=2, nc=5, n_orb=7, seed=25, n_pol=2)
    op, a, Sc, k2, s0 = _oracle_m3(cfg)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(2, op.N)) + 1j * rng.normal(size=(2, op.N))
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype=dtype, max_rhs=2)
    prob.set_m3(1.0)
    if dtype == "f64":
        K3 = O.m3.explicit_kernel(op, a, Sc, 1.0, k2, s0)
        ref = op.delta[None, :] * x + (K3 @ x.T).T
        y = prob.matvec(x).cpu().numpy()
        assert rel_l2(y, ref) < 1e-13
        assert rel_l2(op.apply(x), ref) > 1e-3   # the band is not a no-op
    else:
        x = x.astype(np.complex64).astype(np.complex128)
        off = O.m3.band_offsets(cfg.n_div, 1.0)
        sd = O.m3.dense_shape(off, cfg.n_coarse, cfg.n_div, k2, s0)
        ref = O.m3.apply(op, O.m3.band_blocks(op, a, Sc, off, sd), off, x)
        aop = abs_operator(op)
        ablocks = O.m3.band_blocks(aop, np.abs(a).astype(complex), Sc, off, sd, absolute=True)
        bound = 10 * U32 * np.abs(O.m3.apply(aop, ablocks, off, np.abs(x))) \
            + (FP32_INNER_UNITS + PACKED_PRODUCT_UNITS) * U32 * np.abs(aop.apply_kernel(np.abs(x)))
        y = prob.matvec(x).cpu().numpy().astype(np.complex128)
        assert np.all(np.abs(y - ref) <= bound + 1e-300)
    prob.close()


@pytest.mark.parametrize("cfg,w", [
    (ti.tiny_config(n_coarse=3, n_div=2, nv=3, nc=6, n_orb=9, seed=21, n_pol=3), 1.0),
    (ti.tiny_config(n_coarse=2, n_div=3, nv=2, nc=3, n_orb=6, seed=22, n_pol=2), 0.7),
], ids=["3v6c", "2v3c_ndiv3"])
def test_m3_matvec_fp32_within_rounding_bound(bse, cfg, w):
    """FP32 storage: every output within 10 FP32 units of the sum of |terms| of the
    Method 1 product and of the band (each band term is a product of at most 8 stored
    or rounded factors: x, four overlaps, a_c, the block, the output), plus the FP32
    arithmetic of the restrict, prolong and packed coarse product on the Method 1 kernel
    terms."""
    op, a, Sc, k2, s0 = _oracle_m3(cfg)
    off = O.m3.band_offsets(cfg.n_div, w)
    sd = O.m3.dense_shape(off, cfg.n_coarse, cfg.n_div, k2, s0)
    blocks = O.m3.band_blocks(op, a, Sc, off, sd)
    rng = np.random.default_rng(5)
    x = (rng.normal(size=(cfg.n_pol, op.N)) + 1j * rng.normal(size=(cfg.n_pol, op.N))).astype(np.complex64)
    x = x.astype(np.complex128)
    ref = O.m3.apply(op, blocks, off, x)
    aop = abs_operator(op)
    ablocks = O.m3.band_blocks(aop, np.abs(a).astype(complex), Sc, off, sd, absolute=True)
    bound = 10 * U32 * np.abs(O.m3.apply(aop, ablocks, off, np.abs(x))) \
        + (FP32_INNER_UNITS + PACKED_PRODUCT_UNITS) * U32 * np.abs(aop.apply_kernel(np.abs(x)))
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f32", max_rhs=cfg.n_pol)
    prob.set_m3(w)
    y = prob.matvec(x).cpu().numpy().astype(np.complex128)
    assert np.all(np.abs(y - ref) <= bound + 1e-300)
    prob.close()


def test_m3_haydock_c0_matches_oracle(bse):
    """Chains of H^{M3} (C0, FP64, w = 1): the well-conditioned head of the chain and
    eps2 at broadenings where 200 steps have converged (the same criteria as the
    Method 1 chain)."""
    cfg = ti.get_config("c0")
    op, a, Sc, k2, s0 = _oracle_m3(cfg)
    K3 = O.m3.explicit_kernel(op, a, Sc, 1.0, k2, s0)
    H = np.diag(op.delta).astype(complex) + K3
    bs = bands(cfg)
    P = bs.P_flat()[:1]
    och = O.haydock(lambda v: (H @ v.T).T, P, cfg.steps)
    ra, rb, rpn = och["a"], och["b"], och["pnorm2"]
    prob = bse.problem_from_bands(bs, cfg, dtype="f64", max_rhs=1)
    prob.set_m3(1.0)
    ch = prob.haydock(P, cfg.steps)
    ga, gb = ch["a"].cpu().numpy(), ch["b"].cpu().numpy()
    assert int(ch["steps"][0]) == cfg.steps and int(ch["status"][0]) == bse.BSE_OK
    assert rel_l2(ga[0, :20], ra[0, :20]) < 1e-10
    assert rel_l2(gb[0, 1:21], rb[0, 1:21]) < 1e-10
    om, C = cfg.omega(), cfg.prefactor()
    for eta in (0.3, 0.5):
        e_ref = O.continued_fraction(ra, rb, rpn, C, om, eta)
        e_gpu = prob.continued_fraction(ch, C, om, eta).cpu().numpy()
        assert rel_l2(e_gpu.imag, e_ref.imag) < 1e-10
    # Method 3 moves the spectrum against Method 1 (the band matters at this size)
    ch1 = O.haydock(op.apply, P, cfg.steps)
    e1 = O.continued_fraction(ch1["a"], ch1["b"], ch1["pnorm2"], C, om, 0.3)
    assert rel_l2(O.continued_fraction(ra, rb, rpn, C, om, 0.3).imag, e1.imag) > 1e-3
    prob.close()


def test_m3_operator_hermitian_at_full_size(bse):
    """C1 size (N = 589 824, 3 right-hand sides, FP32, w = 1: 257 offsets, a 23 GB
    band): <x | H y> = <H x | y> for random x, y to FP32 accuracy, and the band
    changes the product."""
    cfg = ti.get_config("c1")
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f32", max_rhs=3)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(3, prob.N)) + 1j * rng.normal(size=(3, prob.N))
    yv = rng.normal(size=(3, prob.N)) + 1j * rng.normal(size=(3, prob.N))
    h1x = prob.matvec(x).cpu().numpy().astype(np.complex128)
    prob.set_m3(1.0)
    assert prob.m3_offsets == 257
    hx = prob.matvec(x).cpu().numpy().astype(np.complex128)
    hy = prob.matvec(yv).cpu().numpy().astype(np.complex128)
    xs = x.astype(np.complex64).astype(np.complex128)
    ys = yv.astype(np.complex64).astype(np.complex128)
    lhs = np.sum(xs.conj() * hy, axis=1)
    rhs = np.sum(hx.conj() * ys, axis=1)
    mag = np.sum(np.abs(xs) * np.abs(hy), axis=1)
    assert np.all(np.abs(lhs - rhs) < 1e-5 * mag)
    assert rel_l2(hx, h1x) > 1e-4
    prob.close()


@pytest.mark.parametrize("n_c,dtype,steps", [(4, "f64", 200), (8, "f32", 400)], ids=["4^3x2", "8^3x2"])
def test_library_m3_closer_than_m1_to_the_dense_mesh(bse, n_c, dtype, steps):
    """The comparison of Sec. 5 through the library: eps2 from M1 and from M3 (w = 1)
    on an n_c^3 x 2 double grid against the BSE built directly on the (2 n_c)^3 dense
    mesh (one division: no interpolation; 36 864 transitions for n_c = 8, a 10.9 GB
    kernel).  Chains of `steps` steps, eta = 0.2 eV; C0 crystal (seed 0, 3v3c)."""
    import time
    cfg = ti.get_config("c0").with_(n_coarse=n_c, steps=steps)
    cfg_d = cfg.with_(n_coarse=2 * n_c, n_div=1)
    om, C, eta = cfg.omega(), cfg.prefactor(), 0.2
    assert abs(cfg_d.prefactor() - C) < 1e-15 * C
    out = {}
    for name, c, w in (("dense", cfg_d, None), ("M1", cfg, None), ("M3", cfg, 1.0)):
        bs = bands(c)
        prob = bse.problem_from_bands(bs, c, dtype=dtype, max_rhs=1)
        if w is not None:
            prob.set_m3(w)
        P = bs.P_flat()[:1]
        prob.haydock(P, 5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch = prob.haydock(P, steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        assert int(ch["status"][0]) == bse.BSE_OK
        out[name] = (prob.continued_fraction(ch, C, om, eta).cpu().numpy().imag[0], dt)
        prob.close()
    ref = out["dense"][0]
    e1, e3 = rel_l2(out["M1"][0], ref), rel_l2(out["M3"][0], ref)
    print(f"\n{n_c}^3 x 2 ({dtype}): eps2 error vs dense mesh M1 {e1:.4f} M3 {e3:.4f}; ms/step dense "
          f"{1e3 * out['dense'][1]:.3f} M1 {1e3 * out['M1'][1]:.3f} M3 {1e3 * out['M3'][1]:.3f}")
    assert e3 < 0.7 * e1


@pytest.mark.parametrize("w", [0.0, 1.5], ids=["diagonal_only", "widest"])
def test_m3_band_edge_widths(bse, w):
    """w = 0: the band is the diagonal block alone (one offset, padded to two with a
    zero block); w = 1.5 on the 8^3 dense mesh of C0: 123 offsets, the widest band
    that does not reach round the mesh (2 floor(w n_div) = 6 < 8), several full
    chunks and a short last one.  FP64 matvec against the explicit kernel."""
    cfg = ti.get_config("c0")
    op, a, Sc, k2, s0 = _oracle_m3(cfg)
    K3 = O.m3.explicit_kernel(op, a, Sc, w, k2, s0)
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f64", max_rhs=1)
    prob.set_m3(w)
    assert prob.m3_offsets == len(O.m3.band_offsets(cfg.n_div, w))
    x = ti.random_vectors(op.N, 1, 77)
    y = prob.matvec(x).cpu().numpy()
    ref = op.delta[None, :] * x + (K3 @ x.T).T
    assert rel_l2(y, ref) < 1e-13
    prob.close()


def test_m3_rejects_a_band_that_wraps(bse):
    cfg = ti.get_config("c0")
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype="f64", max_rhs=1)
    with pytest.raises(bse.BSEError):
        prob.set_m3(2.0)   # 2 floor(w n_div) = 8 reaches the 8^3 dense mesh
    prob.close()


@pytest.mark.parametrize("dtype", ["f32v64", "bf16"])
def test_m3_with_other_storage_forms(bse, dtype):
    """The band with FP64 Lanczos vectors (FP32 band blocks, FP64 x) and with the
    block-scaled BF16 coarse kernel (FP32 band blocks): relative L2 against the FP64
    oracle within the storage form's rounding (FP32: 1e-6; BF16 kernel: 2 BF16 units on
    the whole product)."""
    cfg = ti.tiny_config(n_coarse=3, n_div=2, nv=3, nc=6, n_orb=9, seed=21, n_pol=3)
    op, a, Sc, k2, s0 = _oracle_m3(cfg)
    off = O.m3.band_offsets(cfg.n_div, 1.0)
    blocks = O.m3.band_blocks(op, a, Sc, off, O.m3.dense_shape(off, cfg.n_coarse, cfg.n_div, k2, s0))
    x = ti.random_vectors(op.N, 3, 88)
    x = x / np.linalg.norm(x, axis=1, keepdims=True)
    prob = bse.problem_from_bands(bands(cfg), cfg, dtype=dtype, max_rhs=3)
    prob.set_m3(1.0)
    xs = prob.vector(x)
    y = prob.matvec(xs).cpu().numpy().astype(np.complex128)
    ref = O.m3.apply(op, blocks, off, xs.cpu().numpy().astype(np.complex128))
    tol = 1e-6 if dtype == "f32v64" else 2 * 2.0 ** -8
    assert rel_l2(y, ref) < tol
    prob.close()
