"""The C-ABI library loads and exports what include/bse_dg.h declares; host-side
argument checks reject bad input before any device work (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bse_dg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bse_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def bse():
    from paper_1602_01863_amd import bse as mod
    return mod


def test_every_declared_symbol_is_exported(bse):
    names = _declared()
    assert len(names) >= 15
    lib = bse.library()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(bse.EXPORTED) == names


def test_version_and_sizes(bse):
    assert "gfx950" in bse.bse_version()
    d = bse.Dims(8, 4, 3, 6, 9, 3, bse.BSE_F32, 8)
    assert bse.bse_coarse_kernel_bytes(d) == 9216 * 9216 * 8
    assert bse.bse_overlaps_bytes(d) == 512 * 8 * 45 * 64 * 8
    assert bse.bse_workspace_bytes(d) > 2 * 589824 * 3 * 8
    d64 = bse.Dims(4, 2, 3, 3, 6, 1, bse.BSE_F64, 8)
    assert bse.bse_coarse_kernel_bytes(d64) == 576 * 576 * 16


@pytest.mark.parametrize("fields", [
    dict(n_coarse=0), dict(n_div=0), dict(nv=0), dict(max_rhs=0), dict(max_rhs=5),
    dict(dtype=7), dict(neighbours=4),
])
def test_invalid_dims_rejected(bse, fields):
    base = dict(n_coarse=4, n_div=2, nv=3, nc=3, n_orb=6, max_rhs=1, dtype=0, neighbours=8)
    base.update(fields)
    d = bse.Dims(**base)
    assert bse.bse_workspace_bytes(d) == 0
    assert bse.library().bse_last_error().decode() != ""


def test_plan_create_checks_before_device_work(bse):
    lib = bse.library()
    d = bse.Dims(4, 2, 3, 3, 6, 1, bse.BSE_F64, 8)
    plan = ctypes.c_void_p()
    # NULL inputs
    st = lib.bse_plan_create(ctypes.byref(d), None, None, None, None, 0, None, ctypes.byref(plan))
    assert st == bse.BSE_ERR_INVALID_ARG
    # band counts beyond what the hot path takes (nv nc = 35 > 32; nv + nc = 17 > 16)
    for nv, nc in [(5, 7), (1, 16)]:
        d2 = bse.Dims(4, 2, nv, nc, nv + nc, 1, bse.BSE_F64, 8)
        st = lib.bse_plan_create(ctypes.byref(d2), 1, 1, 1, 256, 1 << 30, None, ctypes.byref(plan))
        assert st == bse.BSE_ERR_UNSUPPORTED
    # a pair without a compiled form but in range passes the band check (and stops at the
    # short workspace, before any device work)
    d3 = bse.Dims(4, 2, 2, 5, 7, 1, bse.BSE_F32, 8)
    st = lib.bse_plan_create(ctypes.byref(d3), 1, 1, 1, 256, 16, None, ctypes.byref(plan))
    assert st == bse.BSE_ERR_WORKSPACE
    # misaligned or short workspace
    st = lib.bse_plan_create(ctypes.byref(d), 1, 1, 1, 8, 1 << 30, None, ctypes.byref(plan))
    assert st == bse.BSE_ERR_WORKSPACE
    st = lib.bse_plan_create(ctypes.byref(d), 1, 1, 1, 256, 16, None, ctypes.byref(plan))
    assert st == bse.BSE_ERR_WORKSPACE
    assert not plan.value


def test_other_entry_points_check_arguments(bse):
    lib = bse.library()
    assert lib.bse_interp_matvec(None, None, None, 1, None) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_haydock_run(None, None, 1, 1, None, None, None, None, None, None) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_continued_fraction(1, 1, 10, 5, 1, 1, 1, 1.0, 1, 1, 0.1, 1, 1, None) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_continued_fraction(1, 1, 10, 11, 1, 1, 1, 1.0, 1, 1, 0.0, 1, 1, None) == bse.BSE_ERR_INVALID_ARG
    d = bse.Dims(4, 2, 3, 3, 6, 1, bse.BSE_F64, 8)
    m = bse.KernelModel(12.0, 0.3, 6.0, 9, 16)
    assert lib.bse_build_coarse_kernel(ctypes.byref(d), 1, 1, ctypes.byref(m), 1, None) == bse.BSE_ERR_INVALID_ARG
    d_big = bse.Dims(4, 2, 3, 6, 20, 1, bse.BSE_F64, 8)
    m = bse.KernelModel(12.0, 0.3, 6.0, 4, 16)
    assert lib.bse_build_coarse_kernel(ctypes.byref(d_big), 1, 1, ctypes.byref(m), 1, None) == bse.BSE_ERR_UNSUPPORTED
    assert lib.bse_plan_set_gemv_splits(None, 4) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_plan_set_restrict_group(None, 1) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_plan_set_coarse_product(None, 0) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_plan_set_converge_closure(None, 16) == bse.BSE_ERR_INVALID_ARG
    # converged chains: NULL plan, then NULL outputs, before any device work
    conv = [1, 3, 100, 20, 1.0, 1, 10, 0.1, 1e-3] + [1] * 7 + [None]
    assert lib.bse_haydock_converge(None, *conv) == bse.BSE_ERR_INVALID_ARG
    conv_null_eps = conv[:14] + [None, None, None]
    assert lib.bse_haydock_converge(1, *conv_null_eps) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_batch_launch(None, None) == bse.BSE_ERR_INVALID_ARG


def test_m3_band_geometry_and_checks(bse):
    """Band offsets |o|^2 <= (w n_div)^2 and the buffer size; widths that reach round
    the periodic mesh, or an unsupported pair count, are rejected on the host."""
    lib = bse.library()
    d = bse.Dims(8, 4, 3, 6, 9, 3, bse.BSE_F32, 8)
    n, nbytes = bse.bse_m3_band_info(d, 1.0)
    assert n == 257
    # table (258 offsets, padded to even, rounded to 256 bytes) + blocks (32768 x 258 x 18 x 18
    # complex FP32) + product (3 x N FP64 complex)
    assert nbytes == 4352 + 32768 * 258 * 324 * 8 + 3 * 589824 * 16
    assert bse.bse_m3_band_info(d, 0.5)[0] == 33 and bse.bse_m3_band_info(d, 0.0)[0] == 1
    n32 = ctypes.c_int32()
    nb = ctypes.c_size_t()
    assert lib.bse_m3_band_info(ctypes.byref(d), 4.0, ctypes.byref(n32), ctypes.byref(nb)) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_m3_band_info(ctypes.byref(d), -1.0, ctypes.byref(n32), ctypes.byref(nb)) == bse.BSE_ERR_INVALID_ARG
    small = bse.Dims(2, 2, 1, 1, 2, 1, bse.BSE_F64, 8)   # dense mesh 4: floor(w n_div) must stay below 2
    assert lib.bse_m3_band_info(ctypes.byref(small), 1.0, ctypes.byref(n32), ctypes.byref(nb)) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_m3_band_info(ctypes.byref(small), 0.5, ctypes.byref(n32), ctypes.byref(nb)) == bse.BSE_OK
    m = bse.KernelModel(12.0, 0.3, 6.0, 4, 16)
    assert lib.bse_build_m3_band(ctypes.byref(d), None, 1, ctypes.byref(m), 1.0, 256, 1 << 40, None) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_build_m3_band(ctypes.byref(d), 1, 1, ctypes.byref(m), 1.0, 256, 16, None) == bse.BSE_ERR_WORKSPACE
    assert lib.bse_build_m3_band(ctypes.byref(d), 1, 1, ctypes.byref(m), 1.0, 8, 1 << 40, None) == bse.BSE_ERR_WORKSPACE
    assert lib.bse_plan_set_m3_band(None, None, 1.0) == bse.BSE_ERR_INVALID_ARG
    assert lib.bse_build_divergence_coefficient(ctypes.byref(d), None, 1, ctypes.byref(m), 1, None) == bse.BSE_ERR_INVALID_ARG



def test_noalloc_backward_rejects_oversized_calls_before_device_work(bse):
    lib = bse.library()
    # non-NULL dummy pointers: the size check comes before any device call
    st = lib.bse_dense_backward_noalloc(8, 8, 8, 8, 8, 8, 8, (1 << 20) // 64 + 1, 8, 64, bse.BSE_ACT_GELU, None)
    assert st == bse.BSE_ERR_WORKSPACE
    st = lib.bse_dense_backward_noalloc(None, 8, 8, 8, 8, 8, 8, 4, 8, 64, bse.BSE_ACT_GELU, None)
    assert st == bse.BSE_ERR_INVALID_ARG
