"""bse_dense_backward_noalloc: the backward pass of a dense layer with dz kept in the
library's own device array, checked through the C ABI against bse_dense_backward with
a caller-owned buffer (same kernels, so the results must agree bit for bit), on
consecutive calls whose sizes shrink, so that a stale scratch tail would show."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LIMIT = 1 << 20   # entries of batch * n_out the scratch array holds


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_01863_amd import bse as mod
    return mod, mod.library()


def _layer(batch, n_in, n_out, seed):
    g = torch.Generator().manual_seed(seed)
    dev = torch.device("cuda", 0)
    x = torch.randn(batch, n_in, generator=g).to(dev)
    W = (torch.randn(n_out, n_in, generator=g) / n_in ** 0.5).to(dev)
    z = torch.randn(batch, n_out, generator=g).to(dev)
    dy = torch.randn(batch, n_out, generator=g).to(dev)
    return x, W, z, dy


def _call(mod, lib, name, x, W, z, dy, act, work=None):
    batch, n_in = x.shape
    n_out = W.shape[0]
    dev = x.device
    dx = torch.full((batch, n_in), float("nan"), device=dev)
    dW = torch.full((n_out, n_in), float("nan"), device=dev)
    db = torch.full((n_out,), float("nan"), device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = [x.data_ptr(), W.data_ptr(), z.data_ptr(), dy.data_ptr(), dx.data_ptr(), dW.data_ptr(), db.data_ptr(),
            batch, n_in, n_out, act]
    if work is not None:
        args.append(work.data_ptr())
    st = getattr(lib, name)(*args, stream)
    assert st == mod.BSE_OK, lib.bse_last_error().decode()
    torch.cuda.synchronize()
    return dx.cpu().numpy(), dW.cpu().numpy(), db.cpu().numpy()


def test_noalloc_backward_matches_the_workspace_call(lib):
    mod, L = lib
    # the largest call the scratch holds, then smaller ones (GELU and linear)
    cases = [(2048, 32, 512, mod.BSE_ACT_GELU, 1), (300, 128, 386, mod.BSE_ACT_GELU, 2),
             (37, 96, 128, mod.BSE_ACT_NONE, 3)]
    assert cases[0][0] * cases[0][2] == LIMIT
    for batch, n_in, n_out, act, seed in cases:
        x, W, z, dy = _layer(batch, n_in, n_out, seed)
        work = torch.full((batch, n_out), float("nan"), device=x.device)
        ref = _call(mod, L, "bse_dense_backward", x, W, z, dy, act, work)
        got = _call(mod, L, "bse_dense_backward_noalloc", x, W, z, dy, act)
        for r, g in zip(ref, got):
            assert np.all(np.isfinite(r))
            assert np.array_equal(r, g), (batch, n_in, n_out)


def test_noalloc_backward_rejects_a_call_past_the_scratch(lib):
    mod, L = lib
    x, W, z, dy = _layer(LIMIT // 64 + 1, 8, 64, 4)
    out = [torch.zeros(1, device=x.device) for _ in range(3)]
    st = L.bse_dense_backward_noalloc(x.data_ptr(), W.data_ptr(), z.data_ptr(), dy.data_ptr(), out[0].data_ptr(),
                                      out[1].data_ptr(), out[2].data_ptr(), x.shape[0], 8, 64, mod.BSE_ACT_GELU,
                                      None)
    assert st == mod.BSE_ERR_WORKSPACE
    assert "scratch" in L.bse_last_error().decode()
