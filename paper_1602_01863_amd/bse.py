"""Python binding of libbse_dg.so (ctypes).

Functions named like the C entry points marshal torch device tensors into raw
pointers and call the library; they compute nothing themselves.  Device memory
and streams come from PyTorch.  ``BSEProblem`` wires the setup calls, the plan
and its workspace together for one Hamiltonian.

The library must have been built (``__graft_entry__.build()`` or
``python -m paper_1602_01863_amd.build``); importing this module without it
raises, there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbse_dg.so")

BSE_OK = 0
BSE_INFO_INVARIANT_SUBSPACE = 1
BSE_INFO_ZERO_START = 2
BSE_ERR_INVALID_ARG = -1
BSE_ERR_HIP = -2
BSE_ERR_NONFINITE = -3
BSE_ERR_UNSUPPORTED = -4
BSE_ERR_WORKSPACE = -5

BSE_F64, BSE_F32, BSE_F32_VEC64, BSE_BF16_KC, BSE_F16_KC = 0, 1, 2, 3, 4
DTYPES = {"f64": BSE_F64, "f32": BSE_F32, "f32v64": BSE_F32_VEC64, "bf16": BSE_BF16_KC, "f16": BSE_F16_KC}

# symbols declared in include/bse_dg.h
EXPORTED = [
    "bse_version", "bse_last_error", "bse_workspace_bytes", "bse_coarse_kernel_bytes",
    "bse_overlaps_bytes", "bse_build_overlaps", "bse_build_transition_energies",
    "bse_build_coarse_kernel", "bse_plan_create", "bse_plan_destroy", "bse_interp_matvec",
    "bse_haydock_run", "bse_haydock_converge", "bse_continued_fraction", "bse_plan_set_timing", "bse_plan_get_timing",
    "bse_plan_set_gemv_splits", "bse_plan_set_coarse_product", "bse_plan_set_converge_closure",
    "bse_plan_set_restrict_group", "bse_batch_create", "bse_batch_launch",
    "bse_batch_destroy", "bse_dense_forward", "bse_dense_backward", "bse_dense_backward_noalloc", "bse_mse_loss", "bse_adam_step",
    "bse_to_bf16", "bse_dense_forward_bf16", "bse_continued_fraction_terminated",
    "bse_build_divergence_coefficient", "bse_m3_band_info", "bse_build_m3_band", "bse_plan_set_m3_band",
]
BSE_ACT_NONE, BSE_ACT_GELU = 0, 1


class BSEError(RuntimeError):
    pass


class Dims(ctypes.Structure):
    _fields_ = [("n_coarse", ctypes.c_int32), ("n_div", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("nc", ctypes.c_int32), ("n_orb", ctypes.c_int32), ("max_rhs", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("neighbours", ctypes.c_int32)]


class KernelModel(ctypes.Structure):
    _fields_ = [("eps_inf", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("kernel_energy", ctypes.c_double), ("g2_max", ctypes.c_int32),
                ("q0_quad", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise BSEError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "bse_version": (ctypes.c_char_p, []),
        "bse_last_error": (ctypes.c_char_p, []),
        "bse_workspace_bytes": (sz, [P(Dims)]),
        "bse_coarse_kernel_bytes": (sz, [P(Dims)]),
        "bse_overlaps_bytes": (sz, [P(Dims)]),
        "bse_build_overlaps": (i32, [P(Dims), vp, vp, vp, vp]),
        "bse_build_transition_energies": (i32, [P(Dims), vp, vp, vp]),
        "bse_build_coarse_kernel": (i32, [P(Dims), vp, vp, P(KernelModel), vp, vp]),
        "bse_plan_create": (i32, [P(Dims), vp, vp, vp, vp, sz, vp, P(vp)]),
        "bse_plan_destroy": (None, [vp]),
        "bse_interp_matvec": (i32, [vp, vp, vp, i32, vp]),
        "bse_haydock_run": (i32, [vp, vp, i32, i32, vp, vp, vp, vp, vp, vp]),
        "bse_haydock_converge": (i32, [vp, vp, i32, i32, i32, dbl, vp, i32, dbl, dbl, vp, vp, vp, vp, vp, vp, vp,
                                         vp]),
        "bse_continued_fraction": (i32, [vp, vp, i32, i32, vp, vp, i32, dbl, vp, i32, dbl, vp, vp, vp]),
        "bse_plan_set_timing": (i32, [vp, i32]),
        "bse_plan_get_timing": (i32, [vp, P(dbl), P(i64)]),
        "bse_plan_set_gemv_splits": (i32, [vp, i32]),
        "bse_plan_set_coarse_product": (i32, [vp, i32]),
        "bse_plan_set_converge_closure": (i32, [vp, i32]),
        "bse_plan_set_restrict_group": (i32, [vp, i32]),
        "bse_batch_create": (i32, [P(vp), i32, P(vp), P(i32), i32, P(vp), P(vp), P(vp), P(vp), P(vp), i32, P(vp)]),
        "bse_batch_launch": (i32, [vp, vp]),
        "bse_batch_destroy": (None, [vp]),
        "bse_dense_forward": (i32, [vp, vp, vp, vp, vp, i32, i32, i32, i32, vp]),
        "bse_dense_backward": (i32, [vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp]),
        "bse_dense_backward_noalloc": (i32, [vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp]),
        "bse_mse_loss": (i32, [vp, vp, vp, vp, i64, vp]),
        "bse_adam_step": (i32, [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, i32, vp]),
        "bse_to_bf16": (i32, [vp, vp, i64, vp]),
        "bse_dense_forward_bf16": (i32, [vp, vp, vp, vp, vp, i32, i32, i32, i32, vp]),
        "bse_continued_fraction_terminated": (i32, [vp, vp, i32, i32, i32, vp, vp, vp, i32, dbl, vp, i32, dbl,
                                                    vp, vp, vp]),
        "bse_build_divergence_coefficient": (i32, [P(Dims), vp, vp, P(KernelModel), vp, vp]),
        "bse_m3_band_info": (i32, [P(Dims), dbl, P(i32), P(sz)]),
        "bse_build_m3_band": (i32, [P(Dims), vp, vp, P(KernelModel), dbl, vp, sz, vp]),
        "bse_plan_set_m3_band": (i32, [vp, vp, dbl]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def library() -> ctypes.CDLL:
    return _lib


def _check(status: int, what: str) -> int:
    if status < 0:
        msg = _lib.bse_last_error().decode(errors="replace")
        raise BSEError(f"{what} failed with status {status}: {msg}")
    return status


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ---- thin wrappers with the C names ---------------------------------------------------
def bse_version() -> str:
    return _lib.bse_version().decode()


def bse_workspace_bytes(dims: Dims) -> int:
    return int(_lib.bse_workspace_bytes(ctypes.byref(dims)))


def bse_coarse_kernel_bytes(dims: Dims) -> int:
    return int(_lib.bse_coarse_kernel_bytes(ctypes.byref(dims)))


def bse_overlaps_bytes(dims: Dims) -> int:
    return int(_lib.bse_overlaps_bytes(ctypes.byref(dims)))


def bse_build_overlaps(dims, vecs_coarse, vecs_dense, d_out, stream=None):
    _check(_lib.bse_build_overlaps(ctypes.byref(dims), _ptr(vecs_coarse), _ptr(vecs_dense), _ptr(d_out),
                                   _stream(stream)), "bse_build_overlaps")


def bse_build_transition_energies(dims, eps_dense, delta_out, stream=None):
    _check(_lib.bse_build_transition_energies(ctypes.byref(dims), _ptr(eps_dense), _ptr(delta_out),
                                              _stream(stream)), "bse_build_transition_energies")


def bse_build_coarse_kernel(dims, vecs_coarse, tau, model: KernelModel, Kc_out, stream=None):
    _check(_lib.bse_build_coarse_kernel(ctypes.byref(dims), _ptr(vecs_coarse), _ptr(tau), ctypes.byref(model),
                                        _ptr(Kc_out), _stream(stream)), "bse_build_coarse_kernel")


def bse_plan_create(dims, Kc, d, delta, workspace, stream=None):
    plan = ctypes.c_void_p()
    _check(_lib.bse_plan_create(ctypes.byref(dims), _ptr(Kc), _ptr(d), _ptr(delta), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream),
                                ctypes.byref(plan)), "bse_plan_create")
    return plan


def bse_plan_destroy(plan):
    _lib.bse_plan_destroy(plan)


def bse_interp_matvec(plan, x, y, n_rhs, stream=None):
    _check(_lib.bse_interp_matvec(plan, _ptr(x), _ptr(y), int(n_rhs), _stream(stream)), "bse_interp_matvec")


def bse_haydock_run(plan, P, n_rhs, n_steps, a, b, pnorm2, steps_done, status, stream=None):
    _check(_lib.bse_haydock_run(plan, _ptr(P), int(n_rhs), int(n_steps), _ptr(a), _ptr(b), _ptr(pnorm2),
                                _ptr(steps_done), _ptr(status), _stream(stream)), "bse_haydock_run")


def bse_haydock_converge(plan, P, n_rhs, max_steps, check_every, prefactor, omega, n_omega, eta, tol, a, b, pnorm2,
                         steps_done, status, eps_re, eps_im, stream=None):
    _check(_lib.bse_haydock_converge(plan, _ptr(P), int(n_rhs), int(max_steps), int(check_every), float(prefactor),
                                     _ptr(omega), int(n_omega), float(eta), float(tol), _ptr(a), _ptr(b),
                                     _ptr(pnorm2), _ptr(steps_done), _ptr(status), _ptr(eps_re), _ptr(eps_im),
                                     _stream(stream)), "bse_haydock_converge")


def bse_continued_fraction(a, b, lda, ldb, pnorm2, steps, n_chains, prefactor, omega, n_omega, eta,
                           eps_re, eps_im, stream=None):
    _check(_lib.bse_continued_fraction(_ptr(a), _ptr(b), int(lda), int(ldb), _ptr(pnorm2), _ptr(steps),
                                       int(n_chains), float(prefactor), _ptr(omega), int(n_omega), float(eta),
                                       _ptr(eps_re), _ptr(eps_im), _stream(stream)), "bse_continued_fraction")


def bse_plan_set_timing(plan, enable):
    """enable: False / 0 off, True / 1 the coarse product, 2 the Method 3 band product."""
    _check(_lib.bse_plan_set_timing(plan, int(enable)), "bse_plan_set_timing")


def bse_plan_get_timing(plan):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.bse_plan_get_timing(plan, ctypes.byref(ms), ctypes.byref(n)), "bse_plan_get_timing")
    return ms.value, n.value


def bse_plan_set_gemv_splits(plan, n_split: int):
    _check(_lib.bse_plan_set_gemv_splits(plan, int(n_split)), "bse_plan_set_gemv_splits")


def bse_plan_set_coarse_product(plan, form: int):
    """0: packed Hermitian tiles (default for the FP32 and FP64 coarse kernels); 1: full stream."""
    _check(_lib.bse_plan_set_coarse_product(plan, int(form)), "bse_plan_set_coarse_product")


def bse_plan_set_converge_closure(plan, k: int):
    """Tail of the fraction in bse_haydock_converge: 0 truncated; k: constant chain of the
    means of the last k coefficients."""
    _check(_lib.bse_plan_set_converge_closure(plan, int(k)), "bse_plan_set_converge_closure")


def bse_plan_set_restrict_group(plan, rhs_per_block: int):
    _check(_lib.bse_plan_set_restrict_group(plan, int(rhs_per_block)), "bse_plan_set_restrict_group")


def bse_batch_create(plans, P_list, n_rhs, n_steps, a, b, pnorm2, steps_done, status, n_branches):
    n = len(plans)
    arr = lambda cls, xs: (cls * n)(*xs)
    vp = ctypes.c_void_p
    batch = ctypes.c_void_p()
    _check(_lib.bse_batch_create(arr(vp, plans), n, arr(vp, [_ptr(t) for t in P_list]),
                                 arr(ctypes.c_int32, [int(r) for r in n_rhs]), int(n_steps),
                                 arr(vp, [_ptr(t) for t in a]), arr(vp, [_ptr(t) for t in b]),
                                 arr(vp, [_ptr(t) for t in pnorm2]), arr(vp, [_ptr(t) for t in steps_done]),
                                 arr(vp, [_ptr(t) for t in status]), int(n_branches), ctypes.byref(batch)),
           "bse_batch_create")
    return batch


def bse_batch_launch(batch, stream=None):
    _check(_lib.bse_batch_launch(batch, _stream(stream)), "bse_batch_launch")


def bse_batch_destroy(batch):
    _lib.bse_batch_destroy(batch)


def default_branches() -> int:
    """Branches of a batch: one per hardware queue the runtime gives this process
    (GPU_MAX_HW_QUEUES, 4 by default), less the one the caller's stream keeps.  With
    more branches than that, two branch streams can share a hardware queue and run one
    after the other (measured: 48-member batch 0.74 s with 4 branches, 0.67 s with 3)."""
    try:
        queues = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    except ValueError:
        queues = 4
    return max(1, min(16, queues - 1))


class BSEBatch:
    """Haydock chains of many problems recorded into HIP graphs, one per branch (bse_batch_*).

    problems: BSEProblem list; P_list: matching [n_rhs, N] start vectors.  The output
    tensors are allocated here and stay attached to the graph; every run() recomputes
    all chains and leaves them in .chains (one dict per problem, as BSEProblem.haydock).
    """

    def __init__(self, problems, P_list, n_steps: int, n_branches: int | None = None):
        if n_branches is None:
            n_branches = default_branches()
        self.problems = list(problems)
        self.P = []
        self.chains = []
        for prob, P in zip(self.problems, P_list):
            P = torch.as_tensor(P)
            if P.dim() == 1:
                P = P[None]
            P = P.to(prob.device).to(torch.complex128).contiguous()
            r, dev = P.shape[0], prob.device
            self.P.append(P)
            self.chains.append(dict(a=torch.empty(r, n_steps, dtype=torch.float64, device=dev),
                                    b=torch.empty(r, n_steps + 1, dtype=torch.float64, device=dev),
                                    pnorm2=torch.empty(r, dtype=torch.float64, device=dev),
                                    steps=torch.empty(r, dtype=torch.int32, device=dev),
                                    status=torch.empty(r, dtype=torch.int32, device=dev)))
        self.n_steps = n_steps
        c = self.chains
        self.batch = bse_batch_create([p.plan for p in self.problems], self.P, [P.shape[0] for P in self.P],
                                      n_steps, [x["a"] for x in c], [x["b"] for x in c], [x["pnorm2"] for x in c],
                                      [x["steps"] for x in c], [x["status"] for x in c], n_branches)

    def run(self, stream=None):
        bse_batch_launch(self.batch, stream)
        return self.chains

    def close(self):
        if getattr(self, "batch", None) is not None:
            torch.cuda.synchronize(self.problems[0].device)   # no launch may still run
            bse_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- learned terminator: network and closed continued fraction -------------------------
def bse_dense_forward(x, W, b, z, y, batch, n_in, n_out, act, stream=None):
    _check(_lib.bse_dense_forward(_ptr(x), _ptr(W), _ptr(b), _ptr(z), _ptr(y), int(batch), int(n_in), int(n_out),
                                  int(act), _stream(stream)), "bse_dense_forward")


def bse_dense_backward(x, W, z, dy, dx, dW, db, batch, n_in, n_out, act, work, stream=None):
    _check(_lib.bse_dense_backward(_ptr(x), _ptr(W), _ptr(z), _ptr(dy), _ptr(dx), _ptr(dW), _ptr(db), int(batch),
                                   int(n_in), int(n_out), int(act), _ptr(work), _stream(stream)),
           "bse_dense_backward")


def bse_dense_backward_noalloc(x, W, z, dy, dx, dW, db, batch, n_in, n_out, act, stream=None):
    _check(_lib.bse_dense_backward_noalloc(_ptr(x), _ptr(W), _ptr(z), _ptr(dy), _ptr(dx), _ptr(dW), _ptr(db),
                                           int(batch), int(n_in), int(n_out), int(act), _stream(stream)),
           "bse_dense_backward_noalloc")


def bse_mse_loss(y, t, dy, loss, n, stream=None):
    _check(_lib.bse_mse_loss(_ptr(y), _ptr(t), _ptr(dy), _ptr(loss), int(n), _stream(stream)), "bse_mse_loss")


def bse_adam_step(p, g, m, v, n, lr, beta1, beta2, eps, t, stream=None):
    _check(_lib.bse_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), int(n), float(lr), float(beta1), float(beta2),
                              float(eps), int(t), _stream(stream)), "bse_adam_step")


def bse_to_bf16(x, y, n, stream=None):
    _check(_lib.bse_to_bf16(_ptr(x), _ptr(y), int(n), _stream(stream)), "bse_to_bf16")


def bse_dense_forward_bf16(x, W, b, y_bf16, y_f32, batch, n_in, n_out, act, stream=None):
    _check(_lib.bse_dense_forward_bf16(_ptr(x), _ptr(W), _ptr(b), _ptr(y_bf16), _ptr(y_f32), int(batch), int(n_in),
                                       int(n_out), int(act), _stream(stream)), "bse_dense_forward_bf16")


def bse_continued_fraction_terminated(a, b, lda, ldb, m, pnorm2, a_inf, b_inf, n_chains, prefactor, omega, n_omega,
                                      eta, eps_re, eps_im, stream=None):
    _check(_lib.bse_continued_fraction_terminated(_ptr(a), _ptr(b), int(lda), int(ldb), int(m), _ptr(pnorm2),
                                                  _ptr(a_inf), _ptr(b_inf), int(n_chains), float(prefactor),
                                                  _ptr(omega), int(n_omega), float(eta), _ptr(eps_re),
                                                  _ptr(eps_im), _stream(stream)),
           "bse_continued_fraction_terminated")


# ---- one Hamiltonian on the device ------------------------------------------------------
# ---- Method 3 (Sec. 4): the divergence treated in a band along the diagonal -----------
def bse_build_divergence_coefficient(dims, vecs_coarse, tau, model: KernelModel, a_out, stream=None):
    _check(_lib.bse_build_divergence_coefficient(ctypes.byref(dims), _ptr(vecs_coarse), _ptr(tau),
                                                 ctypes.byref(model), _ptr(a_out), _stream(stream)),
           "bse_build_divergence_coefficient")


def bse_m3_band_info(dims, w: float):
    """(number of band offsets, bytes of the band buffer)."""
    n = ctypes.c_int32(0)
    nb = ctypes.c_size_t(0)
    _check(_lib.bse_m3_band_info(ctypes.byref(dims), float(w), ctypes.byref(n), ctypes.byref(nb)),
           "bse_m3_band_info")
    return n.value, nb.value


def bse_build_m3_band(dims, d, a_coef, model: KernelModel, w: float, band, stream=None):
    _check(_lib.bse_build_m3_band(ctypes.byref(dims), _ptr(d), _ptr(a_coef), ctypes.byref(model), float(w),
                                  _ptr(band), band.numel() * band.element_size(), _stream(stream)),
           "bse_build_m3_band")


def bse_plan_set_m3_band(plan, band, w: float):
    _check(_lib.bse_plan_set_m3_band(plan, _ptr(band) if band is not None else None, float(w)),
           "bse_plan_set_m3_band")


def _storage(dtype_code: int):
    """(matrix complex dtype, vector complex dtype) for a bse_dtype."""
    if dtype_code == BSE_F64:
        return torch.complex128, torch.complex128
    if dtype_code in (BSE_F32, BSE_BF16_KC, BSE_F16_KC):
        return torch.complex64, torch.complex64
    return torch.complex64, torch.complex128


class BSEProblem:
    """Device-resident inputs, setup products and a plan for one Hamiltonian.

    vecs_coarse [Nkc, nv+nc, n_orb], vecs_dense [Nk, nv+nc, n_orb] (complex128),
    eps_dense [Nk, nv+nc] (eV), tau [n_orb, 3]; all numpy arrays or tensors.
    """

    def __init__(self, n_coarse, n_div, nv, nc, vecs_coarse, vecs_dense, eps_dense, tau, *,
                 dtype="f64", max_rhs=1, neighbours=8, eps_inf=12.0, lam=0.3, kernel_energy=6.0,
                 g2_max=4, q0_quad=16, device="cuda", Kc=None, d=None):
        self.device = torch.device(device)
        n_orb = int(np.shape(vecs_dense)[-1])
        self.dims = Dims(n_coarse, n_div, nv, nc, n_orb, max_rhs, DTYPES[dtype], neighbours)
        self.model = KernelModel(eps_inf, lam, kernel_energy, g2_max, q0_quad)
        self.mat_dtype, self.vec_dtype = _storage(self.dims.dtype)
        self.nk = n_coarse ** 3 * n_div ** 3
        self.N = self.nk * nv * nc
        self.Nc = n_coarse ** 3 * nv * nc
        dev = self.device
        as_t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a,
                                             dtype=dt).to(dev).contiguous()
        self.vecs_coarse = as_t(vecs_coarse, torch.complex128)
        self.vecs_dense = as_t(vecs_dense, torch.complex128)
        self.eps_dense = as_t(eps_dense, torch.float64)
        self.tau = as_t(tau, torch.float64)
        ne = (nv * nv + nc * nc)
        self.d = torch.empty(n_coarse ** 3 * 8 * ne * n_div ** 3, dtype=self.mat_dtype, device=dev)
        assert self.d.numel() * self.d.element_size() == bse_overlaps_bytes(self.dims)
        self.Kc = torch.empty(self.Nc, self.Nc, dtype=self.mat_dtype, device=dev)
        assert self.Kc.numel() * self.Kc.element_size() == bse_coarse_kernel_bytes(self.dims)
        self.delta = torch.empty(self.N, dtype=torch.float64, device=dev)
        if d is None:
            bse_build_overlaps(self.dims, self.vecs_coarse, self.vecs_dense, self.d)
        else:
            self.d.copy_(torch.as_tensor(d).to(dev).reshape(-1))
        bse_build_transition_energies(self.dims, self.eps_dense, self.delta)
        if Kc is None:
            bse_build_coarse_kernel(self.dims, self.vecs_coarse, self.tau, self.model, self.Kc)
        else:
            self.Kc.copy_(torch.as_tensor(Kc).to(dev).reshape(self.Nc, self.Nc))
        nbytes = bse_workspace_bytes(self.dims)
        if nbytes == 0:
            raise BSEError(_lib.bse_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.plan = bse_plan_create(self.dims, self.Kc, self.d, self.delta, self.workspace)

    def close(self):
        if getattr(self, "plan", None) is not None:
            bse_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- products ----------------------------------------------------------------------
    def vector(self, x) -> torch.Tensor:
        """[n_rhs, N] device vector in the plan's vector storage."""
        t = torch.as_tensor(x)
        if t.dim() == 1:
            t = t[None]
        return t.to(self.device).to(self.vec_dtype).contiguous()

    def matvec(self, x) -> torch.Tensor:
        x = self.vector(x)
        y = torch.empty_like(x)
        bse_interp_matvec(self.plan, x, y, x.shape[0])
        return y

    def haydock(self, P, n_steps: int) -> dict:
        P = torch.as_tensor(P)
        if P.dim() == 1:
            P = P[None]
        P = P.to(self.device).to(torch.complex128).contiguous()
        r = P.shape[0]
        dev = self.device
        a = torch.empty(r, n_steps, dtype=torch.float64, device=dev)
        b = torch.empty(r, n_steps + 1, dtype=torch.float64, device=dev)
        pn = torch.empty(r, dtype=torch.float64, device=dev)
        steps = torch.empty(r, dtype=torch.int32, device=dev)
        status = torch.empty(r, dtype=torch.int32, device=dev)
        bse_haydock_run(self.plan, P, r, n_steps, a, b, pn, steps, status)
        return dict(a=a, b=b, pnorm2=pn, steps=steps, status=status)

    def haydock_converge(self, P, max_steps: int, omega, eta: float, prefactor: float, tol: float,
                         check_every: int = 20, closure: int = 0):
        """Chains run until eps2 changes by at most tol (relative to its peak) between
        checks every check_every steps: (chain dict as haydock, eps [n_rhs, n_omega]).
        closure = k > 0 closes each checked fraction by the constant chain of the means of
        the chain's last k coefficients (0: truncated)."""
        bse_plan_set_converge_closure(self.plan, closure)
        P = torch.as_tensor(P)
        if P.dim() == 1:
            P = P[None]
        P = P.to(self.device).to(torch.complex128).contiguous()
        r = P.shape[0]
        dev = self.device
        om = torch.as_tensor(np.asarray(omega, dtype=np.float64)).to(dev)
        a = torch.empty(r, max_steps, dtype=torch.float64, device=dev)
        b = torch.empty(r, max_steps + 1, dtype=torch.float64, device=dev)
        pn = torch.empty(r, dtype=torch.float64, device=dev)
        steps = torch.empty(r, dtype=torch.int32, device=dev)
        status = torch.empty(r, dtype=torch.int32, device=dev)
        er = torch.empty(r, om.numel(), dtype=torch.float64, device=dev)
        ei = torch.empty_like(er)
        bse_haydock_converge(self.plan, P, r, max_steps, check_every, prefactor, om, om.numel(), eta, tol, a, b, pn,
                             steps, status, er, ei)
        return dict(a=a, b=b, pnorm2=pn, steps=steps, status=status), torch.complex(er, ei)

    @staticmethod
    def continued_fraction(chain: dict, prefactor: float, omega, eta: float) -> torch.Tensor:
        a, b = chain["a"], chain["b"]
        dev = a.device
        om = torch.as_tensor(np.asarray(omega, dtype=np.float64)).to(dev)
        n_chains = a.shape[0]
        er = torch.empty(n_chains, om.numel(), dtype=torch.float64, device=dev)
        ei = torch.empty_like(er)
        bse_continued_fraction(a, b, a.shape[1], b.shape[1], chain["pnorm2"], chain["steps"], n_chains,
                               prefactor, om, om.numel(), eta, er, ei)
        return torch.complex(er, ei)

    def set_m3(self, w):
        """Method 3 with band width w (in units of the coarse spacing); None: Method 1.
        Builds a_c and the band on the device and attaches it to the plan."""
        if w is None:
            bse_plan_set_m3_band(self.plan, None, 0.0)
            self.band = self.a_coef = None
            return
        n_off, nbytes = bse_m3_band_info(self.dims, w)
        self.a_coef = torch.empty(self.Nc, self.Nc, dtype=self.mat_dtype, device=self.device)
        bse_build_divergence_coefficient(self.dims, self.vecs_coarse, self.tau, self.model, self.a_coef)
        self.band = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        bse_build_m3_band(self.dims, self.d, self.a_coef, self.model, w, self.band)
        bse_plan_set_m3_band(self.plan, self.band, w)
        self.m3_offsets = n_off

    def set_timing(self, enable):
        """0 off; 1 (or True) the coarse product; 2 the Method 3 band product; 3 the coarse
        product's streaming kernel alone."""
        bse_plan_set_timing(self.plan, int(enable))

    def timing(self):
        return bse_plan_get_timing(self.plan)


def problem_from_bands(bs, cfg, dtype=None, max_rhs=None, neighbours=8, **kw) -> BSEProblem:
    """BSEProblem for a tbinputs BandStructure and its config."""
    if dtype is None:
        dtype = {"c128": "f64", "c64": "f32"}.get(cfg.dtype, cfg.dtype)
    return BSEProblem(cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc, bs.vecs_coarse, bs.vecs_dense, bs.eps_dense,
                      bs.tau, dtype=dtype, max_rhs=max_rhs or cfg.n_pol, neighbours=neighbours,
                      eps_inf=cfg.eps_inf, lam=cfg.lam, kernel_energy=cfg.kernel_energy, g2_max=cfg.g2_max,
                      q0_quad=cfg.q0_quad, **kw)
