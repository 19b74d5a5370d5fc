"""Haydock-Lanczos chain and the macroscopic dielectric function.

Eqs. (ai)-(ci): b_1 = 0, psi_1 = P / ||P||, then for i = 1, 2, ...
    a_i     = <psi_i | H | psi_i>
    b_{i+1} = || H psi_i - a_i psi_i - b_i psi_{i-1} ||
    psi_{i+1} = (H psi_i - a_i psi_i - b_i psi_{i-1}) / b_{i+1}.
The subtractions are taken in the modified order (w = H psi_i - b_i psi_{i-1},
a_i = Re <psi_i | w>, w -= a_i psi_i), which equals the printed form in exact
arithmetic; H is Hermitian so a_i is real.  No reorthogonalisation unless
asked for (the paper mentions none).

Eq. (fraccont): eps_M(w) = 1 - C ||P||^2 / (z - a_1 - b_2^2 / (z - a_2 - ...)),
z = w + i eta, truncated after a_m (no terminator).  C stands for
lim v(q) and is a caller-supplied scalar.

Eq. (epsmacro) by diagonalisation: eps_M(w) = 1 - C sum_l |<l|P>|^2 / (z - E_l).

Arrays use 0-based chain positions: a[..., i] = a_{i+1}; b[..., 0] = b_1 = 0
and b[..., i] = b_{i+1}.
"""

from __future__ import annotations

import numpy as np


def haydock(apply_H, P: np.ndarray, m: int, reorth: bool = False, tol: float = 1e-12,
            round_dtype=None):
    """Run independent chains for every row of P [n_rhs, N].

    apply_H maps [n_rhs, N] -> [n_rhs, N].  Returns dict(a [n_rhs, m],
    b [n_rhs, m+1], pnorm2 [n_rhs], steps [n_rhs]).  A chain stops (its
    remaining coefficients stay 0) when b_{i+1} <= tol * ||w|| (an invariant
    Krylov subspace); steps counts its valid a_i.

    round_dtype (e.g. np.complex64) rounds every stored vector to that type,
    emulating lower-precision vector storage around an FP64 computation.
    """
    P = np.atleast_2d(np.asarray(P, dtype=np.complex128))
    n_rhs, N = P.shape
    a = np.zeros((n_rhs, m))
    b = np.zeros((n_rhs, m + 1))
    pnorm2 = np.real(np.sum(P.conj() * P, axis=1))
    steps = np.zeros(n_rhs, dtype=np.int64)
    active = pnorm2 > 0
    psi = np.zeros_like(P)
    psi[active] = P[active] / np.sqrt(pnorm2[active])[:, None]

    def rnd(v):
        return v if round_dtype is None else v.astype(round_dtype).astype(np.complex128)

    psi = rnd(psi)
    psi_prev = np.zeros_like(P)
    basis = [psi.copy()] if reorth else None
    b_cur = np.zeros(n_rhs)
    for i in range(m):
        if not active.any():
            break
        w = apply_H(psi) - b_cur[:, None] * psi_prev
        ai = np.real(np.sum(psi.conj() * w, axis=1))
        w = w - ai[:, None] * psi
        if reorth:
            for _ in range(2):
                for v in basis:
                    w = w - np.sum(v.conj() * w, axis=1)[:, None] * v
        wn = np.sqrt(np.real(np.sum(w.conj() * w, axis=1)))
        a[active, i] = ai[active]
        steps[active] = i + 1
        stop = active & (wn <= tol * np.sqrt(ai ** 2 + wn ** 2))
        go = active & ~stop
        b[go, i + 1] = wn[go]
        new = np.zeros_like(w)
        new[go] = w[go] / wn[go][:, None]
        active = go
        psi_prev, psi = psi, rnd(new)
        b_cur = np.where(go, wn, 0.0)
        if reorth:
            basis.append(psi.copy())
    return dict(a=a, b=b, pnorm2=pnorm2, steps=steps)


def continued_fraction(a: np.ndarray, b: np.ndarray, pnorm2, prefactor: float,
                       omega: np.ndarray, eta: float, steps=None) -> np.ndarray:
    """eps_M(omega) from chain coefficients, Eq. (fraccont) -> complex [n_rhs, n_omega]."""
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    pnorm2 = np.atleast_1d(pnorm2)
    n_rhs, m = a.shape
    if steps is None:
        steps = np.full(n_rhs, m)
    z = np.asarray(omega, dtype=np.float64) + 1j * eta
    out = np.empty((n_rhs, z.shape[0]), dtype=np.complex128)
    for r in range(n_rhs):
        n = int(steps[r])
        if n == 0 or pnorm2[r] == 0:
            out[r] = 1.0
            continue
        t = z - a[r, n - 1]
        for i in range(n - 2, -1, -1):
            t = z - a[r, i] - b[r, i + 1] ** 2 / t
        out[r] = 1.0 - prefactor * pnorm2[r] / t
    return out


def constant_chain_g(z, a_inf: float, b_inf: float):
    """Resolvent of a semi-infinite chain with constant coefficients a_inf, b_inf:
    g = 1 / (z - a_inf - b_inf^2 g), the root that vanishes as |z| grows, i.e. the
    one with Im g < 0 for Im z > 0 (semicircle of half-width 2 b_inf).

    This is the usual closure of a Lanczos continued fraction once the
    coefficients have settled; the paper leaves the tail of Eq. (fraccont) open.
    """
    z = np.asarray(z, dtype=np.complex128)
    x = z - a_inf
    if b_inf == 0:
        return 1.0 / x
    root = np.sqrt(x * x - 4.0 * b_inf * b_inf)
    g1 = (x - root) / (2.0 * b_inf * b_inf)
    g2 = (x + root) / (2.0 * b_inf * b_inf)
    return np.where(g1.imag <= 0, g1, g2)


def continued_fraction_terminated(a: np.ndarray, b: np.ndarray, pnorm2, prefactor: float,
                                  omega: np.ndarray, eta: float, a_inf, b_inf) -> np.ndarray:
    """eps_M(omega) from m coefficients a_1..a_m, b_1..b_{m+1} closed by the constant
    chain (a_inf, b_inf) beyond a_m: t_m = z - a_m - b_{m+1}^2 g_inf(z), then
    t_i = z - a_i - b_{i+1}^2 / t_{i+1} and eps_M = 1 - C ||P||^2 / t_1."""
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    pnorm2 = np.atleast_1d(pnorm2)
    a_inf = np.atleast_1d(a_inf)
    b_inf = np.atleast_1d(b_inf)
    n_rhs, m = a.shape
    z = np.asarray(omega, dtype=np.float64) + 1j * eta
    out = np.empty((n_rhs, z.shape[0]), dtype=np.complex128)
    for r in range(n_rhs):
        if pnorm2[r] == 0:
            out[r] = 1.0
            continue
        t = z - a[r, m - 1] - b[r, m] ** 2 * constant_chain_g(z, a_inf[r], b_inf[r])
        for i in range(m - 2, -1, -1):
            t = z - a[r, i] - b[r, i + 1] ** 2 / t
        out[r] = 1.0 - prefactor * pnorm2[r] / t
    return out


def eigh_spectrum(H: np.ndarray, P: np.ndarray, prefactor: float, omega: np.ndarray,
                  eta: float) -> np.ndarray:
    """eps_M(omega) from the eigenpairs of a Hermitian H, Eq. (epsmacro)."""
    E, V = np.linalg.eigh(H)
    P = np.atleast_2d(P)
    w = np.abs(V.conj().T @ P.T) ** 2                          # [n_states, n_rhs]
    z = np.asarray(omega, dtype=np.float64) + 1j * eta
    g = 1.0 / (z[None, :] - E[:, None])                          # [n_states, n_omega]
    return 1.0 - prefactor * (w.T @ g)


def ip_spectrum(delta: np.ndarray, P: np.ndarray, prefactor: float, omega: np.ndarray,
                eta: float) -> np.ndarray:
    """Independent-particle limit (K = 0): eps_M = 1 - C sum_t |P_t|^2 / (z - delta_t)."""
    P = np.atleast_2d(P)
    z = np.asarray(omega, dtype=np.float64) + 1j * eta
    g = 1.0 / (z[None, :] - np.asarray(delta)[:, None])
    return 1.0 - prefactor * ((np.abs(P) ** 2) @ g)
