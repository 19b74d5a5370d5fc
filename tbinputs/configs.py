"""Workload descriptions for the synthetic double-grid BSE runs.

Each configuration fixes the tight-binding crystal (orbitals, seed), the two
meshes (coarse points per axis and divisions per axis, Sec. 3), the
transition space (valence and conduction bands), the chain (Haydock steps and
polarisations) and the spectrum grid (omega window and broadening eta).
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class BSEConfig:
    name: str
    n_orb: int            # orbitals per cell of the tight-binding crystal
    nv: int               # valence bands kept in the transition space
    nc: int               # conduction bands kept in the transition space
    n_coarse: int         # coarse points per axis (cubic mesh)
    n_div: int            # divisions per axis (dense = n_coarse * n_div per axis)
    seed: int
    steps: int            # Haydock steps per chain
    n_pol: int            # polarisations (x, y, z ...) run as right-hand sides
    omega_max: float      # eV, spectrum window [0, omega_max]
    n_omega: int
    eta: float            # eV, Lorentzian broadening
    dtype: str            # "c128" or "c64": storage of kernel, overlaps, vectors
    # crystal and kernel model parameters (shared by every workload)
    hop_amplitude: float = 0.5    # eV, |H_R| scale, times exp(-|R|)
    onsite_split: float = 6.0     # eV, valence-orbital / conduction-orbital split
    gap: float = 1.1              # eV, gap after the scissor shift
    eps_inf: float = 12.0         # screening of the model W(q)
    lam: float = 0.3              # screening wavevector of the model W(q)
    g2_max: int = 4               # |G|^2 cut of the plane-wave sums (33 G)
    kernel_energy: float = 6.0    # eV, kernel energy scale (divided by dense N_k)
    q0_quad: int = 16             # midpoint points per axis for the q->0 average
    # finite-difference displaced structure: (delta, direction seed) added to every H_R
    perturb: tuple | None = None
    extra: dict = field(default_factory=dict, compare=False, hash=False)

    # ---- derived sizes -------------------------------------------------------
    @property
    def n_div3(self) -> int:
        return self.n_div ** 3

    @property
    def nk_coarse(self) -> int:
        return self.n_coarse ** 3

    @property
    def nk_dense(self) -> int:
        return self.nk_coarse * self.n_div3

    @property
    def n_pair(self) -> int:
        return self.nv * self.nc

    @property
    def n_trans_coarse(self) -> int:
        return self.nk_coarse * self.n_pair

    @property
    def n_trans(self) -> int:
        return self.nk_dense * self.n_pair

    @property
    def n_bands(self) -> int:
        return self.nv + self.nc

    def omega(self) -> np.ndarray:
        return np.linspace(0.0, self.omega_max, self.n_omega)

    def prefactor(self) -> float:
        """Scalar standing for lim v(q) in the macroscopic dielectric function.

        Spin factor 2 times 4*pi over (cell volume 1 times dense k count).
        """
        return 8.0 * np.pi / self.nk_dense

    def with_(self, **kw) -> "BSEConfig":
        return replace(self, **kw)


CONFIGS = {
    # validation workload: 4^3 coarse, 2 divisions, 3v+3c, FP64
    "c0": BSEConfig(name="c0", n_orb=6, nv=3, nc=3, n_coarse=4, n_div=2, seed=0,
                    steps=200, n_pol=1, omega_max=10.0, n_omega=2000, eta=0.1,
                    dtype="c128"),
    # headline workload: 8^3 coarse, 4 divisions (32^3 dense), 3v+6c, FP32
    "c1": BSEConfig(name="c1", n_orb=9, nv=3, nc=6, n_coarse=8, n_div=4, seed=1,
                    steps=300, n_pol=3, omega_max=15.0, n_omega=3000, eta=0.05,
                    dtype="c64"),
    # precision-form workload: 10^3 coarse, 4 divisions (40^3 dense), 4v+6c
    "c2": BSEConfig(name="c2", n_orb=10, nv=4, nc=6, n_coarse=10, n_div=4, seed=2,
                    steps=400, n_pol=3, omega_max=15.0, n_omega=3000, eta=0.05,
                    dtype="c64"),
}


def get_config(name: str) -> BSEConfig:
    return CONFIGS[name.lower()]


# batching workload: 3 grids x 8 seeded displacement directions x (+delta, -delta)
BATCH_GRIDS = ((4, 2), (6, 3), (8, 4))
BATCH_DIRECTIONS = 8
BATCH_DELTA = 0.01


def batch_configs() -> list:
    """The 48 uneven Hamiltonians of the batching workload.

    One seeded 9-orbital crystal (seed 3) displaced by +-delta (delta = 0.01) along
    8 seeded directions, each structure on 3 grids (4^3 x 2, 6^3 x 3, 8^3 x 4);
    nv = 3, nc = 3 for +delta and 6 for -delta; 3 polarisations, 200 steps, FP32.
    """
    out = []
    for n_coarse, n_div in BATCH_GRIDS:
        for d in range(BATCH_DIRECTIONS):
            for sign in (1, -1):
                nc = 3 if sign > 0 else 6
                out.append(BSEConfig(name=f"c3_{n_coarse}x{n_div}_d{d}{'p' if sign > 0 else 'm'}", n_orb=9, nv=3,
                                     nc=nc, n_coarse=n_coarse, n_div=n_div, seed=3, steps=200, n_pol=3,
                                     omega_max=15.0, n_omega=3000, eta=0.05, dtype="c64",
                                     perturb=(sign * BATCH_DELTA, 1000 + d)))
    return out


def tiny_config(n_coarse=2, n_div=2, nv=2, nc=2, n_orb=None, seed=7, dtype="c128",
                n_pol=1, steps=40, **kw) -> BSEConfig:
    """Small workload for brute-force checks (explicit matrices, eigh)."""
    if n_orb is None:
        n_orb = nv + nc
    return BSEConfig(name=f"tiny{n_coarse}x{n_div}_{nv}v{nc}c", n_orb=n_orb, nv=nv, nc=nc,
                     n_coarse=n_coarse, n_div=n_div, seed=seed, steps=steps, n_pol=n_pol,
                     omega_max=kw.pop("omega_max", 16.0), n_omega=kw.pop("n_omega", 400),
                     eta=kw.pop("eta", 0.1), dtype=dtype, **kw)
