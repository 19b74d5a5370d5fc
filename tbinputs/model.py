"""Periodic tight-binding crystal standing in for the Kohn-Sham inputs.

H(kappa) = sum_R H_R exp(i 2 pi kappa.R) over the 27 lattice vectors
R in {-1,0,1}^3, with kappa in reduced coordinates of a cubic reciprocal
lattice.  H_R is a random Hermitian matrix of size n_orb with amplitude
hop_amplitude * exp(-|R|), and H_{-R} = H_R, so H(kappa) is Hermitian and
periodic (H(kappa + G) = H(kappa)).  The first nv orbitals are pulled down by
onsite_split/2 and the rest pushed up by the same amount, so that the lowest
nv bands form an isolated valence manifold.  Orbitals sit on two sites:
tau = (0,0,0) for the first n_orb//2 orbitals and (1/4,1/4,1/4) for the rest
(the local-field exchange term vanishes identically if every orbital sits on
the same site).

The meshes follow Sec. 3: coarse points kappa_i = i / n_c, and dense points
kappa_{i,j} = (i + j / n_div) / n_c with 0 <= j < n_div per axis.  Dense
points are ordered cell-major: kd = cell * n_div^3 + sub, with
cell = (i1 n_c + i2) n_c + i3 and sub = (j1 n_div + j2) n_div + j3.  The
dense mesh contains the coarse one (sub = 0) and the eigenvectors there are
the very same arrays, so the two meshes share one gauge at common points.

Energies are in eV.  A scissor shift sets the gap (min conduction minus max
valence over the dense mesh) to cfg.gap (Sec. 2 scissors operator).  The
oscillator strengths for q -> 0 along polarisation e are taken as
P_vck(e) = <c k| dH/dkappa_e |v k> / (eps_ck - eps_vk), with the energies
before the scissor shift.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from .configs import BSEConfig

LATTICE_R = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.int64)  # [27,3]


@dataclass
class TBModel:
    n_orb: int
    nv: int
    R: np.ndarray      # [27, 3] integer lattice vectors
    HR: np.ndarray     # [27, n_orb, n_orb] complex128, Hermitian, HR(-R) == HR(R)
    tau: np.ndarray    # [n_orb, 3] reduced orbital positions

    def hamiltonian(self, kpts: np.ndarray) -> np.ndarray:
        """H(kappa) for kpts [n,3] (reduced) -> [n, n_orb, n_orb]."""
        ph = np.exp(2j * np.pi * (kpts @ self.R.T.astype(np.float64)))  # [n, 27]
        return np.einsum("kr,rab->kab", ph, self.HR)

    def velocity(self, kpts: np.ndarray, axis: int) -> np.ndarray:
        """dH/dkappa_axis at kpts -> [n, n_orb, n_orb]."""
        ph = np.exp(2j * np.pi * (kpts @ self.R.T.astype(np.float64)))
        w = 2j * np.pi * self.R[:, axis].astype(np.float64)
        return np.einsum("kr,r,rab->kab", ph, w, self.HR)


@dataclass
class BandStructure:
    cfg: BSEConfig
    kpts_coarse: np.ndarray   # [Nkc, 3]
    kpts_dense: np.ndarray    # [Nkd, 3]
    eps_dense: np.ndarray     # [Nkd, nb] eV, scissor applied to conduction bands
    eps_dense_ks: np.ndarray  # [Nkd, nb] eV, before the scissor
    vecs_dense: np.ndarray    # [Nkd, nb, n_orb] complex128, vecs[k, n, a] = c_{nk,a}
    vecs_coarse: np.ndarray   # [Nkc, nb, n_orb] complex128 (== dense at sub = 0)
    P: np.ndarray             # [n_pol, Nkd, nv, nc] complex128
    tau: np.ndarray           # [n_orb, 3]
    scissor: float

    def P_flat(self) -> np.ndarray:
        """P as [n_pol, N] in transition order t = (kd*nv + v)*nc + c."""
        return self.P.reshape(self.P.shape[0], -1)


def _hermitian(rng, n):
    m = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return (m + m.conj().T) / 2.0


def make_model(cfg: BSEConfig, seed: int | None = None, perturb: tuple | None = None) -> TBModel:
    """Draw the crystal for cfg (seeded).

    perturb = (delta, direction_seed) adds delta * (random Hermitian
    direction, amplitude exp(-|R|)) to every H_R: a finite-difference
    displaced structure.
    """
    seed = cfg.seed if seed is None else seed
    if perturb is None:
        perturb = cfg.perturb
    rng = np.random.default_rng(seed)
    n = cfg.n_orb
    R = LATTICE_R
    HR = np.zeros((len(R), n, n), dtype=np.complex128)
    index = {tuple(r): i for i, r in enumerate(R)}
    split = np.diag([-cfg.onsite_split / 2.0] * cfg.nv + [cfg.onsite_split / 2.0] * (n - cfg.nv))
    for i, r in enumerate(R):
        rt = tuple(r)
        neg = tuple(-x for x in rt)
        if rt < neg:          # filled from its partner below
            continue
        h = cfg.hop_amplitude * np.exp(-np.linalg.norm(r)) * _hermitian(rng, n)
        if rt == (0, 0, 0):
            h = h + split
        HR[i] = h
        HR[index[neg]] = h
    if perturb is not None:
        delta, dseed = perturb
        prng = np.random.default_rng(dseed)
        for i, r in enumerate(R):
            rt = tuple(r)
            neg = tuple(-x for x in rt)
            if rt < neg:
                continue
            h = delta * np.exp(-np.linalg.norm(r)) * _hermitian(prng, n)
            HR[i] = HR[i] + h
            if neg != rt:
                HR[index[neg]] = HR[index[neg]] + h
    tau = np.zeros((n, 3))
    tau[n // 2:, :] = 0.25
    return TBModel(n_orb=n, nv=cfg.nv, R=R, HR=HR, tau=tau)


def coarse_kpoints(n_coarse: int) -> np.ndarray:
    i = np.arange(n_coarse)
    g = np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.float64) / n_coarse


def dense_kpoints(n_coarse: int, n_div: int) -> np.ndarray:
    i = np.arange(n_coarse)
    j = np.arange(n_div)
    ci = np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1).reshape(-1, 1, 3)
    sj = np.stack(np.meshgrid(j, j, j, indexing="ij"), axis=-1).reshape(1, -1, 3)
    k = (ci.astype(np.float64) + sj.astype(np.float64) / n_div) / n_coarse
    return k.reshape(-1, 3)


def band_structure(cfg: BSEConfig, model: TBModel | None = None, chunk: int = 8192) -> BandStructure:
    """Diagonalise the crystal on both meshes and build P for cfg.n_pol polarisations."""
    if model is None:
        model = make_model(cfg)
    nb = cfg.n_bands
    if nb > cfg.n_orb:
        raise ValueError("nv + nc exceeds the orbital count")
    kd = dense_kpoints(cfg.n_coarse, cfg.n_div)
    nkd = kd.shape[0]
    eps = np.empty((nkd, nb))
    vecs = np.empty((nkd, nb, cfg.n_orb), dtype=np.complex128)
    P = np.empty((cfg.n_pol, nkd, cfg.nv, cfg.nc), dtype=np.complex128)
    for s in range(0, nkd, chunk):
        kk = kd[s:s + chunk]
        e, u = np.linalg.eigh(model.hamiltonian(kk))      # u[k, a, n]
        e = e[:, :nb]
        u = u[:, :, :nb]
        eps[s:s + chunk] = e
        vecs[s:s + chunk] = np.transpose(u, (0, 2, 1))
        uv = u[:, :, :cfg.nv]
        uc = u[:, :, cfg.nv:nb]
        de = e[:, cfg.nv:nb][:, None, :] - e[:, :cfg.nv][:, :, None]   # [k, v, c]
        for p in range(cfg.n_pol):
            dh = model.velocity(kk, p % 3)
            m = np.einsum("kac,kab,kbv->kvc", uc.conj(), dh, uv)       # <c|dH|v>
            P[p, s:s + chunk] = m / de
    ndiv3 = cfg.n_div3
    vecs_coarse = vecs[::ndiv3].copy()
    vecs[::ndiv3] = vecs_coarse   # same arrays at the shared points
    scissor = cfg.gap - (eps[:, cfg.nv:].min() - eps[:, :cfg.nv].max())
    eps_sc = eps.copy()
    eps_sc[:, cfg.nv:] += scissor
    return BandStructure(cfg=cfg, kpts_coarse=coarse_kpoints(cfg.n_coarse), kpts_dense=kd,
                         eps_dense=eps_sc, eps_dense_ks=eps, vecs_dense=vecs,
                         vecs_coarse=vecs_coarse, P=P, tau=model.tau.copy(), scissor=scissor)


def random_vectors(n: int, n_rhs: int, seed: int) -> np.ndarray:
    """Seeded complex Gaussian test vectors [n_rhs, n] (complex128)."""
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(n_rhs, n)) + 1j * rng.normal(size=(n_rhs, n))) / np.sqrt(2.0)
