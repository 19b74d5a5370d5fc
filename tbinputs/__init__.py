"""Seeded synthetic band-structure inputs for the double-grid BSE path.

This package is the stand-in for the Kohn-Sham stage that the method takes as
given (Sec. 2: energies and wavefunctions on the coarse and dense meshes, a
scissor shift, and the oscillator matrix elements P evaluated for small q).
It builds a periodic tight-binding crystal and diagonalises it; it holds none
of the method's own arithmetic (no overlaps, weights, kernel, matvec, Lanczos
or continued fraction).  Both the CPU oracle and the HIP path consume what it
produces.
"""

from .configs import CONFIGS, BSEConfig, batch_configs, get_config, tiny_config
from .model import (
    TBModel,
    BandStructure,
    make_model,
    band_structure,
    random_vectors,
    dense_kpoints,
    coarse_kpoints,
)

__all__ = [
    "CONFIGS",
    "BSEConfig",
    "get_config",
    "batch_configs",
    "tiny_config",
    "TBModel",
    "BandStructure",
    "make_model",
    "band_structure",
    "random_vectors",
    "dense_kpoints",
    "coarse_kpoints",
]
