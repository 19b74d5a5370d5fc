"""Plain FP64 CPU oracle of the double-grid on-the-fly BSE / Haydock path.

TEST INFRASTRUCTURE.  Only the tests, the smoke check of the entry module and
the CPU-baseline leg of the benchmark may import or run anything in this
package.  The product path (the HIP library and its Python binding) never
calls it, and this package never calls the product path: the two share no
code.  Both only consume the seeded inputs of ``tbinputs``.

Contents, each following the paper (Gillet, Giantomassi, Gonze, "Efficient
on-the-fly interpolation technique for Bethe-Salpeter calculations of optical
spectra"):

* ``grids``     Sec. 3: coarse/dense meshes, the neighbourhood N(k) of
                Eq. (neighborhood), the dense set S(k~) of Eq. (subspace) and
                the trilinear prefactors f^{lmn}; the one-neighbour prefactor
                of the Rohlfing-Louie scheme (Eq. eqRL).
* ``overlaps``  Eq. (completeness): d_{nk}^{n'k~} = <u_{n'k~}|u_{nk}>.
* ``kernel``    Eqs. (bse2)-(bse3b) and (Wcoul) with the model screened
                interaction of the synthetic crystal: the coarse kernel K_c.
* ``matvec``    Eq. (bse1) diagonal; Eq. (interp1) explicit interpolated
                kernel; Eqs. (matmul1)-(matmul3) on-the-fly product, both with
                the corner sum collapsed first and literally.
* ``lanczos``   Eqs. (ai)-(ci) Haydock-Lanczos chain, Eq. (fraccont)
                continued fraction (also closed by a constant-coefficient
                tail), Eq. (epsmacro) by diagonalisation.
* ``m3``        Sec. 4, Method 3: the divergent part of Eq. (diverg)
                interpolated and combined with the dense-mesh q inside a band
                ||k - k'|| <= w d, as a sparse correction of the Method 1 product.
* ``mlp``       the learned terminator's network (dense layers, GELU, mean
                squared error, Adam): textbook definitions, no part of the
                paper.

Every function here is pinned by a CPU test against something other than
itself (closed forms, invariants, brute force, textbook routines).
"""

from .grids import (
    corner_offsets,
    neighbour_table,
    trilinear_weights,
    nearest_corner_weights,
    dense_index_map,
    fold_int,
)
from .overlaps import overlaps
from .kernel import (
    g_vectors,
    w_model,
    w_q0_average,
    coarse_kernel,
    coarse_kernel_block_rows,
    screening_kappa2,
    s_shape,
    s_q0_average,
    coarse_shape,
    divergence_coefficient,
)
from .matvec import InterpOperator, transition_energies
from .lanczos import (
    haydock,
    continued_fraction,
    continued_fraction_terminated,
    constant_chain_g,
    eigh_spectrum,
    ip_spectrum,
)
from . import m3, mlp

__all__ = [
    "corner_offsets", "neighbour_table", "trilinear_weights", "nearest_corner_weights",
    "dense_index_map", "fold_int", "overlaps", "g_vectors", "w_model", "w_q0_average",
    "coarse_kernel", "coarse_kernel_block_rows", "InterpOperator", "transition_energies",
    "haydock", "continued_fraction", "continued_fraction_terminated", "constant_chain_g",
    "eigh_spectrum", "ip_spectrum", "mlp", "m3", "screening_kappa2", "s_shape", "s_q0_average",
    "coarse_shape", "divergence_coefficient",
]
