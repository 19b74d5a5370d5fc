"""Helpers for the GPU parity tests: layouts and error bounds.

Nothing here computes the method: it only reshapes the library's outputs into
the oracle's layout and evaluates the rounding bound of a product from
absolute values.
"""

from __future__ import annotations

import numpy as np

import oracle as O

U32 = 2.0 ** -24   # unit roundoff of FP32
U64 = 2.0 ** -53


def gpu_overlaps_to_oracle(d, n_c, n_div, nv, nc):
    """Library layout [cell][z][e][sub] -> oracle (Dv [kd, z, v, n1], Dc [kd, z, c, n2])."""
    ncell, ndiv3 = n_c ** 3, n_div ** 3
    ne = nv * nv + nc * nc
    a = np.asarray(d).reshape(ncell, 8, ne, ndiv3).transpose(0, 3, 1, 2).reshape(ncell * ndiv3, 8, ne)
    Dv = a[:, :, :nv * nv].reshape(-1, 8, nv, nv)
    Dc = a[:, :, nv * nv:].reshape(-1, 8, nc, nc)
    return Dv, Dc


def abs_operator(op: O.InterpOperator) -> O.InterpOperator:
    """Same product with every factor replaced by its modulus: applied to |x| it
    bounds the sum of |terms| of each output of op.apply(x)."""
    return O.InterpOperator(np.abs(op.Dv).astype(complex), np.abs(op.Dc).astype(complex), op.f,
                            np.abs(op.Kc).astype(complex), np.abs(op.delta), op.n_c, op.n_div, op.nv, op.nc)


# The packed Hermitian coarse product of the FP32 coarse kernel (the library's default for
# BSE_F32 and BSE_F32_VEC64) computes r = K_c qbar in FP32 arithmetic: qbar is rounded to
# FP32 (1 unit of |qbar|), each FP32 run adds at most 64 FMA terms into one accumulator
# (conjugate-transposed tiles: 16 steps x 2 rows x 2 FMAs per component; plain tiles:
# 16 x 2), which the first-order bound of recursive summation keeps within 64 units of the
# run's sum of |terms|; runs are added in FP64 and each tile partial is rounded to FP32 once
# (1 unit).  Every output of r is therefore within 66 units of sum_j |K_ij| |qbar_j|, and
# the prolong carries that to |C|^H |K| |C| |x| on top of the 10 units of storage rounding.
PACKED_PRODUCT_UNITS = 66

# With FP32 overlaps the restrict and the prolong form their per-(subpoint, corner)
# contractions in FP32 and add the results in FP64.  Restrict: T = sum over 6 c of
# x Dc (12 FMAs per component, 12 units), then Y = sum over 3 v of conj(f Dv) T (6 FMAs,
# 6 units), plus the rounding of an FP64 vector entry to FP32 (1 unit): 19 units of
# sum |f Dv| |x| |Dc|.  Prolong: r rounded to FP32 (1), the 6-term sum over n2 (12), the
# 3-term sum over n1 (6) and the product with f (1): 20 units of sum f |Dv| |r| |Dc|.
# Both reach the output through |C|^H |K| |C| |x|: 39 units on the kernel terms.
FP32_INNER_UNITS = 19 + 20


def product_bound(op: O.InterpOperator, x, unit: float, factors: int = 10, kernel_factors=None):
    """Componentwise bound on |y_gpu - y| for storage rounding of unit `unit`.

    Every term of y = delta x + C^H K C x is a product of at most 7 stored
    factors (x, 2 overlaps, K_c, 2 overlaps, output); FP64 accumulation adds
    well below one FP32 unit.  `factors` units per |term| covers that.
    kernel_factors (default: factors) applies to the kernel terms C^H K C x alone,
    for products whose arithmetic adds its own rounding (PACKED_PRODUCT_UNITS).
    """
    aop = abs_operator(op)
    ax = np.abs(x)
    if kernel_factors is None:
        return factors * unit * np.abs(aop.apply(ax))
    diag = np.abs(aop.delta)[None] * np.atleast_2d(ax)
    kern = aop.apply_kernel(ax)
    return unit * (factors * diag + kernel_factors * np.abs(kern))


def fp32_kernel_factors(packed: bool) -> int:
    """Units of the kernel terms with FP32 overlaps and coarse kernel: storage rounding
    (10), the restrict's and prolong's FP32 contractions, and the packed coarse product's
    own arithmetic when it runs (form 0)."""
    return 10 + FP32_INNER_UNITS + (PACKED_PRODUCT_UNITS if packed else 0)
