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


def product_bound(op: O.InterpOperator, x, unit: float, factors: int = 10):
    """Componentwise bound on |y_gpu - y| for storage rounding of unit `unit`.

    Every term of y = delta x + C^H K C x is a product of at most 7 stored
    factors (x, 2 overlaps, K_c, 2 overlaps, output); FP64 accumulation adds
    well below one FP32 unit.  `factors` units per |term| covers that.
    """
    aop = abs_operator(op)
    return factors * unit * np.abs(aop.apply(np.abs(x)))
