"""Shared builders for the tests: seeded inputs plus the oracle's operator."""

from __future__ import annotations

import functools

import numpy as np

import oracle as O
import tbinputs as ti


@functools.lru_cache(maxsize=None)
def bands(cfg):
    return ti.band_structure(cfg)


@functools.lru_cache(maxsize=None)
def oracle_parts(cfg, weights="trilinear"):
    """(bs, Dv, Dc, f, Kc, delta) computed by the oracle for cfg."""
    bs = bands(cfg)
    Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    f = (O.trilinear_weights(cfg.n_div) if weights == "trilinear"
         else O.nearest_corner_weights(cfg.n_div))
    Kc = O.coarse_kernel(bs.vecs_coarse, bs.tau, cfg.nv, cfg.nc, cfg.n_coarse, cfg.n_div, cfg)
    delta = O.transition_energies(bs.eps_dense, cfg.nv, cfg.nc)
    return bs, Dv, Dc, f, Kc, delta


def oracle_operator(cfg, weights="trilinear", Kc=None):
    bs, Dv, Dc, f, Kc0, delta = oracle_parts(cfg, weights)
    return O.InterpOperator(Dv, Dc, f, Kc0 if Kc is None else Kc, delta, cfg.n_coarse,
                            cfg.n_div, cfg.nv, cfg.nc)


def rel_l2(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
