"""Autotuner for the plan tunables of the double-grid BSE library.

For one problem shape it times short Haydock runs (the whole step: coarse product,
prolong, update + restrict, collapse) over the candidate settings of the two
tunables the library exposes,

  * column splits of the coarse product (`bse_plan_set_gemv_splits`, 0 = the
    library's own choice), and
  * right-hand sides per restrict block (`bse_plan_set_restrict_group`, 1 or 3;
    3 only for three right-hand sides),

keeps the fastest, applies it to the plan and records it in a JSON cache keyed by
the shape (coarse points, divisions, bands, precision, right-hand sides, device).
Every setting gives the same operator; only the summation order of the coarse
product's splits differs, so results agree to rounding.
"""

from __future__ import annotations

import json
import os
import time

import torch

from . import bse

DEFAULT_SPLITS = (0, 8, 16, 24, 32, 48, 64)


def shape_key(prob: "bse.BSEProblem", n_rhs: int) -> str:
    d = prob.dims
    dev = torch.cuda.get_device_name(prob.device)
    return f"{d.n_coarse}x{d.n_div}_{d.nv}v{d.nc}c_dtype{d.dtype}_nb{d.neighbours}_rhs{n_rhs}_{dev}"


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path, db):
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(prob: "bse.BSEProblem", setting: dict) -> None:
    bse.bse_plan_set_gemv_splits(prob.plan, int(setting["splits"]))
    bse.bse_plan_set_restrict_group(prob.plan, int(setting["group"]))


def time_setting(prob, P, setting: dict, steps: int, repeats: int) -> float:
    """Best wall time per step (ms) of `repeats` runs of `steps` steps, on the device."""
    apply(prob, setting)
    prob.haydock(P, 2)                       # warm the setting's kernels
    best = float("inf")
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        prob.haydock(P, steps)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / steps)
    return best


def autotune(prob: "bse.BSEProblem", P, steps: int = 12, repeats: int = 2, splits=DEFAULT_SPLITS,
             cache: str | None = None, force: bool = False) -> dict:
    """Pick and apply the fastest setting for prob with start vectors P ([n_rhs, N]).

    Returns {"splits", "group", "ms_per_step", "key", "cached", "trials"}.
    """
    P = torch.as_tensor(P)
    if P.dim() == 1:
        P = P[None]
    P = P.to(prob.device).to(torch.complex128).contiguous()
    n_rhs = P.shape[0]
    key = shape_key(prob, n_rhs)
    db = _load(cache)
    if not force and key in db:
        setting = dict(db[key])
        apply(prob, setting)
        return dict(setting, key=key, cached=True, trials=[])
    groups = (1, 3) if n_rhs == 3 else (1,)
    trials = []
    for g in groups:
        for sp in splits:
            s = {"splits": sp, "group": g}
            trials.append(dict(s, ms_per_step=time_setting(prob, P, s, steps, repeats)))
    best = min(trials, key=lambda t: t["ms_per_step"])
    setting = {"splits": best["splits"], "group": best["group"], "ms_per_step": best["ms_per_step"],
               "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}
    apply(prob, setting)
    db[key] = setting
    _store(cache, db)
    return dict(setting, key=key, cached=False, trials=trials)
