"""Benchmark: Haydock steps/s of the double-grid on-the-fly BSE path on one MI355X.

Workload (default): 8^3 coarse mesh, 4 divisions per axis (32^3 = 32768 dense k),
3 valence + 6 conduction bands (N = 589,824 transitions), coarse kernel 9216^2
complex FP32, 3 polarisations advanced together, FP64 accumulation and Lanczos
scalars.  A step is one Haydock iteration of all three chains: coarse product,
prolong + diagonal + a_i, update + restrict + b_{i+1}, collapse.  Inputs are
seeded synthetic tight-binding data, resident in HBM before timing starts.

Prints one JSON line (see the keys below).  The CPU baseline times the plain
FP64 oracle on the host for a bounded number of steps of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "hbm_counters_c1_f32.md")
GEMV_SOURCE = os.path.join(ROOT, "paper_1602_01863_amd", "csrc", "gemv.hip")


M3_SUMMARY = os.path.join(ROOT, "profiles", "m3_band_c1_f32.md")
M3_SOURCE = os.path.join(ROOT, "paper_1602_01863_amd", "csrc", "m3.hip")


def measured_m3_traffic(workload: str, dtype: str, w: float):
    """HBM bytes per band-product launch from the committed counter summary (C1, FP32,
    w = 1), or None if it does not cover this run or the kernel source has changed."""
    import hashlib
    import re

    if workload != "c1" or dtype != "f32" or w != 1.0 or not os.path.exists(M3_SUMMARY):
        return None
    text = open(M3_SUMMARY).read()
    m_t = re.search(r"traffic_bytes_per_launch:\s*(\d+)", text)
    m_h = re.search(r"m3_source_sha256_16:\s*([0-9a-f]+)", text)
    if not (m_t and m_h):
        return None
    digest = hashlib.sha256(open(M3_SOURCE, "rb").read()).hexdigest()[:16]
    return int(m_t.group(1)) if digest == m_h.group(1) else None


def measured_traffic(workload: str, dtype: str, key: str = "traffic_bytes_per_launch"):
    """HBM bytes per launch (key: the coarse product's two kernels, or
    traffic_bytes_per_launch_stream for its streaming kernel alone) from the committed
    rocprofv3 counter summary, or None if it does not cover this workload or the kernel
    source has changed since the counters were taken."""
    import hashlib
    import re

    if workload != "c1" or dtype != "f32" or not os.path.exists(COUNTER_SUMMARY):
        return None
    text = open(COUNTER_SUMMARY).read()
    m_t = re.search(key + r":\s*(\d+)", text)
    m_h = re.search(r"gemv_source_sha256_16:\s*([0-9a-f]+)", text)
    if not (m_t and m_h):
        return None
    digest = hashlib.sha256(open(GEMV_SOURCE, "rb").read()).hexdigest()[:16]
    return int(m_t.group(1)) if digest == m_h.group(1) else None


def _args():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=300)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--config", default="c1")
    p.add_argument("--dtype", default=None, help="f32 | f32v64 | f64 | bf16 | f16 (default: workload's)")
    p.add_argument("--splits", type=int, default=0, help="column splits of the coarse product (0 = auto)")
    p.add_argument("--full-stream", action="store_true",
                   help="FP32 coarse kernel: stream the whole K_c instead of the packed Hermitian tiles")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-race", action="store_true", help="skip the converged time-to-eps2 comparison")
    p.add_argument("--race-eta", type=float, default=None,
                   help="broadening (eV) of the converged time-to-eps2 comparison (default: the workload's)")
    p.add_argument("--cpu-steps", type=int, default=8, help="oracle steps timed for the CPU baseline")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    p.add_argument("--batch", action="store_true",
                   help="batching workload: 48 uneven Hamiltonians x 3 polarisations in one HIP graph")
    p.add_argument("--batch-launches", type=int, default=3, help="timed graph launches of the batch")
    p.add_argument("--no-autotune", action="store_true", help="batch: keep the automatic tunables")
    p.add_argument("--no-batch", action="store_true",
                   help="leave the batching workload out of the default line")
    p.add_argument("--time-to-spectrum", action="store_true",
                   help="time to eps2 of the plain FP32 form against the BF16 form, its graph-recorded "
                        "chains and the learned terminator (C1 workload)")
    p.add_argument("--m3", type=float, default=None, metavar="W",
                   help="Method 3 with band width W (units of the coarse spacing); default: Method 1")
    return p.parse_args()


def main():
    args = _args()
    if args.gpus != 1:
        print(f"bench.py: the Haydock path runs on one GPU (--gpus {args.gpus} requested); "
              "sharding the coarse cells over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import tbinputs as ti
    from paper_1602_01863_amd import bse

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.batch:
        batch_bench(args)
        return
    if args.time_to_spectrum:
        spectrum_race(args)
        return
    cfg = ti.get_config(args.config)
    dtype = args.dtype or {"c128": "f64", "c64": "f32"}[cfg.dtype]
    t0 = time.perf_counter()
    bs = ti.band_structure(cfg)
    t_inputs = time.perf_counter() - t0

    # ---- setup on the device (overlaps, transition energies, coarse kernel, plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob = bse.problem_from_bands(bs, cfg, dtype=dtype, max_rhs=cfg.n_pol)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    if args.splits:
        bse.bse_plan_set_gemv_splits(prob.plan, args.splits)
    if args.full_stream:
        bse.bse_plan_set_coarse_product(prob.plan, 1)
    t_m3 = None
    if args.m3 is not None:   # a_c and the band blocks on the device, attached to the plan
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.set_m3(args.m3)
        torch.cuda.synchronize()
        t_m3 = time.perf_counter() - t0
    P = torch.as_tensor(bs.P_flat()).to("cuda").contiguous()

    # ---- untimed spin-up: one chain of the workload's length, so that the measurements
    # below see the GPU at its steady clock rather than right after the host-side setup
    # (a 20-step chain right after setup ran 10% slower than the same chain later)
    prob.haydock(P, cfg.steps)
    torch.cuda.synchronize()

    # ---- dominant kernel (coarse product): HIP events around each launch of one chain
    # run of K steps, on the stream it is launched on
    prob.set_timing(True)
    torch.cuda.synchronize()
    prob.haydock(P, args.steps)
    torch.cuda.synchronize()
    gemv_ms_total, gemv_launches = prob.timing()
    prob.set_timing(False)
    gemv_ms = gemv_ms_total / max(1, gemv_launches)
    # the product's streaming kernel alone, the dominant kernel of the step: the library
    # launches it with an event pair that the runtime stamps with its own start and end
    prob.set_timing(3)
    torch.cuda.synchronize()
    prob.haydock(P, args.steps)
    torch.cuda.synchronize()
    kern_ms_total, kern_launches = prob.timing()
    prob.set_timing(False)
    kern_ms = kern_ms_total / max(1, kern_launches)

    # ---- warmup, then exactly K timed steps (one chain run of K steps)
    if args.warmup > 0:
        prob.haydock(P, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch = prob.haydock(P, args.steps)
    torch.cuda.synchronize()
    t_chain = time.perf_counter() - t0
    ms_per_step = 1e3 * t_chain / args.steps
    steps_per_s = args.steps / t_chain

    # ---- fixed cost of one bse_haydock_run call (chain start, report, launch and
    # synchronisation latency): a one-step chain less one step at the timed rate
    t_one = []
    for _ in range(5):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prob.haydock(P, 1)
        torch.cuda.synchronize()
        t_one.append(time.perf_counter() - t1)
    fixed_ms = 1e3 * min(t_one) - ms_per_step
    Nc, n_rhs = prob.Nc, cfg.n_pol
    lowp = dtype in ("bf16", "f16")
    mat_bytes = {"f64": 16, "f32": 8, "f32v64": 8, "bf16": 4, "f16": 4}[dtype]
    nbk = -(-Nc // 64)
    packed = not args.full_stream
    if lowp:   # 64 x 64 blocks in the format (zero-padded) + one FP32 scale per block
        nblk = nbk * (nbk + 1) // 2 if packed else nbk * nbk   # packed: blocks on and above the diagonal
        kc_bytes = nblk * 64 * 64 * mat_bytes + nblk * 4
    elif packed:   # the 128 x 128 tiles on and above the diagonal (K_c Hermitian)
        nt = -(-Nc // 128)
        kc_bytes = nt * (nt + 1) // 2 * 128 * 128 * mat_bytes
    else:
        kc_bytes = Nc * Nc * mat_bytes
    gemv_bytes = kc_bytes + 2 * Nc * n_rhs * 16                  # K_c once + qbar in + r out
    gemv_flops = 8.0 * Nc * Nc * n_rhs                           # complex MAC = 8 flops
    achieved_gbs = gemv_bytes / (gemv_ms * 1e-3) / 1e9
    kern_bytes = kc_bytes + Nc * n_rhs * 16                      # the streaming kernel: K_c once + qbar in
    kern_gbs = kern_bytes / (kern_ms * 1e-3) / 1e9
    kern_name = ("k_hemv_mfma" if lowp and packed else "k_gemv_mfma" if lowp
                 else "k_hemv64" if packed and dtype == "f64" else "k_hemv" if packed else "k_gemv2")
    # matrix-core work actually issued: per 64 x 64 block and 16-row group, four 16x16x32
    # products (16 columns: 4 rhs x re/im x leading/remainder)
    # issued 16x16x32 products: 16 per stored block for P1, 16 more per off-diagonal block
    # for P2 in the packed form (padding columns and the hi/lo split included)
    mfma_flops = ((16 * nbk * nbk if not packed else 16 * nbk * (nbk + 1) // 2 + 16 * nbk * (nbk - 1) // 2)
                  * (2.0 * 16 * 16 * 32)) if lowp else 0.0

    # ---- Method 3: the band product, timed the same way
    m3 = None
    if args.m3 is not None:
        prob.set_timing(2)
        torch.cuda.synchronize()
        prob.haydock(P, args.steps)
        torch.cuda.synchronize()
        band_ms_total, band_launches = prob.timing()
        prob.set_timing(False)
        band_ms = band_ms_total / max(1, band_launches)
        npair = cfg.nv * cfg.nc
        elem = 16 if dtype == "f64" else 8
        vbytes = 16 if dtype in ("f64", "f32v64") else 8
        # blocks once (without the padding offsets) + x once + the FP64 product written
        band_bytes = (cfg.nk_dense * prob.m3_offsets * npair * npair * elem
                      + n_rhs * prob.N * (vbytes + 16))
        m3 = {"w": args.m3, "offsets": prob.m3_offsets, "band_buffer_bytes": int(prob.band.numel()),
              "build_s": round(t_m3, 3), "band_product_avg_ms": round(band_ms, 5),
              "band_product_launches": band_launches, "band_product_bytes": int(band_bytes),
              "band_product_GBps": round(band_bytes / (band_ms * 1e-3) / 1e9, 1)}

    # ---- time to a converged eps2 at the workload's broadening, FP32 and BF16 forms
    race = None
    if args.config == "c1" and dtype == "f32" and args.m3 is None and not args.no_race:
        race = converged_race(bs, cfg, P, prob, eta=args.race_eta)

    # ---- time to eps2 on the host from a ready plan (chain + continued fraction + copy)
    om = cfg.omega()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch2 = prob.haydock(P, cfg.steps)
    eps = prob.continued_fraction(ch2, cfg.prefactor(), om, cfg.eta)
    eps_host = eps.cpu().numpy()
    t_eps = time.perf_counter() - t0
    status = ch2["status"].cpu().numpy().tolist()

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    # ---- algorithmic bytes of a whole step (for the step-level bandwidth)
    N, ncell, ndiv3 = prob.N, cfg.nk_coarse, cfg.n_div3
    ne = cfg.nv ** 2 + cfg.nc ** 2
    vec_bytes = 8 if dtype in ("f32", "bf16", "f16") else 16
    d_bytes = ncell * 8 * ne * ndiv3 * (16 if dtype == "f64" else 8)
    step_bytes = (gemv_bytes + 2 * d_bytes                    # K_c; overlaps in prolong and restrict
                  + n_rhs * N * vec_bytes * 6                  # psi_i x2, psi_{i-1}, w write/read, u write
                  + N * 8)                                     # transition energies (FP64)
    if m3 is not None:
        step_bytes += m3["band_product_bytes"] + n_rhs * N * 16       # band blocks, x; product read back
    out = {
        "metric": "Haydock steps/s",
        "value": round(steps_per_s, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f32v64": "f32/f64-vectors", "f64": "f64", "bf16": "bf16-kernel/f32",
                  "f16": "f16-kernel/f32"}[dtype],
        "data": "synthetic (seeded tight-binding crystal)",
        "config": {
            "workload": (f"{cfg.name}: {cfg.n_coarse}^3 coarse x {cfg.n_div}^3 divisions "
                         f"({cfg.nk_dense} dense k), {cfg.nv}v+{cfg.nc}c, N={N}, Kc {Nc}^2, "
                         f"{n_rhs} polarisations per step, {dtype} storage, FP64 accumulation"
                         + (f", Method 3 band w={args.m3}" if args.m3 is not None else "")),
            "n_coarse": cfg.n_coarse, "n_div": cfg.n_div, "nv": cfg.nv, "nc": cfg.nc, "N": N,
            "N_coarse": Nc, "polarisations": n_rhs, "parallelism": "single GPU",
        },
        "chain_steps_per_s": round(steps_per_s * n_rhs, 2),
        "fixed_ms_per_call": round(fixed_ms, 4),
        "step_algorithmic_bytes": int(step_bytes),
        "step_GBps": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "coarse_product": {
            "avg_ms": round(gemv_ms, 5), "launches": gemv_launches,
            "TFLOPs": round(gemv_flops / (gemv_ms * 1e-3) / 1e12, 3),
            "engine": ("matrix cores 16x16x32 " + dtype + ", FP32 in-block accumulation, blocks on and above the "
                       "diagonal (HBM-bound)") if lowp and packed
            else ("matrix cores 16x16x32 " + dtype + ", FP32 in-block accumulation (HBM-bound)") if lowp
            else ("VALU FP64 FMA on the packed Hermitian tiles (HBM-bound; no MFMA)") if packed and dtype == "f64"
            else ("VALU FP32 FMA on the packed Hermitian tiles, FP32 runs of 16 steps summed in FP64 "
                  "(HBM-bound; no MFMA)") if packed
            else "VALU FP64 FMA on " + ("FP64" if dtype == "f64" else "FP32") + " storage (HBM-bound; no MFMA)",
            "MFMA_TFLOPs_issued": round(mfma_flops / (gemv_ms * 1e-3) / 1e12, 3) if lowp else None,
            "MFMA_peak_TFLOPs": 2500.0 if lowp else None,
            "span": ("k_hemv_mfma + k_hm_reduce" if lowp and packed else "k_gemv_mfma + k_gemv_reduce" if lowp
                     else "k_hemv64 + k_hemv_reduce" if packed and dtype == "f64"
                     else "k_hemv + k_hemv_reduce" if packed else "k_gemv2 + k_gemv_reduce"),
            "algorithmic_bytes": int(gemv_bytes),
            "GBps": round(achieved_gbs, 1),
            "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.config, dtype),
        },
        "roofline": {
            "kernel": f"{kern_name}: the coarse product's streaming kernel (r = K_c qbar"
                      + (", packed Hermitian " + ("blocks" if lowp else "tiles") if packed else "")
                      + "), without the kernel that adds its partials",
            "bound": "hbm",
            "achieved": round(kern_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(kern_gbs / HBM_PEAK_GBS, 4),
            "avg_ms": round(kern_ms, 5),
            "algorithmic_bytes": int(kern_bytes),
            "traffic": measured_traffic(args.config, dtype, "traffic_bytes_per_launch_stream"),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
        "method3": m3,
        "time_to_eps2": race,
        "time_to_eps2_s": round(t_eps, 4),
        "setup_s": round(t_setup, 3),
        "inputs_s": round(t_inputs, 2),
        "chain_status": status,
        "eps2_peak": float(np.max(eps_host.imag)),
    }

    if m3 is not None:   # the band product is the dominant kernel of a Method 3 step
        ach = m3["band_product_GBps"]
        out["roofline"] = {"kernel": "Method 3 band product y = Delta x (k_m3_apply)", "bound": "hbm",
                           "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(ach / HBM_PEAK_GBS, 4),
                           "traffic": measured_m3_traffic(args.config, dtype, args.m3),
                           "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"}
        out["coarse_product_roofline_frac"] = round(achieved_gbs / HBM_PEAK_GBS, 4)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, bs, args.cpu_steps)
        if m3 is not None:
            out["cpu_baseline"] = m3_cpu_baseline(cfg, args.m3, out["cpu_baseline"])
    prob.close()
    if not args.no_batch and args.m3 is None:
        # the batching workload (48 Hamiltonians, 144 chains in HIP graphs), summarised
        del prob
        torch.cuda.empty_cache()
        b = run_batch(args, with_cpu=False)
        out["batch"] = {k: b[k] for k in ("metric", "value", "unit", "batch_s", "per_chain_steps_per_s",
                                          "graph_launches_per_batch", "sequential_host_launched_s",
                                          "speedup_vs_sequential", "chain_status", "inputs_s")}
        out["batch"]["workload"] = b["config"]["workload"]
        out["batch"]["roofline_frac"] = b["roofline"]["frac"] if b["roofline"] else None
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """The batching workload on its own: one JSON line (see run_batch)."""
    print(json.dumps(run_batch(args, with_cpu=not args.no_cpu_baseline)), flush=True)


def run_batch(args, with_cpu):
    """48 uneven Hamiltonians (16 displaced structures x 3 grids, nv 3, nc 3 or 6) with 3
    polarisations each = 144 Haydock chains of 200 steps, recorded once into a HIP graph
    and launched as one unit; tunables picked per shape by the autotuner.  Returns the
    aggregate and per-chain rates and the same chains run one plan after the other
    without the graph."""
    import torch

    import tbinputs as ti
    from paper_1602_01863_amd import bse
    from paper_1602_01863_amd.autotune import autotune, apply

    cfgs = ti.batch_configs()
    t0 = time.perf_counter()
    bss = [ti.band_structure(c) for c in cfgs]
    t_inputs = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    probs = [bse.problem_from_bands(b, c, dtype="f32", max_rhs=c.n_pol) for b, c in zip(bss, cfgs)]
    Ps = [torch.as_tensor(b.P_flat()).to("cuda").contiguous() for b in bss]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    # one tuning per shape, applied to every member of that shape
    t0 = time.perf_counter()
    tuned = {}
    for c, p, P in zip(cfgs, probs, Ps):
        if args.no_autotune:
            break
        key = (c.n_coarse, c.n_div, c.nc)
        if key not in tuned:
            tuned[key] = autotune(p, P, steps=10, repeats=2)
        else:
            apply(p, tuned[key])
    t_tune = time.perf_counter() - t0
    steps = cfgs[0].steps
    n_chains = sum(c.n_pol for c in cfgs)
    # the same chains one plan after the other, host-launched (reference)
    for p, P in zip(probs, Ps):
        p.haydock(P, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, P in zip(probs, Ps):
        p.haydock(P, steps)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    n_branches = bse.default_branches()
    batch = bse.BSEBatch(probs, Ps, steps, n_branches=n_branches)
    batch.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_launches):
        batch.run()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.batch_launches
    status = sorted({int(s) for ch in batch.chains for s in ch["status"].cpu().tolist()})
    shapes = {f"{k[0]}^3x{k[1]} 3v{k[2]}c": {"splits": v["splits"], "rhs_per_restrict_block": v["group"],
                                             "ms_per_step": round(v["ms_per_step"], 4)} for k, v in tuned.items()}
    out = {
        "metric": "batched Haydock chain-steps/s",
        "value": round(n_chains * steps / t_batch, 1),
        "unit": "chain-steps/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic (seeded tight-binding crystal, 16 displaced structures)",
        "config": {"workload": f"batching: {len(cfgs)} Hamiltonians x 3 polarisations = {n_chains} chains "
                               f"of {steps} steps (grids 4^3x2, 6^3x3, 8^3x4; nv 3, nc 3 or 6)",
                   "hamiltonians": len(cfgs), "chains": n_chains, "steps": steps,
                   "transitions_total": int(sum(p.N for p in probs)), "graph_branches": n_branches},
        "batch_s": round(t_batch, 4),
        "per_chain_steps_per_s": round(steps / t_batch, 1),
        "graph_launches_per_batch": n_branches,
        "kernel_launches_per_batch_without_graph": int(sum(3 + 5 * steps for _ in probs)),
        "sequential_host_launched_s": round(t_eager, 4),
        "speedup_vs_sequential": round(t_eager / t_batch, 3),
        "roofline": batch_roofline(cfgs, probs, steps, t_batch),
        "cpu_baseline": batch_cpu_baseline(cfgs, bss, steps) if with_cpu else None,
        "chain_status": status,
        "autotuned": shapes,
        "inputs_s": round(t_inputs, 1), "setup_s": round(t_setup, 2), "tune_s": round(t_tune, 2),
    }
    batch.close()
    for p in probs:
        p.close()
    return out


def batch_roofline(cfgs, probs, steps, t_batch):
    """Aggregate algorithmic HBM bytes of every member's steps (the packed K_c tiles on and
    above the diagonal once, the overlaps in prolong and restrict, the Lanczos vectors, the
    transition energies) over the batch time, against the HBM peak."""
    total = 0.0
    for c, p in zip(cfgs, probs):
        ne = c.nv ** 2 + c.nc ** 2
        d_bytes = c.nk_coarse * 8 * ne * c.n_div3 * 8
        nbk = (p.Nc + 127) // 128
        kc_bytes = nbk * (nbk + 1) // 2 * 128 * 128 * 8   # FP32 members: packed Hermitian tiles
        step = kc_bytes + 2 * p.Nc * c.n_pol * 16 + 2 * d_bytes + c.n_pol * p.N * 8 * 6 + p.N * 8
        total += step * steps
    ach = total / t_batch / 1e9
    return {"kernel": "all step kernels of the 48 members (aggregate)", "bound": "hbm",
            "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "algorithmic_bytes": int(total)}


def m3_cpu_baseline(cfg, w, m1, n_sample=256):
    """The oracle's Method 3 step: its Method 1 step (measured above) plus the band
    product, timed on a bounded sample (n_sample dense points x every offset, blocks of
    the band's shape) and scaled to all dense points."""
    import numpy as np

    import oracle as O

    off = O.m3.band_offsets(cfg.n_div, w)
    npair = cfg.nv * cfg.nc
    rng = np.random.default_rng(0)
    blocks = rng.normal(size=(n_sample, len(off), npair, npair)) + 0j
    x = rng.normal(size=(cfg.n_pol, cfg.n_trans)) + 0j
    ks = np.arange(n_sample)
    t0 = time.perf_counter()
    O.m3.band_product(blocks, off, x, cfg.n_coarse, cfg.n_div, ks)
    t_band = (time.perf_counter() - t0) * cfg.nk_dense / n_sample
    t_step = 1.0 / m1["value"] + t_band
    return {"value": round(1.0 / t_step, 4), "unit": "steps/s", "cores": m1["cores"], "kind": "oracle",
            "sample": (m1["sample"] + f"; plus the band product of {len(off)} offsets timed on {n_sample} of the "
                       f"{cfg.nk_dense} dense points and scaled ({t_band:.1f} s per step); the band build is setup")}


def batch_cpu_baseline(cfgs, bss, steps, sample_steps=2):
    """The oracle on a bounded sample of the batch: one member of each grid and band
    shape runs `sample_steps` Haydock steps (after its untimed setup); the batch's
    oracle time is estimated as every member's steps at its shape's measured rate."""
    import oracle as O

    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    per_step = {}
    for c, bs in zip(cfgs, bss):
        key = (c.n_coarse, c.n_div, c.nc)
        if key in per_step:
            continue
        Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, c.n_coarse, c.n_div, c.nv, c.nc)
        Kc = O.coarse_kernel(bs.vecs_coarse, bs.tau, c.nv, c.nc, c.n_coarse, c.n_div, c)
        delta = O.transition_energies(bs.eps_dense, c.nv, c.nc)
        op = O.InterpOperator(Dv, Dc, O.trilinear_weights(c.n_div), Kc, delta, c.n_coarse, c.n_div, c.nv, c.nc)
        t0 = time.perf_counter()
        O.haydock(op.apply, bs.P_flat(), sample_steps)
        per_step[key] = (time.perf_counter() - t0) / sample_steps
    t_total = sum(per_step[(c.n_coarse, c.n_div, c.nc)] * steps for c in cfgs)
    n_chain_steps = sum(c.n_pol for c in cfgs) * steps
    return {"value": round(n_chain_steps / t_total, 2), "unit": "chain-steps/s", "cores": int(cores),
            "kind": "oracle",
            "sample": (f"{sample_steps} Haydock steps (3 polarisations) of one member per shape "
                       f"({len(per_step)} shapes) with the FP64 NumPy oracle after its untimed setup; "
                       f"the batch's {len(cfgs)} members x {steps} steps estimated at those rates")}


def spectrum_race(args):
    """Time from a ready plan to eps2 on the host (chains, continued fraction, copy) on
    the headline workload, for the plain FP32 form and for the BF16 form alone, with its
    chains recorded into a HIP graph, and closed by the learned terminator (64 steps,
    the full plain chain when the error estimate exceeds 1e-3).  Each eps2 is compared
    with the plain FP32 one (relative L2), at the workload's broadening and two wider
    ones.  Prints one JSON line."""
    import numpy as np
    import torch

    import tbinputs as ti
    from paper_1602_01863_amd import bse
    from paper_1602_01863_amd import terminator as T

    cfg = ti.get_config(args.config)
    bs = ti.band_structure(cfg)
    om, C, steps = cfg.omega(), cfg.prefactor(), cfg.steps
    etas = (cfg.eta, 0.2, 0.5)
    P = torch.as_tensor(bs.P_flat()).to("cuda").contiguous()
    probs = {dt: bse.problem_from_bands(bs, cfg, dtype=dt, max_rhs=cfg.n_pol) for dt in ("f32", "bf16")}
    graph = bse.BSEBatch([probs["bf16"]], [P], steps, n_branches=1)
    net = T.TerminatorMLP.load(T.default_weights_path())

    def eps2(prob, ch, eta):
        return prob.continued_fraction(ch, C, om, eta).cpu().numpy().imag

    forms = {
        "f32": lambda eta: (eps2(probs["f32"], probs["f32"].haydock(P, steps), eta), None),
        "bf16": lambda eta: (eps2(probs["bf16"], probs["bf16"].haydock(P, steps), eta), None),
        "bf16_graph": lambda eta: (eps2(probs["bf16"], graph.run()[0], eta), None),
        "bf16_terminator": lambda eta: _terminated(T, probs["bf16"], P, net, steps, C, om, eta),
    }
    out_forms = {}
    ref = {}
    for name, fn in forms.items():
        fn(etas[0])   # warm
        rows = {}
        for eta in etas:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, fb = fn(eta)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if name == "f32":
                ref[eta] = e
            err = float(np.linalg.norm(e - ref[eta]) / np.linalg.norm(ref[eta]))
            rows[str(eta)] = {"s": round(dt, 4), "eps2_rel_err_vs_f32": err}
            if fb is not None:
                rows[str(eta)]["fallback_fraction"] = float(np.mean(fb))
        out_forms[name] = rows
    graph.close()
    for p in probs.values():
        p.close()
    out = {"metric": "time to eps2 from a ready plan", "unit": "s", "higher_is_better": False, "n_gpus": 1,
           "data": "synthetic (seeded tight-binding crystal)",
           "config": {"workload": f"{cfg.name}: {cfg.n_coarse}^3 x {cfg.n_div}, {cfg.nv}v{cfg.nc}c, N={cfg.n_trans}, "
                                  f"{steps} steps x {cfg.n_pol} polarisations, {cfg.n_omega} omega points"},
           "forms": out_forms}
    print(json.dumps(out), flush=True)


def converged_race(bs, cfg, P, prob_f32, tol=1e-3, ref_steps=1800, check_every=20, cap=3000, eta=None):
    """Time to a converged eps2 at the workload's broadening (Sec. 2 after Eq. fraccont:
    chains run until the spectrum stops changing), from a ready plan to eps on the host,
    for the plain FP32 form and the BF16 coarse kernel, with bse_haydock_converge (a check
    every check_every steps; stop when eps2 moved by at most tol of its peak).  Each
    spectrum is compared (relative L2 of eps2, worst polarisation) with the converged
    FP64 spectrum: an FP64 chain of ref_steps steps (at eta = 0.05 eV its own change
    from 1200 to 1800 steps is ~1e-8)."""
    import numpy as np
    import torch

    from paper_1602_01863_amd import bse

    om, C = cfg.omega(), cfg.prefactor()
    eta = cfg.eta if eta is None else eta
    p64 = bse.problem_from_bands(bs, cfg, dtype="f64", max_rhs=cfg.n_pol)
    ch = p64.haydock(P, ref_steps)
    ref = p64.continued_fraction(ch, C, om, eta).cpu().numpy().imag
    p64.close()
    del p64
    torch.cuda.empty_cache()
    out = {"eta_eV": eta, "tolerance": 1e-3, "stop_rule": f"max change <= {tol} x peak, checked every "
           f"{check_every} steps", "reference": f"FP64 chain of {ref_steps} steps", "forms": {}}
    probs = {"f32": prob_f32, "bf16": bse.problem_from_bands(bs, cfg, dtype="bf16", max_rhs=cfg.n_pol)}
    # "_closed": every checked fraction closed by the constant chain of the chain's last 16
    # coefficients (the square-root terminator), so the stop rule sees the closed spectrum
    runs = [("f32", "f32", 0), ("bf16", "bf16", 0), ("f32_closed", "f32", 16), ("bf16_closed", "bf16", 16)]
    for name, pk, closure in runs:
        prob = probs[pk]
        prob.haydock_converge(P, cap, om, eta, C, tol, check_every, closure=closure)   # warm
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chc, eps = prob.haydock_converge(P, cap, om, eta, C, tol, check_every, closure=closure)
            e2 = eps.cpu().numpy().imag
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        err = max(float(np.linalg.norm(e2[r] - ref[r]) / np.linalg.norm(ref[r])) for r in range(cfg.n_pol))
        out["forms"][name] = {"seconds": round(best, 4), "steps": chc["steps"].cpu().numpy().tolist(),
                              "eps2_rel_err": float("%.3g" % err), "within": bool(err <= 1e-3)}
    prob_f32.haydock_converge(P, 1, om, eta, C, tol, check_every, closure=0)   # leave the plan as it was
    probs["bf16"].close()
    f = out["forms"]
    out["bf16_speedup_vs_f32"] = round(f["f32"]["seconds"] / f["bf16"]["seconds"], 3)
    out["closure_speedup_f32"] = round(f["f32"]["seconds"] / f["f32_closed"]["seconds"], 3)
    fastest = min((v["seconds"], k) for k, v in f.items() if v["within"])
    out["fastest_within"] = {"form": fastest[1], "seconds": fastest[0],
                             "speedup_vs_f32": round(f["f32"]["seconds"] / fastest[0], 3)}
    return out


def _terminated(T, prob, P, net, steps, C, om, eta):
    """eps2 closed by the terminator after 64 steps, with the full-chain fallback."""
    eps, fb = T.run_with_fallback(prob, P, net, steps, C, om, eta, threshold=1e-3)
    return eps.imag, fb


def cpu_baseline(cfg, bs, n_steps):
    """Time the plain FP64 oracle's Haydock steps on the host (same workload)."""
    import numpy as np

    import oracle as O

    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    Kc = O.coarse_kernel(bs.vecs_coarse, bs.tau, cfg.nv, cfg.nc, cfg.n_coarse, cfg.n_div, cfg)
    delta = O.transition_energies(bs.eps_dense, cfg.nv, cfg.nc)
    op = O.InterpOperator(Dv, Dc, O.trilinear_weights(cfg.n_div), Kc, delta, cfg.n_coarse, cfg.n_div,
                          cfg.nv, cfg.nc)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.haydock(op.apply, bs.P_flat(), n_steps)
    t = time.perf_counter() - t0
    return {"value": round(n_steps / t, 4), "unit": "steps/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"{n_steps} Haydock steps of the same workload (all {cfg.n_pol} polarisations per "
                       f"step) with the FP64 NumPy oracle, after its untimed setup of {t_setup:.0f} s "
                       f"(overlaps, coarse kernel)")}


if __name__ == "__main__":
    main()
