"""Write the oracle's Haydock chains for a workload as golden text.

Runs only the seeded inputs (tbinputs) and the CPU oracle.  Two chains per
polarisation are written:

* ``<name>_oracle_chain.txt``        plain FP64 (the parity reference);
* ``<name>_oracle_chain_f32emu.txt`` the same computation with the coarse
  kernel, the overlaps and every stored Lanczos vector rounded to complex64,
  arithmetic still FP64: the rounding floor of FP32 storage.

Each row: pol, pnorm2, steps, a_1..a_m, b_1..b_{m+1}.

With --long M only the FP64 chain is written, M steps long, as
``<name>_oracle_chain_<M>.txt``: long enough for the spectrum at the workload's
broadening to have converged (the reference of the converged-spectrum checks).

Usage: python tests/golden/make_oracle_chains.py c1 [--long 1200]
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O      # noqa: E402
import tbinputs as ti   # noqa: E402


def _rows(ch):
    out = []
    for r in range(ch["a"].shape[0]):
        out.append(np.concatenate([[r, ch["pnorm2"][r], ch["steps"][r]], ch["a"][r], ch["b"][r]]))
    return np.array(out)


def main(name: str, long_steps: int = 0):
    cfg = ti.get_config(name)
    if long_steps:
        cfg = cfg.with_(steps=long_steps)
    t0 = time.time()
    bs = ti.band_structure(cfg)
    Dv, Dc = O.overlaps(bs.vecs_coarse, bs.vecs_dense, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    Kc = O.coarse_kernel(bs.vecs_coarse, bs.tau, cfg.nv, cfg.nc, cfg.n_coarse, cfg.n_div, cfg)
    delta = O.transition_energies(bs.eps_dense, cfg.nv, cfg.nc)
    f = O.trilinear_weights(cfg.n_div)
    print(f"setup {time.time() - t0:.1f} s", flush=True)
    header = (f"Oracle Haydock chains, workload {cfg.name}: {cfg.n_coarse}^3 coarse, n_div "
              f"{cfg.n_div}, nv {cfg.nv}, nc {cfg.nc}, seed {cfg.seed}, {cfg.steps} steps, "
              f"{cfg.n_pol} polarisations.\nWritten by tests/golden/make_oracle_chains.py "
              f"{name} (oracle only).\nColumns: pol, pnorm2, steps, a_1..a_m, b_1..b_(m+1)")
    op = O.InterpOperator(Dv, Dc, f, Kc, delta, cfg.n_coarse, cfg.n_div, cfg.nv, cfg.nc)
    t0 = time.time()
    ch = O.haydock(op.apply, bs.P_flat(), cfg.steps)
    print(f"fp64 chain {time.time() - t0:.1f} s", flush=True)
    if long_steps:
        np.savetxt(os.path.join(HERE, f"{name}_oracle_chain_{long_steps}.txt"), _rows(ch), fmt="%.17e",
                   header=header.replace("(oracle only)", f"--long {long_steps} (oracle only)"))
        return
    np.savetxt(os.path.join(HERE, f"{name}_oracle_chain.txt"), _rows(ch), fmt="%.17e",
               header=header)
    c64 = np.complex64
    op32 = O.InterpOperator(Dv.astype(c64).astype(complex), Dc.astype(c64).astype(complex), f,
                            Kc.astype(c64).astype(complex), delta, cfg.n_coarse, cfg.n_div,
                            cfg.nv, cfg.nc)
    t0 = time.time()
    ch32 = O.haydock(op32.apply, bs.P_flat(), cfg.steps, round_dtype=c64)
    print(f"f32-storage chain {time.time() - t0:.1f} s", flush=True)
    np.savetxt(os.path.join(HERE, f"{name}_oracle_chain_f32emu.txt"), _rows(ch32), fmt="%.17e",
               header=header.replace("Oracle Haydock chains",
                                     "Oracle Haydock chains with complex64 storage rounding"))
    om = cfg.omega()
    e64 = O.continued_fraction(ch["a"], ch["b"], ch["pnorm2"], cfg.prefactor(), om, cfg.eta)
    e32 = O.continued_fraction(ch32["a"], ch32["b"], ch32["pnorm2"], cfg.prefactor(), om, cfg.eta)
    for r in range(cfg.n_pol):
        err = np.linalg.norm(e32[r].imag - e64[r].imag) / np.linalg.norm(e64[r].imag)
        ea = np.linalg.norm(ch32["a"][r, :50] - ch["a"][r, :50]) / np.linalg.norm(ch["a"][r, :50])
        eb = np.linalg.norm(ch32["b"][r, 1:51] - ch["b"][r, 1:51]) / np.linalg.norm(ch["b"][r, 1:51])
        print(f"pol {r}: f32-storage floor  eps2 rel-L2 {err:.3e}  a[:50] {ea:.3e}  b[:50] {eb:.3e}")


if __name__ == "__main__":
    args = sys.argv[1:]
    long_steps = 0
    if "--long" in args:
        k = args.index("--long")
        long_steps = int(args[k + 1])
        del args[k:k + 2]
    main(args[0] if args else "c1", long_steps)
