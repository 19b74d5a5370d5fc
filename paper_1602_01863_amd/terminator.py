"""Learned continued-fraction terminator.

A Haydock chain that is cut after m steps leaves the tail of Eq. (fraccont)
unknown; the paper runs the chain until the spectrum stops changing.  Here a small
dense network (4 layers, width 128, GELU) predicts, from the first M_IN = 64
coefficients of a chain, the next M_OUT = 192 coefficients and the asymptotic pair
(a_inf, b_inf) that closes the fraction as a constant chain.  The chain can then
stop after 64 steps, plus 32 that check the prediction (the error estimate: how far
the closed spectrum moves when those computed coefficients replace the predicted
ones); when the estimate says the closed spectrum is not good enough, the full plain
chain is run instead (the fallback, which is also the reference in the tests).

Everything runs in the library's kernels: training (FP32 dense layers, GELU, mean
squared error, Adam) and inference (BF16 on the matrix cores), the chains (the
method's own Haydock runs) and the closed continued fraction.  PyTorch only holds
device memory.

Normalisation of one chain from its first 64 coefficients a_1..a_64, b_2..b_65:
centre c = mean(a_1..a_64), scale s = 2 mean(b_2..b_65) (about the half-width of the
band the chain sees); inputs (a_n - c) / s and b_n / s.  The targets are residuals
against the method's own closure without the network (the constant chain given by
the means of the last 16 computed a_n and b_n): the network learns corrections to
that closure, and a network that predicts zero reproduces it.  The tail targets are
smoothed with a 32-step moving average: the broadened spectrum depends on the slow
trend of the coefficients, while their step-to-step fluctuations past the converged
head are rounding-driven and not predictable from the head (fitting them made the
closed spectra worse than the plain closure in our measurements).
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import bse

M_IN = 64
M_OUT = 192
WIDTH = 128
N_IN = 2 * M_IN
N_OUT = 2 * M_OUT + 2
SIZES = (N_IN, WIDTH, WIDTH, WIDTH, N_OUT)
TAIL_AVG = 64          # steps after M_IN + M_OUT averaged into the asymptotic targets
CHAIN_LEN = M_IN + M_OUT + TAIL_AVG


# ---- normalisation -------------------------------------------------------------------
def normalise(a, b):
    """(inputs [n, 128], centre [n], scale [n]) from a [n, >= 64], b [n, >= 65]."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = a[:, :M_IN].mean(axis=1)
    s = 2.0 * b[:, 1:M_IN + 1].mean(axis=1)
    s = np.where(s > 0, s, 1.0)
    x = np.concatenate([(a[:, :M_IN] - c[:, None]) / s[:, None], b[:, 1:M_IN + 1] / s[:, None]], axis=1)
    return x, c, s


HEAD_K = 16            # computed coefficients averaged into the method's own closure
SMOOTH = 32            # moving-average window of the tail targets


def head_closure(a, b, k=HEAD_K):
    """The method's own closure without the network: (a_inf, b_inf) = means of the last
    k computed coefficients a_{65-k}..a_64 and b_{66-k}..b_65."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return a[:, M_IN - k:M_IN].mean(axis=1), b[:, M_IN + 1 - k:M_IN + 1].mean(axis=1)


def moving_average(seg, w):
    """Row-wise moving average of window w, ends padded with the first / last value."""
    if w <= 1:
        return seg
    k = np.ones(w) / w
    pad = np.concatenate([seg[:, :1].repeat(w // 2, 1), seg, seg[:, -1:].repeat(w - 1 - w // 2, 1)], axis=1)
    return np.stack([np.convolve(r, k, mode="valid") for r in pad])


def targets(a, b, c, s, smooth=SMOOTH):
    """Normalised residual targets [n, 386] from chains of CHAIN_LEN steps: the tail
    a_65..a_256, b_66..b_257 (moving-averaged) and the means of the next TAIL_AVG
    coefficients, minus the head closure."""
    ha, hb = head_closure(a, b)
    at = (a[:, M_IN:M_IN + M_OUT] - ha[:, None]) / s[:, None]
    bt = (b[:, M_IN + 1:M_IN + M_OUT + 1] - hb[:, None]) / s[:, None]
    ainf = (a[:, M_IN + M_OUT:CHAIN_LEN].mean(axis=1) - ha) / s
    binf = (b[:, M_IN + M_OUT + 1:CHAIN_LEN + 1].mean(axis=1) - hb) / s
    return np.concatenate([moving_average(at, smooth), moving_average(bt, smooth), ainf[:, None], binf[:, None]],
                          axis=1)


def denormalise(y, a, b, s):
    """Predicted (a_65..a_256, b_66..b_257, a_inf, b_inf) in eV from the network's
    residuals y and the computed head a, b."""
    y = np.asarray(y, dtype=np.float64)
    ha, hb = head_closure(a, b)
    at = y[:, :M_OUT] * s[:, None] + ha[:, None]
    bt = np.abs(y[:, M_OUT:2 * M_OUT] * s[:, None] + hb[:, None])
    ainf = y[:, 2 * M_OUT] * s + ha
    binf = np.abs(y[:, 2 * M_OUT + 1] * s + hb)
    return at, bt, ainf, binf


# ---- the network on the device ----------------------------------------------------------
class TerminatorMLP:
    """Dense GELU network with parameters in device memory, trained by the library's kernels."""

    def __init__(self, seed: int = 0, device="cuda", sizes=SIZES):
        self.sizes = tuple(sizes)
        self.device = torch.device(device)
        rng = np.random.default_rng(seed)
        self.W, self.b = [], []
        for n_in, n_out in zip(self.sizes[:-1], self.sizes[1:]):
            lim = 1.0 / math.sqrt(n_in)
            self.W.append(torch.tensor(rng.uniform(-lim, lim, size=(n_out, n_in)), dtype=torch.float32,
                                       device=self.device))
            self.b.append(torch.zeros(n_out, dtype=torch.float32, device=self.device))
        self._adam = None
        self.step = 0

    @property
    def n_layers(self):
        return len(self.W)

    def _act(self, i):
        return bse.BSE_ACT_GELU if i < self.n_layers - 1 else bse.BSE_ACT_NONE

    # -- FP32 forward with cache, backward --------------------------------------------------
    def forward(self, x: torch.Tensor, cache: bool = False):
        h = x.contiguous()
        saved = []
        for i in range(self.n_layers):
            n_out = self.sizes[i + 1]
            z = torch.empty(h.shape[0], n_out, dtype=torch.float32, device=self.device)
            y = torch.empty_like(z)
            bse.bse_dense_forward(h, self.W[i], self.b[i], z, y, h.shape[0], self.sizes[i], n_out, self._act(i))
            saved.append((h, z))
            h = y
        return (h, saved) if cache else h

    def backward(self, saved, dy: torch.Tensor):
        grads = [None] * self.n_layers
        g = dy.contiguous()
        for i in range(self.n_layers - 1, -1, -1):
            h, z = saved[i]
            n_in, n_out = self.sizes[i], self.sizes[i + 1]
            dW = torch.empty_like(self.W[i])
            db = torch.empty_like(self.b[i])
            dx = torch.empty(h.shape[0], n_in, dtype=torch.float32, device=self.device) if i > 0 else None
            work = torch.empty(h.shape[0], n_out, dtype=torch.float32, device=self.device)
            bse.bse_dense_backward(h, self.W[i], z, g, dx, dW, db, h.shape[0], n_in, n_out, self._act(i), work)
            grads[i] = (dW, db)
            g = dx
        return grads

    def loss_and_grads(self, x, t):
        y, saved = self.forward(x, cache=True)
        dy = torch.empty_like(y)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        bse.bse_mse_loss(y, t.contiguous(), dy, loss, y.numel())
        return loss, self.backward(saved, dy)

    def adam(self, grads, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        if self._adam is None:
            self._adam = [(torch.zeros_like(p), torch.zeros_like(p)) for p in self.params()]
        self.step += 1
        for p, g, (m, v) in zip(self.params(), [x for pair in grads for x in pair], self._adam):
            bse.bse_adam_step(p, g, m, v, p.numel(), lr, beta1, beta2, eps, self.step)

    def params(self):
        out = []
        for W, b in zip(self.W, self.b):
            out += [W, b]
        return out

    # -- BF16 inference ----------------------------------------------------------------------
    def prepare_bf16(self):
        self.Wb = []
        for W in self.W:
            wb = torch.empty(W.shape, dtype=torch.int16, device=self.device)
            bse.bse_to_bf16(W, wb, W.numel())
            self.Wb.append(wb)

    def infer_bf16(self, x: torch.Tensor) -> torch.Tensor:
        """FP32 outputs of the network run in BF16 on the matrix cores."""
        if not hasattr(self, "Wb"):
            self.prepare_bf16()
        n = x.shape[0]
        h = torch.empty(n, self.sizes[0], dtype=torch.int16, device=self.device)
        bse.bse_to_bf16(x.contiguous(), h, x.numel())
        for i in range(self.n_layers):
            n_out = self.sizes[i + 1]
            last = i == self.n_layers - 1
            yb = None if last else torch.empty(n, n_out, dtype=torch.int16, device=self.device)
            yf = torch.empty(n, n_out, dtype=torch.float32, device=self.device) if last else None
            bse.bse_dense_forward_bf16(h, self.Wb[i], self.b[i], yb, yf, n, self.sizes[i], n_out, self._act(i))
            h = yb if not last else yf
        return h

    # -- persistence ---------------------------------------------------------------------------
    def save(self, path, **meta):
        arrs = {f"W{i}": W.cpu().numpy() for i, W in enumerate(self.W)}
        arrs.update({f"b{i}": b.cpu().numpy() for i, b in enumerate(self.b)})
        arrs["sizes"] = np.array(self.sizes)
        for k, v in meta.items():
            arrs[f"meta_{k}"] = np.asarray(v)
        np.savez(path, **arrs)

    @classmethod
    def load(cls, path, device="cuda"):
        z = np.load(path, allow_pickle=False)
        net = cls(device=device, sizes=tuple(int(v) for v in z["sizes"]))
        for i in range(net.n_layers):
            net.W[i] = torch.tensor(z[f"W{i}"], dtype=torch.float32, device=net.device)
            net.b[i] = torch.tensor(z[f"b{i}"], dtype=torch.float32, device=net.device)
        return net


def train(net: TerminatorMLP, x: np.ndarray, t: np.ndarray, epochs=40, batch=256, lr=1e-3, seed=0, log=None):
    """Minibatch Adam on the mean squared error; returns the loss of every epoch."""
    dev = net.device
    X = torch.tensor(x, dtype=torch.float32, device=dev)
    T = torch.tensor(t, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n), device=dev)
        tot = torch.zeros(1, dtype=torch.float64, device=dev)
        nb = 0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            loss, grads = net.loss_and_grads(X[idx].contiguous(), T[idx].contiguous())
            net.adam(grads, lr=lr * (0.5 * (1 + math.cos(math.pi * ep / epochs))))
            tot += loss
            nb += 1
        hist.append(float(tot.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return hist


# ---- chains from the method -------------------------------------------------------------
def polarisation_mix(P3: np.ndarray, n: int, rng) -> np.ndarray:
    """n random unit combinations of the 3 Cartesian P vectors ([3, N] -> [n, N])."""
    e = rng.normal(size=(n, P3.shape[0]))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    return e @ P3


def generate_chains(cfgs, steps=CHAIN_LEN, rhs=4, dtype=None, seed=0, workers=8, log=None):
    """Run the method's Haydock chains on the problems of cfgs (rhs random polarisations
    each) and return (a [n, steps], b [n, steps + 1]) as FP64 host arrays."""
    import tbinputs as ti

    rng = np.random.default_rng(seed)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        bss = list(ex.map(ti.band_structure, cfgs))
    A, B = [], []
    for k, (cfg, bs) in enumerate(zip(cfgs, bss)):
        dt = dtype or {"c128": "f64", "c64": "f32"}[cfg.dtype]
        prob = bse.problem_from_bands(bs, cfg, dtype=dt, max_rhs=rhs)
        P = polarisation_mix(bs.P_flat(), rhs, rng)
        ch = prob.haydock(P, steps)
        ok = ch["status"].cpu().numpy() == bse.BSE_OK
        A.append(ch["a"].cpu().numpy()[ok])
        B.append(ch["b"].cpu().numpy()[ok])
        prob.close()
        if log and (k + 1) % 200 == 0:
            log(f"chains: {k + 1} / {len(cfgs)} problems")
    return np.concatenate(A), np.concatenate(B)


def training_configs(n_c0: int, n_c1: int, seed0: int = 10_000):
    """Seeded problems of the C0 family (4^3 x 2, 6 orbitals, 3v3c, FP64) and of the C1
    family at 2 divisions (8^3 x 2, 9 orbitals, 3v6c, FP32); seeds from seed0 up."""
    import tbinputs as ti

    out = []
    for i in range(n_c0):
        out.append(ti.get_config("c0").with_(name=f"t0_{i}", seed=seed0 + i, n_pol=3))
    for i in range(n_c1):
        out.append(ti.get_config("c1").with_(name=f"t1_{i}", seed=seed0 + n_c0 + i, n_div=2))
    return out


# ---- spectra --------------------------------------------------------------------------
def closed_spectrum(a, b, pnorm2, a_inf, b_inf, prefactor, omega, eta, device="cuda"):
    """eps_M of chains a [n, m], b [n, m + 1] closed by (a_inf, b_inf), on the device."""
    a = torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(device)
    b = torch.as_tensor(np.ascontiguousarray(b), dtype=torch.float64).to(device)
    n, m = a.shape
    pn = torch.as_tensor(np.asarray(pnorm2, dtype=np.float64)).to(device)
    ai = torch.as_tensor(np.asarray(a_inf, dtype=np.float64)).to(device)
    bi = torch.as_tensor(np.asarray(b_inf, dtype=np.float64)).to(device)
    om = torch.as_tensor(np.asarray(omega, dtype=np.float64)).to(device)
    er = torch.empty(n, om.numel(), dtype=torch.float64, device=device)
    ei = torch.empty_like(er)
    bse.bse_continued_fraction_terminated(a, b, m, m + 1, m, pn, ai, bi, n, prefactor, om, om.numel(), eta, er, ei)
    return (er + 1j * ei).cpu().numpy()


def predict_tail(net: TerminatorMLP, a, b, bf16=True):
    """(a [n, 256], b [n, 257], a_inf, b_inf): 64 computed coefficients + the network's
    192 and its asymptotic pair."""
    x, c, s = normalise(a, b)
    X = torch.tensor(x, dtype=torch.float32, device=net.device)
    y = (net.infer_bf16(X) if bf16 else net.forward(X)).cpu().numpy()
    at, bt, ainf, binf = denormalise(y, a, b, s)
    A = np.concatenate([a[:, :M_IN], at], axis=1)
    B = np.concatenate([b[:, :M_IN + 1], bt], axis=1)
    return A, B, ainf, binf


K_CHECK = 32           # computed coefficients past the network's input that check its prediction


def terminated_eps(net, a, b, pnorm2, prefactor, omega, eta, threshold=1e-3, bf16=True):
    """eps_M closed by the network's tail, checked against K_CHECK more computed steps.

    a, b hold M_IN + K_CHECK computed coefficients per chain.  The network predicts
    a_65..a_256 from the first 64; the delivered spectrum (closure B) takes the computed
    a_65..a_96, b_66..b_97 in place of the predicted ones and the prediction from there
    on.  The error estimate is how far the spectrum moves when those 32 computed
    coefficients replace the predicted ones,
        est = ||eps2(B) - eps2(A)|| / ||eps2(B)||,  A = the 64 computed + all predicted,
    i.e. the evidence the chain itself gives on the prediction (the paper's own stop rule
    compares spectra of successive chain lengths in the same way).  Chains with
    est > threshold are marked for the fallback (the full plain chain)."""
    A, B, ainf, binf = predict_tail(net, a, b, bf16=bf16)
    e_a = closed_spectrum(A, B, pnorm2, ainf, binf, prefactor, omega, eta)
    A2, B2 = A.copy(), B.copy()
    A2[:, M_IN:M_IN + K_CHECK] = a[:, M_IN:M_IN + K_CHECK]
    B2[:, M_IN + 1:M_IN + K_CHECK + 1] = b[:, M_IN + 1:M_IN + K_CHECK + 1]
    e_b = closed_spectrum(A2, B2, pnorm2, ainf, binf, prefactor, omega, eta)
    est = np.linalg.norm(e_b.imag - e_a.imag, axis=1) / np.maximum(np.linalg.norm(e_b.imag, axis=1), 1e-300)
    return e_b, est, est > threshold


def run_with_fallback(prob, P, net, n_full, prefactor, omega, eta, threshold=1e-3):
    """Spectrum of the chains of prob for the start vectors P ([n_rhs, N]): 96 steps
    closed by the network when its error estimate is <= threshold, else the plain chain of
    n_full steps (the fallback).  Returns (eps_M [n_rhs, n_omega], fell_back [n_rhs])."""
    m = M_IN + K_CHECK
    ch = prob.haydock(P, m)
    a, b = ch["a"].cpu().numpy(), ch["b"].cpu().numpy()
    pn = ch["pnorm2"].cpu().numpy()
    eps, est, fb = terminated_eps(net, a[:, :m], b[:, :m + 1], pn, prefactor, omega, eta, threshold)
    if fb.any():
        full = prob.haydock(P, n_full)
        plain = prob.continued_fraction(full, prefactor, omega, eta).cpu().numpy()
        eps[fb] = plain[fb]
    return eps, fb


def default_weights_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "terminator_mlp.npz")


# ---- command line: train the network, evaluate it against long plain chains ---------------
def evaluation_configs(n: int, seed0: int = 90_000):
    """Held-out problems at the C1 size (8^3 x 4, 9 orbitals, 3v6c); seeds disjoint from training."""
    import tbinputs as ti

    return [ti.get_config("c1").with_(name=f"e1_{i}", seed=seed0 + i) for i in range(n)]


def evaluate(net, n_problems=8, ref_steps=600, etas=(0.05, 0.1, 0.2), log=None):
    """Errors of eps2 from 64 steps (truncated; closed by the head; closed by the network)
    and from 300 plain steps, against the ref_steps-step chains (relative L2 per chain,
    averaged), on held-out C1-size problems with the 3 Cartesian polarisations."""
    import tbinputs as ti

    cfgs = evaluation_configs(n_problems)
    with ThreadPoolExecutor(max_workers=8) as ex:
        bss = list(ex.map(ti.band_structure, cfgs))
    rows = {}
    A, B, PN = [], [], []
    for cfg, bs in zip(cfgs, bss):
        prob = bse.problem_from_bands(bs, cfg, dtype="f32", max_rhs=3)
        ch = prob.haydock(bs.P_flat(), ref_steps)
        A.append(ch["a"].cpu().numpy())
        B.append(ch["b"].cpu().numpy())
        PN.append(ch["pnorm2"].cpu().numpy())
        prob.close()
    a, b, pn = np.concatenate(A), np.concatenate(B), np.concatenate(PN)
    cfg = cfgs[0]
    om = cfg.omega()
    C = cfg.prefactor()
    zeros = np.zeros(len(a))

    def trunc(m, eta):
        # the plain fraction cut after a_m: b_{m+1} = 0 removes the closure term
        bm = b[:, :m + 1].copy()
        bm[:, m] = 0.0
        return closed_spectrum(a[:, :m], bm, pn, zeros, zeros, C, om, eta)

    for eta in etas:
        ref = trunc(ref_steps, eta).imag
        errs = lambda e: np.linalg.norm(e.imag - ref, axis=1) / np.linalg.norm(ref, axis=1)
        err = lambda e: float(np.mean(errs(e)))
        A, Bq, ainf, binf = predict_tail(net, a, b)
        e_net64 = closed_spectrum(A, Bq, pn, ainf, binf, C, om, eta)
        e_net, est, fb = terminated_eps(net, a, b, pn, C, om, eta)
        ha, hb = head_closure(a, b)
        e_head = closed_spectrum(a[:, :M_IN], b[:, :M_IN + 1], pn, ha, hb, C, om, eta)
        true = errs(e_net)
        acc = ~fb
        rows[str(eta)] = {"truncated_64": err(trunc(M_IN, eta)), "head_closure_64": err(e_head),
                          "network_64": err(e_net64), "network_96_checked": err(e_net),
                          "plain_96": err(trunc(M_IN + K_CHECK, eta)), "plain_300": err(trunc(300, eta)),
                          "fallback_fraction": float(fb.mean()), "estimate_mean": float(est.mean()),
                          "accepted": int(acc.sum()), "false_accepts": int((acc & (true > 1e-3)).sum()),
                          "worst_accepted_error": float(true[acc].max()) if acc.any() else None}
        if log:
            log(f"eta {eta}: {rows[str(eta)]}")
    return rows


def main(argv=None):
    import argparse
    import json
    import time

    ap = argparse.ArgumentParser(prog="python -m paper_1602_01863_amd.terminator")
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train", help="generate chains with the method and train the network")
    tr.add_argument("--c0", type=int, default=2500, help="C0-family problems (4 chains each)")
    tr.add_argument("--c1", type=int, default=2500, help="C1-family problems at 2 divisions (4 chains each)")
    tr.add_argument("--epochs", type=int, default=60)
    tr.add_argument("--out", default=default_weights_path())
    ev = sub.add_parser("evaluate", help="held-out C1-size chains against 600-step plain chains")
    ev.add_argument("--weights", default=default_weights_path())
    ev.add_argument("--problems", type=int, default=8)
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    if args.cmd == "train":
        t0 = time.perf_counter()
        a, b = generate_chains(training_configs(args.c0, args.c1), log=log)
        t_gen = time.perf_counter() - t0
        x, c, s = normalise(a, b)
        t = targets(a, b, c, s)
        log(f"{len(a)} chains in {t_gen:.0f} s")
        net = TerminatorMLP(seed=0)
        t0 = time.perf_counter()
        hist = train(net, x, t, epochs=args.epochs, log=log)
        t_train = time.perf_counter() - t0
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        net.save(args.out, n_chains=len(a), loss=np.array(hist), chain_len=CHAIN_LEN, c0=args.c0, c1=args.c1,
                 gen_s=t_gen, train_s=t_train)
        log(json.dumps({"chains": len(a), "loss_first": hist[0], "loss_last": hist[-1], "gen_s": round(t_gen, 1),
                        "train_s": round(t_train, 1), "out": args.out}))
    else:
        net = TerminatorMLP.load(args.weights)
        rows = evaluate(net, n_problems=args.problems, log=log)
        log(json.dumps(rows))


if __name__ == "__main__":
    main()
