"""Training and evaluation of the HOS surrogate on trajectories the library
itself generates on the GPU.

Data: seeded JONSWAP seas (Hs/lambda_p ~ U[0.01, 0.03], gamma 3.3, deep
water, lambda_p = 2 pi, g = 1) on n x n modes over `periods` peak
wavelengths, HOS order 3, dt = Tp / 64; every `stride` steps a pair (network
input at t, residual target over the linear propagator at t + stride dt).
All arithmetic (HOS steps, features, linear propagation, targets, forward,
backward, Adam) runs in the HIP library; torch only holds device buffers and
draws minibatch indices.

  python -m paper_2005_12716_amd.train --trajectories 2000 --steps 200 --iters 20000 --out fno.npz
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

import synth
from paper_2005_12716_amd import lib

LAM = 2.0 * math.pi  # peak wavelength (k_p = 1, g = 1, T_p = 2 pi)


def sea_hos(n: int, periods: float, seed: int, order_m: int = 3) -> lib.Hos:
    L = periods * LAM
    d = lib.hos_desc(3, n, n, L, L, -1.0, order_m=order_m, dt=LAM / 64)
    sp = synth.surrogate_sea(seed)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=sp["hs_over_lambda"] * LAM, kp=1.0, gamma=sp["gamma"],
                              phases=synth.mode_phases(sp["phase_seed"], n, n // 2 + 1))
    return lib.Hos(d, eh, ph)


def default_scales(stride: int, base_substeps: int = 0) -> dict:
    """Input scale sigma = Hs/4 at Hs/lambda_p = 0.02 for eta and, through the
    linear dispersion (phis ~ g/omega eta, omega_p = 1), for phis; residual
    scale rho in proportion to the base's one-call error at s = 10 (about
    4e-2 linear, 7e-3 with one integrating-factor RK4 substep, 2e-4 with
    two): 0.05, 0.005, 0.0002; for the RK4 bases scaled by (s / 10)^5, the
    order of a fourth-order step's error over one call."""
    sig = 0.02 * LAM / 4.0
    rho = {0: 0.05, 1: 0.005}.get(base_substeps, 0.0002)
    if base_substeps > 0:
        rho *= (stride / 10.0) ** 5
    return {"stride_s": stride, "sigma_eta": sig, "sigma_phi": sig, "rho": rho, "base_substeps": base_substeps}


class Pairs:
    """Device store of (input, target) pairs: inputs [count][in_channels][n][n]
    (the state, then for 4 channels its linear propagation), targets
    [count][2][n][n], FP32."""

    def __init__(self, count: int, n: int, in_channels: int = 2):
        self.x = torch.empty((count, in_channels, n, n), dtype=torch.float32, device="cuda")
        self.t = torch.empty((count, 2, n, n), dtype=torch.float32, device="cuda")
        self.in_channels = in_channels
        self.count = 0


def generate(net: lib.Fno, scales: dict, seeds, steps: int, periods: float, store: Pairs, log=None):
    n = net.desc.n
    stride = scales["stride_s"]
    sd = lib.surrogate_desc(**scales)
    lin = torch.empty((2, n, n), dtype=torch.float32, device="cuda")
    xn = torch.empty_like(lin)
    for j, seed in enumerate(seeds):
        h = sea_hos(n, periods, seed)
        sur = lib.Surrogate(h, net, sd)
        for _ in range(steps // stride):
            i = store.count
            li = store.x[i, 2:4] if store.in_channels == 4 else lin
            sur.features(store.x[i, 0:2], li)
            h.step(stride)
            sur.features(xn, want_lin=False)
            sur.target(xn, li, store.t[i])
            store.count += 1
        sur.close()
        h.close()
        if log and (j + 1) % max(1, len(seeds) // 10) == 0:
            torch.cuda.synchronize()
            log(f"generated {j + 1}/{len(seeds)} trajectories ({store.count} pairs)")
    torch.cuda.synchronize()


def train(net: lib.Fno, store: Pairs, iters: int, batch: int, lr: float, seed: int = 0, log=None,
          log_every: int = 200):
    """Adam with a cosine learning-rate decay to lr/20; minibatches drawn
    without replacement per epoch (seeded)."""
    rng = np.random.default_rng(seed)
    n = net.desc.n
    xb = torch.empty((batch, store.in_channels, n, n), dtype=torch.float32, device="cuda")
    tb = torch.empty((batch, 2, n, n), dtype=torch.float32, device="cuda")
    order = rng.permutation(store.count)
    pos = 0
    hist = []
    t0 = time.time()
    for it in range(iters):
        if pos + batch > store.count:
            order = rng.permutation(store.count)
            pos = 0
        idx = torch.as_tensor(order[pos:pos + batch], device="cuda")
        pos += batch
        torch.index_select(store.x[:store.count], 0, idx, out=xb)
        torch.index_select(store.t[:store.count], 0, idx, out=tb)
        a = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * it / max(1, iters))))
        loss = net.train_step(xb, tb, a)
        hist.append(loss)
        if log and ((it + 1) % log_every == 0 or it == iters - 1):
            log(f"iter {it + 1}/{iters} loss {np.mean(hist[-log_every:]):.4e} lr {a:.2e} "
                f"({time.time() - t0:.0f} s)")
    return hist


def one_call_errors(net: lib.Fno, scales: dict, seeds, calls: int, periods: float, base_only: bool = True):
    """Per-call relative state error of the network (and of the base
    prediction alone, the network not evaluated) on held-out seas: every
    call judged by HOS, whose state is kept (tol = inf)."""
    n = net.desc.n
    out = {"network": [], "base_only": []}
    for name, only in (("network", False), ("base_only", True)):
        if only and not base_only:
            continue
        sd = lib.surrogate_desc(tol=1e30, audit_every=1, cooldown=0, drift_tol=0.0, base_only=only, **scales)
        for seed in seeds:
            h = sea_hos(n, periods, seed)
            sur = lib.Surrogate(h, net, sd)
            errs = []
            for _ in range(calls):
                sur.advance(1)
                errs.append(sur.stats.last_audit_err)
            out[name].append(errs)
            sur.close()
            h.close()
    return {k: np.array(v) for k, v in out.items() if v}


def rel_state_error(e, p, er, pr) -> float:
    """Relative L2 error of the half spectra (e, p) against (er, pr), max over
    the two fields, with the Parseval weights of the half spectrum (1 for the
    p = 0 column, 2 for the others): the measure of the rollout's judge."""
    w = np.full(er.shape[1], 2.0)
    w[0] = 1.0

    def one(a, b):
        return math.sqrt(float(np.sum(w * np.abs(a - b) ** 2)) / float(np.sum(w * np.abs(b) ** 2)))

    return max(one(e, er), one(p, pr))


def zero_output(desc: lib.FnoDesc, vec: np.ndarray) -> np.ndarray:
    P = lib.fno_unpack(desc, vec)
    P["Q2"] = np.zeros_like(P["Q2"])
    P["c2"] = np.zeros_like(P["c2"])
    return lib.fno_pack(desc, P)


def rollout(net: lib.Fno, scales: dict, seeds, calls: int, periods: float, tol: float, audit_every: int,
            cooldown: int, base_only: bool = False, drift_tol=None):
    """Rollout with the HOS fallback/judge (drift bound drift_tol, default
    tol), of the network or (base_only) of the base prediction alone;
    offline error against a plain HOS run of the same seas; effective HOS
    steps per second."""
    n = net.desc.n
    res = []
    for seed in seeds:
        h = sea_hos(n, periods, seed)
        ref = sea_hos(n, periods, seed)
        sd = lib.surrogate_desc(tol=tol, audit_every=audit_every, cooldown=cooldown, base_only=base_only,
                                drift_tol=drift_tol, **scales)
        sur = lib.Surrogate(h, net, sd)
        torch.cuda.synchronize()
        t0 = time.time()
        st = sur.advance(calls)
        torch.cuda.synchronize()
        dt = time.time() - t0
        ref.step(calls * scales["stride_s"])
        e, p, _ = h.state()
        er, pr, _ = ref.state()
        off = rel_state_error(e, p, er, pr)
        st = dict(st)
        st.update(seed=seed, offline_err=float(off), seconds=dt,
                  effective_steps_per_s=calls * scales["stride_s"] / dt)
        res.append(st)
        sur.close()
        h.close()
        ref.close()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--periods", type=float, default=20.0)
    ap.add_argument("--channels", type=int, default=64)
    ap.add_argument("--layers", type=int, default=8)
    ap.add_argument("--p-modes", type=int, default=32)
    ap.add_argument("--q-modes", type=int, default=31)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--in-channels", type=int, default=4, choices=(2, 4))
    ap.add_argument("--trajectories", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--stride", type=int, default=10)
    ap.add_argument("--base-substeps", type=int, default=1,
                    help="base prediction: 0 exact linear propagation, n integrating-factor RK4 substeps")
    ap.add_argument("--iters", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--test-seeds", type=int, default=8)
    ap.add_argument("--calls", type=int, default=20)
    ap.add_argument("--out", default=None, help="weights file (.npz) to write")
    ap.add_argument("--report", default=None, help="JSON report to write")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    lib.load()
    desc = lib.fno_desc(a.n, a.channels, a.layers, a.p_modes, a.q_modes, a.hidden, max_batch=a.batch,
                        in_channels=a.in_channels)
    vec0 = lib.fno_init(desc, 0)
    net = lib.Fno(desc, vec0)
    scales = default_scales(a.stride, a.base_substeps)
    store = Pairs(a.trajectories * (a.steps // a.stride), a.n, a.in_channels)
    t0 = time.time()
    generate(net, scales, range(1000, 1000 + a.trajectories), a.steps, a.periods, store, log)
    t_gen = time.time() - t0
    log(f"{store.count} pairs in {t_gen:.1f} s")
    t0 = time.time()
    hist = train(net, store, a.iters, a.batch, a.lr, log=log)
    t_train = time.time() - t0
    del store
    test = range(3000, 3000 + a.test_seeds)
    errs = one_call_errors(net, scales, test, a.calls, a.periods)
    roll = rollout(net, scales, test, a.calls, a.periods, tol=1e-3, audit_every=4, cooldown=4)
    roll_base = rollout(net, scales, test, a.calls, a.periods, tol=1e-3, audit_every=4, cooldown=4, base_only=True)
    rep = {
        "config": vars(a), "scales": scales, "pairs": a.trajectories * (a.steps // a.stride),
        "generate_s": t_gen, "train_s": t_train, "train_ms_per_iter": 1e3 * t_train / max(1, a.iters),
        "loss_first": float(np.mean(hist[:50])), "loss_last": float(np.mean(hist[-200:])),
        "one_call_err_network_mean": float(errs["network"].mean()),
        "one_call_err_network_max": float(errs["network"].max()),
        "one_call_err_base_mean": float(errs["base_only"].mean()),
        "one_call_err_base_max": float(errs["base_only"].max()),
        "rollout": roll,
        "rollout_base_only": roll_base,
    }
    log(json.dumps({k: v for k, v in rep.items() if k != "rollout"}))
    for r in roll + roll_base:
        log(json.dumps(r))
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)
    if a.out:
        np.savez(a.out, params=net.get(0), adam_m=net.get(2), adam_v=net.get(3),
                 desc=np.array([a.n, a.channels, a.layers, a.p_modes, a.q_modes, a.hidden, a.in_channels]),
                 scales=json.dumps(scales))
    net.close()
    return rep


if __name__ == "__main__":
    main()
    sys.exit(0)
