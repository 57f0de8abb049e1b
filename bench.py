#!/usr/bin/env python3
"""Benchmark of the incident-wave hot path on one MI355X.

Workload (the irregular-sea configuration of the metric): 3D deep-water
JONSWAP sea, Hs/lambda_p = 0.02, gamma = 3.3, cos^2 spreading, phases from
seed 1, 512 x 256 modes over 40 x 20 peak wavelengths, order M = 3 with full
dealiasing, FP32 transforms with FP64 state and phases, RK4 dt = Tp/64;
interpolation of all 11 fields to the 1,996,800 cell centres of a structured
O-mesh around a vertical cylinder of radius 0.1 lambda_p (grid refinement
n = 4, a 4 x 4 lambda_p window, 48 layers).

One step = one RK4 HOS step + mean-level modes A, A_t + coefficient-grid
evaluation + interpolation to every cell centre (the whole CFD-side update).
value = cell-centre field points per second = points x 11 fields / step time.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LAM = 2 * math.pi
NX, NY = 512, 256
LX, LY = 40 * LAM, 20 * LAM
HS = 0.02 * LAM
M = 3
NFIELDS = 11
PEAK_HBM = 8.0e12  # B/s, MI355X HBM3E


def workload():
    import numpy as np
    import synth
    pts = synth.cylinder_cloud(LX, LY, HS)
    gx, gy = 4 * NX, 4 * NY
    dx = LX / gx
    ix0 = int(math.floor((LX / 2 - 2.05 * LAM) / dx)) - 2
    wx = int(math.ceil(4.1 * LAM / dx)) + 6
    iy0 = int(math.floor((LY / 2 - 2.05 * LAM) / dx)) - 2
    wy = wx
    zl = synth.clustered_layers(pts[2].min() - 1e-9, pts[2].max() + 1e-9, 48, HS / 16)
    phases = synth.mode_phases(1, NY, NX // 2 + 1)
    return pts, (gx, gy, ix0, iy0, wx, wy), np.asarray(zl), phases


def batched_setup(lib, torch, pts_scale=1.0, fields=None):
    """The batched configuration: 64 seeded JONSWAP realisations with mode
    grids uniform over the even 5-smooth sizes in [128, 512] per axis,
    Hs/lambda_p ~ U[0.01, 0.03], M = 3, each interpolated (n = 4 window, 32
    layers) to 100k..1M box-cloud points clustered toward z = 0."""
    import numpy as np
    import synth
    reals = synth.batch_realisations(3)
    hoses, cells, outs, npts = [], [], [], 0
    mask = lib.ALL_FIELDS if fields is None else fields
    nf = bin(mask).count("1")
    for r in reals:
        nx, ny = r["nx"], r["ny"]
        lx, ly = nx * LAM / 12.8, ny * LAM / 12.8
        hs = r["hs_over_lambda"] * LAM
        d = lib.hos_desc(3, nx, ny, lx, ly, -1.0, order_m=M, dt=LAM / 64)
        eh, ph = lib.sea_spectrum(d, kind=0, hs=hs, kp=1.0, gamma=3.3,
                                  phases=synth.mode_phases(r["phase_seed"], ny, nx // 2 + 1))
        h = lib.Hos(d, eh, ph)
        n = max(1000, int(r["npts"] * pts_scale))
        x0, y0 = lx / 2 - 2 * LAM, ly / 2 - 2 * LAM
        p = synth.box_cloud(r["phase_seed"], n, x0, y0, 4 * LAM, 4 * LAM, -0.5 * LAM, 0.1 * LAM)
        gx, gy = 4 * nx, 4 * ny
        dx, dy = lx / gx, ly / gy
        ix0, iy0 = int(math.floor(x0 / dx)) - 2, int(math.floor(y0 / dy)) - 2
        wx, wy = int(math.ceil(4 * LAM / dx)) + 6, int(math.ceil(4 * LAM / dy)) + 6
        zl = synth.clustered_layers(-0.5 * LAM - 1e-9, 0.1 * LAM + 1e-9, 32, 0.01 * LAM)
        gd = lib.grid_desc(gx, gy, zl, (ix0, iy0, wx, wy))
        c = h.bind(gd, torch.tensor(p, device="cuda"))
        hoses.append(h)
        cells.append(c)
        outs.append(torch.empty((nf, n), dtype=torch.float32, device="cuda"))
        npts += n
    return hoses, cells, outs, npts, mask, nf


def run_batched(lib, torch, steps):
    import tempfile
    hoses, cells, outs, npts, mask, nf = batched_setup(lib, torch)
    b = lib.Batch(hoses, cells, [mask] * len(hoses), outs, nsteps=1)
    with tempfile.TemporaryDirectory() as td:
        k, tune_ms = b.autotune(os.path.join(td, "tune.json"))
    b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        b.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res = {"realisations": len(hoses), "points": npts, "branches": k, "ms_per_launch": ms,
           "realisation_steps_per_s": len(hoses) * 1e3 / ms,
           "cell_field_pts_per_s": npts * nf * 1e3 / ms}
    b.close()
    for c in cells:
        c.close()
    for h in hoses:
        h.close()
    return res


def algorithmic_bytes(kind, ctx):
    """Compulsory HBM bytes per launch of a kernel class (inputs read once,
    outputs written once), as listed in the design notes."""
    n, L, wx, wy, nxh, py = ctx["n"], ctx["nl"], ctx["wx"], ctx["wy"], NX // 2 + 1, ctx["py"]
    fvol, fsrf = 8, 2
    if kind == "interp":
        return 60.0 * n + 4.0 * (fvol * L * wx * wy + fsrf * wx * wy)
    if kind == "xeval":
        return fvol * L * wy * nxh * 8.0 + fvol * L * wy * wx * 4.0
    if kind == "yinv_eval":
        return 3 * NY * nxh * 16.0 + (fvol * L + fsrf) * wy * nxh * 8.0
    if kind in ("xpass", "yinv", "yfwd"):
        # HOS step per launch, averaged: survey model 4 T_rhs 16 P bytes per step
        t_rhs = 5 + M * (M + 1) // 2 + (M - 1) + 2
        return 4 * t_rhs * 16.0 * (2 * NX) * py / ctx["hos_launches_per_step"]
    return None


def cpu_baseline(pts, win, zl, phases, budget_s=20.0):
    """The FP64 oracle on a bounded sample of one step, scaled to the whole
    step: one RK4 step, the modes, the coefficient grids of 2 of the 48
    layers (x 24) and the interpolation of 100k of the points (x n/100k)."""
    import numpy as np
    from oracle import Grid, hos, sea
    from oracle import reconstruct as rc
    g = Grid(nx=NX, ny=NY, lx=LX, ly=LY, depth=-1.0, order_m=M)
    eh, ph = sea.jonswap(g, HS, 1.0, 3.3, phases)
    gx, gy, ix0, iy0, wx, wy = win
    t0 = time.perf_counter()
    eh, ph = hos.rk4_step(g, eh, ph, LAM / 64)
    t_hos = time.perf_counter() - t0
    t0 = time.perf_counter()
    A = hos.mean_level_modes(g, eh, ph)
    At, eth = hos.mean_level_modes_t(g, eh, ph)
    t_modes = time.perf_counter() - t0
    fields = [f for f in range(11) if f != rc.P]
    t0 = time.perf_counter()
    rc.eval_grid(g, A, At, eh, eth, gx, gy, zl[:2], fields, window=(ix0, iy0, wx, wy), prefilter=True)
    t_eval = (time.perf_counter() - t0) * (zl.size / 2)
    coef = rc.eval_grid(g, A, At, eh, eth, gx, gy, zl, [rc.ETA], window=(ix0, iy0, wx, wy), prefilter=True)
    # a coefficient grid for interpolation timing (values do not matter for the timing)
    shape = (zl.size, wy, wx)
    rng = np.random.default_rng(0)
    for f in fields:
        if f not in (rc.ETA, rc.ETA_T):
            coef[f] = rng.standard_normal(shape)
    coef[rc.ETA_T] = coef[rc.ETA]
    nsamp = 100_000
    sel = pts[:, :nsamp]
    t0 = time.perf_counter()
    rc.interp_points(g, coef, zl, gx, gy, (ix0, iy0, wx, wy), sel, list(range(11)))
    t_interp = (time.perf_counter() - t0) * (pts.shape[1] / nsamp)
    total = t_hos + t_modes + t_eval + t_interp
    return {
        "value": pts.shape[1] * NFIELDS / total,
        "unit": "cell-centre field pts/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("1 RK4 step at 512x256 + modes + coefficient grids of 2/48 layers (x24) + interpolation of "
                   f"{nsamp} of {pts.shape[1]} points (scaled); numpy FP64, single thread"),
        "seconds": {"hos_step": t_hos, "modes": t_modes, "eval_scaled": t_eval, "interp_scaled": t_interp},
        "hos_steps_per_s": 1.0 / t_hos,
        "cpu": platform.processor() or platform.machine(),
        "nproc": os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the workload is a single "
              "realisation and this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2005_12716_amd import lib

    torch.cuda.set_device(0)
    pts, win, zl, phases = workload()
    gx, gy, ix0, iy0, wx, wy = win
    d = lib.hos_desc(3, NX, NY, LX, LY, -1.0, order_m=M, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=HS, kp=1.0, gamma=3.3, phases=phases)
    h = lib.Hos(d, eh, ph)
    gd = lib.grid_desc(gx, gy, zl, (ix0, iy0, wx, wy))
    xyz = torch.tensor(pts, device="cuda")
    cells = h.bind(gd, xyz)
    out = torch.empty((NFIELDS, cells.n), dtype=torch.float32, device="cuda")
    _, nbad = cells.interp(lib.ALL_FIELDS, out)
    assert nbad == 0, f"{nbad} points outside the grid"
    print(f"# workload: {cells.n} points, window {wx}x{wy} of {gx}x{gy}, {zl.size} layers", file=sys.stderr, flush=True)

    def step():
        h.step(1)
        cells.interp(lib.ALL_FIELDS, out, count=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    print(f"# end-to-end {ms_step:.3f} ms/step", file=sys.stderr, flush=True)

    # HOS step alone
    nh = 4 * args.steps
    e0.record()
    h.step(nh)
    e1.record()
    torch.cuda.synchronize()
    ms_hos = e0.elapsed_time(e1) / nh
    # interpolation alone (modes cached; coefficient grids re-evaluated each call)
    e0.record()
    for _ in range(args.steps):
        cells.interp(lib.ALL_FIELDS, out, count=False)
    e1.record()
    torch.cuda.synchronize()
    ms_interp = e0.elapsed_time(e1) / args.steps
    print(f"# hos {ms_hos:.3f} ms/step, interp+eval {ms_interp:.3f} ms", file=sys.stderr, flush=True)

    # per-kernel pass: the same steps with every launch bracketed by HIP events
    h.profile(True)
    for _ in range(args.steps):
        step()
    prof = h.profile_read()
    h.profile(False)
    launches_per_step = {k: c / args.steps for k, (_, c) in prof.items()}
    hos_launches = sum(launches_per_step[k] for k in ("yinv", "xpass", "yfwd"))
    py = 2 * NY
    ctx = {"n": cells.n, "nl": zl.size, "wx": wx, "wy": wy, "py": py,
           "hos_launches_per_step": max(hos_launches, 1)}
    kinds = sorted(prof, key=lambda k: -prof[k][0])
    dom = kinds[0]
    tot_ms, cnt = prof[dom]
    avg_s = tot_ms / cnt / 1e3
    ab = algorithmic_bytes(dom, ctx)
    roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": None, "traffic": None, "avg_launch_ms": tot_ms / cnt,
            "share_of_step": tot_ms / args.steps / ms_step}
    if ab is not None:
        ach = ab / avg_s / 1e9
        roof.update({"achieved": ach, "frac": ach / (PEAK_HBM / 1e9), "algorithmic_bytes_per_launch": ab})
    breakdown = {k: {"ms_per_step": prof[k][0] / args.steps, "launches_per_step": launches_per_step[k]}
                 for k in kinds if prof[k][1] > 0}

    res = {
        "metric": "cell-centre field pts/s (end-to-end CFD update: HOS step + modes + grid + interpolation)",
        "value": cells.n * NFIELDS / (ms_step / 1e3),
        "unit": "cell-centre field pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 transforms / f64 state",
        "data": "synthetic",
        "config": {"workload": "3D JONSWAP 512x256 modes M=3 (40x20 lambda_p, Hs/lambda_p=0.02, gamma=3.3, seed 1) "
                               "-> 1,996,800-point cylinder O-mesh, 11 fields, n=4 window, 48 layers",
                   "points": cells.n, "modes": [NX, NY], "order_m": M, "padded": [2 * NX, py],
                   "grid": [gx, gy], "window": [ix0, iy0, wx, wy], "layers": int(zl.size)},
        "hos_steps_per_s": 1e3 / ms_hos,
        "hos_mode_steps_per_s": NX * NY * 1e3 / ms_hos,
        "interp_eval_pts_per_s": cells.n * NFIELDS / (ms_interp / 1e3),
        "roofline": roof,
        "kernels": breakdown,
    }
    cells.close()
    h.close()
    if not args.no_batched:
        print("# batched configuration", file=sys.stderr, flush=True)
        res["batched"] = run_batched(lib, torch, max(2, args.steps // 4))
        print(f"# batched {res['batched']['ms_per_launch']:.2f} ms per launch", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(pts, win, zl, phases)
        res["cpu_baseline"] = cb
        res["speedup_vs_cpu_baseline"] = res["value"] / cb["value"]
        res["hos_speedup_vs_cpu_baseline"] = res["hos_steps_per_s"] / cb["hos_steps_per_s"]
    print(json.dumps(res))


if __name__ == "__main__":
    main()
