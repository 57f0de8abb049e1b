#!/usr/bin/env python3
"""Benchmark of the incident-wave hot path on one MI355X.

Headline workload (the largest single-GPU configuration): the steep large
sea - 3D deep-water JONSWAP, Hs/lambda_p = 0.04, gamma = 5, cos^2 spreading,
phases from seed 5, 1024 x 1024 modes over 40 x 40 peak wavelengths, order
M = 5 with full dealiasing (3072^2 product grid), FP32 transforms with FP64
state, phases and vertical factors, RK4 dt = Tp/64 - mapped at every CFD step
to the 20,000,000 cell centres of a jittered hex mesh (500 x 250 x 160 cells
over 8 x 4 lambda_p, z in [-lambda_p/2, 0.2 lambda_p] clustered about the
mean level, +-10 % jitter, seed 6) through a coefficient grid refined four
times (4096^2 nodes, windowed on the mesh with a stencil halo, 64 layers).

One step = one RK4 HOS step + mean-level modes A, A_t + coefficient-grid
evaluation + interpolation of all 11 fields to every cell centre (the whole
CFD-side update), timed as two calls (step, then interpolate) and as one call
that interpolates the current state while the step advances it; value =
cell-centre field points per second = points x 11 fields / the faster step.

Other configurations are reported as keys: the 512 x 256, M = 3 sea with the
2M-point cylinder O-mesh, the 2D regular wave (steps/s), the batched
realisations, and the learned surrogate.
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
NFIELDS = 11
PEAK_HBM = 8.0e12  # B/s, MI355X HBM3E
# headline: steep large sea
N5, M5 = 1024, 5
L5 = 40 * LAM
HS5 = 0.04 * LAM
GAMMA5 = 5.0
# the 512 x 256, M = 3 sea with the cylinder O-mesh
NX, NY = 512, 256
LX, LY = 40 * LAM, 20 * LAM
HS = 0.02 * LAM
M = 3


def workload5():
    """Hex-mesh cell centres, grid window and layers of the steep large sea."""
    import numpy as np
    import synth
    x0, y0, wx, wy = L5 / 2 - 4 * LAM, L5 / 2 - 2 * LAM, 8 * LAM, 4 * LAM
    pts, mesh = synth.hex_cloud(6, x0, y0, wx, wy, -0.5 * LAM, 0.2 * LAM, 500, 250, 160, HS5 / 16)
    gx = 4 * N5
    dx = L5 / gx
    win = (gx, gx, int(math.floor(x0 / dx)) - 2, int(math.floor(y0 / dx)) - 2, int(math.ceil(wx / dx)) + 6,
           int(math.ceil(wy / dx)) + 6)
    zl = synth.clustered_layers(mesh["ze"][0] - 1e-9, mesh["ze"][-1] + 1e-9, 64, HS5 / 16)
    phases = synth.mode_phases(5, N5, N5 // 2 + 1)
    return pts, win, np.asarray(zl), phases


def workload():
    """Cylinder O-mesh, grid window and layers of the 512 x 256, M = 3 sea."""
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


padding_choice = {}


def batched_setup(lib, torch, pts_scale=1.0, fields=None, streams=None, padding=None):
    """The batched configuration: 64 seeded JONSWAP realisations with mode
    grids uniform over the even 5-smooth sizes in [128, 512] per axis,
    Hs/lambda_p ~ U[0.01, 0.03], M = 3, each interpolated (n = 4 window, 32
    layers) to 100k..1M box-cloud points clustered toward z = 0.  padding:
    the product-grid policy of every realisation (1 or 2), or "tune" for the
    library's timed choice per grid size (the choices are returned in
    `padding_choice`, keyed "nx x ny")."""
    import numpy as np
    import synth
    reals = synth.batch_realisations(3)
    hoses, cells, outs, npts = [], [], [], 0
    mask = lib.ALL_FIELDS if fields is None else fields
    nf = bin(mask).count("1")
    padding_choice.clear()
    for r in reals:
        nx, ny = r["nx"], r["ny"]
        lx, ly = nx * LAM / 12.8, ny * LAM / 12.8
        hs = r["hs_over_lambda"] * LAM
        d = lib.hos_desc(3, nx, ny, lx, ly, -1.0, order_m=M, dt=LAM / 64)
        if padding == "tune":
            key = f"{nx}x{ny}"
            if key not in padding_choice:
                padding_choice[key] = lib.tune_padding(d)[0]
            d.dealias = padding_choice[key]
        elif padding is not None:
            d.dealias = padding
        eh, ph = lib.sea_spectrum(d, kind=0, hs=hs, kp=1.0, gamma=3.3,
                                  phases=synth.mode_phases(r["phase_seed"], ny, nx // 2 + 1))
        h = lib.Hos(d, eh, ph, stream=streams[len(hoses) % len(streams)] if streams else None)
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


def run_batched(lib, torch, steps, fixed=False):
    """fixed: product-grid policy 2 for every realisation and the graph's
    default branch count (no timed choices: a short run for counter passes)."""
    import tempfile
    t0 = time.time()
    hoses, cells, outs, npts, mask, nf = batched_setup(lib, torch, padding=2 if fixed else "tune")
    setup_s = time.time() - t0
    b = lib.Batch(hoses, cells, [mask] * len(hoses), outs, nsteps=1)
    if fixed:
        k, tune_ms = None, None
    else:
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
           "setup_s": setup_s, "padding_2_sizes": sorted(kk for kk, v in padding_choice.items() if v == 2),
           "padding_1_sizes": sorted(kk for kk, v in padding_choice.items() if v == 1),
           "realisation_steps_per_s": len(hoses) * 1e3 / ms,
           "cell_field_pts_per_s": npts * nf * 1e3 / ms}
    # compulsory HBM bytes of one launch, lower bound: the HOS intermediates
    # (the library's count, from one eager profiled step of every realisation)
    # plus the interpolated outputs (4 B per point and field); coefficient
    # grids and point data not counted
    hos_bytes = 0.0
    for h in hoses:
        h.profile(True)
        h.step(1)
        torch.cuda.synchronize()
        pb = h.profile_bytes()
        h.profile(False)
        hos_bytes += sum(pb.get(kk, 0.0) for kk in ("yinv", "xpass", "yfwd"))
    out_bytes = 4.0 * npts * nf
    res["compulsory_bytes_lower_bound"] = {"hos": hos_bytes, "interp_outputs": out_bytes,
                                           "GB_per_s": (hos_bytes + out_bytes) / (ms / 1e3) / 1e9,
                                           "frac_of_hbm_peak": (hos_bytes + out_bytes) / (ms / 1e3) / PEAK_HBM}
    b.close()
    for c in cells:
        c.close()
    for h in hoses:
        h.close()
    return res


def run_surrogate(lib, torch, steps, train_trajectories=100, train_iters=1000, base_substeps=2):
    """The learned configuration: the spectral neural operator (256^2 over 20
    lambda_p, 64 channels, 8 layers, p < 32, |q| <= 31, width 128, input the
    state and its linear propagation), trained here briefly on the GPU
    (train_trajectories seeded JONSWAP seas x 200 HOS steps, stride s = 10,
    train_iters Adam steps of batch 8), then: network-only calls, plain HOS,
    and the judged rollout (tol 1e-3, audit every 4th call, cool-down 4) on
    held-out seas."""
    import numpy as np
    from paper_2005_12716_amd import train as T
    desc = lib.fno_desc(in_channels=4, max_batch=8)
    vec0 = lib.fno_init(desc, 0)
    net = lib.Fno(desc, vec0)
    scales = T.default_scales(10, base_substeps)
    store = T.Pairs(train_trajectories * 20, 256, 4)
    t0 = time.perf_counter()
    T.generate(net, scales, range(1000, 1000 + train_trajectories), 200, 20.0, store)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist = T.train(net, store, train_iters, 8, 1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del store
    errs = T.one_call_errors(net, scales, range(3000, 3003), 5, 20.0)
    # network-only calls and base-only calls (no audits), plain HOS on the same sea
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms_by = {}
    for only in (False, True):
        h = T.sea_hos(256, 20.0, 3000)
        sd = lib.surrogate_desc(tol=1e30, audit_every=1 << 30, cooldown=0, probation=0, drift_tol=0.0,
                                base_only=only, **scales)
        sur = lib.Surrogate(h, net, sd)
        sur.advance(2)
        torch.cuda.synchronize()
        e0.record()
        sur.advance(steps)
        e1.record()
        torch.cuda.synchronize()
        ms_by[only] = e0.elapsed_time(e1) / steps
        sur.close()
        h.close()
    ms_call, ms_base = ms_by[False], ms_by[True]
    h = T.sea_hos(256, 20.0, 3000)
    e0.record()
    h.step(10 * steps)
    e1.record()
    torch.cuda.synchronize()
    ms_hos = e0.elapsed_time(e1) / (10 * steps)
    h.close()
    x = torch.zeros((8, 4, 256, 256), dtype=torch.float32, device="cuda")
    y = torch.empty((8, 2, 256, 256), dtype=torch.float32, device="cuda")
    net.forward(x[:1], y[:1])
    e0.record()
    for _ in range(steps):
        net.forward(x, y)
    e1.record()
    torch.cuda.synchronize()
    ms_fwd8 = e0.elapsed_time(e1) / steps
    roll = T.rollout(net, scales, range(3000, 3003), 20, 20.0, tol=1e-3, audit_every=4, cooldown=4)
    roll_base = T.rollout(net, scales, range(3000, 3003), 20, 20.0, tol=1e-3, audit_every=4, cooldown=4,
                          base_only=True)
    net.close()
    keys = ("seed", "calls", "surrogate_calls", "hos_calls", "bound_calls", "audits", "fallbacks", "max_audit_err",
            "drift_est", "offline_err", "effective_steps_per_s")
    return {
        "network": {"n": 256, "channels": 64, "layers": 8, "p_modes": 32, "q_modes": 31, "hidden": 128,
                    "in_channels": 4, "params": int(vec0.size)},
        "stride_s": 10,
        "training": {"trajectories": train_trajectories, "pairs": train_trajectories * 20, "iters": train_iters,
                     "batch": 8, "generate_s": t_gen, "train_s": t_train,
                     "ms_per_iter": 1e3 * t_train / train_iters,
                     "loss_first": float(np.mean(hist[:50])), "loss_last": float(np.mean(hist[-100:]))},
        "base": ("exact linear propagation" if base_substeps == 0 else
                 f"{base_substeps} integrating-factor RK4 substep(s) over the stride"),
        "one_call_rel_err": {"network": float(errs["network"].mean()),
                             "base_only": float(errs["base_only"].mean())},
        "ms_per_network_call": ms_call,
        "ms_per_base_only_call": ms_base,
        "network_forward_ms_per_sample_b8": ms_fwd8 / 8,
        "hos_ms_per_step_256": ms_hos,
        "network_only_steps_per_s": 10 * 1e3 / ms_call,
        "base_only_steps_per_s": 10 * 1e3 / ms_base,
        "plain_hos_steps_per_s": 1e3 / ms_hos,
        "judge": "tol 1e-3 per judged call, drift bound 1e-3 on the estimated accumulated error, every 4th call "
                 "judged, probation 2, cool-down 4",
        "judged_rollout": [{k: r[k] for k in keys} for r in roll],
        "judged_rollout_base_only": [{k: r[k] for k in keys} for r in roll_base],
    }


def run_fv_divergence(lib, torch):
    """Divergence diagnostic of the paper's zero-padding demonstration
    (Sec. 3.2.3-3.2.4): 2D JONSWAP Tp = 0.7 s, Hs = 0.028 m, gamma 3.3, 128
    modes over 10 lambda_p, one period of HOS; CFD cells lambda_p/100 x Hs/20
    down to -0.1 lambda_p; finite-volume divergence of the interpolated
    velocity for refinements n = 1, 2, 4 (RMS and max, 1/s)."""
    import numpy as np
    import synth
    g0, tp, hs = 9.81, 0.7, 0.028
    lam = g0 * tp * tp / (2 * math.pi)
    d = lib.hos_desc(2, 128, 1, 10 * lam, 1.0, -1.0, order_m=3, dt=tp / 64, g=g0, rho=1000.0)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=hs, kp=2 * math.pi / lam, gamma=3.3, phases=synth.mode_phases(579, 1, 65))
    h = lib.Hos(d, eh, ph)
    h.step(64)
    dx, dz = lam / 100, hs / 20
    zbot = -0.1 * lam
    nzc = int(round(-zbot / dz))
    xe = np.arange(1001) * dx
    ze = zbot + np.arange(nzc + 1) * dz
    zl = np.linspace(zbot - 2 * dz, 2 * dz, 41)
    out = {}
    for n in (1, 2, 4):
        _, rms, mx = h.fv_divergence(lib.grid_desc(128 * n, 1, zl), xe, None, ze)
        out[f"n{n}"] = {"rms_per_s": rms, "max_per_s": mx}
    h.close()
    return out


def kernel_profile(h, step, steps):
    """Per-kernel-class time (HIP start/stop events stamped by the runtime at
    kernel start and end, summed over the launches) and bytes of `steps`
    calls of `step`, from the library's profiler."""
    h.profile(True)
    for _ in range(steps):
        step()
    prof = h.profile_read()
    comp = h.profile_bytes()
    model = h.profile_transform_bytes()
    h.profile(False)
    out = {}
    for k, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        out[k] = {"ms_per_step": ms / steps, "launches_per_step": cnt / steps, "avg_launch_ms": ms / cnt,
                  "compulsory_bytes_per_launch": comp.get(k, 0.0) / cnt,
                  "model_bytes_per_launch": model.get(k, 0.0) / cnt}
    return out


def hos_model_bytes(kernels, m, px, py):
    """Algorithmic bytes per launch of the HOS classes under the survey's
    two-pass transform model, counted per CFD step as the step's transforms
    (4 right-hand sides of T = 5 + M(M+1)/2 inverse and (M-1) + 2 forward
    real transforms each, plus the mean-level modes' M(M-1)/2 inverse and
    M-1 forward ones), each streaming its product-grid field once per pass
    (8 B per point in FP32), spread evenly over the class's launches."""
    p = float(px) * py
    t_inv, t_fwd = 4 * (5 + m * (m + 1) // 2) + m * (m - 1) // 2, 4 * ((m - 1) + 2) + (m - 1)
    per_step = {"yinv": 8.0 * p * t_inv, "yfwd": 8.0 * p * t_fwd, "xpass": 8.0 * p * (t_inv + t_fwd)}
    for k, b in per_step.items():
        if k in kernels:
            d = kernels[k]
            d["transforms_performed_bytes_per_launch"] = d["model_bytes_per_launch"]
            d["model_bytes_per_launch"] = b / d["launches_per_step"]
    return kernels


def roofline_of(kernels, traffic_file=False):
    """Roofline entry of the dominant kernel class (largest share of the
    profiled step): achieved = algorithmic bytes per launch under the
    two-pass transform model (the HOS, evaluation and gather byte model) /
    average launch duration; the library's compulsory bytes (every distinct
    input read once, every output written once) are given beside it."""
    tot = sum(v["ms_per_step"] for v in kernels.values())
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    d = kernels[dom]
    t = d["avg_launch_ms"] / 1e3
    ach = d["model_bytes_per_launch"] / t / 1e9
    comp = d["compulsory_bytes_per_launch"] / t / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": ach / (PEAK_HBM / 1e9), "traffic": measured_traffic(dom) if traffic_file else None,
            "byte_model": ("two-pass transform bytes: every real transform of the step (4 right-hand sides + the "
                           "mean-level modes; evaluation: every (field, layer) job on the refined grid) streams its "
                           "grid field once per pass, read and written; gather: 16 B + 4 B per field per point + grid"),
            "model_bytes_per_launch": d["model_bytes_per_launch"],
            "compulsory_bytes_per_launch": d["compulsory_bytes_per_launch"],
            "achieved_compulsory": comp, "frac_compulsory": comp / (PEAK_HBM / 1e9),
            "avg_launch_ms": d["avg_launch_ms"], "launches_per_step": d["launches_per_step"],
            "share_of_profiled_step": d["ms_per_step"] / tot, "profiled_step_ms": tot}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "xpass_steep_sea_1024x1024_m5_traffic.md")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none or a source it names has changed
    since the counters were taken (hash of each source file)."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    srcs = []
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            k, v = k.strip(), v.strip().strip("`")
            if k.startswith("source_sha256 "):
                srcs.append((k.split(" ", 1)[1].strip(), v))
            else:
                kv[k] = v
    if kv.get("kernel_class") != kernel or not srcs:
        return None
    for path, sha in srcs:
        src = os.path.join(ROOT, path)
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != sha:
            return None
    return float(kv["hbm_bytes_per_launch"])


def cpu_info():
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


_POOL = {}  # state the pool workers inherit at fork (the coefficient grid is large)


def _eval_one(z):
    """One (layer, field) coefficient grid of the oracle (pool worker)."""
    from threadpoolctl import threadpool_limits
    from oracle import reconstruct as rc
    S = _POOL
    with threadpool_limits(1):
        t0 = time.perf_counter()
        rc.eval_grid(S["g"], S["A"], S["At"], S["eh"], S["eth"], S["gx"], S["gy"], [z], [rc.U], window=S["win"],
                     prefilter=True)
        return time.perf_counter() - t0


def _interp_chunk(sel):
    from threadpoolctl import threadpool_limits
    from oracle import reconstruct as rc
    S = _POOL
    with threadpool_limits(1):
        t0 = time.perf_counter()
        rc.interp_points(S["g"], S["coef"], S["zl"], S["gx"], S["gy"], S["win"], S["sp"][:, sel], list(range(11)))
        return time.perf_counter() - t0


def cpu_baseline(pts, win, zl, phases, pool_workers=None):
    """The FP64 oracle on a bounded sample of the steep-sea CFD update,
    scaled to one update: one right-hand side (x 4 for the RK4 step), the
    mean-level modes and their time derivative, the coefficient grids of 2 of
    the 64 x 8 + 2 (layer, field) planes (scaled), and the interpolation of
    100,000 of the 20M points (scaled).  Timed on one thread (BLAS pools
    limited to 1); the evaluation and interpolation samples are also timed
    over a process pool on every host core (the oracle's FFTs are serial, so
    the right-hand side and the modes keep their one-thread times)."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    from threadpoolctl import threadpool_limits
    from oracle import Grid, hos, sea
    from oracle import reconstruct as rc
    g = Grid(nx=N5, ny=N5, lx=L5, ly=L5, depth=-1.0, order_m=M5)
    eh, ph = sea.jonswap(g, HS5, 1.0, GAMMA5, phases, "cos2")
    gx, gy, ix0, iy0, wx, wy = win
    window = (ix0, iy0, wx, wy)
    npl = zl.size * 8 + 2
    nsamp = 100_000
    sel = np.linspace(0, pts.shape[1] - 1, nsamp).astype(np.int64)
    sp = pts[:, sel]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        hos.rhs(g, eh, ph)
        t_rhs = time.perf_counter() - t0
        t0 = time.perf_counter()
        A = hos.mean_level_modes(g, eh, ph)
        At, eth = hos.mean_level_modes_t(g, eh, ph)
        t_modes = time.perf_counter() - t0
        t0 = time.perf_counter()
        rc.eval_grid(g, A, At, eh, eth, gx, gy, zl[[0, zl.size // 2]], [rc.U], window=window, prefilter=True)
        t_eval = (time.perf_counter() - t0) * npl / 2
        # a coefficient grid for the interpolation timing (values do not matter for the timing)
        rng = np.random.default_rng(0)
        shape = (zl.size, wy, wx)
        coef = {f: (rng.standard_normal(shape).astype(np.float64) if f not in (rc.ETA, rc.ETA_T)
                    else rng.standard_normal((1, wy, wx))[0]) for f in range(11) if f != rc.P}
        t0 = time.perf_counter()
        rc.interp_points(g, coef, zl, gx, gy, window, sp, list(range(11)))
        t_interp = (time.perf_counter() - t0) * pts.shape[1] / nsamp
    total = 4 * t_rhs + t_modes + t_eval + t_interp
    model, nproc = cpu_info()
    res = {
        "value": pts.shape[1] * NFIELDS / total,
        "unit": "cell-centre field pts/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"steep sea 1024x1024 M=5: one right-hand side (x4 for the RK4 step) + modes A, A_t + "
                   f"coefficient grids of 2 of {npl} (layer, field) planes (scaled) + interpolation of {nsamp} of "
                   f"{pts.shape[1]} points (scaled); numpy FP64, one thread"),
        "seconds": {"rhs": t_rhs, "step_4rhs": 4 * t_rhs, "modes": t_modes, "eval_scaled": t_eval,
                    "interp_scaled": t_interp, "update": total},
        "hos_steps_per_s": 1.0 / (4 * t_rhs),
        "cpu": model,
        "nproc": nproc,
    }
    # all host cores: the independent evaluation planes and point chunks over a pool
    workers = pool_workers or max(1, min(nproc or 1, 16))
    if workers > 1:
        import multiprocessing as mp
        _POOL.update(g=g, A=A, At=At, eh=eh, eth=eth, gx=gx, gy=gy, win=window, coef=coef, zl=zl, sp=sp)
        z_s = [float(zl[(i * 7) % zl.size]) for i in range(workers)]
        with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
            list(ex.map(_interp_chunk, [np.arange(2)] * workers))  # start the workers
            t0 = time.perf_counter()
            list(ex.map(_eval_one, z_s))
            t_eval_pool = (time.perf_counter() - t0) * npl / workers
            chunks = np.array_split(np.arange(nsamp), workers)
            t0 = time.perf_counter()
            list(ex.map(_interp_chunk, chunks))
            t_interp_pool = (time.perf_counter() - t0) * pts.shape[1] / nsamp
        _POOL.clear()
        tot_pool = 4 * t_rhs + t_modes + t_eval_pool + t_interp_pool
        res["all_cores"] = {"value": pts.shape[1] * NFIELDS / tot_pool, "cores": workers,
                            "seconds": {"eval_scaled": t_eval_pool, "interp_scaled": t_interp_pool, "update": tot_pool},
                            "note": "evaluation planes and point chunks over a process pool; the right-hand side "
                                    "and the modes are serial FFT work and keep their one-thread times"}
    return res


def run_steep(lib, torch, steps, warmup, inputs):
    """The headline: the steep large sea's CFD update at 20M cell centres."""
    pts, win, zl, phases = inputs
    gx, gy, ix0, iy0, wx, wy = win
    d = lib.hos_desc(3, N5, N5, L5, L5, -1.0, order_m=M5, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=HS5, kp=1.0, gamma=GAMMA5, phases=phases)
    h = lib.Hos(d, eh, ph)
    gd = lib.grid_desc(gx, gy, zl, (ix0, iy0, wx, wy))
    t0 = time.perf_counter()
    cells = h.bind(gd, torch.tensor(pts, device="cuda"))
    t_bind = time.perf_counter() - t0
    out = torch.empty((NFIELDS, cells.n), dtype=torch.float32, device="cuda")
    _, nbad = cells.interp(lib.ALL_FIELDS, out)
    assert nbad == 0, f"{nbad} points outside the grid"
    print(f"# steep sea: {cells.n} points, window {wx}x{wy} of {gx}x{gy}, {zl.size} layers, bind {t_bind:.1f} s",
          file=sys.stderr, flush=True)

    def step():
        h.step(1)
        cells.interp(lib.ALL_FIELDS, out, count=False)

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, k):
        torch.cuda.synchronize()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    for _ in range(warmup):
        step()
    ms_step = timed(step, steps)
    print(f"# steep sea: step then interpolation {ms_step:.3f} ms", file=sys.stderr, flush=True)
    for _ in range(2):
        cells.interp_step(lib.ALL_FIELDS, out, 1)
    ms_pipe = timed(lambda: cells.interp_step(lib.ALL_FIELDS, out, 1), steps)
    print(f"# steep sea: concurrent {ms_pipe:.3f} ms", file=sys.stderr, flush=True)
    ms_hos = timed(lambda: h.step(1), steps)
    ms_interp = timed(lambda: cells.interp(lib.ALL_FIELDS, out, count=False), steps)
    print(f"# steep sea: hos {ms_hos:.3f} ms, modes+grid+gather {ms_interp:.3f} ms", file=sys.stderr, flush=True)
    kernels = hos_model_bytes(kernel_profile(h, step, max(3, steps // 4)), M5, 3 * N5, 3 * N5)
    cells.close()
    h.close()
    return {"ms_step": ms_step, "ms_pipe": ms_pipe, "ms_hos": ms_hos, "ms_interp": ms_interp, "points": int(pts.shape[1]),
            "win": win, "layers": int(zl.size), "kernels": kernels, "bind_s": t_bind}


def run_cylinder(lib, torch, steps, warmup):
    """The 512 x 256, M = 3 sea with the 1,996,800-point cylinder O-mesh (n =
    4 window, 48 layers): CFD update, HOS step, graph launch, kernel
    breakdown; then the direct sums, the cell-side passes and the stream-
    function wave on the same cells."""
    import numpy as np
    import synth
    pts, win, zl, phases = workload()
    gx, gy, ix0, iy0, wx, wy = win
    d = lib.hos_desc(3, NX, NY, LX, LY, -1.0, order_m=M, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=HS, kp=1.0, gamma=3.3, phases=phases)
    h = lib.Hos(d, eh, ph)
    gd = lib.grid_desc(gx, gy, zl, (ix0, iy0, wx, wy))
    cells = h.bind(gd, torch.tensor(pts, device="cuda"))
    out = torch.empty((NFIELDS, cells.n), dtype=torch.float32, device="cuda")
    _, nbad = cells.interp(lib.ALL_FIELDS, out)
    assert nbad == 0

    def step():
        h.step(1)
        cells.interp(lib.ALL_FIELDS, out, count=False)

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, k):
        torch.cuda.synchronize()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    for _ in range(warmup):
        step()
    ms_step = timed(step, steps)
    for _ in range(2):
        cells.interp_step(lib.ALL_FIELDS, out, 1)
    ms_pipe = timed(lambda: cells.interp_step(lib.ALL_FIELDS, out, 1), steps)
    gb = lib.Batch([h], [cells], [lib.ALL_FIELDS], [out], nsteps=1)
    gb.run()
    ms_graph = timed(gb.run, steps)
    gb.close()
    ms_hos = timed(lambda: h.step(1), 4 * steps)
    ms_interp = timed(lambda: cells.interp(lib.ALL_FIELDS, out, count=False), steps)
    kernels = hos_model_bytes(kernel_profile(h, step, steps), M, 2 * NX, 2 * NY)
    best = min(ms_step, ms_pipe, ms_graph)
    res = {
        "workload": "3D JONSWAP 512x256 modes M=3 (40x20 lambda_p, Hs/lambda_p=0.02, gamma=3.3, seed 1) -> "
                    "1,996,800-point cylinder O-mesh, 11 fields, n=4 window, 48 layers",
        "points": cells.n, "ms_per_step": best,
        "cell_field_pts_per_s": cells.n * NFIELDS / (best / 1e3),
        "eager_ms_per_step": ms_step, "concurrent_ms_per_step": ms_pipe, "graph_ms_per_step": ms_graph,
        "hos_steps_per_s": 1e3 / ms_hos, "hos_mode_steps_per_s": NX * NY * 1e3 / ms_hos,
        "interp_eval_pts_per_s": cells.n * NFIELDS / (ms_interp / 1e3),
        "roofline": roofline_of(kernels), "kernels": kernels,
    }
    # direct analytical evaluation (the exact FP64 modal sums, every mode at
    # every point) at the first 65536 cell centres, at the same state
    sub = cells._xyz[:, :65536].contiguous()
    h.eval_points_direct(sub, lib.ALL_FIELDS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.eval_points_direct(sub, lib.ALL_FIELDS)
    torch.cuda.synchronize()
    ms_direct = (time.perf_counter() - t0) * 1e3
    nmodes = NY * (NX // 2 + 1)
    res["direct_eval"] = {"points": int(sub.shape[1]), "modes": nmodes, "fields": NFIELDS, "dtype": "f64",
                          "ms": ms_direct, "point_modes_per_s": sub.shape[1] * nmodes / (ms_direct / 1e3)}
    # cell-side passes on every cell: incident volume fraction from the
    # interpolated eta (cell heights of the mesh's z-levels), modified
    # pressure, relaxation of alpha and three velocity rows (every cell in
    # the zone); bytes = inputs read + outputs written
    ncell = cells.n
    fl = cells.interp(lib.P | lib.ETA)[0]
    p_c, eta_c = fl[0].contiguous(), fl[1].contiguous()  # bit order: P before ETA
    dzc = np.diff(synth.cylinder_z_edges(HS, LAM)).astype(np.float32)
    dz_c = torch.tensor(np.tile(dzc, ncell // dzc.size), device="cuda")
    zc = cells._xyz[2].contiguous()
    xr = torch.linspace(0.0, 1.0, ncell, dtype=torch.float32, device="cuda")
    alpha = torch.empty(ncell, dtype=torch.float32, device="cuda")
    ps = torch.empty_like(alpha)
    ucv = torch.randn(3, ncell, dtype=torch.float32, device="cuda")
    acfd = torch.rand(ncell, dtype=torch.float32, device="cuda")

    def wall(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    cs = {}
    for name, fn, nb in [("alpha", lambda: h.cells_alpha(eta_c, zc, dz_c, out=alpha), 20),
                         ("pstar", lambda: h.cells_pstar(p_c, alpha, 1.2, out=ps), 12),
                         ("relax", lambda: h.cells_relax(xr, alpha, acfd, ucv), 40)]:
        ms = wall(fn)
        cs[name] = {"ms": ms, "bytes_per_cell": nb, "GB_per_s": nb * ncell / (ms / 1e3) / 1e9,
                    "frac_of_hbm_peak": nb * ncell / (ms / 1e3) / PEAK_HBM}
    res["cell_side"] = {"cells": ncell, **cs}
    # stream-function regular wave (ka = 0.24, N = 9, kh = 2) at every cell, all fields
    sd, ssol = lib.stream_solve(2.0, 0.48, LAM, 9)
    sout = torch.empty((NFIELDS, ncell), dtype=torch.float64, device="cuda")
    ms_stream = wall(lambda: lib.stream_eval(sd, ssol, 0.3, cells._xyz, lib.ALL_FIELDS, out=sout), reps=5)
    res["stream_wave_eval"] = {"points": ncell, "modes": 9, "fields": NFIELDS, "dtype": "f64", "ms": ms_stream,
                               "cell_field_pts_per_s": ncell * NFIELDS / (ms_stream / 1e3)}
    cells.close()
    h.close()
    return res


def run_regular_2d(lib, torch, steps):
    """The 2D regular wave: Stokes-2 initial state, ka = 0.1, kh = 2, 256
    modes over 4 wavelengths, M = 3 with full dealiasing, FP64, RK4 T/64;
    steps/s over two periods (128 steps), then the fold to 64 nodes x 32
    layers and the interpolation of 10k points (seed 0)."""
    import numpy as np
    import synth
    h0 = 2.0
    k = 2 * math.pi * 4 / (4 * LAM)
    depth = h0 / k
    lx = 4 * LAM
    omega = math.sqrt(k * math.tanh(k * depth))
    d = lib.hos_desc(2, 256, 1, lx, 1.0, depth, order_m=3, dt=(2 * math.pi / omega) / 64, precision=1)
    eh, ph = lib.sea_spectrum(d, kind=1, mode=4, ka=0.1)
    h = lib.Hos(d, eh, ph)
    h.step(4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    h.step(128)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 128
    zl = np.linspace(-depth, 0.0, 32)
    gd = lib.grid_desc(64, 1, zl)
    pts = synth.uniform_points_2d(0, 10000, 0.0, lx, -depth, 0.0)
    cells = h.bind(gd, torch.tensor(pts, device="cuda"))
    out = torch.empty((NFIELDS, cells.n), dtype=torch.float32, device="cuda")
    cells.interp(lib.ALL_FIELDS, out)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        cells.interp(lib.ALL_FIELDS, out, count=False)
    e1.record()
    torch.cuda.synchronize()
    ms_i = e0.elapsed_time(e1) / steps
    cells.close()
    h.close()
    return {"workload": "2D Stokes wave ka=0.1 kh=2, 256 modes over 4 wavelengths, M=3, FP64, RK4 T/64",
            "hos_steps_per_s": 1e3 / ms, "ms_per_step": ms,
            "interp_10k_points_ms": ms_i, "interp_cell_field_pts_per_s": 10000 * NFIELDS / (ms_i / 1e3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline only (no other configurations)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-fixed", action="store_true",
                    help="batched leg with product-grid policy 2 everywhere and no branch autotuning (counter passes)")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-trajectories", type=int, default=100)
    ap.add_argument("--surrogate-iters", type=int, default=1000)
    ap.add_argument("--only", choices=["cylinder", "regular_wave_2d", "batched", "surrogate"], default=None,
                    help="run one secondary configuration alone and print its record (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run plain 256 MiB device copies (reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the workload is a single "
              "realisation and the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.only:
        import torch
        from paper_2005_12716_amd import lib
        torch.cuda.set_device(0)
        run = {"cylinder": lambda: run_cylinder(lib, torch, max(20, args.steps), args.warmup),
               "regular_wave_2d": lambda: run_regular_2d(lib, torch, args.steps),
               "batched": lambda: run_batched(lib, torch, max(2, args.steps // 4), args.batched_fixed),
               "surrogate": lambda: run_surrogate(lib, torch, max(5, args.steps), args.surrogate_trajectories,
                                                  args.surrogate_iters)}[args.only]
        print(json.dumps({args.only: run()}))
        return

    # the oracle first, before anything touches the GPU, so that its pool
    # workers fork from a process without a GPU context
    inputs = workload5()
    cb = None
    if not args.no_cpu_baseline:
        print("# oracle on the host", file=sys.stderr, flush=True)
        cb = cpu_baseline(*inputs)
        print(f"# oracle {cb['value']:.3g} cell-centre field pts/s", file=sys.stderr, flush=True)

    import torch
    from paper_2005_12716_amd import lib

    torch.cuda.set_device(0)
    st = run_steep(lib, torch, args.steps, args.warmup, inputs)
    best = min(st["ms_step"], st["ms_pipe"])
    n = st["points"]
    gx, gy, ix0, iy0, wx, wy = st["win"]
    res = {
        "metric": "cell-centre field pts/s (end-to-end CFD update: HOS step + modes + grid + interpolation)",
        "value": n * NFIELDS / (best / 1e3),
        "unit": "cell-centre field pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 transforms / f64 state, phases and vertical factors",
        "data": "synthetic",
        "config": {"workload": "steep large sea: 3D JONSWAP 1024x1024 modes M=5 (40x40 lambda_p, Hs/lambda_p=0.04, "
                               "gamma=5, seed 5) -> 20,000,000-point jittered hex mesh (500x250x160, seed 6), "
                               "11 fields, n=4 window, 64 layers",
                   "execution": ("interpolation concurrent with the step (swense_interp_step)" if st["ms_pipe"] < st["ms_step"]
                                 else "step, then interpolation (swense_hos_step + swense_interp_cells)"),
                   "points": n, "modes": [N5, N5], "order_m": M5, "padded": [3 * N5, 3 * N5],
                   "grid": [gx, gy], "window": [ix0, iy0, wx, wy], "layers": st["layers"]},
        "eager_ms_per_step": st["ms_step"],
        "concurrent_ms_per_step": st["ms_pipe"],
        "hos_ms_per_step": st["ms_hos"],
        "hos_steps_per_s": 1e3 / st["ms_hos"],
        "hos_mode_steps_per_s": N5 * N5 * 1e3 / st["ms_hos"],
        "interp_eval_ms": st["ms_interp"],
        "bind_s": st["bind_s"],
        "roofline": roofline_of(st["kernels"], traffic_file=True),
        "kernels": st["kernels"],
    }
    if not args.no_extra:
        print("# cylinder O-mesh configuration", file=sys.stderr, flush=True)
        res["cylinder_512x256"] = run_cylinder(lib, torch, max(20, args.steps), args.warmup)
        print("# 2D regular wave", file=sys.stderr, flush=True)
        res["regular_wave_2d"] = run_regular_2d(lib, torch, args.steps)
        res["fv_divergence_paper_demo"] = run_fv_divergence(lib, torch)
        if not args.no_batched:
            print("# batched configuration", file=sys.stderr, flush=True)
            res["batched"] = run_batched(lib, torch, max(2, args.steps // 4))
            print(f"# batched {res['batched']['ms_per_launch']:.2f} ms per launch", file=sys.stderr, flush=True)
        if not args.no_surrogate:
            print("# surrogate configuration (brief training, then rollout)", file=sys.stderr, flush=True)
            res["surrogate"] = run_surrogate(lib, torch, max(5, args.steps), args.surrogate_trajectories,
                                             args.surrogate_iters)
            print(f"# surrogate {res['surrogate']['ms_per_network_call']:.2f} ms per call", file=sys.stderr, flush=True)
    if cb is not None:
        res["cpu_baseline"] = cb
        res["speedup_vs_cpu_baseline"] = res["value"] / cb["value"]
        res["hos_speedup_vs_cpu_baseline"] = res["hos_steps_per_s"] / cb["hos_steps_per_s"]
    print(json.dumps(res))


if __name__ == "__main__":
    main()
