"""Writes steep_sea_16steps.npz, the oracle's reference for the steep large
sea after 16 RK4 steps: 1024 x 1024 modes over 40 x 40 peak wavelengths,
deep water, order M = 5 with full dealiasing, JONSWAP Hs/lambda_p = 0.04,
gamma = 5, cos^2 spreading, phases seed 5, dt = Tp/64 (nondimensional g = 1,
k_p = 1).  Stored:

* the FP64 state (eta_hat, phis_hat) on the modes p < 128, |q| < 128 (the
  energetic part of the spectrum and its first harmonics), the norms of the
  whole half spectra and of the part outside that block;
* 2000 cell centres of the 20M-point hex mesh (every 10000th, plus the 16
  nearest to the mean level and 16 spread over the top layer of cells) and
  the oracle's interpolated values of all 11 fields there: coefficient grids
  refined four times (4096^2 nodes) on the mesh window with a 3-node halo,
  64 layers clustered about the mean level, periodic cubic spline
  horizontally and 4-point Lagrange vertically;
* at each of those points, the RMS over the horizontal plane at the point's
  height of each field (Parseval over the kept modes): far above the crests
  the continued fields are sums of terms grown by e^{kz}, and the attainable
  accuracy of single-precision transforms there is relative to that size.

Only the oracle and the seeded generators are called.  Takes about 15
minutes on one core (the evaluation planes run over a process pool):
    python tests/golden/make_steep_sea.py
"""
from __future__ import annotations

import math
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import Grid, hos, sea  # noqa: E402
from oracle import reconstruct as rc  # noqa: E402

LAM = 2 * math.pi
N, M = 1024, 5
L = 40 * LAM
HS = 0.04 * LAM
NSTEPS = 16
PB = 128  # block of stored modes: p < PB, |q| < PB
GX = 4 * N

_S = {}


def _rms_at(args):
    """Plane RMS of volume field f at every height in zs (Parseval over the
    kept modes p < nx/2, q != ny/2; modes p > 0 count twice)."""
    f, zs = args
    S = _S
    g = S["g"]
    hx = g.nx // 2
    keep = np.arange(g.ny) != g.ny // 2
    w = np.where(np.arange(hx) == 0, 1.0, 2.0)[None, :]
    out = np.empty(len(zs))
    for k, z in enumerate(zs):
        fh = rc.field_spectrum(g, f, S["A"], S["At"], float(z))[keep, :hx]
        out[k] = math.sqrt(float(np.sum(w * np.abs(fh) ** 2)))
    return out


def _plane(args):
    f, z = args
    S = _S
    fh = rc.field_spectrum(S["g"], f, S["A"], S["At"], z)
    nodes = rc.node_values(S["g"], fh, GX, GX, prefilter=True)
    return rc._window(nodes, *S["win"], GX, GX)


def main():
    g = Grid(nx=N, ny=N, lx=L, ly=L, depth=-1.0, order_m=M)
    e0, p0 = sea.jonswap(g, HS, 1.0, 5.0, synth.mode_phases(5, N, N // 2 + 1), "cos2")
    e, p = hos.run(g, e0, p0, LAM / 64, NSTEPS, lambda n, ee, pp: print(f"step {n}", flush=True))
    rows = np.r_[0:PB, N - PB + 1:N]
    eb, pb = e[rows, :PB], p[rows, :PB]
    mask = np.ones(e.shape, dtype=bool)
    mask[np.ix_(rows, np.arange(PB))] = False
    A = hos.mean_level_modes(g, e, p)
    At, eth = hos.mean_level_modes_t(g, e, p)
    x0, y0, wx, wy = L / 2 - 4 * LAM, L / 2 - 2 * LAM, 8 * LAM, 4 * LAM
    pts, mesh = synth.hex_cloud(6, x0, y0, wx, wy, -0.5 * LAM, 0.2 * LAM, 500, 250, 160, HS / 16)
    dx = L / GX
    win = (int(math.floor(x0 / dx)) - 2, int(math.floor(y0 / dx)) - 2, int(math.ceil(wx / dx)) + 6,
           int(math.ceil(wy / dx)) + 6)
    zl = np.asarray(synth.clustered_layers(mesh["ze"][0] - 1e-9, mesh["ze"][-1] + 1e-9, 64, HS / 16))
    n = pts.shape[1]
    near = np.argsort(np.abs(pts[2]))[:16]
    top = np.flatnonzero(pts[2] > mesh["ze"][-2])[:: max(1, np.count_nonzero(pts[2] > mesh["ze"][-2]) // 16)][:16]
    idx = np.unique(np.concatenate([np.arange(0, n, 10000), near, top]))[:2000]
    sp = pts[:, idx]
    _S.update(g=g, A=A, At=At, win=win)
    vol = [rc.PHI, rc.U, rc.V, rc.W, rc.PHI_T, rc.U_T, rc.V_T, rc.W_T]
    coef = {}
    with ProcessPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        for f in vol:
            coef[f] = np.stack(list(ex.map(_plane, [(f, float(z)) for z in zl])))
            print(f"field {f}", flush=True)
    coef[rc.ETA] = rc._window(rc.node_values(g, e, GX, GX, prefilter=True), *win, GX, GX)
    coef[rc.ETA_T] = rc._window(rc.node_values(g, eth, GX, GX, prefilter=True), *win, GX, GX)
    vals, nbad = rc.interp_points(g, coef, zl, GX, GX, win, sp, list(range(11)))
    assert nbad == 0
    with ProcessPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        rms = dict(zip(vol, ex.map(_rms_at, [(f, sp[2]) for f in vol])))
    hx = N // 2
    keep = np.arange(N) != N // 2
    wts = np.where(np.arange(hx) == 0, 1.0, 2.0)[None, :]
    srms = [math.sqrt(float(np.sum(wts * np.abs(x[keep, :hx]) ** 2))) for x in (e, eth)]
    plane_rms = np.zeros((11, sp.shape[1]))
    for f in vol:
        plane_rms[f] = rms[f]
    plane_rms[rc.ETA] = srms[0]
    plane_rms[rc.ETA_T] = srms[1]
    # pressure: rho (|phi_t| + |grad phi|^2) scale at the height, plus rho g |z|
    plane_rms[rc.P] = g.rho * (rms[rc.PHI_T] + rms[rc.U] ** 2 + rms[rc.V] ** 2 + rms[rc.W] ** 2 + g.g * np.abs(sp[2]))
    np.savez_compressed(os.path.join(HERE, "steep_sea_16steps.npz"),
                        eta_block=eb, phis_block=pb, block_rows=rows, block_cols=np.arange(PB),
                        eta_norm=np.linalg.norm(e), phis_norm=np.linalg.norm(p),
                        eta_outside_norm=np.linalg.norm(e[mask]), phis_outside_norm=np.linalg.norm(p[mask]),
                        point_index=idx, points=sp, values=np.stack([vals[f] for f in range(11)]),
                        plane_rms=plane_rms)
    print("written", flush=True)


if __name__ == "__main__":
    main()
