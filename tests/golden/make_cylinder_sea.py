"""Writes cylinder_sea_128steps.npz, the oracle's reference for the 512 x 256
irregular sea after 128 RK4 steps (two peak periods): modes over 40 x 20 peak
wavelengths, deep water, order M = 3 with full dealiasing, JONSWAP
Hs/lambda_p = 0.02, gamma = 3.3, cos^2 spreading, phases seed 1, dt = Tp/64
(nondimensional g = 1, k_p = 1).  Stored:

* the FP64 state (eta_hat, phis_hat) on the modes p < 128, |q| < 64, the
  norms of the whole half spectra and of the part outside that block;
* 2000 of the 1,996,800 cell centres of the cylinder O-mesh (every 998th)
  and the oracle's interpolated values of all 11 fields there: coefficient
  grids refined four times (2048 x 1024 nodes) on a 4.1 x 4.1 lambda_p window
  with a halo, 48 layers clustered about the mean level, periodic cubic
  spline horizontally and 4-point Lagrange vertically.

Only the oracle and the seeded generators are called.  A few minutes on
one core:
    python tests/golden/make_cylinder_sea.py
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import Grid, hos, sea  # noqa: E402
from oracle import reconstruct as rc  # noqa: E402

LAM = 2 * math.pi
NX, NY, M = 512, 256, 3
LX, LY = 40 * LAM, 20 * LAM
HS = 0.02 * LAM
NSTEPS = 128
PB, QB = 128, 64


def window_and_layers(pts):
    """The cylinder mesh's grid window (n = 4) and 48 layers."""
    gx, gy = 4 * NX, 4 * NY
    dx = LX / gx
    ix0 = int(math.floor((LX / 2 - 2.05 * LAM) / dx)) - 2
    wx = int(math.ceil(4.1 * LAM / dx)) + 6
    iy0 = int(math.floor((LY / 2 - 2.05 * LAM) / dx)) - 2
    zl = np.asarray(synth.clustered_layers(pts[2].min() - 1e-9, pts[2].max() + 1e-9, 48, HS / 16))
    return (gx, gy), (ix0, iy0, wx, wx), zl


def main():
    g = Grid(nx=NX, ny=NY, lx=LX, ly=LY, depth=-1.0, order_m=M)
    e0, p0 = sea.jonswap(g, HS, 1.0, 3.3, synth.mode_phases(1, NY, NX // 2 + 1), "cos2")
    e, p = hos.run(g, e0, p0, LAM / 64, NSTEPS)
    rows = np.r_[0:QB, NY - QB + 1:NY]
    mask = np.ones(e.shape, dtype=bool)
    mask[np.ix_(rows, np.arange(PB))] = False
    A = hos.mean_level_modes(g, e, p)
    At, eth = hos.mean_level_modes_t(g, e, p)
    pts = synth.cylinder_cloud(LX, LY, HS)
    (gx, gy), win, zl = window_and_layers(pts)
    idx = np.arange(0, pts.shape[1], 998)[:2000]
    sp = pts[:, idx]
    fields = [f for f in range(11) if f != rc.P]
    coef = rc.eval_grid(g, A, At, e, eth, gx, gy, zl, fields, window=win, prefilter=True)
    vals, nbad = rc.interp_points(g, coef, zl, gx, gy, win, sp, list(range(11)))
    assert nbad == 0
    np.savez_compressed(os.path.join(HERE, "cylinder_sea_128steps.npz"),
                        eta_block=e[rows, :PB], phis_block=p[rows, :PB], block_rows=rows, block_cols=np.arange(PB),
                        eta_norm=np.linalg.norm(e), phis_norm=np.linalg.norm(p),
                        eta_outside_norm=np.linalg.norm(e[mask]), phis_outside_norm=np.linalg.norm(p[mask]),
                        point_index=idx, points=sp, values=np.stack([vals[f] for f in range(11)]))
    print("written", flush=True)


if __name__ == "__main__":
    main()
