"""GPU finite-volume divergence of the interpolated velocity (Sec. 3.2.3)
against the oracle's (same interpolant at the face centres, same face sums),
and the paper's demonstration that x4 zero-padding refinement of the
intermediate grid cuts it by two orders of magnitude (Sec. 3.2.4)."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import Grid, hos, sea
from oracle import reconstruct as rc

pytestmark = pytest.mark.gpu


def _oracle_div(G, A, At, eh, eth, gx, gy, zl, win, xe, ye, ze, three):
    coef = rc.eval_grid(G, A, At, eh, eth, gx, gy, zl, [rc.U, rc.V, rc.W] if three else [rc.U, rc.W],
                        prefilter=True, window=win)
    fu, fv, fw = rc.face_centres(xe, ye, ze)
    nx, ny, nz = xe.size - 1, ye.size - 1, ze.size - 1
    uu, _ = rc.interp_points(G, coef, zl, gx, gy, win, fu, [rc.U])
    ww, _ = rc.interp_points(G, coef, zl, gx, gy, win, fw, [rc.W])
    vv = None
    if three:
        v, _ = rc.interp_points(G, coef, zl, gx, gy, win, fv, [rc.V])
        vv = v[rc.V].reshape(nz, ny + 1, nx)
    return rc.fv_divergence(uu[rc.U].reshape(nz, ny, nx + 1), vv, ww[rc.W].reshape(nz + 1, ny, nx), xe, ye, ze), \
        np.abs(uu[rc.U]).max()


def test_paper_demo_refinement_on_gpu(gpu_lib):
    from paper_2005_12716_amd import lib
    g0, tp, hs = 9.81, 0.7, 0.028
    lam = g0 * tp * tp / (2 * math.pi)
    d = lib.hos_desc(2, 128, 1, 10 * lam, 1.0, -1.0, order_m=3, dt=tp / 64, g=g0, rho=1000.0)
    G = Grid(nx=128, ny=1, lx=10 * lam, ly=1.0, depth=-1.0, order_m=3, g=g0, rho=1000.0)
    eh, ps = sea.jonswap(G, hs, 2 * math.pi / lam, 3.3, synth.mode_phases(579, 1, G.nxh))
    h = lib.Hos(d, eh, ps)
    h.step(64)
    e, p, _ = h.state()
    A = hos.mean_level_modes(G, e, p)
    At, eth = hos.mean_level_modes_t(G, e, p)
    dx, dz = lam / 100, hs / 20
    zbot = -0.1 * lam
    nzc = int(round(-zbot / dz))
    xe = np.arange(1001) * dx
    ze = zbot + np.arange(nzc + 1) * dz
    ye = np.array([0.0, 1.0])
    zl = np.linspace(zbot - 2 * dz, 2 * dz, 41)
    rms = {}
    for n in (1, 4):
        gd = lib.grid_desc(128 * n, 1, zl)
        div, r, mx = h.fv_divergence(gd, xe, None, ze)
        ref, umax = _oracle_div(G, A, At, e, eth, 128 * n, 1, zl, None, xe, ye, ze, False)
        got = div.cpu().numpy()
        scale = umax / dx
        assert np.sqrt(np.mean((got - ref) ** 2)) <= 2e-5 * scale, n
        assert abs(r - math.sqrt(float(np.mean(got.astype(np.float64) ** 2)))) <= 1e-6 * r
        assert abs(mx - np.abs(got).max()) <= 1e-6 * mx
        rms[n] = r
    print("FV divergence RMS (1/s): n=1", rms[1], "n=4", rms[4])
    assert rms[1] / rms[4] > 50, rms
    h.close()


def test_fv_divergence_3d_window_matches_oracle(gpu_lib):
    from paper_2005_12716_amd import lib
    lamp = 2 * math.pi
    nx, ny = 64, 32
    d = lib.hos_desc(3, nx, ny, nx * lamp / 6.4, ny * lamp / 6.4, -1.0, order_m=3, dt=lamp / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=0.03 * lamp, kp=1.0, gamma=3.3,
                              phases=synth.mode_phases(21, ny, nx // 2 + 1))
    h = lib.Hos(d, eh, ph)
    G = Grid(nx=nx, ny=ny, lx=d.lx, ly=d.ly, depth=-1.0, order_m=3)
    A = hos.mean_level_modes(G, eh, ph)
    At, eth = hos.mean_level_modes_t(G, eh, ph)
    gx, gy = 2 * nx, 2 * ny
    ddx, ddy = d.lx / gx, d.ly / gy
    win = (20, 10, 40, 30)
    xe = (24 + np.linspace(0.0, 28.0, 17)) * ddx
    ye = (14 + np.linspace(0.0, 18.0, 9)) * ddy
    ze = np.linspace(-1.0, 0.15, 7)
    zl = np.linspace(-1.1, 0.25, 16)
    gd = lib.grid_desc(gx, gy, zl, win)
    div, r, mx = h.fv_divergence(gd, xe, ye, ze)
    ref, umax = _oracle_div(G, A, At, eh, eth, gx, gy, zl, win, xe, ye, ze, True)
    got = div.cpu().numpy()
    scale = umax / min(np.diff(xe).min(), np.diff(ye).min(), np.diff(ze).min())
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 2e-5 * scale
    h.close()
