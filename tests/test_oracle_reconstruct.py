"""Pins of the oracle's reconstruction (Sec. 3.2, 3.3): grid evaluation
against brute-force modal sums, zero divergence per mode (also above the
mean level), the interpolation scheme against an independent periodic
spline and its convergence orders, and the paper's zero-padding
divergence reduction (Sec. 3.2.4)."""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import synth
from oracle import Grid, hos, sea
from oracle import reconstruct as rc

LAM = 2 * math.pi


def _state(nx, ny, depth, M=3, steps=4, seed=21, hs=0.03):
    g = Grid(nx=nx, ny=ny, lx=nx * LAM / 6.4, ly=max(ny, 1) * LAM / 6.4 if ny > 1 else 1.0,
             depth=depth, order_m=M)
    eh, ph = sea.jonswap(g, hs * LAM, 1.0, 3.3, synth.mode_phases(seed, ny, g.nxh))
    eh, ph = hos.run(g, eh, ph, LAM / 64, steps)
    A = hos.mean_level_modes(g, eh, ph)
    At, eth = hos.mean_level_modes_t(g, eh, ph)
    return g, eh, ph, A, At, eth


@pytest.mark.parametrize("ny,depth", [(1, 1.2), (8, -1.0), (8, 1.2)])
@pytest.mark.parametrize("n", [0.5, 1, 2, 4])
def test_eval_grid_equals_brute_force(ny, depth, n):
    nx = 16
    g, eh, ph, A, At, eth = _state(nx, ny, depth)
    gx = int(nx * n)
    gy = int(ny * n) if ny > 1 else 1
    zl = np.array([-1.1, -0.4, 0.0, 0.3])
    fields = list(range(11))
    win = (3, 1 if ny > 1 else 0, gx - 5, gy - 2 if ny > 1 else 1)
    out = rc.eval_grid(g, A, At, eh, eth, gx, gy, zl, fields, window=win)
    xs = g.lx * ((win[0] + np.arange(win[2])) % gx) / gx
    ys = g.ly * ((win[1] + np.arange(win[3])) % gy) / gy if ny > 1 else np.zeros(1)
    X, Y = np.meshgrid(xs, ys)
    for li, z in enumerate(zl):
        pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)])
        ref = rc.analytic_at_points(g, A, At, eh, eth, pts, fields)
        for f in fields:
            got = out[f][li] if f in rc.VOLUME else out[f]
            scale = max(1e-300, np.abs(ref[f]).max())
            if f == rc.P:
                scale = max(scale, 1.0)
            assert np.abs(got.ravel() - ref[f]).max() <= 1e-12 * scale, (f, z)


@pytest.mark.parametrize("depth", [1.2, -1.0])
def test_divergence_free_per_mode_on_nodes(depth):
    """du/dx + dv/dy (spectral) + dw/dz (4th-order difference in z) = 0 on
    every node, below and above z = 0 (extension into the air)."""
    g, eh, ph, A, At, eth = _state(16, 8, depth)
    KX, KY, _ = g.kvec()
    for z in (-1.0, -0.2, 0.0, 0.25):
        ux = rc.node_values(g, 1j * KX * rc.field_spectrum(g, rc.U, A, At, z), 32, 16)
        vy = rc.node_values(g, 1j * KY * rc.field_spectrum(g, rc.V, A, At, z), 32, 16)
        d = 1e-3
        wz = sum(c * rc.node_values(g, rc.field_spectrum(g, rc.W, A, At, z + s * d), 32, 16)
                 for c, s in ((-1, 2), (8, 1), (-8, -1), (1, -2))) / (12 * d)
        scale = np.abs(ux).max()
        assert np.abs(ux + vy + wz).max() < 1e-8 * scale


def test_lagrange_reproduces_cubics_and_bspline_reproduces_linear():
    rng = np.random.default_rng(0)
    zl = np.sort(rng.uniform(-2, 1, 9))
    z = rng.uniform(zl[0], zl[-1], 200)
    l0, w, dw, ok = rc.lagrange_weights(zl, z)
    assert ok.all()
    poly = lambda t: 0.3 * t ** 3 - t ** 2 + 2 * t - 0.7  # noqa: E731
    dpoly = lambda t: 0.9 * t ** 2 - 2 * t + 2  # noqa: E731
    got = sum(w[a] * poly(zl[l0 + a]) for a in range(4))
    dgot = sum(dw[a] * poly(zl[l0 + a]) for a in range(4))
    assert np.allclose(got, poly(z), atol=1e-12) and np.allclose(dgot, dpoly(z), atol=1e-11)
    t = rng.uniform(0, 1, 100)
    wb = rc.bspline_weights(t)
    assert np.allclose(wb.sum(0), 1) and np.allclose(wb[0] * -1 + wb[2] + 2 * wb[3], t)


def test_horizontal_interpolant_is_the_periodic_cubic_spline():
    """Against scipy's periodic CubicSpline through the node values."""
    g, eh, ph, A, At, eth = _state(32, 1, 1.2)
    zl = np.array([-1.0, -0.5, -0.2, 0.0])
    for gx in (32, 64):
        vals = rc.eval_grid(g, A, At, eh, eth, gx, 1, zl, [rc.U, rc.ETA])
        coef = rc.eval_grid(g, A, At, eh, eth, gx, 1, zl, [rc.U, rc.ETA], prefilter=True)
        xn = g.lx * np.arange(gx + 1) / gx
        rng = np.random.default_rng(gx)
        x = rng.uniform(0, g.lx, 300)
        pts = np.stack([x, np.zeros_like(x), np.full_like(x, -0.5)])
        got, nbad = rc.interp_points(g, coef, zl, gx, 1, None, pts, [rc.U, rc.ETA])
        assert nbad == 0
        for f, row in ((rc.U, vals[rc.U][1, 0]), (rc.ETA, vals[rc.ETA][0])):
            cs = CubicSpline(xn, np.append(row, row[0]), bc_type="periodic")
            assert np.abs(got[f] - cs(x)).max() < 1e-12 * np.abs(row).max()


def test_interpolation_convergence_orders():
    """Errors against brute-force modal sums at random points fall at order
    4 for values and order 3 for the divergence of the interpolant as both
    the node spacing and the layer spacing halve."""
    g, eh, ph, A, At, eth = _state(16, 8, 1.5, hs=0.02)
    rng = np.random.default_rng(3)
    npts = 400
    pts = np.stack([rng.uniform(0, g.lx, npts), rng.uniform(0, g.ly, npts), rng.uniform(-1.0, 0.0, npts)])
    ref = rc.analytic_at_points(g, A, At, eh, eth, pts, [rc.U, rc.W])
    hs, ev, ed = [], [], []
    for n in (2, 4, 8):
        gx, gy = 16 * n, 8 * n
        zl = np.linspace(-1.2, 0.2, 6 * n + 1)
        coef = rc.eval_grid(g, A, At, eh, eth, gx, gy, zl, [rc.U, rc.V, rc.W], prefilter=True)
        got, nbad = rc.interp_points(g, coef, zl, gx, gy, None, pts, [rc.U, rc.W])
        div = rc.divergence_of_interpolant(g, coef, zl, gx, gy, None, pts)
        assert nbad == 0
        hs.append(1.0 / n)
        ev.append(max(np.abs(got[rc.U] - ref[rc.U]).max(), np.abs(got[rc.W] - ref[rc.W]).max()))
        ed.append(np.sqrt(np.mean(div * div)))
    sv = np.polyfit(np.log(hs), np.log(ev), 1)[0]
    sd = np.polyfit(np.log(hs), np.log(ed), 1)[0]
    assert abs(sv - 4) < 0.4, (sv, ev)
    assert abs(sd - 3) < 0.4, (sd, ed)


def test_out_of_range_points_are_counted():
    g, eh, ph, A, At, eth = _state(16, 1, 1.0)
    zl = np.linspace(-1.0, 0.0, 8)
    coef = rc.eval_grid(g, A, At, eh, eth, 16, 1, zl, [rc.U], prefilter=True, window=(2, 0, 10, 1))
    dx = g.lx / 16
    pts = np.array([[3.5 * dx, 4.5 * dx, 1.2 * dx, 10.5 * dx, 5.0 * dx],
                    [0, 0, 0, 0, 0], [-0.5, 0.1, -0.5, -0.5, -0.5]])
    got, nbad = rc.interp_points(g, coef, zl, 16, 1, (2, 0, 10, 1), pts, [rc.U])
    # z above the top layer, x stencil before the window, x stencil past it
    assert nbad == 3
    assert np.isfinite(got[rc.U][[0, 4]]).all() and np.isnan(got[rc.U][[1, 2, 3]]).all()


def test_paper_zero_padding_divergence_reduction():
    """Sec. 3.2.4: 2D JONSWAP (Tp = 0.7 s, Hs = 0.028 m, gamma = 3.3,
    Lx = 10 lambda_p, N = 128), CFD cells (lambda_p/100, Hs/20); refining the
    HOS grid x4 by zero padding cuts the finite-volume divergence of the
    interpolated velocity by about two orders of magnitude, down to the
    floor of the face-centre approximation."""
    g0, tp, hs = 9.81, 0.7, 0.028
    lam = g0 * tp * tp / (2 * math.pi)
    G = Grid(nx=128, ny=1, lx=10 * lam, ly=1.0, depth=-1.0, order_m=3, g=g0, rho=1000.0)
    eh, ps = sea.jonswap(G, hs, 2 * math.pi / lam, 3.3, synth.mode_phases(579, 1, G.nxh))
    eh, ps = hos.run(G, eh, ps, tp / 64, 64)
    A = hos.mean_level_modes(G, eh, ps)
    At, eth = hos.mean_level_modes_t(G, eh, ps)
    dx, dz = lam / 100, hs / 20
    zbot = -0.1 * lam
    nzc = int(round(-zbot / dz))
    xe = np.arange(1001) * dx
    ze = zbot + np.arange(nzc + 1) * dz
    ye = np.array([0.0, 1.0])
    fu, _, fw = rc.face_centres(xe, ye, ze)
    zl = np.linspace(zbot - 2 * dz, 2 * dz, 41)
    rms = {}
    for n in (1, 4):
        coef = rc.eval_grid(G, A, At, eh, eth, 128 * n, 1, zl, [rc.U, rc.W], prefilter=True)
        uu, _ = rc.interp_points(G, coef, zl, 128 * n, 1, None, fu, [rc.U])
        ww, _ = rc.interp_points(G, coef, zl, 128 * n, 1, None, fw, [rc.W])
        div = rc.fv_divergence(uu[rc.U].reshape(nzc, 1, 1001), None, ww[rc.W].reshape(nzc + 1, 1, 1000), xe, ye, ze)
        rms[n] = math.sqrt(float(np.mean(div * div)))
    ua = rc.analytic_at_points(G, A, At, eh, eth, fu, [rc.U])[rc.U]
    wa = rc.analytic_at_points(G, A, At, eh, eth, fw, [rc.W])[rc.W]
    div = rc.fv_divergence(ua.reshape(nzc, 1, 1001), None, wa.reshape(nzc + 1, 1, 1000), xe, ye, ze)
    floor = math.sqrt(float(np.mean(div * div)))
    assert rms[1] / rms[4] > 50, rms
    assert rms[4] < 1.1 * floor, (rms, floor)
