"""GPU parity of the reconstruction (Sec. 3.2, 3.3): grid evaluation with
pad / fold / window and every field, interpolation to scattered points,
the divergence of the interpolant, and out-of-range handling, against the
FP64 oracle on the same state.  Outputs are FP32: relative L2 per field
below 1e-5 (1e-6 typical)."""
import math

import numpy as np

import c18
import pytest
import torch

import synth
from oracle import Grid, hos
from oracle import reconstruct as rc

pytestmark = pytest.mark.gpu
LAM = 2 * math.pi
BITS = [1 << i for i in range(11)]


def rel(a, b):
    """Both C18 measures at once: the larger of the relative L2 error and the
    maximum absolute error over the largest reference magnitude."""
    return c18.both(a, b)


def _state(lib, dim, nx, ny, depth, M=3, steps=3, precision=0, hs=0.03):
    lx = nx * LAM / 6.4
    ly = ny * LAM / 6.4 if dim == 3 else 1.0
    d = lib.hos_desc(dim, nx, ny, lx, ly, depth, order_m=M, dt=LAM / 64, precision=precision)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=hs * LAM, kp=1.0, gamma=3.3, phases=synth.mode_phases(9, ny, nx // 2 + 1))
    g = Grid(nx=nx, ny=ny, lx=lx, ly=ly, depth=depth, order_m=M)
    h = lib.Hos(d, eh, ph)
    h.step(steps)
    er, pr = hos.run(g, eh, ph, d.dt, steps)
    A = hos.mean_level_modes(g, er, pr)
    At, eth = hos.mean_level_modes_t(g, er, pr)
    return h, g, (er, pr, A, At, eth)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("dim,nx,ny,depth,gx,gy,win", [
    (3, 32, 16, -1.0, 64, 32, None),
    (3, 32, 16, 1.2, 128, 64, (10, 5, 70, 30)),
    (3, 30, 20, 1.2, 20, 10, None),               # fold
    (3, 24, 16, -1.0, 96, 64, (90, 60, 12, 8)),   # window wrapping the period
    (2, 64, 1, 1.5, 256, 1, (16, 0, 100, 1)),
    (2, 64, 1, -1.0, 40, 1, None),                # fold in 2D
])
def test_eval_grid_parity(gpu_lib, dim, nx, ny, depth, gx, gy, win, precision):
    from paper_2005_12716_amd import lib
    h, g, (er, pr, A, At, eth) = _state(lib, dim, nx, ny, depth, precision=precision)
    zl = np.array([-1.3, -0.6, -0.2, 0.0, 0.1, 0.35])
    gd = lib.grid_desc(gx, gy, zl, win)
    out = h.eval_grid(gd, lib.ALL_FIELDS).cpu().numpy()
    ix0, iy0, wx, wy = win if win is not None else (0, 0, gx, gy)
    ref = rc.eval_grid(g, A, At, er, eth, gx, gy, zl, list(range(11)), window=(ix0, iy0, wx, wy))
    nl = zl.size
    vol = out[: 9 * nl * wy * wx].reshape(9, nl, wy, wx)
    srf = out[9 * nl * wy * wx:].reshape(2, wy, wx)
    for f in range(9):
        r = ref[f]
        if np.linalg.norm(r) == 0:
            assert np.abs(vol[f]).max() == 0
            continue
        assert rel(vol[f], r) < 1e-5, (f, rel(vol[f], r))
    for k, f in enumerate([rc.ETA, rc.ETA_T]):
        assert rel(srf[k], ref[f]) < 1e-5
    h.close()


def test_eval_grid_subset_mask_layout(gpu_lib):
    from paper_2005_12716_amd import lib
    h, g, (er, pr, A, At, eth) = _state(lib, 3, 24, 12, -1.0)
    zl = np.array([-0.5, 0.0])
    gd = lib.grid_desc(48, 24, zl)
    mask = lib.W | lib.P | lib.ETA_T
    out = h.eval_grid(gd, mask).cpu().numpy()
    assert out.size == h.grid_size(gd, mask) == 2 * 2 * 24 * 48 + 24 * 48
    ref = rc.eval_grid(g, A, At, er, eth, 48, 24, zl, [rc.W, rc.P, rc.ETA_T])
    n = 2 * 24 * 48
    assert rel(out[:n].reshape(2, 24, 48), ref[rc.W]) < 1e-5
    assert rel(out[n:2 * n].reshape(2, 24, 48), ref[rc.P]) < 1e-5
    assert rel(out[2 * n:].reshape(24, 48), ref[rc.ETA_T]) < 1e-5
    h.close()


@pytest.mark.parametrize("dim,nx,ny,gx,gy,win", [
    (3, 32, 16, 64, 32, None),
    (3, 32, 16, 128, 64, (20, 10, 60, 40)),
    (2, 64, 1, 256, 1, None),
])
def test_interp_parity(gpu_lib, dim, nx, ny, gx, gy, win):
    from paper_2005_12716_amd import lib
    h, g, (er, pr, A, At, eth) = _state(lib, dim, nx, ny, 1.4)
    zl = np.linspace(-1.4, 0.3, 13)
    gd = lib.grid_desc(gx, gy, zl, win)
    rng = np.random.default_rng(1)
    n = 5000
    ix0, iy0, wx, wy = win if win is not None else (0, 0, gx, gy)
    dx, dy = g.lx / gx, (g.ly / gy if dim == 3 else 1.0)
    x = rng.uniform((ix0 + 1) * dx, (ix0 + wx - 2) * dx, n) if win else rng.uniform(0, g.lx, n)
    y = (rng.uniform((iy0 + 1) * dy, (iy0 + wy - 2) * dy, n) if win else rng.uniform(0, g.ly, n)) if dim == 3 else np.zeros(n)
    z = rng.uniform(-1.4, 0.3, n)
    pts = np.stack([x, y, z])
    cells = h.bind(gd, torch.tensor(pts, device="cuda"))
    out, nbad = cells.interp(lib.ALL_FIELDS)
    out = out.cpu().numpy()
    assert nbad == 0
    coef = rc.eval_grid(g, A, At, er, eth, gx, gy, zl, [f for f in range(11) if f != rc.P], prefilter=True,
                        window=(ix0, iy0, wx, wy))
    ref, nb = rc.interp_points(g, coef, zl, gx, gy, (ix0, iy0, wx, wy), pts, list(range(11)))
    assert nb == 0
    for f in range(11):
        if np.linalg.norm(ref[f]) == 0:
            assert np.abs(out[f]).max() == 0
            continue
        assert rel(out[f], ref[f]) < 1e-5, (f, rel(out[f], ref[f]))
    div = cells.divergence().cpu().numpy()
    dref = rc.divergence_of_interpolant(g, coef, zl, gx, gy, (ix0, iy0, wx, wy), pts)
    # the divergence is a small difference of O(k u) terms: compare on that scale
    scale = np.linalg.norm(out[1]) * 2 * math.pi / g.lx * (nx / 2)
    assert np.linalg.norm(div - dref) / scale < 1e-5
    cells.close()
    h.close()


@pytest.mark.parametrize("nx,ny,gx,gy", [(256, 256, 512, 768), (512, 256, 1536, 1024), (1024, 256, 2048, 512),
                                         # 2/3/5-smooth mode counts whose refined lengths have no
                                         # compile-time transform: runtime-plan residue y pass
                                         (192, 150, 384, 600), (160, 360, 320, 1080), (128, 480, 256, 960)])
def test_interp_residue_forms(gpu_lib, nx, ny, gx, gy):
    """Refinements of 2, 3 and 4 times the mode count: the evaluation's
    residue-form transforms (one wavefront per output residue of the refined
    grid; compile-time lengths at 256 to 1024 modes, runtime plans for the
    2/3/5-smooth counts), with 6 layers (below the skeleton threshold, so
    the plane x pass runs): all 11 fields at 4000 points of a window against
    the oracle."""
    from paper_2005_12716_amd import lib
    h, g, (er, pr, A, At, eth) = _state(lib, 3, nx, ny, -1.0, steps=2)
    zl = np.linspace(-1.0, 0.2, 6)
    win = (gx // 3, gy // 3, gx // 4, gy // 4)
    gd = lib.grid_desc(gx, gy, zl, win)
    ix0, iy0, wx, wy = win
    rng = np.random.default_rng(nx + gx)
    n = 4000
    dx, dy = g.lx / gx, g.ly / gy
    pts = np.stack([rng.uniform((ix0 + 1) * dx, (ix0 + wx - 2) * dx, n),
                    rng.uniform((iy0 + 1) * dy, (iy0 + wy - 2) * dy, n), rng.uniform(-1.0, 0.2, n)])
    cells = h.bind(gd, torch.tensor(pts, device="cuda"))
    out, nbad = cells.interp(lib.ALL_FIELDS)
    out = out.cpu().numpy()
    assert nbad == 0
    coef = rc.eval_grid(g, A, At, er, eth, gx, gy, zl, [f for f in range(11) if f != rc.P], prefilter=True,
                        window=win)
    ref, nb = rc.interp_points(g, coef, zl, gx, gy, win, pts, list(range(11)))
    assert nb == 0
    for f in range(11):
        assert rel(out[f], ref[f]) < 1e-5, (f, rel(out[f], ref[f]))
    cells.close()
    h.close()


def test_out_of_range_and_empty(gpu_lib):
    from paper_2005_12716_amd import lib
    h, g, _ = _state(lib, 3, 16, 8, -1.0)
    zl = np.linspace(-1.0, 0.0, 6)
    gd = lib.grid_desc(32, 16, zl, (4, 2, 16, 8))
    dx, dy = g.lx / 32, g.ly / 16
    pts = np.array([[8.5 * dx, 8.5 * dx, 4.5 * dx, 18.7 * dx, 8.5 * dx],
                    [5.5 * dy, 5.5 * dy, 5.5 * dy, 5.5 * dy, 2.2 * dy],
                    [-0.5, 0.2, -0.5, -0.5, -0.5]])
    cells = h.bind(gd, torch.tensor(pts, device="cuda"))
    out, nbad = cells.interp(lib.U | lib.ETA)
    out = out.cpu().numpy()
    assert nbad == 4
    assert np.isfinite(out[:, 0]).all() and np.isnan(out[:, 1:]).all()
    cells.close()
    empty = h.bind(gd, torch.zeros((3, 0), dtype=torch.float64, device="cuda"))
    o, nb = empty.interp(lib.U)
    assert o.numel() == 0 and nb == 0
    empty.close()
    h.close()


def test_cylinder_cloud_sampled_parity(gpu_lib):
    """The 2M-point cylinder cloud on the 512 x 256 sea: every field at a
    seeded sample of 2000 points against the oracle's interpolation of its
    own coefficient grids (window 4 x 4 peak wavelengths, n = 4, 48 layers)."""
    from paper_2005_12716_amd import lib
    nx, ny = 512, 256
    lx, ly = 40 * LAM, 20 * LAM
    hs = 0.02 * LAM
    d = lib.hos_desc(3, nx, ny, lx, ly, -1.0, order_m=3, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=hs, kp=1.0, gamma=3.3, phases=synth.mode_phases(1, ny, nx // 2 + 1))
    h = lib.Hos(d, eh, ph)
    pts = synth.cylinder_cloud(lx, ly, hs)
    gx, gy = 4 * nx, 4 * ny
    dx = lx / gx
    ix0 = int(math.floor((lx / 2 - 2.05 * LAM) / dx)) - 2
    wx = int(math.ceil(4.1 * LAM / dx)) + 6
    iy0 = int(math.floor((ly / 2 - 2.05 * LAM) / dx)) - 2
    wy = wx
    zl = synth.clustered_layers(pts[2].min() - 1e-9, pts[2].max() + 1e-9, 48, hs / 16)
    gd = lib.grid_desc(gx, gy, zl, (ix0, iy0, wx, wy))
    cells = h.bind(gd, torch.tensor(pts, device="cuda"))
    out, nbad = cells.interp(lib.ALL_FIELDS)
    assert nbad == 0
    sel = np.sort(np.random.default_rng(0).choice(pts.shape[1], 2000, replace=False))
    out = out[:, torch.tensor(sel, device="cuda")].cpu().numpy()
    g = Grid(nx=nx, ny=ny, lx=lx, ly=ly, depth=-1.0, order_m=3)
    A = hos.mean_level_modes(g, eh, ph)
    At, eth = hos.mean_level_modes_t(g, eh, ph)
    coef = rc.eval_grid(g, A, At, eh, eth, gx, gy, zl, [f for f in range(11) if f != rc.P], prefilter=True,
                        window=(ix0, iy0, wx, wy))
    ref, nb = rc.interp_points(g, coef, zl, gx, gy, (ix0, iy0, wx, wy), pts[:, sel], list(range(11)))
    assert nb == 0
    for f in range(11):
        if f in (rc.V, rc.V_T, rc.U, rc.U_T, rc.W, rc.W_T, rc.PHI, rc.PHI_T, rc.ETA, rc.ETA_T, rc.P):
            assert rel(out[f], ref[f]) < 1e-5, (f, rel(out[f], ref[f]))
    cells.close()
    h.close()


def test_interp_step_equals_interp_then_step(gpu_lib):
    """The concurrent interpolate-and-advance call gives the fields of the
    state at its start and the advanced state, bit for bit as the two calls
    made one after the other; repeated calls keep doing so."""
    import torch
    from paper_2005_12716_amd import lib
    lam = 2 * math.pi
    nx, ny = 64, 32
    d = lib.hos_desc(3, nx, ny, nx * lam / 6.4, ny * lam / 6.4, -1.0, order_m=3, dt=lam / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=0.03 * lam, kp=1.0, gamma=3.3,
                              phases=synth.mode_phases(12, ny, nx // 2 + 1))
    pts = synth.box_cloud(5, 4000, 1.0, 1.0, d.lx - 2.0, d.ly - 2.0, -1.0, 0.2)
    gd = lib.grid_desc(2 * nx, 2 * ny, np.linspace(-1.05, 0.25, 12))
    a, b = lib.Hos(d, eh, ph), lib.Hos(d, eh, ph)
    ca = a.bind(gd, torch.tensor(pts, device="cuda"))
    cb = b.bind(gd, torch.tensor(pts, device="cuda"))
    mask = lib.ALL_FIELDS
    for _ in range(3):
        oa = ca.interp_step(mask, nsteps=2)
        ob, _ = cb.interp(mask)
        b.step(2)
        torch.cuda.synchronize()
        assert torch.equal(oa, ob)
        sa, sb = a.state(), b.state()
        assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1]) and sa[2] == sb[2]
    for o in (ca, cb, a, b):
        o.close()
