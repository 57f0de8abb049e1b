"""The allocation-free interpolation entry point (swense_interp_cells_noalloc)
against swense_interp_cells through the C ABI: the same kernels, so the
outputs must agree bit for bit.  Two calls in a row on one GPU, the second
with a smaller input (fewer points, a narrower window, fewer layers, a
structured cloud instead of a random one); no device memory is taken by
the calls; an input beyond the fixed scratch is rejected before any launch."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

LAM = 2 * math.pi


def _sea(lib, nx=128, ny=64):
    d = lib.hos_desc(3, nx, ny, nx * LAM / 12.8, ny * LAM / 12.8, -1.0, order_m=3, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=0.02 * LAM, kp=1.0, gamma=3.3,
                              phases=synth.mode_phases(21, ny, nx // 2 + 1))
    h = lib.Hos(d, eh, ph)
    h.step(3)
    return d, h


def test_noalloc_matches_interp_cells(gpu_lib):
    import torch
    from paper_2005_12716_amd import lib
    d, h = _sea(lib)
    gx, gy = 4 * d.nx, 4 * d.ny
    # first input: 60k random points in a 3 x 2 lambda box, 24 layers (tiled gather)
    x0, y0 = d.lx / 2 - 1.5 * LAM, d.ly / 2 - LAM
    p1 = synth.box_cloud(5, 60000, x0, y0, 3 * LAM, 2 * LAM, -0.4 * LAM, 0.05 * LAM)
    dx, dy = d.lx / gx, d.ly / gy
    w1 = (int(math.floor(x0 / dx)) - 2, int(math.floor(y0 / dy)) - 2, int(math.ceil(3 * LAM / dx)) + 6,
          int(math.ceil(2 * LAM / dy)) + 6)
    z1 = synth.clustered_layers(-0.4 * LAM - 1e-9, 0.05 * LAM + 1e-9, 24, 0.01 * LAM)
    c1 = h.bind(lib.grid_desc(gx, gy, z1, w1), torch.tensor(p1, device="cuda"))
    # second input, smaller: a structured 40 x 30 x 12 cloud (shared columns), 12 layers
    xs = x0 + LAM * (np.arange(40) + 0.5) / 40
    ys = y0 + 0.5 * LAM * (np.arange(30) + 0.5) / 30
    zs = np.linspace(-0.3 * LAM, 0.0, 12)
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    p2 = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    w2 = (int(math.floor(x0 / dx)) - 2, int(math.floor(y0 / dy)) - 2, int(math.ceil(LAM / dx)) + 6,
          int(math.ceil(0.5 * LAM / dy)) + 6)
    z2 = np.linspace(-0.32 * LAM, 0.02 * LAM, 12)
    c2 = h.bind(lib.grid_desc(gx, gy, z2, w2), torch.tensor(p2, device="cuda"))
    mask = lib.ALL_FIELDS
    ref1, nb1 = c1.interp(mask)
    ref2, nb2 = c2.interp(mask)
    assert nb1 == 0 and nb2 == 0
    out1 = torch.full_like(ref1, float("nan"))
    out2 = torch.full_like(ref2, float("nan"))
    assert torch.equal(ref1, ref1) and torch.equal(ref2, ref2)  # torch's own work buffers, before the count
    for _ in range(2):  # twice, so that the second pair finds the first's contents in the scratch
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        _, n1 = c1.interp_noalloc(mask, out1)
        _, n2 = c2.interp_noalloc(mask, out2)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0  # no device memory taken by the calls
        assert n1 == 0 and n2 == 0
        assert torch.equal(out1, ref1), float((out1 - ref1).abs().max())
        assert torch.equal(out2, ref2), float((out2 - ref2).abs().max())
        out1.fill_(float("nan"))
        out2.fill_(float("nan"))
    # a later state: both entry points again, noalloc first this time
    h.step(2)
    a2, _ = c2.interp_noalloc(mask)
    b2, _ = c2.interp(mask)
    assert torch.equal(a2, b2)
    c1.close()
    c2.close()
    h.close()


def test_noalloc_rejects_oversized_scratch(gpu_lib):
    import torch
    from paper_2005_12716_amd import lib
    d, h = _sea(lib)
    gx, gy = 8 * d.nx, 8 * d.ny
    zl = np.linspace(-0.5 * LAM, 0.1 * LAM, 80)  # 80 layers on the whole 1024 x 512 grid: > 128 MiB
    pts = synth.box_cloud(6, 1000, 1.0, 1.0, d.lx - 2.0, d.ly - 2.0, -0.4 * LAM, 0.05 * LAM)
    c = h.bind(lib.grid_desc(gx, gy, zl), torch.tensor(pts, device="cuda"))
    with pytest.raises(lib.SwenseError) as ei:
        c.interp_noalloc(lib.ALL_FIELDS)
    assert ei.value.code == lib.ENOMEM
    # the handle still works, through either entry point, for a smaller mask
    out, nb = c.interp(lib.ETA)
    assert nb == 0 and bool(torch.isfinite(out).all())
    c.close()
    h.close()
