"""Caller-owned device workspaces through the C ABI: a realisation and a
bound cloud whose every device buffer the caller allocated (torch uint8
buffers sized by the workspace queries) give bit for bit the results of
library-allocated handles, their interpolation calls take no device memory,
and too-small workspaces or larger field masks are refused with ENOMEM.  A
batch graph captured before a member's buffers grew is captured again
rather than writing to the freed ones."""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
LAM = 2 * math.pi


def _setup(lib, nx=96, ny=48):
    d = lib.hos_desc(3, nx, ny, nx * LAM / 12.8, ny * LAM / 12.8, -1.0, order_m=3, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=0.02 * LAM, kp=1.0, gamma=3.3,
                              phases=synth.mode_phases(31, ny, nx // 2 + 1))
    x0, y0 = d.lx / 2 - 1.2 * LAM, d.ly / 2 - LAM
    pts = synth.box_cloud(8, 40000, x0, y0, 2.4 * LAM, 2 * LAM, -0.4 * LAM, 0.05 * LAM)
    gx, gy = 4 * nx, 4 * ny
    dx, dy = d.lx / gx, d.ly / gy
    win = (int(math.floor(x0 / dx)) - 2, int(math.floor(y0 / dy)) - 2, int(math.ceil(2.4 * LAM / dx)) + 6,
           int(math.ceil(2 * LAM / dy)) + 6)
    zl = synth.clustered_layers(-0.4 * LAM - 1e-9, 0.05 * LAM + 1e-9, 20, 0.01 * LAM)
    return d, eh, ph, pts, lib.grid_desc(gx, gy, zl, win)


def test_caller_workspaces_match_and_allocate_nothing(gpu_lib):
    from paper_2005_12716_amd import lib
    d, eh, ph, pts, gd = _setup(lib)
    ref = lib.Hos(d, eh, ph)
    wsh = torch.empty(lib.hos_workspace_bytes(d), dtype=torch.uint8, device="cuda")
    h = lib.Hos(d, eh, ph, workspace=wsh)
    xyz = torch.tensor(pts, device="cuda")
    mask = lib.U | lib.W | lib.P | lib.ETA
    cref = ref.bind(gd, xyz)
    wsc = torch.empty(h.cells_workspace_bytes(gd, pts.shape[1], mask), dtype=torch.uint8, device="cuda")
    c = h.bind(gd, xyz, workspace=wsc, ws_mask=mask)
    out = torch.empty((4, pts.shape[1]), dtype=torch.float32, device="cuda")
    for it in range(3):
        ref.step(2)
        h.step(2)
        a, _ = cref.interp(mask)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        _, nb = c.interp(mask, out)
        h.step(1)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0, it  # nothing allocated by the calls
        ref.step(1)
        assert nb == 0
        assert torch.equal(out, a), float((out - a).abs().max())
    e1, p1, t1 = h.state()
    e0, p0, t0 = ref.state()
    assert np.array_equal(e1, e0) and np.array_equal(p1, p0) and t1 == t0
    # concurrent interpolation + step on the caller's workspaces
    a = cref.interp_step(mask, nsteps=1)
    b = c.interp_step(mask, nsteps=1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # a mask needing more coefficient fields than the workspace holds
    with pytest.raises(lib.SwenseError) as ei:
        c.interp(lib.ALL_FIELDS)
    assert ei.value.code == lib.ENOMEM
    c.close()
    cref.close()
    h.close()
    ref.close()


def test_too_small_cells_workspace(gpu_lib):
    from paper_2005_12716_amd import lib
    d, eh, ph, pts, gd = _setup(lib, 64, 32)
    h = lib.Hos(d, eh, ph)
    n = pts.shape[1]
    need = h.cells_workspace_bytes(gd, n, lib.U)
    assert need < h.cells_workspace_bytes(gd, n, lib.ALL_FIELDS)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(lib.SwenseError) as ei:
        h.bind(gd, torch.tensor(pts, device="cuda"), workspace=small, ws_mask=lib.U)
    assert ei.value.code == lib.ENOMEM
    with pytest.raises(lib.SwenseError) as ei:
        lib.Hos(d, eh, ph, workspace=torch.empty(lib.hos_workspace_bytes(d) - 256, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == lib.ENOMEM
    h.close()


def test_batch_recaptures_after_buffers_grow(gpu_lib):
    """A member's interpolation with a larger mask (a larger coefficient grid
    and more evaluation rows) between two launches reallocates buffers the
    captured graph writes; the next launch captures again and still matches
    the realisations stepped and interpolated one by one."""
    from paper_2005_12716_amd import lib
    mask = lib.U
    items = []
    for i, (nx, ny) in enumerate([(64, 32), (80, 40)]):
        d, eh, ph, pts, gd = _setup(lib, nx, ny)
        h = lib.Hos(d, eh, ph)
        c = h.bind(gd, torch.tensor(pts, device="cuda"))
        out = torch.zeros((1, pts.shape[1]), dtype=torch.float32, device="cuda")
        solo = lib.Hos(d, eh, ph)
        cs = solo.bind(gd, torch.tensor(pts, device="cuda"))
        items.append((h, c, out, solo, cs))
    b = lib.Batch([it[0] for it in items], [it[1] for it in items], [mask] * 2, [it[2] for it in items], nsteps=1)
    b.run()
    for it in items:
        it[3].step(1)
    # grow every member's buffers outside the graph
    for it in items:
        big, _ = it[1].interp(lib.ALL_FIELDS)
    torch.cuda.synchronize()
    for _ in range(2):
        b.run()
        for it in items:
            it[3].step(1)
    torch.cuda.synchronize()
    for h, c, out, solo, cs in items:
        ref, _ = cs.interp(mask)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), float((out - ref).abs().max())
    b.close()
    for h, c, out, solo, cs in items:
        cs.close()
        solo.close()
        c.close()
        h.close()
