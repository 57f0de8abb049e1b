"""Batched realisations of uneven size in one graph launch: every
realisation must end exactly where stepping it alone ends (same kernels in
the same order per realisation), for several launches in a row, for every
autotuned branch count, and it must agree with the FP64 oracle."""
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import Grid, hos

pytestmark = pytest.mark.gpu
LAM = 2 * math.pi
SIZES = [(32, 16), (48, 24), (40, 20), (30, 18), (64, 32)]


def _make(lib, nx, ny, seed, npts=3000):
    lx, ly = nx * LAM / 6.4, ny * LAM / 6.4
    d = lib.hos_desc(3, nx, ny, lx, ly, -1.0, order_m=3, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=0.025 * LAM, kp=1.0, gamma=3.3,
                              phases=synth.mode_phases(seed, ny, nx // 2 + 1))
    pts = synth.box_cloud(seed, npts, 0.0, 0.0, lx, ly, -1.0, 0.2)
    zl = np.linspace(-1.05, 0.25, 10)
    gd = lib.grid_desc(2 * nx, 2 * ny, zl)
    return d, eh, ph, pts, gd


def _build(lib, with_cells=True):
    items = []
    for i, (nx, ny) in enumerate(SIZES):
        d, eh, ph, pts, gd = _make(lib, nx, ny, 40 + i)
        h = lib.Hos(d, eh, ph)
        c = h.bind(gd, torch.tensor(pts, device="cuda")) if with_cells else None
        out = torch.zeros((3, pts.shape[1]), dtype=torch.float32, device="cuda") if with_cells else None
        items.append((d, eh, ph, h, c, out, gd, pts))
    return items


def test_batch_matches_individual_runs(gpu_lib):
    from paper_2005_12716_amd import lib
    mask = lib.U | lib.W | lib.P
    items = _build(lib)
    b = lib.Batch([it[3] for it in items], [it[4] for it in items], [mask] * len(items),
                  [it[5] for it in items], nsteps=2)
    for _ in range(3):
        b.run()
    torch.cuda.synchronize()
    for (d, eh, ph, h, c, out, gd, pts) in items:
        e_b, p_b, t_b = h.state()
        ref = lib.Hos(d, eh, ph)
        ref.step(6)
        e_r, p_r, t_r = ref.state()
        assert np.array_equal(e_b, e_r) and np.array_equal(p_b, p_r)
        assert abs(t_b - t_r) < 1e-12
        rc = ref.bind(gd, torch.tensor(pts, device="cuda"))
        o_r, _ = rc.interp(mask)
        assert torch.equal(out, o_r)
        g = Grid(nx=d.nx, ny=d.ny, lx=d.lx, ly=d.ly, depth=-1.0, order_m=3, dealias=d.dealias)
        er, pr = hos.run(g, eh, ph, d.dt, 6)
        assert np.linalg.norm(e_b - er) / np.linalg.norm(er) < 1e-6
        rc.close()
        ref.close()
    b.close()
    for it in items:
        it[4].close()
        it[3].close()


def test_batch_autotune_and_cache(gpu_lib, tmp_path):
    from paper_2005_12716_amd import lib
    items = _build(lib, with_cells=False)
    b = lib.Batch([it[3] for it in items], nsteps=1)
    cache = str(tmp_path / "tune.json")
    k, ms = b.autotune(cache)
    assert k in (1, 2, 4) and ms > 0
    assert os.path.exists(cache) and "batch" in open(cache).read()
    k2, ms2 = b.autotune(cache)
    assert k2 == k and ms2 == -1.0
    # autotuning leaves the states untouched
    for (d, eh, ph, h, *_rest) in items:
        e, p, t = h.state()
        assert np.array_equal(e, eh)
        assert t == 0.0
    b.run()
    torch.cuda.synchronize()
    for (d, eh, ph, h, *_rest) in items:
        ref = lib.Hos(d, eh, ph)
        ref.step(1)
        assert np.array_equal(h.state()[0], ref.state()[0])
        ref.close()
    b.close()
    for it in items:
        it[3].close()


def test_batched_configuration_recipe_sampled(gpu_lib):
    """The 64-realisation batched recipe (mode grids over the even 5-smooth
    sizes in [128, 512], Hs/lambda_p in [0.01, 0.03], n = 4 windows, 32
    layers) with the point counts scaled down and the product-grid policy of
    each size chosen by the padding tuner, as the bench runs it: one graph
    launch of one step each, sampled against the oracle on each
    realisation's own product grid (states of 6 realisations, fields of the 2
    smallest and the 2 largest at 300 points each)."""
    import bench
    from oracle import reconstruct as rc
    from paper_2005_12716_amd import lib
    hoses, cells, outs, npts, mask, nf = bench.batched_setup(lib, torch, pts_scale=0.01, padding="tune")
    assert len(hoses) == 64
    inits = [h.state() for h in hoses]
    b = lib.Batch(hoses, cells, [mask] * 64, outs, nsteps=1)
    b.run()
    torch.cuda.synchronize()
    sizes = [(h.desc.nx * h.desc.ny, i) for i, h in enumerate(hoses)]
    check = [i for _, i in sorted(sizes)[:4]] + [i for _, i in sorted(sizes)[-2:]]
    for i in check:
        h = hoses[i]
        d = h.desc
        g = Grid(nx=d.nx, ny=d.ny, lx=d.lx, ly=d.ly, depth=-1.0, order_m=3, dealias=d.dealias)
        er, pr = hos.run(g, inits[i][0], inits[i][1], d.dt, 1)
        e, p, _ = h.state()
        assert np.linalg.norm(e - er) / np.linalg.norm(er) < 1e-6
    for i in check[:2] + check[-2:]:
        h, c, out = hoses[i], cells[i], outs[i].cpu().numpy()
        d = h.desc
        g = Grid(nx=d.nx, ny=d.ny, lx=d.lx, ly=d.ly, depth=-1.0, order_m=3, dealias=d.dealias)
        e, p, _ = h.state()
        A = hos.mean_level_modes(g, e, p)
        At, eth = hos.mean_level_modes_t(g, e, p)
        gd = c.gd
        zl = np.ctypeslib.as_array(gd.z, shape=(gd.nl,)).copy()
        win = (gd.ix0, gd.iy0, gd.wx, gd.wy)
        coef = rc.eval_grid(g, A, At, e, eth, gd.gx, gd.gy, zl, [f for f in range(11) if f != rc.P],
                            prefilter=True, window=win)
        pts = c.xyz_host
        sel = np.arange(0, pts.shape[1], max(1, pts.shape[1] // 300))
        ref, nb = rc.interp_points(g, coef, zl, gd.gx, gd.gy, win, pts[:, sel], list(range(11)))
        assert nb == 0
        errs = [float(np.linalg.norm(out[f, sel] - ref[f]) / np.linalg.norm(ref[f])) for f in range(11)]
        print(f"realisation {i} ({d.nx} x {d.ny}): largest field error {max(errs):.2e}")
        for f in range(11):
            assert errs[f] <= 1e-5, (f, errs[f])
    b.close()
    for c in cells:
        c.close()
    for h in hoses:
        h.close()
