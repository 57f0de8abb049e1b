"""GPU cell-side use of the incident fields (incident volume fraction,
modified incident pressure, relaxation blending; Sec. 3.2.2, 2.1.3, 4.2)
against the oracle on the same seeded FP32 inputs: element by element
within one FP32 rounding, over a ragged count of a million cells with the
edge cases (interface on a face, cells fully wet or dry, zone coordinates
outside [0, 1]); then on the metric's cylinder cloud with the interpolated
elevation."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cells as oc

pytestmark = pytest.mark.gpu
LAM = 2 * math.pi
N = 1_000_003


def _hos(lib, nx=32, ny=16, rho=1000.0):
    d = lib.hos_desc(3, nx, ny, nx * LAM / 6.4, ny * LAM / 6.4, -1.0, order_m=3, dt=LAM / 64, rho=rho)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=0.02 * LAM, kp=1.0, gamma=3.3, phases=synth.mode_phases(2, ny, nx // 2 + 1))
    return lib.Hos(d, eh, ph)


def _inputs(seed):
    rng = np.random.default_rng(seed)
    zc = rng.uniform(-1.0, 1.0, N)
    dz = rng.uniform(0.005, 0.2, N).astype(np.float32)
    eta = rng.uniform(-0.3, 0.3, N).astype(np.float32)
    # interface exactly on the bottom face, the top face and the centre
    eta[:3] = [0.0, 0.0, 0.0]
    zc[:3] = [float(dz[0]) / 2, -float(dz[1]) / 2, 0.0]
    return eta, zc, dz


def _d(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def test_alpha_matches_oracle(gpu_lib):
    from paper_2005_12716_amd import lib
    h = _hos(lib)
    eta, zc, dz = _inputs(1)
    got = h.cells_alpha(_d(eta), _d(zc), _d(dz)).cpu().numpy()
    ref = oc.incident_alpha(eta, zc, dz)
    assert np.abs(got - ref).max() <= 6e-8
    assert got[0] == 0.0 and got[1] == 1.0 and got[2] == 0.5
    assert (got == 0).any() and (got == 1).any() and ((got > 0) & (got < 1)).any()
    h.close()


def test_pstar_matches_oracle(gpu_lib):
    from paper_2005_12716_amd import lib
    h = _hos(lib, rho=1000.0)
    rng = np.random.default_rng(2)
    p = rng.uniform(-5e3, 2e4, N).astype(np.float32)
    a = rng.uniform(0, 1, N).astype(np.float32)
    a[:2] = [0.0, 1.0]
    got = h.cells_pstar(_d(p), _d(a), 1.2).cpu().numpy()
    ref = oc.pstar(p, a, 1000.0, 1.2)
    assert np.all(np.abs(got - ref) <= 1.2e-7 * np.abs(ref) + 1e-30)
    assert got[1] == p[1]
    # in place
    pd = _d(p)
    h.cells_pstar(pd, _d(a), 1.2, out=pd)
    assert np.array_equal(pd.cpu().numpy(), got)
    h.close()


@pytest.mark.parametrize("ncomp,with_alpha", [(3, True), (2, True), (3, False), (0, True)])
def test_relax_matches_oracle(gpu_lib, ncomp, with_alpha):
    from paper_2005_12716_amd import lib
    h = _hos(lib)
    rng = np.random.default_rng(3 + ncomp)
    x = rng.uniform(-0.5, 1.5, N).astype(np.float32)
    x[:4] = [0.0, 1.0, 0.5, -1.0]
    ai = rng.uniform(0, 1, N).astype(np.float32)
    ac = rng.uniform(0, 1, N).astype(np.float32)
    uc = rng.standard_normal((max(ncomp, 1), N)).astype(np.float32)[:ncomp]
    ad, ucd = _d(ac), (_d(uc) if ncomp else None)
    h.cells_relax(_d(x), _d(ai) if with_alpha else None, ad if with_alpha else None, ucd)
    ra, ru = oc.relax(x, ai, ac, uc if ncomp else np.zeros((1, N)))
    if with_alpha:
        got = ad.cpu().numpy()
        assert np.abs(got - ra).max() <= 6e-8
        assert got[0] == ac[0] and got[3] == ac[3] and got[1] == ai[1]
    else:
        assert np.array_equal(ad.cpu().numpy(), ac)
    if ncomp:
        gu = ucd.cpu().numpy()
        # one FP32 rounding, plus the FP64 rounding of omega: near x = 1 the
        # factor 1 - omega is a cancellation, so an ulp of omega (contracted
        # or not) shifts it by ~1e-16 absolute
        assert np.all(np.abs(gu - ru) <= 6e-8 * np.abs(ru) + 1e-15 * np.abs(uc))
        assert np.array_equal(gu[:, 0], uc[:, 0]) and np.all(gu[:, 1] == 0)
    h.close()


def test_empty_and_bad_arguments(gpu_lib):
    from paper_2005_12716_amd import lib
    h = _hos(lib)
    e = torch.zeros(0, dtype=torch.float32, device="cuda")
    assert h.cells_alpha(e, torch.zeros(0, dtype=torch.float64, device="cuda"), e).numel() == 0
    x = torch.zeros(4, dtype=torch.float32, device="cuda")
    rc = h.L.swense_cells_relax(h.h, 4, 4, x.data_ptr(), None, None, x.data_ptr())
    assert rc != lib.OK
    h.close()


def test_cylinder_cloud_alpha_from_interpolated_eta(gpu_lib):
    """The metric's workload: eta interpolated at the 1,996,800 cell centres,
    the cells' heights from the mesh's z-levels; alpha against the oracle on
    those same eta values, and wet below the troughs, dry above the crests."""
    from paper_2005_12716_amd import lib
    nx, ny = 512, 256
    lx, ly = 40 * LAM, 20 * LAM
    hs = 0.02 * LAM
    d = lib.hos_desc(3, nx, ny, lx, ly, -1.0, order_m=3, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=hs, kp=1.0, gamma=3.3, phases=synth.mode_phases(1, ny, nx // 2 + 1))
    h = lib.Hos(d, eh, ph)
    pts = synth.cylinder_cloud(lx, ly, hs)
    ze = synth.cylinder_z_edges(hs, LAM)
    dzc = np.diff(ze).astype(np.float32)
    dz = np.tile(dzc, pts.shape[1] // dzc.size)
    gx, gy = 4 * nx, 4 * ny
    dx = lx / gx
    ix0 = int(math.floor((lx / 2 - 2.05 * LAM) / dx)) - 2
    wx = int(math.ceil(4.1 * LAM / dx)) + 6
    iy0 = int(math.floor((ly / 2 - 2.05 * LAM) / dx)) - 2
    zl = synth.clustered_layers(pts[2].min() - 1e-9, pts[2].max() + 1e-9, 48, hs / 16)
    gd = lib.grid_desc(gx, gy, zl, (ix0, iy0, wx, wx))
    xyz = torch.tensor(pts, device="cuda")
    cells = h.bind(gd, xyz)
    eta, _ = cells.interp(lib.ETA)
    eta = eta[0].contiguous()
    a = h.cells_alpha(eta, xyz[2].contiguous(), _d(dz)).cpu().numpy()
    e = eta.cpu().numpy()
    ref = oc.incident_alpha(e, pts[2], dz)
    assert np.abs(a - ref).max() <= 6e-8
    assert np.all(a[pts[2] + dz / 2 < e.min()] == 1.0) and np.all(a[pts[2] - dz / 2 > e.max()] == 0.0)
    cells.close()
    h.close()
