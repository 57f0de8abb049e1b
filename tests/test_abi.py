"""Host-side checks of the C ABI: the library loads, exports every function
include/*.h declare, and its host set-up routine (initial sea
spectra, no GPU involved) matches the oracle."""
import math
import os
import re

import numpy as np
import pytest

import synth
from oracle import Grid, sea

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    import glob
    txt = "".join(open(p).read() for p in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(swense_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["swense_hos_init", "swense_hos_step", "swense_eval_grid", "swense_cells_bind", "swense_interp_cells"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2005_12716_amd import lib
    L = lib.load()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) <= set(lib.EXPORTED) | {"swense_version"}
    assert L.swense_version().startswith(b"swense")


@pytest.mark.parametrize("dim,nx,ny,spread", [(3, 32, 16, 0), (3, 24, 20, 1), (2, 64, 1, 0)])
def test_sea_spectrum_matches_oracle_jonswap(dim, nx, ny, spread):
    from paper_2005_12716_amd import lib
    lam = 2 * math.pi
    lx, ly = nx * lam / 6.4, (ny * lam / 6.4 if ny > 1 else 1.0)
    d = lib.hos_desc(dim, nx, ny, lx, ly, -1.0)
    phases = synth.mode_phases(3, ny, nx // 2 + 1)
    e, p = lib.sea_spectrum(d, kind=0, hs=0.02 * lam, kp=1.0, gamma=3.3, spreading=spread, phases=phases)
    g = Grid(nx=nx, ny=ny, lx=lx, ly=ly, depth=-1.0)
    er, pr = sea.jonswap(g, 0.02 * lam, 1.0, 3.3, phases, "cos2" if spread == 0 else "uni")
    assert np.abs(e - er).max() <= 1e-13 * np.abs(er).max()
    assert np.abs(p - pr).max() <= 1e-13 * np.abs(pr).max()


@pytest.mark.parametrize("depth", [2.0, -1.0])
def test_sea_spectrum_matches_oracle_stokes(depth):
    from paper_2005_12716_amd import lib
    lam = 2 * math.pi
    d = lib.hos_desc(2, 256, 1, 4 * lam, 1.0, depth)
    e, p = lib.sea_spectrum(d, kind=1, mode=4, ka=0.1)
    g = Grid(nx=256, ny=1, lx=4 * lam, ly=1.0, depth=depth)
    er, pr, _ = sea.stokes2(g, 4, 0.1)
    assert np.abs(e - er).max() < 1e-16 and np.abs(p - pr).max() < 1e-15


def test_bad_descriptors_are_rejected_without_gpu_work():
    from paper_2005_12716_amd import lib
    d = lib.hos_desc(2, 63, 1, 1.0, 1.0, -1.0)
    with pytest.raises(lib.SwenseError):
        lib.sea_spectrum(d, kind=1, mode=4, ka=0.1)


@pytest.mark.parametrize("in_channels", [2, 4])
def test_network_parameter_packing_matches_the_library(in_channels):
    """The packed parameter vector of the binding has the length the library
    expects (host-only call), and unpacking inverts packing (FP32 values)."""
    from oracle import fno as F
    from paper_2005_12716_amd import lib
    cfg = F.FnoConfig(n=64, channels=6, layers=3, p_modes=5, q_modes=4, hidden=10, in_channels=in_channels)
    desc = lib.fno_desc(cfg.n, cfg.channels, cfg.layers, cfg.p_modes, cfg.q_modes, cfg.hidden, max_batch=2,
                        in_channels=in_channels)
    P = F.init_params(cfg, np.random.default_rng(0))
    vec = lib.fno_pack(desc, P)
    assert vec.size == lib.load().swense_fno_param_count(lib.C.byref(desc))
    Q = lib.fno_unpack(desc, vec)
    for k in P:
        ref = P[k].astype(np.complex64) if np.iscomplexobj(P[k]) else P[k].astype(np.float32)
        assert np.array_equal(Q[k], ref.astype(Q[k].dtype)), k


def test_invalid_descriptors_are_rejected_before_any_device_work():
    """Argument checks of the ABI run on the host first: bad descriptors give
    SWENSE_EINVAL (no GPU needed to reach them)."""
    import ctypes as C
    from paper_2005_12716_amd import lib
    L = lib.load()
    eh = np.zeros((16, 17), dtype=np.complex128)
    bad = [lib.hos_desc(3, 31, 16, 1.0, 1.0, -1.0),          # odd nx
           lib.hos_desc(3, 32, 16, 1.0, 1.0, -1.0, order_m=0),  # order 0
           lib.hos_desc(3, 32, 16, -1.0, 1.0, -1.0),         # negative length
           lib.hos_desc(2, 32, 4, 1.0, 1.0, -1.0),           # 2D with ny > 1
           lib.hos_desc(3, 32, 16, 1.0, 1.0, -1.0, precision=2),
           lib.hos_desc(3, 32, 16, 1.0, 1.0, -1.0, dealias=3)]
    for d in bad:
        h = C.c_void_p()
        rc = L.swense_hos_init(C.byref(d), eh.ctypes.data_as(C.c_void_p), eh.ctypes.data_as(C.c_void_p), lib.SPECTRAL,
                               None, C.byref(h))
        assert rc == lib.EINVAL and not h.value
    for fd in [lib.fno_desc(n=96), lib.fno_desc(channels=7), lib.fno_desc(p_modes=200), lib.fno_desc(q_modes=100),
               lib.fno_desc(max_batch=0), lib.fno_desc(in_channels=0)]:
        f = C.c_void_p()
        params = np.zeros(8, dtype=np.float32)
        assert L.swense_fno_create(C.byref(fd), params.ctypes.data_as(C.c_void_p), None, C.byref(f)) == lib.EINVAL
        assert not f.value
    assert L.swense_surrogate_create(None, None, None, C.byref(C.c_void_p())) == lib.EINVAL
    assert L.swense_hos_step(None, 1) == lib.EINVAL
    best, ms = C.c_int(-5), np.zeros(2)
    for d, n in [(bad[0], 3), (lib.hos_desc(3, 32, 16, 1.0, 1.0, -1.0, dealias=0), 3),
                 (lib.hos_desc(3, 32, 16, 1.0, 1.0, -1.0), 0)]:
        assert L.swense_hos_tune_padding(C.byref(d), n, None, C.byref(best), ms.ctypes.data_as(C.POINTER(C.c_double))) == lib.EINVAL
    assert L.swense_gemm_bf16(0, 4, 4, None, None, None, None) == lib.EINVAL


@pytest.mark.parametrize("depth,height,n", [(2.0, 0.2, 16), (1.0, 0.25, 12), (10.0, 0.5, 20)])
def test_stream_solve_matches_oracle(depth, height, n):
    """The library's host solve of the stream-function wave (its own Newton
    iteration) against the oracle's, same collocation system."""
    from paper_2005_12716_amd import lib
    from oracle import stream
    L = 2 * math.pi
    _, sol = lib.stream_solve(depth, height, L, n)
    ref = stream.solve(depth, height, L, n)
    v = np.concatenate([ref["eta"], ref["B"], [ref["c"], ref["Q"], ref["R"]]])
    assert np.abs(sol - v).max() < 1e-11 * max(1.0, np.abs(v).max())


def _oracle_stream_si(depth, height, wavelength, n, g):
    """The oracle's solve of the same wave in nondimensional form (g = k = 1)
    and its unknowns taken back to the wave's own units by dimensional
    analysis (lengths / k, velocities x sqrt(g/k))."""
    from oracle import stream
    k = 2 * math.pi / wavelength
    vs = math.sqrt(g / k)
    nd = stream.solve(k * depth, k * height, 2 * math.pi, n, g=1.0)
    return {"eta": nd["eta"] / k, "B": nd["B"], "c": nd["c"] * vs, "Q": nd["Q"] * vs / k, "R": nd["R"] * vs * vs,
            "k": k, "d": depth, "N": n, "g": g}


@pytest.mark.parametrize("depth,height,wavelength,n", [(50.0, 4.0, 150.0, 16), (200.0, 8.0, 300.0, 16),
                                                      (500.0, 30.0, 1000.0, 20), (20.0, 2.0, 100.0, 12)])
def test_stream_solve_full_scale_si(depth, height, wavelength, n):
    """Ocean-scale waves in SI units (g = 9.81): the host solve converges and
    its unknowns equal the oracle's nondimensional solution taken back to SI
    units, each block to 1e-11 of its own scale."""
    from paper_2005_12716_amd import lib
    _, sol = lib.stream_solve(depth, height, wavelength, n, g=9.81, rho=1025.0)
    ref = _oracle_stream_si(depth, height, wavelength, n, 9.81)
    N = n
    assert np.abs(sol[: N + 1] - ref["eta"]).max() < 1e-11 * height
    assert np.abs(sol[N + 1: 2 * N + 1] - ref["B"]).max() < 1e-11 * np.abs(ref["B"]).max()
    for i, name in enumerate(["c", "Q", "R"]):
        assert abs(sol[2 * N + 1 + i] - ref[name]) < 1e-11 * abs(ref[name]), name
    assert sol[0] - sol[N] == pytest.approx(height, rel=1e-12)


def test_stream_solve_rejects_bad_input():
    from paper_2005_12716_amd import lib
    with pytest.raises(lib.SwenseError):
        lib.stream_solve(-1.0, 0.1, 2 * math.pi, 8)
    with pytest.raises(lib.SwenseError):
        lib.stream_solve(1.0, 0.1, 2 * math.pi, 100)


def test_hos_workspace_query_and_too_small_workspace():
    """The workspace query and the size and alignment checks of
    swense_hos_init_ws run on the host: a workspace below the queried size is
    refused with ENOMEM and a misaligned one with EINVAL before any device
    work (the pointers below are never dereferenced)."""
    import ctypes as C
    from paper_2005_12716_amd import lib
    L = lib.load()
    lam = 2 * math.pi
    d = lib.hos_desc(3, 64, 32, 64 * lam / 6.4, 32 * lam / 6.4, -1.0, order_m=3, dt=lam / 64)
    need = lib.hos_workspace_bytes(d)
    nc = 32 * 33
    assert need > 2 * nc * 16  # at least the FP64 state
    d5 = lib.hos_desc(3, 64, 32, 64 * lam / 6.4, 32 * lam / 6.4, -1.0, order_m=5, dt=lam / 64)
    assert lib.hos_workspace_bytes(d5) > need  # more series terms, larger product grid
    e = np.zeros((32, 33), dtype=np.complex128)
    h = C.c_void_p()
    fake = C.c_void_p(1 << 20)  # aligned, never touched
    assert L.swense_hos_init_ws(C.byref(d), lib._ptr(e), lib._ptr(e), lib.SPECTRAL, None, fake, need - 256,
                                C.byref(h)) == lib.ENOMEM
    assert L.swense_hos_init_ws(C.byref(d), lib._ptr(e), lib._ptr(e), lib.SPECTRAL, None, C.c_void_p((1 << 20) + 64),
                                need, C.byref(h)) == lib.EINVAL
    bad = lib.hos_desc(3, 63, 32, 1.0, 1.0, -1.0)
    with pytest.raises(lib.SwenseError):
        lib.hos_workspace_bytes(bad)


def test_dft_basis_covers_the_rows_read():
    """Host-only check of the evaluation's DFT coefficient pass: for every
    even mode count up to 8192, the rows its chunks read stay inside the
    basis rows allocated per node tile."""
    from paper_2005_12716_amd import lib
    assert lib.load().swense_selfcheck_launch_geometry(8192) == 0
