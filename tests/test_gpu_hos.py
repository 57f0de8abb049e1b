"""GPU parity of the HOS step (Sec. 3.1.2) against the FP64 oracle, through
the C ABI.  Tolerances: FP64 path to round-off; mixed precision (FP32
transforms of the nonlinear remainder, FP64 state) at relative L2 1e-6 per
right-hand side and 1e-5 on the state after full runs."""
import math

import numpy as np

import c18
import pytest

import synth
from oracle import Grid, hos

pytestmark = pytest.mark.gpu
LAM = 2 * math.pi


def rel(a, b):
    """Both C18 measures at once: the larger of the relative L2 error and the
    maximum absolute error over the largest reference magnitude."""
    return c18.both(a, b)


def _case(lib, dim, nx, ny, depth, M, precision=0, dealias=1, hs=0.03, seed=5, dt=LAM / 64):
    lx = nx * LAM / 6.4
    ly = ny * LAM / 6.4 if dim == 3 else 1.0
    d = lib.hos_desc(dim, nx, ny, lx, ly, depth, order_m=M, dt=dt, dealias=dealias, precision=precision)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=hs * LAM, kp=1.0, gamma=3.3, phases=synth.mode_phases(seed, ny, nx // 2 + 1))
    g = Grid(nx=nx, ny=ny, lx=lx, ly=ly, depth=depth, order_m=M, dealias=dealias)
    return d, g, eh, ph


CASES = [
    # dim, nx, ny, depth, M, dealias
    (2, 64, 1, 1.5, 3, 1),
    (2, 60, 1, -1.0, 5, 1),
    (3, 32, 16, -1.0, 3, 1),
    (3, 24, 20, 2.0, 4, 1),
    (3, 30, 18, -1.0, 2, 0),
    (3, 16, 8, 1.0, 1, 1),
    (3, 40, 10, -1.0, 5, 1),
]


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("dim,nx,ny,depth,M,dealias", CASES)
def test_rhs_parity(gpu_lib, dim, nx, ny, depth, M, dealias, precision):
    from paper_2005_12716_amd import lib
    d, g, eh, ph = _case(lib, dim, nx, ny, depth, M, precision, dealias)
    h = lib.Hos(d, eh, ph)
    et, pt = h.rhs()
    er, pr = hos.rhs(g, eh, ph)
    tol = 1e-12 if precision == 1 else 2e-6
    assert rel(et, er) < tol and rel(pt, pr) < tol, (rel(et, er), rel(pt, pr))
    h.close()


# Padded y lengths 256 ... 4096 (powers of two) and 768, 1536, 3072: the y
# transforms run one kx column per workgroup, on the four-wavefront FFT or
# on three sub-transforms and a radix-3 combine.
WG_CASES = [
    # dim, nx, ny, depth, M, dealias   -> padded Py
    (3, 64, 128, -1.0, 3, 1),  # 256
    (3, 32, 256, 2.0, 3, 1),   # 512, finite depth
    (3, 16, 512, -1.0, 3, 1),  # 1024
    (3, 8, 1024, -1.0, 3, 1),  # 2048
    (3, 8, 2048, 1.5, 3, 1),   # 4096
    # three times a power of two: the three-way workgroup transform
    (3, 8, 384, -1.0, 3, 1),   # 768
    (3, 8, 768, 2.0, 3, 1),    # 1536
    (3, 8, 512, -1.0, 5, 1),   # 1536, order 5
    (3, 8, 1024, -1.0, 5, 1),  # 3072, order 5
]


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("dim,nx,ny,depth,M,dealias", WG_CASES)
def test_rhs_parity_workgroup_y_transforms(gpu_lib, dim, nx, ny, depth, M, dealias, precision):
    test_rhs_parity(gpu_lib, dim, nx, ny, depth, M, dealias, precision)


# Padded x lengths 768, 1536 and 3072 (three times a power of two): in FP32
# the x pass transforms each row as three sub-transforms and a radix-3
# combine.  (At 3072 points the FP64 x pass does not fit a workgroup's LDS.)
X3_CASES = [
    # dim, nx, ny, depth, M, dealias, precisions   -> padded Px
    (3, 384, 8, -1.0, 3, 1, (1, 0)),   # 768
    (3, 768, 8, 1.5, 3, 1, (1, 0)),    # 1536
    (3, 512, 8, -1.0, 5, 1, (1, 0)),   # 1536, order 5
    (3, 1024, 8, 2.0, 5, 1, (0,)),     # 3072, order 5
]


# Padded x lengths between the powers of two (5-smooth, up to 1024: the
# batched configuration's sizes), on the runtime-planned wavefront FFT.
RT_CASES = [
    # dim, nx, ny, depth, M, dealias   -> padded Px
    (3, 300, 8, -1.0, 3, 1),   # 600
    (3, 360, 8, 1.5, 4, 1),    # 960, order 4
    (2, 480, 1, -1.0, 3, 1),   # 960, 2D
]


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("dim,nx,ny,depth,M,dealias", RT_CASES)
def test_rhs_parity_runtime_rows(gpu_lib, dim, nx, ny, depth, M, dealias, precision):
    test_rhs_parity(gpu_lib, dim, nx, ny, depth, M, dealias, precision)


# Padded y lengths of 2 and 3 times a 2/3/5-smooth mode count that have no
# compile-time transform: the residue-form y passes with runtime plans of the
# mode count (one wavefront per residue).
YRR_CASES = [
    # dim, nx, ny, depth, M, dealias   -> padded Py = rs ny
    (3, 32, 150, -1.0, 3, 1),  # 300 = 2 x 150
    (3, 24, 160, 2.0, 3, 1),   # 320 = 2 x 160, finite depth
    (3, 16, 120, -1.0, 5, 1),  # 360 = 3 x 120
    (3, 16, 90, 1.5, 5, 1),    # 270 = 3 x 90, finite depth
    (3, 32, 16, -1.0, 3, 1),   # 32 = 2 x 16
]


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("dim,nx,ny,depth,M,dealias", YRR_CASES)
def test_rhs_parity_runtime_residue_y(gpu_lib, dim, nx, ny, depth, M, dealias, precision):
    test_rhs_parity(gpu_lib, dim, nx, ny, depth, M, dealias, precision)


@pytest.mark.parametrize("dim,nx,ny,depth,M,dealias", YRR_CASES[:2])
def test_steps_parity_runtime_residue_y(gpu_lib, dim, nx, ny, depth, M, dealias):
    test_steps_parity(gpu_lib, dim, nx, ny, depth, M, dealias, 0)


@pytest.mark.parametrize("dim,nx,ny,depth,M,dealias,precisions", X3_CASES)
def test_rhs_parity_three_way_x_transforms(gpu_lib, dim, nx, ny, depth, M, dealias, precisions):
    for precision in precisions:
        test_rhs_parity(gpu_lib, dim, nx, ny, depth, M, dealias, precision)


# Product grids of policy 2 (the smallest 2^k or 3 2^k at or above the
# (M+1)/2 rule) against the oracle on the same product grid.
P2_CASES = [
    # dim, nx, ny, depth, M, dealias   -> padded (policy 1 -> policy 2)
    (3, 40, 10, -1.0, 5, 2),   # 120 x 30 -> 128 x 32
    (3, 24, 20, 2.0, 4, 2),    # 60 x 50 -> 64 x 64, finite depth
    (3, 300, 8, -1.0, 3, 2),   # 600 x 16 -> 768 x 16
    (2, 480, 1, -1.0, 3, 2),   # 960 -> 1024, 2D
    (3, 144, 200, 1.5, 3, 2),  # 288 x 400 -> 384 x 512
]


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("dim,nx,ny,depth,M,dealias", P2_CASES)
def test_rhs_parity_padding_policy_2(gpu_lib, dim, nx, ny, depth, M, dealias, precision):
    test_rhs_parity(gpu_lib, dim, nx, ny, depth, M, dealias, precision)


@pytest.mark.parametrize("dim,nx,ny,depth,M,dealias", P2_CASES[:2])
def test_steps_parity_padding_policy_2(gpu_lib, dim, nx, ny, depth, M, dealias):
    test_steps_parity(gpu_lib, dim, nx, ny, depth, M, dealias, 0)


def test_padding_tuner(gpu_lib):
    """The tuner times both policies where their lengths differ and returns
    the faster; where they coincide it returns 1 untimed.  A realisation
    built with its choice steps like one built with the other policy."""
    from paper_2005_12716_amd import lib
    d, g, eh, ph = _case(lib, 3, 144, 200, 1.5, 3)
    best, ms = lib.tune_padding(d, nsteps=2)
    assert best in (1, 2) and np.all(ms > 0) and ms[best - 1] <= ms[2 - best]
    same, ms1 = lib.tune_padding(_case(lib, 3, 64, 64, -1.0, 3)[0])
    assert same == 1 and np.all(ms1 == -1.0)
    outs = []
    for pol in (1, 2):
        d.dealias = pol
        h = lib.Hos(d, eh, ph)
        h.step(4)
        outs.append(h.state()[:2])
        h.close()
    assert rel(outs[0][0], outs[1][0]) < 1e-6 and rel(outs[0][1], outs[1][1]) < 1e-6


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("dim,nx,ny,depth,M,dealias", CASES[:4])
def test_steps_parity(gpu_lib, dim, nx, ny, depth, M, dealias, precision):
    from paper_2005_12716_amd import lib
    d, g, eh, ph = _case(lib, dim, nx, ny, depth, M, precision, dealias)
    h = lib.Hos(d, eh, ph)
    h.step(12)
    e, p, t = h.state()
    er, pr = hos.run(g, eh, ph, d.dt, 12)
    tol = 1e-11 if precision == 1 else 1e-6
    assert rel(e, er) < tol and rel(p, pr) < tol, (rel(e, er), rel(p, pr))
    assert abs(t - 12 * d.dt) < 1e-12
    h.close()


@pytest.mark.parametrize("precision", [1, 0])
def test_modes_and_energy_parity(gpu_lib, precision):
    from paper_2005_12716_amd import lib
    d, g, eh, ph = _case(lib, 3, 32, 16, 1.5, 3, precision)
    h = lib.Hos(d, eh, ph)
    h.step(3)
    er, pr = hos.run(g, eh, ph, d.dt, 3)
    a, at, et = h.modes()
    A = hos.mean_level_modes(g, er, pr)
    At, eth = hos.mean_level_modes_t(g, er, pr)
    tol = 1e-11 if precision == 1 else 1e-6
    assert rel(a, A) < tol and rel(at, At) < tol and rel(et, eth) < tol, (rel(a, A), rel(at, At), rel(et, eth))
    E = h.energy()
    assert abs(E - hos.energy(g, er, pr)) < (1e-11 if precision == 1 else 1e-6) * abs(E)
    h.close()


@pytest.mark.parametrize("dim,nx,ny", [(3, 24, 10), (2, 48, 1)])
def test_physical_state_roundtrip(gpu_lib, dim, nx, ny):
    from paper_2005_12716_amd import lib
    d, g, eh, ph = _case(lib, dim, nx, ny, -1.0, 3, 0)
    eta, phis = hos.state_to_phys(g, eh, ph)
    h = lib.Hos(d, eta, phis, layout=lib.PHYSICAL)
    e, p, _ = h.state(lib.SPECTRAL)
    assert np.abs(e - eh).max() < 1e-15 * 100 and np.abs(p - ph).max() < 1e-13
    e2, p2, _ = h.state(lib.PHYSICAL)
    assert np.abs(e2 - eta).max() < 1e-14 and np.abs(p2 - phis).max() < 1e-13
    h.close()


def test_stokes_regular_wave_full_run_fp64(gpu_lib):
    """2D Stokes wave, ka = 0.1, kh = 2, 4 wavelengths, 256 modes, M = 3,
    RK4 with T/64 over two periods, FP64 throughout."""
    from paper_2005_12716_amd import lib
    d = lib.hos_desc(2, 256, 1, 4 * LAM, 1.0, 2.0, order_m=3, precision=1)
    eh, ph = lib.sea_spectrum(d, kind=1, mode=4, ka=0.1)
    w = math.sqrt(math.tanh(2.0))
    d.dt = 2 * math.pi / w / 64
    h = lib.Hos(d, eh, ph)
    h.step(128)
    e, p, _ = h.state()
    g = Grid(nx=256, ny=1, lx=4 * LAM, ly=1.0, depth=2.0, order_m=3)
    er, pr = hos.run(g, eh, ph, d.dt, 128)
    assert rel(e, er) < 1e-11 and rel(p, pr) < 1e-11
    h.close()


def test_irregular_sea_512x256_mixed_precision(gpu_lib):
    """Full-size mode grid (512 x 256 over 40 x 20 peak wavelengths, JONSWAP
    Hs/lambda_p = 0.02, M = 3, dt = Tp/64): 8 steps against the oracle,
    relative L2 of eta and phis below 1e-5."""
    from paper_2005_12716_amd import lib
    nx, ny = 512, 256
    d = lib.hos_desc(3, nx, ny, 40 * LAM, 20 * LAM, -1.0, order_m=3, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=0.02 * LAM, kp=1.0, gamma=3.3, phases=synth.mode_phases(1, ny, nx // 2 + 1))
    h = lib.Hos(d, eh, ph)
    h.step(8)
    e, p, _ = h.state()
    g = Grid(nx=nx, ny=ny, lx=40 * LAM, ly=20 * LAM, depth=-1.0, order_m=3)
    er, pr = hos.run(g, eh, ph, d.dt, 8)
    assert rel(e, er) < 1e-5 and rel(p, pr) < 1e-5, (rel(e, er), rel(p, pr))
    h.close()


def test_invalid_descriptors(gpu_lib):
    from paper_2005_12716_amd import lib
    eh = np.zeros((16, 9), dtype=np.complex128)
    for bad in [lib.hos_desc(3, 14, 16, 1.0, 1.0, -1.0), lib.hos_desc(3, 16, 7, 1.0, 1.0, -1.0),
                lib.hos_desc(3, 16, 16, 1.0, 1.0, -1.0, order_m=0), lib.hos_desc(2, 16, 4, 1.0, 1.0, -1.0)]:
        with pytest.raises(lib.SwenseError):
            lib.Hos(bad, eh, eh)


def test_nonfinite_state_is_reported(gpu_lib):
    from paper_2005_12716_amd import lib
    d, g, eh, ph = _case(lib, 3, 16, 8, -1.0, 3, 0)
    eh = eh.copy()
    eh[1, 2] = np.nan
    h = lib.Hos(d, eh, ph)
    with pytest.raises(lib.SwenseError) as ei:
        h.state()
    assert ei.value.code == lib.EUNSTABLE
    h.close()


def test_first_stage_reuses_the_evaluated_rhs_bitwise(gpu_lib):
    """Evaluating the mean-level modes between steps leaves the right-hand
    side of the current state in place; the next step's first RK stage takes
    it instead of recomputing it, with bit-identical results."""
    from paper_2005_12716_amd import lib
    d, g, eh, ph = _case(lib, 3, 32, 16, -1.0, 3)
    a, b = lib.Hos(d, eh, ph), lib.Hos(d, eh, ph)
    for _ in range(3):
        a.step(1)
        a.modes()
    b.step(3)
    ea, pa, ta = a.state()
    eb, pb, tb = b.state()
    assert np.array_equal(ea, eb) and np.array_equal(pa, pb) and ta == tb
    a.close()
    b.close()


@pytest.mark.parametrize("precision,nsub,depth", [(0, 1, -1.0), (0, 2, 1.5), (1, 2, -1.0)])
def test_integrating_factor_step_matches_oracle(gpu_lib, precision, nsub, depth):
    """The coarse integrating-factor RK4 step (the surrogate's base) against
    the oracle's: FP32 transforms of the nonlinear part (1e-6), FP64 (1e-12)."""
    from paper_2005_12716_amd import lib
    d, g, eh, ph = _case(lib, 3, 32, 16, depth, 3, precision=precision)
    h = lib.Hos(d, eh, ph)
    tau = 10 * d.dt
    h.step_exp(tau, nsub)
    e, p, t = h.state()
    er, pr = eh, ph
    for _ in range(nsub):
        er, pr = hos.ifrk4_step(g, er, pr, tau / nsub)
    tol = 1e-6 if precision == 0 else 1e-12
    assert rel(e, er) < tol and rel(p, pr) < tol
    assert abs(t - tau) < 1e-12
    h.close()
