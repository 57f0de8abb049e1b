"""Pins of the oracle's spectral conventions and of the seeded generators
against definitions written out by hand (direct trigonometric sums, a
published SplitMix64 test vector, closed-form derivatives)."""
import math

import numpy as np
import pytest

import synth
from oracle import Grid
from oracle import reconstruct as rc


def _direct_sum(grid, fh, xs, ys):
    """sum over the half spectrum, p > 0 doubled (Hermitian partner)."""
    out = np.zeros((ys.size, xs.size))
    X, Y = np.meshgrid(xs, ys)
    kx, ky = grid.kx(), grid.ky()
    for q in range(grid.ny):
        for p in range(grid.nxh):
            w = 1.0 if p == 0 else 2.0
            out += w * np.real(fh[q, p] * np.exp(1j * (kx[p] * X + ky[q] * Y)))
    return out


def _rand_spec(grid, seed):
    rng = np.random.default_rng(seed)
    fh = rng.standard_normal((grid.ny, grid.nxh)) + 1j * rng.standard_normal((grid.ny, grid.nxh))
    fh *= grid.nyquist_mask()
    # Hermitian p = 0 column
    if grid.ny > 1:
        for q in range(1, grid.ny // 2):
            fh[grid.ny - q, 0] = np.conj(fh[q, 0])
    fh[0, 0] = fh[0, 0].real
    return fh


def test_splitmix64_published_vector():
    # SplitMix64 seeded with 0: first output 0xE220A8397B1DCDAF (Steele et al.)
    u = synth.splitmix64_uniform(np.array([0], dtype=np.uint64))[0]
    assert u == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53


@pytest.mark.parametrize("nx,ny,M,dealias,expect", [
    # (M+1) n / 2 -> policy 1 (next even 2/3/5-smooth) or 2 (next 2^a or 3 2^a)
    (150, 480, 3, 1, (300, 960)), (150, 480, 3, 2, (384, 1024)),
    (500, 160, 3, 2, (1024, 384)), (40, 10, 5, 2, (128, 32)),
    (24, 20, 4, 2, (64, 64)), (1024, 1, 5, 2, (3072, 1)), (25, 25, 4, 1, (64, 64)), (25, 25, 4, 2, (64, 64)),
])
def test_product_grid_lengths(nx, ny, M, dealias, expect):
    g = Grid(nx=nx, ny=ny, lx=1.0, ly=1.0, depth=-1.0, order_m=M, dealias=dealias)
    assert g.padded() == expect


@pytest.mark.parametrize("dealias", [1, 2])
def test_products_of_m_factors_alias_nothing_into_the_kept_band(dealias):
    """The rule's defining property on both policies: the kept modes of a
    product of M band-limited fields formed on the product grid equal those
    of the exact product (a direct sum on a grid fine enough for all of its
    modes)."""
    g = Grid(nx=10, ny=6, lx=3.0, ly=2.0, depth=-1.0, order_m=3, dealias=dealias)
    fs = [_rand_spec(g, 10 + i) for i in range(g.order_m)]
    prod = np.ones(g.padded()[::-1])
    for f in fs:
        prod = prod * g.to_phys(f)
    got = g.to_spec(prod)
    # exact: the same product sampled on a grid of at least (M N) points per axis
    big = Grid(nx=10, ny=6, lx=3.0, ly=2.0, depth=-1.0, order_m=7, dealias=1)
    pe = np.ones(big.padded()[::-1])
    for f in fs:
        pe = pe * big.to_phys(f)
    assert np.allclose(got, big.to_spec(pe), atol=1e-12, rtol=0)


@pytest.mark.parametrize("nx,ny", [(8, 1), (12, 1), (8, 6), (10, 4)])
def test_to_phys_equals_direct_sum(nx, ny):
    g = Grid(nx=nx, ny=ny, lx=3.0, ly=2.0, depth=1.0, order_m=3)
    fh = _rand_spec(g, 1)
    px, py = g.padded()
    xs = g.lx * np.arange(px) / px
    ys = g.ly * np.arange(py) / py if ny > 1 else np.zeros(1)
    assert np.allclose(g.to_phys(fh), _direct_sum(g, fh, xs, ys), atol=1e-12, rtol=0)
    # truncation of a band-limited field returns the modes
    assert np.allclose(g.to_spec(g.to_phys(fh)), fh, atol=1e-13)


@pytest.mark.parametrize("gx,gy", [(8, 6), (16, 12), (32, 24), (5, 3), (6, 4)])
def test_node_values_pad_and_fold_equal_direct_sum(gx, gy):
    g = Grid(nx=8, ny=6, lx=3.0, ly=2.0, depth=1.0)
    fh = _rand_spec(g, 2)
    xs = g.lx * np.arange(gx) / gx
    ys = g.ly * np.arange(gy) / gy
    assert np.allclose(rc.node_values(g, fh, gx, gy), _direct_sum(g, fh, xs, ys), atol=1e-12)


def test_prefilter_interpolates_nodes():
    """Cubic B-spline with prefiltered coefficients reproduces node values
    (1/6, 4/6, 1/6 at the nodes)."""
    g = Grid(nx=16, ny=8, lx=3.0, ly=2.0, depth=1.0)
    fh = _rand_spec(g, 3)
    for gx, gy in [(16, 8), (32, 16), (12, 6)]:
        v = rc.node_values(g, fh, gx, gy)
        c = rc.node_values(g, fh, gx, gy, prefilter=True)
        r = (c + np.roll(c, 1, 1) / 4 + np.roll(c, -1, 1) / 4) * 4 / 6
        r = (r + np.roll(r, 1, 0) / 4 + np.roll(r, -1, 0) / 4) * 4 / 6
        assert np.allclose(r, v, atol=1e-12)


@pytest.mark.parametrize("depth", [0.7, -1.0])
def test_dz_symbol_matches_derivatives_of_basis(depth):
    """j-th z-derivative at z=0 of cosh(k(z+h))/cosh(kh) (or e^{kz})."""
    g = Grid(nx=8, ny=4, lx=3.0, ly=2.0, depth=depth)
    _, _, K = g.kvec()
    for j in range(1, 6):
        s = g.dz_symbol(j)
        for k, sv in zip(K.ravel(), s.ravel()):
            if depth > 0:
                ref = k ** j * (math.sinh(k * depth) if j % 2 else math.cosh(k * depth)) / math.cosh(k * depth)
            else:
                ref = k ** j
            assert abs(sv - ref) <= 1e-12 * max(1.0, abs(ref))


def test_vertical_factors_closed_form():
    g = Grid(nx=8, ny=1, lx=3.0, ly=1.0, depth=0.9)
    K = np.array([0.0, 0.5, 2.0, 7.0])
    for z in (-0.9, -0.3, 0.0, 0.2):
        C, S = rc.vertical_factors(g, K, z)
        assert np.allclose(C, np.cosh(K * (z + 0.9)) / np.cosh(K * 0.9), rtol=1e-14)
        assert np.allclose(S, np.sinh(K * (z + 0.9)) / np.cosh(K * 0.9), rtol=1e-14, atol=1e-300)


def test_generators_shapes_and_ranges():
    ph = synth.mode_phases(5, 4, 3)
    assert ph.shape == (4, 3) and ph.min() >= 0 and ph.max() < 2 * math.pi
    assert np.array_equal(synth.mode_phases(5, 8, 5)[:4, :3][:2], ph[:2])
    c = synth.cylinder_cloud(80 * math.pi, 40 * math.pi, 0.02 * 2 * math.pi)
    assert c.shape == (3, 1_996_800)
    r = np.hypot(c[0] - 40 * math.pi, c[1] - 20 * math.pi)
    assert r.min() > 0.1 * 2 * math.pi and r.max() < 2 * 2 * math.pi
    assert c[2].min() > -math.pi - 1e-9 and c[2].max() < 0.1 * 2 * math.pi + 1e-9
    assert len(synth.even_5smooth(128, 512)) == 26
