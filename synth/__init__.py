"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the wave method itself: it draws random
numbers (SplitMix64, counter-based) and lays out geometry (point clouds,
vertical layer positions, realisation lists).  Spectra, amplitudes and every
step of the solver live on either side of the parity boundary, never here.

Everything is nondimensional with peak wavenumber k_p = 1 (lambda_p = 2*pi)
and g = 1 unless a caller passes other values.
"""
from __future__ import annotations

import math
import numpy as np

__all__ = [
    "splitmix64_uniform", "mode_phases", "uniform_points_2d",
    "cylinder_cloud", "hex_cloud", "hex_cloud_z_edges", "box_cloud", "clustered_layers",
    "uniform_layers", "batch_realisations", "even_5smooth",
]

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_uniform(keys: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014) applied to one counter
    per element; returns U[0,1) from the top 53 bits.  `keys` is uint64."""
    z = (np.asarray(keys, dtype=np.uint64) + _GOLDEN)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _key(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    base = (np.uint64(seed & 0xFFFFFF) << np.uint64(40)) | (np.uint64(stream & 0xFF) << np.uint64(32))
    return base | idx.astype(np.uint64)


def mode_phases(seed: int, ny: int, nxh: int) -> np.ndarray:
    """Random phases in [0, 2*pi) for the half spectrum [ny][nxh]; the counter
    for mode (p, q) is (seed, p, q) so a phase does not depend on the grid size."""
    q = np.arange(ny, dtype=np.uint64)[:, None]
    p = np.arange(nxh, dtype=np.uint64)[None, :]
    idx = (p << np.uint64(16)) | q
    return 2.0 * math.pi * splitmix64_uniform(_key(seed, 1, idx))


def _uniform_stream(seed: int, stream: int, n: int) -> np.ndarray:
    return splitmix64_uniform(_key(seed, stream, np.arange(n, dtype=np.uint64)))


def uniform_points_2d(seed: int, n: int, x0: float, x1: float, z0: float, z1: float) -> np.ndarray:
    """n points uniform in [x0,x1) x [z0,z1); returns [3][n] (x, y=0, z)."""
    ux = _uniform_stream(seed, 2, n)
    uz = _uniform_stream(seed, 3, n)
    out = np.zeros((3, n))
    out[0] = x0 + (x1 - x0) * ux
    out[2] = z0 + (z1 - z0) * uz
    return out


def _geometric_edges(start: float, first: float, total: float, n: int) -> np.ndarray:
    """n cells from `start` spanning `total` whose sizes grow geometrically from
    `first`.  Returns n+1 edges.  Ratio found by bisection."""
    if abs(first * n - total) < 1e-14 * total:
        r = 1.0
    else:
        lo, hi = (1.0 + 1e-12, 10.0) if first * n < total else (1e-6, 1.0 - 1e-12)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            s = first * (mid ** n - 1.0) / (mid - 1.0)
            if (s < total) == (first * n < total):
                lo = mid
            else:
                hi = mid
        r = 0.5 * (lo + hi)
    sizes = first * r ** np.arange(n)
    sizes *= total / sizes.sum()
    return start + np.concatenate([[0.0], np.cumsum(sizes)])


def cylinder_z_edges(hs: float, lam: float) -> np.ndarray:
    """Vertical cell edges of the cylinder mesh: 48 uniform cells of Hs/16 in
    |z| <= 1.5 Hs, 24 cells stretched down to -lambda/2, 8 up to +0.1 lambda."""
    dz = hs / 16.0
    mid = -1.5 * hs + dz * np.arange(49)
    below = _geometric_edges(-1.5 * hs, dz, lam / 2 - 1.5 * hs, 24)
    below = (-1.5 * hs) - (below - (-1.5 * hs))  # mirror downwards
    above = _geometric_edges(1.5 * hs, dz, 0.1 * lam - 1.5 * hs, 8)
    return np.concatenate([below[::-1][:-1], mid, above[1:]])


def cylinder_cloud(lx: float, ly: float, hs: float, lam: float = 2 * math.pi,
                   n_r: int = 130, n_theta: int = 192, scale: float = 1.0) -> np.ndarray:
    """Cell centres of a structured O-mesh around a vertical cylinder of radius
    0.1 lambda at the domain centre, out to radius 2 lambda, geometric radial
    cells (first lambda/400), n_theta sectors and the 80 z-levels of
    `cylinder_z_edges`.  `scale` shrinks n_r and n_theta for smaller clouds.
    Returns [3][n] float64 ordered (z fastest, then r, then theta) so points
    in one vertical column are contiguous."""
    n_r = max(2, int(round(n_r * scale)))
    n_theta = max(4, int(round(n_theta * scale)))
    r_edges = _geometric_edges(0.1 * lam, lam / 400.0, 1.9 * lam, n_r)
    rc = 0.5 * (r_edges[1:] + r_edges[:-1])
    th = (np.arange(n_theta) + 0.5) * (2 * math.pi / n_theta)
    ze = cylinder_z_edges(hs, lam)
    zc = 0.5 * (ze[1:] + ze[:-1])
    cx, cy = 0.5 * lx, 0.5 * ly
    R, T = np.meshgrid(rc, th, indexing="xy")  # [n_theta][n_r]
    xs = (cx + R * np.cos(T)).ravel()
    ys = (cy + R * np.sin(T)).ravel()
    ncol = xs.size
    out = np.empty((3, ncol * zc.size))
    out[0] = np.repeat(xs, zc.size)
    out[1] = np.repeat(ys, zc.size)
    out[2] = np.tile(zc, ncol)
    return out


def _tanh_levels(z0: float, z1: float, n: int, zc: float, dz_min: float) -> np.ndarray:
    """n+1 edges in [z0,z1] clustered around zc with smallest spacing ~dz_min."""
    s = np.linspace(0.0, 1.0, n + 1)
    # map s -> z with sinh stretching about zc; pick the strength by bisection
    a0 = (zc - z0) / (z1 - z0)

    def edges(beta):
        lo = np.arcsinh((0 - a0) * beta)
        hi = np.arcsinh((1 - a0) * beta)
        return z0 + (z1 - z0) * (a0 + np.sinh(lo + (hi - lo) * s) / beta)

    lo_b, hi_b = 1e-3, 1e4
    for _ in range(200):
        mid = math.sqrt(lo_b * hi_b)
        e = edges(mid)
        if np.min(np.diff(e)) > dz_min:
            lo_b = mid
        else:
            hi_b = mid
    return edges(lo_b)


def hex_cloud_z_edges(z0: float, z1: float, nz: int, dz_min: float) -> np.ndarray:
    """Unjittered vertical cell edges of hex_cloud (nz cells on [z0, z1],
    clustered about z = 0 with smallest cell dz_min)."""
    return _tanh_levels(z0, z1, nz, 0.0, dz_min)


def hex_cloud(seed: int, x0: float, y0: float, wx: float, wy: float, z0: float, z1: float,
              nx: int, ny: int, nz: int, dz_min: float, jitter: float = 0.1) -> tuple[np.ndarray, dict]:
    """Cell centres of a box mesh (uniform horizontally, sinh-clustered about
    z=0 vertically) with +-jitter (fraction of the local cell size) applied to
    every centre, mimicking a hex-dominant unstructured mesh.  Returns
    ([3][n] float64 points, mesh dict with the unjittered edges)."""
    xe = x0 + wx * np.arange(nx + 1) / nx
    ye = y0 + wy * np.arange(ny + 1) / ny
    ze = hex_cloud_z_edges(z0, z1, nz, dz_min)
    xc, yc, zc = (0.5 * (e[1:] + e[:-1]) for e in (xe, ye, ze))
    dzc = np.diff(ze)
    n = nx * ny * nz
    # order: z fastest, then x, then y
    Z = np.tile(zc, nx * ny)
    DZ = np.tile(dzc, nx * ny)
    X = np.tile(np.repeat(xc, nz), ny)
    Y = np.repeat(yc, nx * nz)
    jx = 2 * _uniform_stream(seed, 4, n) - 1
    jy = 2 * _uniform_stream(seed, 5, n) - 1
    jz = 2 * _uniform_stream(seed, 6, n) - 1
    out = np.empty((3, n))
    out[0] = X + jitter * (wx / nx) * jx
    out[1] = Y + jitter * (wy / ny) * jy
    out[2] = Z + jitter * DZ * jz
    return out, {"xe": xe, "ye": ye, "ze": ze}


def box_cloud(seed: int, n: int, x0: float, y0: float, wx: float, wy: float,
              zlo: float, zhi: float) -> np.ndarray:
    """n points jittered in a box, clustered toward z = 0 as
    z = sign(u) |u|^2 * extent (u uniform in [-1,1))."""
    ux = _uniform_stream(seed, 7, n)
    uy = _uniform_stream(seed, 8, n)
    uz = 2 * _uniform_stream(seed, 9, n) - 1
    out = np.empty((3, n))
    out[0] = x0 + wx * ux
    out[1] = y0 + wy * uy
    z = np.sign(uz) * uz * uz
    out[2] = np.where(z < 0, -z * zlo, z * zhi)
    return out


def uniform_layers(z0: float, z1: float, n: int) -> np.ndarray:
    return z0 + (z1 - z0) * np.arange(n) / (n - 1)


def clustered_layers(z0: float, z1: float, n: int, dz_min: float) -> np.ndarray:
    """n ascending layer heights on [z0, z1], clustered about z = 0."""
    return _tanh_levels(z0, z1, n - 1, 0.0, dz_min)


def even_5smooth(lo: int, hi: int) -> list[int]:
    out = []
    for v in range(lo, hi + 1):
        if v % 2:
            continue
        w = v
        for f in (2, 3, 5):
            while w % f == 0:
                w //= f
        if w == 1:
            out.append(v)
    return out


def batch_realisations(seed: int, count: int = 64, lo: int = 128, hi: int = 512,
                       pts_lo: int = 100_000, pts_hi: int = 1_000_000) -> list[dict]:
    """The uneven batch: mode counts i.i.d. over the even 5-smooth integers in
    [lo, hi], Hs/lambda_p ~ U[0.01, 0.03], point counts ~ U{pts_lo..pts_hi},
    and a per-realisation phase seed."""
    sizes = even_5smooth(lo, hi)
    u = _uniform_stream(seed, 10, 5 * count).reshape(count, 5)
    out = []
    for r in range(count):
        nx = sizes[min(len(sizes) - 1, int(u[r, 0] * len(sizes)))]
        ny = sizes[min(len(sizes) - 1, int(u[r, 1] * len(sizes)))]
        out.append({
            "nx": nx, "ny": ny,
            "hs_over_lambda": 0.01 + 0.02 * u[r, 2],
            "npts": pts_lo + int(u[r, 3] * (pts_hi - pts_lo + 1)),
            "phase_seed": 1000 * (seed + 1) + r,
        })
    return out


def surrogate_sea(seed: int) -> dict:
    """Training/test sea of the surrogate: Hs/lambda_p ~ U[0.01, 0.03] drawn
    from the seed, JONSWAP gamma 3.3, phases from the same seed."""
    u = _uniform_stream(seed, 20, 1)
    return {"hs_over_lambda": 0.01 + 0.02 * float(u[0]), "gamma": 3.3, "phase_seed": seed}
