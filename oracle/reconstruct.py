"""Reconstruction of the incident fields (Sec. 3.2, 3.3), FP64.

* Analytical evaluation (Sec. 3.2, the modal formulas for u and w): at any
  point, phi = sum_k A_k C(k,z) e^{i k.x}, u = sum A ik_x C e^{ik.x},
  v = sum A ik_y C e^{ik.x}, w = sum A k S(k,z) e^{ik.x}, with
  C = cosh k(z+h)/cosh kh and S = sinh k(z+h)/cosh kh (deep water: e^{kz}).
  The same formula is used above z = 0 (extension into the air, Sec. 3.3).
* Pressure (Bernoulli; dynamic condition of Sec. 3.1 and Sec. 2.4.1):
  p = -rho (phi_t + 1/2 |grad phi|^2 + g z), total pressure incl. hydrostatic.
* Intermediate grid (Sec. 3.2.2): one inverse transform per layer z_l onto
  gx x gy uniformly spaced nodes.  Zero-padding refinement (Sec. 3.2.4):
  gx > nx inserts zero modes at high |k|; gx < nx folds (alias-sums) modes,
  which still gives the exact modal sum at the nodes.  A window of nodes may
  be cut out.
* Interpolation to cell centres (Sec. 3.2.2, "cubic spline scheme"):
  reading = periodic cubic spline horizontally (cubic B-spline on a
  coefficient grid obtained by dividing every mode by
  beta(k dx) = (4 + 2 cos(k dx))/6 per axis, which makes the spline
  interpolate the node values exactly), times 4-point cubic Lagrange
  vertically on the (arbitrary, ascending) layer heights, stencil shifted
  inward at the ends.
* Divergence error (Sec. 3.2.3): sum_f u_f . A_f / dV with face-centre
  values, on structured meshes; plus the analytic divergence of the
  interpolant.
"""
from __future__ import annotations

import math

import numpy as np

from .spectral import Grid

PHI, U, V, W, P, PHI_T, U_T, V_T, W_T, ETA, ETA_T = range(11)
FIELD_NAMES = ["phi", "u", "v", "w", "p", "phi_t", "u_t", "v_t", "w_t", "eta", "eta_t"]
VOLUME = [PHI, U, V, W, P, PHI_T, U_T, V_T, W_T]
SURFACE = [ETA, ETA_T]


def vertical_factors(grid: Grid, K: np.ndarray, z: float):
    """(C, S) at height z for wavenumber magnitudes K, overflow-safe:
    C = (e^{kz} + e^{-k(z+2h)})/(1 + e^{-2kh}), S likewise with a minus."""
    if grid.deep:
        e = np.exp(K * z)
        return e, e
    h = grid.depth
    a = np.exp(K * z)
    b = np.exp(-K * (z + 2 * h))
    d = 1.0 + np.exp(-2 * K * h)
    return (a + b) / d, (a - b) / d


def field_spectrum(grid: Grid, f: int, A, At, z: float):
    """Half spectrum of volume field f (not P) at height z."""
    KX, KY, K = grid.kvec()
    C, S = vertical_factors(grid, K, z)
    base = A if f in (PHI, U, V, W) else At
    ff = f if f <= W else [PHI, U, V, W][f - PHI_T]  # time derivatives use A_t
    if ff == PHI:
        return base * C
    if ff == U:
        return base * (1j * KX) * C
    if ff == V:
        return base * (1j * KY) * C
    if ff == W:
        return base * K * S
    raise ValueError(f)


def _beta(theta):
    return (4.0 + 2.0 * np.cos(theta)) / 6.0


def node_values(grid: Grid, fh: np.ndarray, gx: int, gy: int, prefilter: bool = False) -> np.ndarray:
    """Exact modal sum at the nodes (i Lx/gx, j Ly/gy) of a gx x gy grid,
    by Hermitian completion, folding/padding into a gx x gy spectrum and an
    inverse complex FFT.  With prefilter, returns the periodic cubic B-spline
    coefficients that interpolate those node values."""
    ny, nx = grid.ny, grid.nx
    if gx >= nx and (gy >= ny or ny == 1):
        # zero-padding only: place the half spectrum and inverse real FFT
        hx = nx // 2
        big = np.zeros((gy, gx // 2 + 1), dtype=np.complex128)
        sub = fh[:, :hx].copy()
        if prefilter:
            bx = _beta(2 * math.pi * np.arange(hx) / gx)
            qs = np.arange(ny)
            qs = np.where(qs < ny // 2, qs, qs - ny) if ny > 1 else qs
            by = _beta(2 * math.pi * qs / gy) if ny > 1 else np.ones(1)
            sub = sub / (by[:, None] * bx[None, :])
        if ny == 1:
            big[0, :hx] = sub[0]
        else:
            hy = ny // 2
            big[:hy, :hx] = sub[:hy]
            big[gy - (ny - hy - 1):, :hx] = sub[hy + 1:]
        return np.fft.irfft2(big, s=(gy, gx)) * (gx * gy)
    full = np.zeros((ny, nx), dtype=np.complex128)
    nxh = grid.nxh
    full[:, :nxh] = fh
    qneg = (-np.arange(ny)) % ny
    for p in range(nxh, nx):
        full[:, p] = np.conj(fh[qneg, nx - p])
    ps = np.arange(nx)
    ps = np.where(ps < nx // 2, ps, ps - nx)
    qs = np.arange(ny)
    qs = np.where(qs < ny // 2, qs, qs - ny) if ny > 1 else qs
    if prefilter:
        bx = _beta(2 * math.pi * ps / gx)
        by = _beta(2 * math.pi * qs / gy) if ny > 1 else np.ones(1)
        full = full / (by[:, None] * bx[None, :])
    G = np.zeros((gy, gx), dtype=np.complex128)
    np.add.at(G, ((qs % gy)[:, None], (ps % gx)[None, :]), full)
    return np.real(np.fft.ifft2(G)) * (gx * gy)


def _window(arr, ix0, iy0, wx, wy, gx, gy):
    ix = (ix0 + np.arange(wx)) % gx
    iy = (iy0 + np.arange(wy)) % gy
    return arr[..., iy[:, None], ix[None, :]]


def eval_grid(grid: Grid, A, At, eta_hat, eta_t_hat, gx: int, gy: int, z_layers,
              fields, window=None, prefilter: bool = False) -> dict:
    """Fields on the intermediate grid.  Volume fields -> [L][wy][wx],
    surface fields -> [wy][wx].  window = (ix0, iy0, wx, wy) or None."""
    if grid.ny == 1:
        gy = 1
    ix0, iy0, wx, wy = window if window is not None else (0, 0, gx, gy)
    out = {}
    need = set(fields)
    if P in need:
        need |= {PHI_T, U, V, W}
    for f in sorted(need):
        if f in SURFACE:
            fh = eta_hat if f == ETA else eta_t_hat
            out[f] = _window(node_values(grid, fh, gx, gy, prefilter), ix0, iy0, wx, wy, gx, gy)
            continue
        if f == P:
            continue
        if f == V and grid.ny == 1 or f == V_T and grid.ny == 1:
            out[f] = np.zeros((len(z_layers), wy, wx))
            continue
        layers = []
        for z in z_layers:
            fh = field_spectrum(grid, f, A, At, float(z))
            layers.append(_window(node_values(grid, fh, gx, gy, prefilter), ix0, iy0, wx, wy, gx, gy))
        out[f] = np.stack(layers)
    if P in fields:
        if prefilter:
            raise ValueError("pressure has no coefficient grid; it is formed at the points")
        zz = np.asarray(z_layers, dtype=np.float64)[:, None, None]
        out[P] = -grid.rho * (out[PHI_T] + 0.5 * (out[U] ** 2 + out[V] ** 2 + out[W] ** 2) + grid.g * zz)
    return {f: out[f] for f in fields}


def analytic_at_points(grid: Grid, A, At, eta_hat, eta_t_hat, pts: np.ndarray, fields) -> dict:
    """Brute-force analytical evaluation: the modal sums at every point
    (cost proportional to modes x points, as the paper notes)."""
    x, y, z = pts
    ny, nx = grid.ny, grid.nx
    KX, KY, K = grid.kvec()
    res = {}
    need = set(fields)
    if P in need:
        need |= {PHI_T, U, V, W}
    weights = np.full(KX.shape, 2.0)
    weights[:, 0] = 1.0  # p = 0 column carries both signs of q itself
    for f in sorted(need):
        if f == P:
            continue
        acc = np.zeros(x.shape)
        if f in SURFACE:
            base = eta_hat if f == ETA else eta_t_hat
        for qi in range(ny):
            for p in range(grid.nxh):
                if f in SURFACE:
                    a = base[qi, p]
                    if a == 0:
                        continue
                    ph = np.exp(1j * (KX[qi, p] * x + KY[qi, p] * y))
                    acc += weights[qi, p] * np.real(a * ph)
                    continue
                b = A[qi, p] if f in (PHI, U, V, W) else At[qi, p]
                if b == 0:
                    continue
                kk = K[qi, p]
                C, S = vertical_factors(grid, np.array(kk), z)
                ff = f if f <= W else [PHI, U, V, W][f - PHI_T]
                mult = {PHI: C, U: 1j * KX[qi, p] * C, V: 1j * KY[qi, p] * C, W: kk * S}[ff]
                ph = np.exp(1j * (KX[qi, p] * x + KY[qi, p] * y))
                acc += weights[qi, p] * np.real(b * mult * ph)
        res[f] = acc
    if P in fields:
        res[P] = -grid.rho * (res[PHI_T] + 0.5 * (res[U] ** 2 + res[V] ** 2 + res[W] ** 2) + grid.g * z)
    return {f: res[f] for f in fields}


# ------------------------------------------------------------------------------------
# interpolation
def bspline_weights(t):
    """Uniform cubic B-spline weights for nodes i-1, i, i+1, i+2, t in [0,1)."""
    t2 = t * t
    t3 = t2 * t
    return np.stack([(1 - t) ** 3 / 6, (3 * t3 - 6 * t2 + 4) / 6, (-3 * t3 + 3 * t2 + 3 * t + 1) / 6, t3 / 6])


def bspline_dweights(t):
    """d/dt of `bspline_weights`."""
    t2 = t * t
    return np.stack([-(1 - t) ** 2 / 2, 1.5 * t2 - 2 * t, -1.5 * t2 + t + 0.5, 0.5 * t2])


def lagrange_weights(zl: np.ndarray, z: np.ndarray):
    """4-point Lagrange weights (and their z-derivatives) on the layer
    heights; returns (l0, w[4][n], dw[4][n], inside)."""
    L = zl.size
    inside = (z >= zl[0]) & (z <= zl[-1])
    l = np.clip(np.searchsorted(zl, z, side="right") - 1, 0, L - 2)
    l0 = np.clip(l - 1, 0, L - 4)
    nodes = np.stack([zl[l0 + a] for a in range(4)])
    w = np.ones((4, z.size))
    dw = np.zeros((4, z.size))
    for a in range(4):
        for b in range(4):
            if b == a:
                continue
            w[a] *= (z - nodes[b]) / (nodes[a] - nodes[b])
        for c in range(4):
            if c == a:
                continue
            term = 1.0 / (nodes[a] - nodes[c])
            for b in range(4):
                if b == a or b == c:
                    continue
                term = term * (z - nodes[b]) / (nodes[a] - nodes[b])
            dw[a] += term
    return l0, w, dw, inside


def _hstencil(coord, d, g0, wlen, gfull):
    """Node indices (window-local, 4 x n) and B-spline weights along one
    axis; returns (idx, w, dw, ok)."""
    s = coord / d
    i = np.floor(s).astype(np.int64)
    t = s - i
    idx = np.stack([i - 1, i, i + 1, i + 2]) - g0
    if wlen == gfull:
        idx = idx % gfull
        ok = np.ones(coord.shape, dtype=bool)
    else:
        ok = (idx[0] >= 0) & (idx[3] < wlen)
        idx = np.clip(idx, 0, wlen - 1)
    return idx, bspline_weights(t), bspline_dweights(t) / d, ok


def interp_points(grid: Grid, coef: dict, z_layers, gx: int, gy: int, window, pts: np.ndarray,
                  fields, deriv: bool = False):
    """Interpolate coefficient grids (from eval_grid(..., prefilter=True))
    to points.  Returns (values dict, count of points out of range).  With
    deriv, also returns d/dx, d/dy, d/dz of each volume field."""
    x, y, z = pts
    zl = np.asarray(z_layers, dtype=np.float64)
    if grid.ny == 1:
        gy = 1
    ix0, iy0, wx, wy = window if window is not None else (0, 0, gx, gy)
    ixs, wxs, dwxs, okx = _hstencil(x, grid.lx / gx, ix0, wx, gx)
    if grid.ny > 1:
        iys, wys, dwys, oky = _hstencil(y, grid.ly / gy, iy0, wy, gy)
    else:
        iys = np.zeros((1, x.size), dtype=np.int64)
        wys = np.ones((1, x.size))
        dwys = np.zeros((1, x.size))
        oky = np.ones(x.size, dtype=bool)
    l0, wz, dwz, okz = lagrange_weights(zl, z)
    ok_h = okx & oky
    ok = ok_h & okz
    out, der = {}, {}
    need = set(fields)
    if P in need:
        need |= {PHI_T, U, V, W}
    for f in sorted(need):
        if f == P:
            continue
        c = coef[f]
        if f in SURFACE:
            acc = np.zeros(x.size)
            for b in range(iys.shape[0]):
                for a in range(4):
                    acc += wys[b] * wxs[a] * c[iys[b], ixs[a]]
            out[f] = np.where(ok_h, acc, np.nan)
            continue
        acc = np.zeros(x.size)
        dx = np.zeros(x.size); dy = np.zeros(x.size); dz = np.zeros(x.size)
        for cc in range(4):
            lay = l0 + cc
            for b in range(iys.shape[0]):
                for a in range(4):
                    v = c[lay, iys[b], ixs[a]]
                    acc += wz[cc] * wys[b] * wxs[a] * v
                    if deriv:
                        dx += wz[cc] * wys[b] * dwxs[a] * v
                        dy += wz[cc] * dwys[b] * wxs[a] * v
                        dz += dwz[cc] * wys[b] * wxs[a] * v
        out[f] = np.where(ok, acc, np.nan)
        if deriv:
            der[f] = tuple(np.where(ok, d, np.nan) for d in (dx, dy, dz))
    if P in fields:
        out[P] = -grid.rho * (out[PHI_T] + 0.5 * (out[U] ** 2 + out[V] ** 2 + out[W] ** 2) + grid.g * z)
    nbad = int(np.count_nonzero(~ok))
    res = {f: out[f] for f in fields}
    if deriv:
        return res, nbad, der
    return res, nbad


def divergence_of_interpolant(grid: Grid, coef: dict, z_layers, gx, gy, window, pts):
    """du/dx + dv/dy + dw/dz of the interpolant at the points."""
    _, _, der = interp_points(grid, coef, z_layers, gx, gy, window, pts, [U, V, W], deriv=True)
    return der[U][0] + der[V][1] + der[W][2]


def fv_divergence(face_u, face_v, face_w, xe, ye, ze):
    """Finite-volume divergence sum_f u_f . A_f / dV on a structured box
    mesh from face-centre velocities (Sec. 3.2.3).
    face_u: [nz][ny][nx+1], face_v: [nz][ny+1][nx] (or None in 2D),
    face_w: [nz+1][ny][nx].  Edges xe, ye, ze.  Returns [nz][ny][nx]."""
    dx = np.diff(xe)[None, None, :]
    dz = np.diff(ze)[:, None, None]
    div = (face_u[:, :, 1:] - face_u[:, :, :-1]) / dx + (face_w[1:] - face_w[:-1]) / dz
    if face_v is not None:
        dy = np.diff(ye)[None, :, None]
        div = div + (face_v[:, 1:, :] - face_v[:, :-1, :]) / dy
    return div


def face_centres(xe, ye, ze):
    """Face-centre coordinates of a structured box mesh: (fx, fy, fz) as
    [3][n] arrays in the layouts fv_divergence expects."""
    xc, yc, zc = (0.5 * (e[1:] + e[:-1]) for e in (xe, ye, ze))

    def pts(a, b, c):
        Z, Y, X = np.meshgrid(c, b, a, indexing="ij")
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    return pts(xe, yc, zc), pts(xc, ye, zc), pts(xc, yc, ze)
