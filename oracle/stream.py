"""Regular waves by stream-function theory (Sec. 3.1.1) and their analytical
evaluation at points (Sec. 3.2.1), FP64 (test infrastructure only: used by
tests and the smoke check, never by the library).

Fourier approximation in the frame moving with the wave (X = x - c t, Y =
z + d above the bed): stream function
  psi = -ubar Y + sqrt(g/k^3) sum_{j=1..N} B_j sinh(j k Y)/cosh(j k d) cos(j k X),
which satisfies Laplace's equation and the bed condition.  Unknowns: the
surface heights eta_m at X_m = m pi/(N k), m = 0..N (crest to trough),
B_1..B_N, ubar, the volume flux Q and the Bernoulli constant R.
Equations: the surface is a streamline (psi = -Q) and Bernoulli holds on it
(|grad psi|^2 / 2 + g eta = R) at the N + 1 points, the mean of eta over a
wavelength is zero (trapezoidal rule), eta_0 - eta_N = H.  Reading: no mean
Eulerian current, so the phase speed is c = ubar.  Solved by Newton's
method with a central-difference Jacobian and numpy's dense solver, the wave
height raised in four steps from the linear guess.

Fields in the fixed frame (z from the mean level): u = psi_Y + c, w =
-psi_X, phi with grad phi = (u, w), eta from the cosine series through the
eta_m; time derivatives by d/dt = -c d/dX; pressure from Bernoulli with the
constant chosen so that p = 0 on the free surface:
  p = rho (R - c^2/2) - rho (phi_t + (u^2 + w^2)/2 + g z).
"""
from __future__ import annotations

import math

import numpy as np


def _hyper(j, k, Y, d):
    """cosh(jkY)/cosh(jkd) and sinh(jkY)/cosh(jkd) in overflow-safe form."""
    a = np.exp(j * k * (Y - d))
    b = np.exp(-j * k * (Y + d))
    den = 1.0 + np.exp(-2.0 * j * k * d)
    return (a + b) / den, (a - b) / den


def residual(v, N, k, d, H, g):
    eta, B = v[: N + 1], v[N + 1: 2 * N + 1]
    ubar, Q, R = v[2 * N + 1: 2 * N + 4]
    X = np.arange(N + 1) * math.pi / (N * k)
    Y = eta + d
    j = np.arange(1, N + 1)[:, None]
    s = math.sqrt(g / k ** 3)
    ch, sh = _hyper(j, k, Y[None, :], d)
    cx, sx = np.cos(j * k * X[None, :]), np.sin(j * k * X[None, :])
    psi = -ubar * Y + s * np.sum(B[:, None] * sh * cx, axis=0)
    U = -ubar + s * np.sum(B[:, None] * j * k * ch * cx, axis=0)
    W = s * np.sum(B[:, None] * j * k * sh * sx, axis=0)
    kin = psi + Q
    dyn = 0.5 * (U ** 2 + W ** 2) + g * eta - R
    mean = (0.5 * eta[0] + np.sum(eta[1:N]) + 0.5 * eta[N]) / N
    return np.concatenate([kin, dyn, [mean, eta[0] - eta[N] - H]])


def solve(depth: float, height: float, wavelength: float, N: int, g: float = 1.0, steps: int = 4):
    """Returns dict(eta[N+1], B[N], c, Q, R, k, d, N, g)."""
    k = 2 * math.pi / wavelength
    d = depth
    th = math.tanh(k * d)
    c0 = math.sqrt(g * th / k)
    v = np.zeros(2 * N + 4)
    for i in range(1, steps + 1):
        Hs = height * i / steps
        if i == 1:
            v[: N + 1] = 0.5 * Hs * np.cos(np.arange(N + 1) * math.pi / N)
            v[N + 1] = 0.5 * k * Hs / math.sqrt(th)
            v[2 * N + 1] = c0
            v[2 * N + 2] = c0 * d
            v[2 * N + 3] = 0.5 * c0 * c0
        else:  # extrapolate the surface and coefficients with the height
            v[: 2 * N + 1] *= i / (i - 1)
        for _ in range(50):
            r = residual(v, N, k, d, Hs, g)
            if np.max(np.abs(r)) < 1e-14:
                break
            J = np.empty((v.size, v.size))
            for i in range(v.size):
                e = np.zeros(v.size)
                e[i] = 1e-7 * max(1.0, abs(v[i]))
                J[:, i] = (residual(v + e, N, k, d, Hs, g) - residual(v - e, N, k, d, Hs, g)) / (2 * e[i])
            v = v - np.linalg.solve(J, r)
        assert np.max(np.abs(residual(v, N, k, d, Hs, g))) < 1e-12, "stream-function solve did not converge"
    return {"eta": v[: N + 1], "B": v[N + 1: 2 * N + 1], "c": v[2 * N + 1], "Q": v[2 * N + 2], "R": v[2 * N + 3],
            "k": k, "d": d, "N": N, "g": g}


def eta_coefficients(sol):
    """E_0..E_N of eta(X) = sum_j E_j cos(j k X) through the N + 1 surface points."""
    N, eta = sol["N"], sol["eta"]
    m = np.arange(N + 1)
    w = np.ones(N + 1)
    w[0] = w[N] = 0.5
    E = np.array([(2.0 / N) * np.sum(w * eta * np.cos(jj * m * math.pi / N)) for jj in range(N + 1)])
    E[0] *= 0.5
    E[N] *= 0.5
    return E


def fields(sol, x, z, t, rho: float = 1.0):
    """phi, u, w, p, phi_t, u_t, w_t, eta, eta_t at points (x, z) and time t."""
    N, k, d, g, c = sol["N"], sol["k"], sol["d"], sol["g"], sol["c"]
    B = sol["B"]
    x, z = np.asarray(x, dtype=np.float64), np.asarray(z, dtype=np.float64)
    X = x - c * t
    Y = z + d
    s = math.sqrt(g / k ** 3)
    j = np.arange(1, N + 1)[:, None]
    ch, sh = _hyper(j, k, Y[None, :], d)
    cx, sx = np.cos(j * k * X[None, :]), np.sin(j * k * X[None, :])
    Bj = B[:, None]
    phi = s * np.sum(Bj * ch * sx, axis=0)
    u = s * np.sum(Bj * j * k * ch * cx, axis=0)
    w = s * np.sum(Bj * j * k * sh * sx, axis=0)
    phi_t = -c * u
    u_t = c * s * np.sum(Bj * (j * k) ** 2 * ch * sx, axis=0)
    w_t = -c * s * np.sum(Bj * (j * k) ** 2 * sh * cx, axis=0)
    E = eta_coefficients(sol)
    jj = np.arange(N + 1)[:, None]
    eta = np.sum(E[:, None] * np.cos(jj * k * X[None, :]), axis=0)
    eta_t = c * np.sum(E[:, None] * jj * k * np.sin(jj * k * X[None, :]), axis=0)
    p = rho * (sol["R"] - 0.5 * c * c) - rho * (phi_t + 0.5 * (u ** 2 + w ** 2) + g * z)
    return {"phi": phi, "u": u, "w": w, "p": p, "phi_t": phi_t, "u_t": u_t, "w_t": w_t, "eta": eta, "eta_t": eta_t}
