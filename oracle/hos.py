"""High-Order Spectral (HOS) free-surface step, FP64 (Sec. 3.1.2).

Unknowns: surface elevation eta and surface potential phis = phi(x, eta)
(definition of the surface potential, Sec. 3.1.2), both as half spectra.

Evolution (the 2D HOS equations of Sec. 3.1.2; the 3D form follows from the
free-surface kinematic and dynamic conditions of Sec. 3.1 by the chain rule
with grad = (d/dx, d/dy)):
    eta_t  = (1 + |grad eta|^2) W - grad phis . grad eta
    phis_t = -g eta - 1/2 |grad phis|^2 + 1/2 (1 + |grad eta|^2) W^2
where W is the vertical velocity at the surface.

Reading (the paper cites West et al. 1987 and Dommermuth & Yue 1987 for
HOS and does not give the series): W follows the West et al. order-M
expansion.  With g_{m,j} = d^j/dz^j phi^(m) at z = 0 (by FFT of
D_z^j phihat^(m)),
    phi^(1)(x,0)   = phis
    phi^(m+1)(x,0) = - sum_{j=1..m} eta^j/j! g_{m+1-j, j}
    W^(m)          = sum_{j=0..m-1} eta^j/j! g_{m-j, j+1}
and the evolution terms are truncated consistently at order M:
    eta_t  = W_M + |grad eta|^2 W_{M-2} - [M>=2] grad phis . grad eta
    phis_t = -g eta - [M>=2] 1/2 |grad phis|^2 + 1/2 [W^2]_M + 1/2 |grad eta|^2 [W^2]_{M-2}
with W_K = sum_{m<=K} W^(m), [W^2]_K = sum_{m=2..K} sum_{l=1..m-1} W^(l) W^(m-l).
Products are formed on the (M+1)/2 dealiased grid; Nyquist modes are zeroed
after every truncation; the mean of eta_t is set to 0; the mean of phis_t
(the Bernoulli constant) is kept.  Time integration: classical fixed-step
RK4 on the spectral state (the paper names no integrator).
"""
from __future__ import annotations

import math

import numpy as np

from .spectral import Grid


def grad_phys(grid: Grid, fh: np.ndarray):
    KX, KY, _ = grid.kvec()
    fx = grid.to_phys(1j * KX * fh)
    fy = grid.to_phys(1j * KY * fh) if grid.ny > 1 else np.zeros_like(fx)
    return fx, fy


def series(grid: Grid, eta: np.ndarray, phis_hat: np.ndarray, order: int | None = None):
    """Order-M Dirichlet series.  Given physical eta on the product grid and
    the surface value's half spectrum, returns (modes [phihat^(1..M)], g)
    where g[(m, j)] are the physical vertical derivatives used by W."""
    M = grid.order_m if order is None else order
    modes = [phis_hat]
    g = {}
    for m in range(1, M + 1):
        for j in range(1, M - m + 2):
            g[(m, j)] = grid.to_phys(grid.dz_symbol(j) * modes[m - 1])
        if m < M:
            acc = np.zeros_like(eta)
            for j in range(1, m + 1):
                acc += eta ** j / math.factorial(j) * g[(m + 1 - j, j)]
            modes.append(grid.to_spec(-acc) * grid.nyquist_mask())
    return modes, g


def w_orders(grid: Grid, eta: np.ndarray, g: dict, order: int | None = None):
    """W^(m), m = 1..M, physical."""
    M = grid.order_m if order is None else order
    out = []
    for m in range(1, M + 1):
        acc = np.zeros_like(eta)
        for j in range(0, m):
            acc += eta ** j / math.factorial(j) * g[(m - j, j + 1)]
        out.append(acc)
    return out


def _wsum(W, K):
    s = np.zeros_like(W[0])
    for m in range(1, K + 1):
        s += W[m - 1]
    return s


def _w2sum(W, K):
    s = np.zeros_like(W[0])
    for m in range(2, K + 1):
        for l in range(1, m):
            s += W[l - 1] * W[m - l - 1]
    return s


def rhs(grid: Grid, eta_hat: np.ndarray, phis_hat: np.ndarray, want_phys: bool = False):
    """Time derivatives (eta_t_hat, phis_t_hat) of the spectral state."""
    M = grid.order_m
    eta = grid.to_phys(eta_hat)
    ex, ey = grad_phys(grid, eta_hat)
    px, py = grad_phys(grid, phis_hat)
    _, g = series(grid, eta, phis_hat)
    W = w_orders(grid, eta, g)
    ge2 = ex * ex + ey * ey
    eta_t = _wsum(W, M)
    phi_t = -grid.g * eta
    if M >= 3:
        eta_t = eta_t + ge2 * _wsum(W, M - 2)
    if M >= 2:
        eta_t = eta_t - (px * ex + py * ey)
        phi_t = phi_t - 0.5 * (px * px + py * py)
    phi_t = phi_t + 0.5 * _w2sum(W, M)
    if M >= 4:
        phi_t = phi_t + 0.5 * ge2 * _w2sum(W, M - 2)
    eth = grid.to_spec(eta_t) * grid.nyquist_mask()
    pth = grid.to_spec(phi_t) * grid.nyquist_mask()
    eth[0, 0] = 0.0
    if want_phys:
        return eth, pth, {"eta": eta, "W": W, "eta_t": eta_t, "phi_t": phi_t}
    return eth, pth


def rk4_step(grid: Grid, eta_hat, phis_hat, dt: float):
    k1 = rhs(grid, eta_hat, phis_hat)
    k2 = rhs(grid, eta_hat + 0.5 * dt * k1[0], phis_hat + 0.5 * dt * k1[1])
    k3 = rhs(grid, eta_hat + 0.5 * dt * k2[0], phis_hat + 0.5 * dt * k2[1])
    k4 = rhs(grid, eta_hat + dt * k3[0], phis_hat + dt * k3[1])
    e = eta_hat + dt / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
    p = phis_hat + dt / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
    return e, p


def linear_propagate(grid: Grid, eta_hat, phis_hat, tau: float):
    """Exact solution over tau of the linear part of the evolution (the
    M = 1 equations eta_t = k tanh(kh) phis, phis_t = -g eta), mode by mode:
    eta <- cos(w tau) eta + (kt/w) sin(w tau) phis, phis <- cos(w tau) phis -
    (g/w) sin(w tau) eta with kt = k tanh(kh) (deep: k), w = sqrt(g kt);
    k = 0: phis <- phis - g tau eta."""
    _, _, K = grid.kvec()
    kt = K * np.tanh(K * grid.depth) if grid.depth > 0 else K
    w = np.sqrt(grid.g * kt)
    c, s = np.cos(w * tau), np.sin(w * tau)
    safe = np.where(w > 0, w, 1.0)
    a = np.where(w > 0, kt * s / safe, 0.0)
    b = np.where(w > 0, grid.g * s / safe, grid.g * tau)
    return c * eta_hat + a * phis_hat, c * phis_hat - b * eta_hat


def nonlinear_rhs(grid: Grid, eta_hat, phis_hat):
    """The right-hand side minus its linear part (kt phis, -g eta)."""
    _, _, K = grid.kvec()
    kt = K * np.tanh(K * grid.depth) if grid.depth > 0 else K
    et, pt = rhs(grid, eta_hat, phis_hat)
    ne = et - kt * phis_hat * grid.nyquist_mask()
    ne[0, 0] = 0.0
    return ne, pt + grid.g * eta_hat * grid.nyquist_mask()


def ifrk4_step(grid: Grid, eta_hat, phis_hat, h: float):
    """One integrating-factor (Lawson) RK4 step of size h: classical RK4 on
    v(t) = E(-t) X(t), E the exact linear propagator, so that only the
    nonlinear part N is integrated numerically:
      k1 = N(X), k2 = N(E_h/2 (X + h/2 k1)), k3 = N(E_h/2 X + h/2 k2),
      k4 = N(E_h X + h E_h/2 k3),
      X <- E_h X + h/6 (E_h k1 + 2 E_h/2 (k2 + k3) + k4).
    (A time integrator for the surrogate's base step, not in the paper.)"""
    def E(x, t):
        return linear_propagate(grid, x[0], x[1], t)

    def add(x, y, a=1.0):
        return x[0] + a * y[0], x[1] + a * y[1]

    X = (eta_hat, phis_hat)
    k1 = nonlinear_rhs(grid, *X)
    k2 = nonlinear_rhs(grid, *E(add(X, k1, 0.5 * h), 0.5 * h))
    k3 = nonlinear_rhs(grid, *add(E(X, 0.5 * h), k2, 0.5 * h))
    k4 = nonlinear_rhs(grid, *add(E(X, h), E(k3, 0.5 * h), h))
    s = add(add(E(k1, h), E(add(k2, k3), 0.5 * h), 2.0), k4)
    return add(E(X, h), s, h / 6.0)


def run(grid: Grid, eta_hat, phis_hat, dt: float, nsteps: int, callback=None):
    for n in range(nsteps):
        eta_hat, phis_hat = rk4_step(grid, eta_hat, phis_hat, dt)
        if callback is not None:
            callback(n + 1, eta_hat, phis_hat)
    return eta_hat, phis_hat


def energy(grid: Grid, eta_hat, phis_hat) -> float:
    """E = 1/2 int phis eta_t dA + 1/2 g int eta^2 dA, with eta_t from the
    order-M right-hand side (kinetic energy as the surface flux of phi)."""
    eth, _ = rhs(grid, eta_hat, phis_hat)
    shape = (grid.nx, grid.ny)
    phis = grid.to_phys(phis_hat, shape)
    et = grid.to_phys(eth, shape)
    eta = grid.to_phys(eta_hat, shape)
    return 0.5 * grid.integrate(phis * et) + 0.5 * grid.g * grid.integrate(eta * eta)


def mean_level_modes(grid: Grid, eta_hat, phis_hat):
    """Modal amplitudes A^phi of the potential at z = 0 (the coefficients of
    the cosh basis, Sec. 3.1 and Sec. 3.2): A = sum_m phihat^(m)."""
    eta = grid.to_phys(eta_hat)
    modes, _ = series(grid, eta, phis_hat)
    return sum(modes)


def mean_level_modes_t(grid: Grid, eta_hat, phis_hat):
    """Modal amplitudes of d(phi)/dt at z = 0, plus eta_t_hat.

    Reading (the paper only says the pressure is reconstructed like the
    velocity): phi_t is harmonic and satisfies the seabed condition, and by
    the chain rule its surface value is phis_t - W eta_t.  So the same order-M
    Dirichlet series is solved with surface data f = phis_t - [M>=2] W_M eta_t
    (the product is second order and is dropped at M = 1 so that M = 1 stays
    exactly linear)."""
    M = grid.order_m
    eth, pth, extra = rhs(grid, eta_hat, phis_hat, want_phys=True)
    eta = extra["eta"]
    f = grid.to_phys(pth)
    if M >= 2:
        f = f - _wsum(extra["W"], M) * grid.to_phys(eth)
    fh = grid.to_spec(f) * grid.nyquist_mask()
    modes, _ = series(grid, eta, fh)
    return sum(modes), eth


def state_from_phys(grid: Grid, eta: np.ndarray, phis: np.ndarray):
    shape = eta.shape
    return grid.to_spec(eta.reshape(shape)) * grid.nyquist_mask(), grid.to_spec(phis) * grid.nyquist_mask()


def state_to_phys(grid: Grid, eta_hat, phis_hat):
    shape = (grid.nx, grid.ny)
    return grid.to_phys(eta_hat, shape), grid.to_phys(phis_hat, shape)


def hermite_in_time(y0, dy0, y1, dy1, t0: float, t1: float, t: float):
    """Values between two outputs of the wave model (the CFD step is several
    times shorter than the HOS step: Sec. 4.3 and the validation cases).
    Reading (the paper is silent): cubic Hermite interpolation in time of a
    modal amplitude from its values and time derivatives at t0 and t1 -
    (A, A_t) and (eta_hat, eta_t_hat) - and the derivative of that cubic as
    the time derivative at t.  Returns (y(t), y'(t))."""
    dt = t1 - t0
    s = (t - t0) / dt
    h00, h10, h01, h11 = 2 * s**3 - 3 * s**2 + 1, s**3 - 2 * s**2 + s, -2 * s**3 + 3 * s**2, s**3 - s**2
    d00, d10, d01, d11 = 6 * s**2 - 6 * s, 3 * s**2 - 4 * s + 1, -6 * s**2 + 6 * s, 3 * s**2 - 2 * s
    y = h00 * y0 + h10 * dt * dy0 + h01 * y1 + h11 * dt * dy1
    dy = (d00 * y0 + d10 * dt * dy0 + d01 * y1 + d11 * dt * dy1) / dt
    return y, dy
