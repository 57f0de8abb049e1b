"""Initial sea states (FP64 spectra), the oracle's side of the set-up step.

Regular wave: second-order Stokes wave.  The paper initialises regular waves
with stream-function theory (Sec. 3.1.1) and gives no formula; the oracle
uses the textbook second-order Stokes solution, which is the same wave to
O((ka)^2).

Irregular sea: JONSWAP spectrum (Sec. 3.1.2 and the reconstruction example
of Sec. 3.2.2 give Tp, Hs and gamma only).  Reading: standard JONSWAP shape
with sigma = 0.07 / 0.09, mapped to wavenumber by deep-water dispersion,
optional cos^2 directional spreading, amplitudes scaled so Hs = 4 sqrt(m0)
on the discrete modes, random phases supplied by the caller.
"""
from __future__ import annotations

import math

import numpy as np

from .spectral import Grid


def stokes2(grid: Grid, mode: int, ka: float, phase: float = 0.0):
    """Half spectra (eta_hat, phis_hat) of a second-order Stokes wave on mode
    `mode` along x.  Linear dispersion w^2 = g k tanh(kh).
    eta  = a cos t + a2 cos 2t,   a2 = (k a^2/4) cosh kh (2 + cosh 2kh)/sinh^3 kh
    phis = phi1(x,0) + phi2(x,0) + eta1 * dphi1/dz(x,0), where
    phi1 = (g a / w) cosh k(z+h)/cosh kh sin t and
    phi2 = (3/8) w a^2 cosh 2k(z+h)/sinh^4 kh sin 2t  (deep water: a2 = k a^2/2, phi2 = 0)."""
    k = 2 * math.pi * mode / grid.lx
    a = ka / k
    g = grid.g
    if grid.deep:
        w = math.sqrt(g * k)
        a2 = 0.5 * k * a * a
        b2 = 0.0
    else:
        h = grid.depth
        w = math.sqrt(g * k * math.tanh(k * h))
        a2 = (k * a * a / 4) * math.cosh(k * h) * (2 + math.cosh(2 * k * h)) / math.sinh(k * h) ** 3
        b2 = 0.375 * w * a * a * math.cosh(2 * k * h) / math.sinh(k * h) ** 4
    b1 = g * a / w                       # phi1(x,0) = b1 sin t
    b_cross = 0.5 * w * a * a            # a cos t * (w a sin t) = (w a^2 / 2) sin 2t
    eta = np.zeros((grid.ny, grid.nxh), dtype=np.complex128)
    phi = np.zeros_like(eta)
    e1 = np.exp(1j * phase)
    # cos t -> coefficient 1/2 at +k ; sin t -> coefficient 1/(2i) at +k
    eta[0, mode] += 0.5 * a * e1
    eta[0, 2 * mode] += 0.5 * a2 * e1 * e1
    phi[0, mode] += b1 / (2j) * e1
    phi[0, 2 * mode] += (b2 + b_cross) / (2j) * e1 * e1
    return eta, phi, {"k": k, "a": a, "omega": w, "a2": a2}


def jonswap_omega(omega: np.ndarray, omega_p: float, gamma: float, g: float) -> np.ndarray:
    """JONSWAP frequency spectrum with unit Phillips constant: the
    Pierson-Moskowitz shape g^2 w^-5 exp(-5/4 (w_p/w)^4), which peaks at w_p,
    times the peak enhancement gamma^r with r = exp(-(w - w_p)^2 / (2 s^2 w_p^2))
    and the published widths s = 0.07 below the peak and 0.09 above it."""
    sig = np.where(omega <= omega_p, 0.07, 0.09)
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        s = g * g * omega ** -5.0 * np.exp(-1.25 * (omega_p / omega) ** 4) \
            * gamma ** np.exp(-((omega - omega_p) ** 2) / (2 * sig * sig * omega_p * omega_p))
    return np.where(omega > 0, s, 0.0)


def spreading_cos2(theta: np.ndarray) -> np.ndarray:
    """Directional spreading D(theta) = (2/pi) cos^2(theta) on |theta| < pi/2,
    zero behind; theta is measured from the +x axis (the mean direction)."""
    theta = np.asarray(theta, dtype=np.float64)
    return np.where(np.abs(theta) < math.pi / 2, (2 / math.pi) * np.cos(theta) ** 2, 0.0)


def jonswap(grid: Grid, hs: float, kp: float, gamma: float, phases: np.ndarray,
            spreading: str = "cos2"):
    """Half spectra (eta_hat, phis_hat) of a linear JONSWAP sea.

    S(k, theta) = S_w(w(k)) dw/dk D(theta) / k with w = sqrt(g k) and
    D = (2/pi) cos^2(theta) on |theta| < pi/2 ("cos2"), or all energy on
    ky = 0 ("uni", also used in 2D).  Each mode with kx > 0 carries the
    component a cos(k.x + phase); a = sqrt(2 S dkx dky).  Potential of the
    linear wave travelling along +k: phis_hat = -i (g/w) eta_hat."""
    g = grid.g
    KX, KY, K = grid.kvec()
    dkx = 2 * math.pi / grid.lx
    dky = 2 * math.pi / grid.ly if grid.ny > 1 else 1.0
    wp = math.sqrt(g * kp)
    w = np.sqrt(g * K)
    with np.errstate(divide="ignore", invalid="ignore"):
        sk = jonswap_omega(w, wp, gamma, g) * np.where(w > 0, g / (2 * w), 0.0)
    if grid.ny == 1 or spreading == "uni":
        # all energy on the ky = 0 row: a = sqrt(2 S_k(kx) dkx)
        dens = np.where((KY == 0) & (KX > 0), sk / dky, 0.0)
    else:
        d = spreading_cos2(np.arctan2(KY, KX))
        with np.errstate(divide="ignore", invalid="ignore"):
            dens = np.where((K > 0) & (KX > 0), sk * d / K, 0.0)
    amp = np.sqrt(2 * dens * dkx * dky)
    amp[:, -1] = 0.0
    if grid.ny > 1:
        amp[grid.ny // 2, :] = 0.0
    m0 = 0.5 * float(np.sum(amp * amp))
    amp *= hs / (4 * math.sqrt(m0))
    eta = 0.5 * amp * np.exp(1j * phases)
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(w > 0, -1j * (g / w) * eta, 0.0)
    return eta.astype(np.complex128), phi.astype(np.complex128)
