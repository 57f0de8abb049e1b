"""Cell-side use of the incident fields in the CFD solver, FP64 (test
infrastructure: only tests, the smoke check and the bench's CPU baseline
use this package).

* Incident volume fraction (Sec. 3.2.2, the VOF field reconstructed from the
  free-surface elevation eta_I): reading = the fraction of a cell's height
  below eta_I taken at the cell centre, alpha_I = clamp((eta_I - z_lo) /
  (z_hi - z_lo), 0, 1) with z_lo, z_hi = z_c -+ dz/2.  The paper shows the
  reconstructed field but gives no formula; cells are treated as vertical
  prisms with a flat interface across the cell.
* Modified incident pressure (Sec. 2.1.3, Eq. pIStar): p_I* = rho p_I /
  rho_I with rho the two-phase density; reading = the VOF mixture
  rho = alpha rho_water + (1 - alpha) rho_air, rho_I = rho_water.
* Relaxation zones (Sec. 4.2, Eq. weightFunction, swUcRelax, swVOFRelax):
  weight omega(x) = -2 x^3 + 3 x^2 of the non-dimensional distance x in
  [0, 1] from the inner boundary of the zone (x = 1 at the outer boundary);
  the complementary velocity becomes (1 - omega) u_C and the volume
  fraction omega alpha_I + (1 - omega) alpha_CFD.  Outside a zone (x <= 0)
  nothing changes; x is clamped to [0, 1].
"""
from __future__ import annotations

import numpy as np


def incident_alpha(eta: np.ndarray, zc: np.ndarray, dz: np.ndarray) -> np.ndarray:
    """Fraction of each cell's height [zc - dz/2, zc + dz/2] below eta."""
    eta, zc, dz = (np.asarray(a, dtype=np.float64) for a in (eta, zc, dz))
    zlo = zc - 0.5 * dz
    return np.clip((eta - zlo) / dz, 0.0, 1.0)


def pstar(p: np.ndarray, alpha: np.ndarray, rho_water: float, rho_air: float) -> np.ndarray:
    """p_I* = rho p_I / rho_I with rho = alpha rho_water + (1 - alpha) rho_air."""
    p, alpha = (np.asarray(a, dtype=np.float64) for a in (p, alpha))
    rho = alpha * rho_water + (1.0 - alpha) * rho_air
    return rho * p / rho_water


def relax_weight(x: np.ndarray) -> np.ndarray:
    """omega = -2 x^3 + 3 x^2 on x clamped to [0, 1]."""
    x = np.clip(np.asarray(x, dtype=np.float64), 0.0, 1.0)
    return -2.0 * x ** 3 + 3.0 * x ** 2


def relax(x: np.ndarray, alpha_i: np.ndarray, alpha_cfd: np.ndarray, uc: np.ndarray):
    """Relaxed (alpha, u_C): omega alpha_I + (1 - omega) alpha_CFD and
    (1 - omega) u_C (uc: [3][n] or [2][n])."""
    w = relax_weight(x)
    alpha_i, alpha_cfd, uc = (np.asarray(a, dtype=np.float64) for a in (alpha_i, alpha_cfd, uc))
    return w * alpha_i + (1.0 - w) * alpha_cfd, (1.0 - w)[None, :] * uc
