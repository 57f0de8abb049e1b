"""Pins of the oracle's interpolation in time between outputs of the wave
model: exact on cubics, the end values and slopes, the derivative of the
value, and fourth-order agreement with the HOS trajectory itself."""
import math

import numpy as np

import synth
from oracle import Grid, hos, sea


def test_exact_on_cubics_and_at_the_ends():
    c = np.array([0.3, -1.2, 0.7, 2.1])
    f = lambda t: c[0] + c[1] * t + c[2] * t**2 + c[3] * t**3
    df = lambda t: c[1] + 2 * c[2] * t + 3 * c[3] * t**2
    t0, t1 = 0.4, 1.1
    for t in (0.4, 0.55, 0.8, 1.1):
        y, dy = hos.hermite_in_time(f(t0), df(t0), f(t1), df(t1), t0, t1, t)
        assert abs(y - f(t)) < 1e-13 and abs(dy - df(t)) < 1e-12


def test_derivative_is_the_slope_of_the_value():
    rng = np.random.default_rng(1)
    y0, dy0, y1, dy1 = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    t, h = 0.37, 1e-6
    yp, _ = hos.hermite_in_time(y0, dy0, y1, dy1, 0.0, 1.0, t + h)
    ym, _ = hos.hermite_in_time(y0, dy0, y1, dy1, 0.0, 1.0, t - h)
    _, dy = hos.hermite_in_time(y0, dy0, y1, dy1, 0.0, 1.0, t)
    assert abs((yp - ym) / (2 * h) - dy) < 1e-8


def test_fourth_order_against_the_hos_trajectory():
    """Mean-level modes between two HOS outputs T_p/8 apart against the HOS
    state at that time: the error falls by about 16 when the gap halves."""
    lam = 2 * math.pi
    g = Grid(nx=32, ny=16, lx=5 * lam, ly=2.5 * lam, depth=-1.0, order_m=3)
    e, p = sea.jonswap(g, 0.03 * lam, 1.0, 3.3, synth.mode_phases(4, 16, 17), "cos2")
    dt = lam / 256
    errs = []
    for gap in (32, 16):
        e1, p1 = hos.run(g, e, p, dt, gap)
        em, pm = hos.run(g, e, p, dt, gap // 2)
        A0, A1, Am = (hos.mean_level_modes(g, a, b) for a, b in ((e, p), (e1, p1), (em, pm)))
        At0, _ = hos.mean_level_modes_t(g, e, p)
        At1, _ = hos.mean_level_modes_t(g, e1, p1)
        a, _ = hos.hermite_in_time(A0, At0, A1, At1, 0.0, gap * dt, gap * dt / 2)
        errs.append(np.linalg.norm(a - Am) / np.linalg.norm(Am))
    assert errs[0] < 5e-3 and 10 < errs[0] / errs[1] < 24, errs
