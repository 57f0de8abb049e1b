"""Pins of the oracle's initial sea state (the JONSWAP seas of Sec. 3.1.2 and
the reconstruction example of Sec. 3.2.2, which give only Tp, Hs and gamma).

The reading is the standard JONSWAP shape with the published peak widths
0.07 / 0.09 and cos^2 directional spreading.  Each pin below is a property
that shape must have, fixed by the mathematics or by an independent
published fit, not a retyped formula:

* the Pierson-Moskowitz base (gamma = 1) integrates to g^2 / (5 w_p^4) with a
  unit Phillips constant (closed form) and peaks exactly at w_p;
* the enhancement at the peak is exactly gamma, and the enhancement falls to
  half its logarithm at w_p (1 -+ s sqrt(2 ln 2)) with s = 0.07 below and
  0.09 above (so the peak is wider on the high-frequency side);
* the zeroth moment relative to Pierson-Moskowitz follows the widely used
  normalisation 1 / (1 - 0.287 ln gamma) (a fit good to about 1 % for
  gamma in [1, 5]);
* the spreading integrates to one over direction, with D(0) = 2/pi, and on a
  square grid the modes (5, 0), (4, 3), (3, 4) of equal |k| carry amplitudes
  in the ratio cos(theta) = 1 : 0.8 : 0.6;
* on a fine one-dimensional grid, the frequency spectrum recovered from the
  discrete amplitudes peaks at the mode nearest w_p and sums to Hs^2 / 16.

Planted mistakes (a swapped pair of widths, a missing factor 2 in the
enhancement exponent, a wrong base exponent or coefficient, a spreading
normalised to 1/pi) are run through the same checks and must fail one of
them.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import Grid, sea

LAM = 2 * math.pi


def _m0(spec, wp, gamma, g):
    f = lambda w: float(spec(np.array([w]), wp, gamma, g)[0])  # noqa: E731
    return quad(f, 0.05 * wp, 40 * wp, limit=800, points=[0.8 * wp, wp, 1.2 * wp])[0]


def _shape_failures(spec):
    """Every pin of the frequency spectrum that `spec` violates."""
    bad = []
    g = 9.81
    for wp in (0.7, 1.0, 2.5):
        # base shape: closed-form moment and peak position
        m0 = _m0(spec, wp, 1.0, g)
        if abs(m0 / (g * g / (5 * wp ** 4)) - 1) > 1e-6:
            bad.append(("pm_m0", wp, m0))
        w = np.linspace(0.5 * wp, 2 * wp, 300001)
        for gamma in (1.0, 3.3, 5.0):
            pk = w[np.argmax(spec(w, wp, gamma, g))]
            if abs(pk / wp - 1) > 2e-5:
                bad.append(("peak", wp, gamma, pk))
        # enhancement at the peak and its half-log widths on both sides
        for gamma in (2.0, 3.3, 5.0):
            pm = lambda x: spec(np.array([x]), wp, 1.0, g)[0]  # noqa: E731
            js = lambda x: spec(np.array([x]), wp, gamma, g)[0]  # noqa: E731
            if abs(js(wp) / pm(wp) - gamma) > 1e-12 * gamma:
                bad.append(("enh", wp, gamma))
            for side, s in ((-1, 0.07), (1, 0.09)):
                x = wp * (1 + side * s * math.sqrt(2 * math.log(2)))
                r = math.log(js(x) / pm(x)) / math.log(gamma)
                if abs(r - 0.5) > 1e-9:
                    bad.append(("width", side, wp, gamma, r))
    # moment against the published normalisation fit
    for gamma in (1.0, 2.0, 3.3, 5.0):
        r = _m0(spec, 1.0, gamma, g) / (g * g / 5.0)
        if abs(r * (1 - 0.287 * math.log(gamma)) - 1) > 0.01:
            bad.append(("m0_fit", gamma, r))
    return bad


# -- planted mistakes: each is the oracle's spectrum with one plausible slip
def _swapped_widths(w, wp, gamma, g):
    sig = np.where(w <= wp, 0.09, 0.07)
    return g * g * w ** -5.0 * np.exp(-1.25 * (wp / w) ** 4) \
        * gamma ** np.exp(-((w - wp) ** 2) / (2 * sig * sig * wp * wp))


def _no_half(w, wp, gamma, g):
    sig = np.where(w <= wp, 0.07, 0.09)
    return g * g * w ** -5.0 * np.exp(-1.25 * (wp / w) ** 4) \
        * gamma ** np.exp(-((w - wp) ** 2) / (sig * sig * wp * wp))


def _exp4(w, wp, gamma, g):
    sig = np.where(w <= wp, 0.07, 0.09)
    return g * g * w ** -4.0 * np.exp(-1.25 * (wp / w) ** 4) \
        * gamma ** np.exp(-((w - wp) ** 2) / (2 * sig * sig * wp * wp))


def _coef1(w, wp, gamma, g):
    sig = np.where(w <= wp, 0.07, 0.09)
    return g * g * w ** -5.0 * np.exp(-1.0 * (wp / w) ** 4) \
        * gamma ** np.exp(-((w - wp) ** 2) / (2 * sig * sig * wp * wp))


def _gamma_sq(w, wp, gamma, g):
    sig = np.where(w <= wp, 0.07, 0.09)
    return g * g * w ** -5.0 * np.exp(-1.25 * (wp / w) ** 4) \
        * (gamma * gamma) ** np.exp(-((w - wp) ** 2) / (2 * sig * sig * wp * wp))


def test_jonswap_shape_pins():
    assert _shape_failures(sea.jonswap_omega) == []


@pytest.mark.parametrize("mutant", [_swapped_widths, _no_half, _exp4, _coef1, _gamma_sq])
def test_jonswap_pins_catch_planted_mistakes(mutant):
    assert _shape_failures(mutant), mutant.__name__


def _spreading_failures(D):
    bad = []
    tot = quad(lambda t: float(D(np.array([t]))[0]), -math.pi, math.pi, points=[-math.pi / 2, 0, math.pi / 2])[0]
    if abs(tot - 1) > 1e-10:
        bad.append(("integral", tot))
    if abs(float(D(np.array([0.0]))[0]) - 2 / math.pi) > 1e-15:
        bad.append(("peak",))
    if float(D(np.array([math.pi * 0.75]))[0]) != 0.0:
        bad.append(("behind",))
    return bad


def test_spreading_normalised_and_one_sided():
    assert _spreading_failures(sea.spreading_cos2) == []
    # planted: normalised to 1/pi, and a cos spreading in place of cos^2
    assert _spreading_failures(lambda t: np.where(np.abs(t) < math.pi / 2, np.cos(t) ** 2 / math.pi, 0.0))
    assert _spreading_failures(lambda t: np.where(np.abs(t) < math.pi / 2, 0.5 * np.cos(t), 0.0))


def test_discrete_sea_directional_amplitudes():
    """Square grid, equal |k| = 5 dk: amplitudes go as cos(theta) (the
    amplitude is the square root of S D dkx dky), mirrored in ky, and modes
    across the mean direction carry nothing."""
    n = 32
    g = Grid(nx=n, ny=n, lx=n * LAM / 6.4, ly=n * LAM / 6.4, depth=-1.0, order_m=3)
    eh, _ = sea.jonswap(g, 0.02 * LAM, 1.0, 3.3, synth.mode_phases(3, n, g.nxh))
    a = np.abs(eh)
    ref = a[0, 5]
    assert ref > 0
    assert abs(a[3, 4] / ref - 0.8) < 1e-12 and abs(a[4, 3] / ref - 0.6) < 1e-12
    assert abs(a[n - 3, 4] / ref - 0.8) < 1e-12 and abs(a[n - 4, 3] / ref - 0.6) < 1e-12
    assert a[5, 0] == 0.0 and a[n - 5, 0] == 0.0


def test_discrete_unidirectional_spectrum_peak_and_hs():
    """1D sea over 200 peak wavelengths (dk = kp/200): the frequency spectrum
    recovered from the amplitudes, S_w = (a^2/2)/dk * dk/dw with dk/dw = 2w/g
    in deep water, peaks at the mode nearest w_p and its modes hold Hs^2/16."""
    n = 4096
    g = Grid(nx=n, ny=1, lx=200 * LAM, ly=1.0, depth=-1.0, order_m=3)
    hs = 0.02 * LAM
    eh, _ = sea.jonswap(g, hs, 1.0, 3.3, synth.mode_phases(4, 1, g.nxh))
    a = 2 * np.abs(eh[0])
    k = 2 * math.pi * np.arange(g.nxh) / g.lx
    w = np.sqrt(g.g * k)
    sw = 0.5 * a * a / (k[1] - k[0]) * 2 * w / g.g
    i = int(np.argmax(sw))
    assert abs(w[i] - 1.0) <= 0.5 * (w[i + 1] - w[i - 1]), w[i]
    assert abs(0.5 * np.sum(a * a) - hs * hs / 16) < 1e-14
