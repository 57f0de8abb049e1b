"""Pins of the stream-function oracle: the linear (Airy) limit, Stokes'
third-order dispersion and second-harmonic amplitude, the free-surface
conditions between the collocation points (converging with N), and the
pressure vanishing on the free surface."""
import math

import numpy as np

from oracle import stream


def test_airy_limit():
    L, d = 2 * math.pi, 1.2
    k = 1.0
    H = 1e-5
    sol = stream.solve(d, H, L, 8)
    th = math.tanh(k * d)
    assert abs(sol["c"] - math.sqrt(th / k)) < 1e-9
    # deviations are the second-order terms, relative size k H
    assert abs(sol["B"][0] - 0.5 * k * H / math.sqrt(th)) < 1e-4 * k * H
    m = np.arange(9)
    assert np.allclose(sol["eta"], 0.5 * H * np.cos(m * math.pi / 8), atol=1e-4 * H)


def test_stokes_dispersion_and_second_harmonic():
    L, d = 2 * math.pi, 2.0   # k = 1, kh = 2
    for ka in (0.05, 0.1):
        # H from the first-harmonic amplitude a (H = 2a to this order)
        sol = stream.solve(d, 2 * ka, L, 16)
        th = math.tanh(d)
        c3 = math.sqrt(th * (1 + ka ** 2 * (9 - 10 * th ** 2 + 9 * th ** 4) / (8 * th ** 4)))
        assert abs(sol["c"] - c3) / c3 < 2 * ka ** 4
        E = stream.eta_coefficients(sol)
        a2 = (ka ** 2 / 4) * math.cosh(d) * (2 + math.cosh(2 * d)) / math.sinh(d) ** 3
        assert abs(E[2] - a2) / a2 < 3 * ka, (ka, E[2], a2)


def test_surface_conditions_between_points_converge():
    L, d, H = 2 * math.pi, 1.5, 0.3   # ka ~ 0.15
    errs = []
    for N in (8, 16):
        sol = stream.solve(d, H, L, N)
        # half-way between collocation points, on the interpolated surface
        X = (np.arange(N) + 0.5) * math.pi / (N * sol["k"])
        f = stream.fields(sol, X, np.zeros_like(X), 0.0)
        eta = f["eta"]
        f = stream.fields(sol, X, eta, 0.0)
        # dynamic: p = 0 on the surface; kinematic: eta_t + u eta_x = w
        h = 1e-6
        ex = (stream.fields(sol, X + h, np.zeros_like(X), 0.0)["eta"]
              - stream.fields(sol, X - h, np.zeros_like(X), 0.0)["eta"]) / (2 * h)
        errs.append(max(np.abs(f["p"]).max(), np.abs(f["eta_t"] + f["u"] * ex - f["w"]).max()))
    assert errs[1] < 1e-6 and errs[1] < errs[0] / 20, errs


def test_pressure_vanishes_at_the_collocation_points():
    sol = stream.solve(1.0, 0.2, 2 * math.pi, 12)
    X = np.arange(13) * math.pi / (12 * sol["k"])
    f = stream.fields(sol, X, sol["eta"], 0.0)
    assert np.abs(f["p"]).max() < 1e-10
    assert np.abs(f["eta"] - sol["eta"]).max() < 1e-13
