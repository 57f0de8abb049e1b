"""Pins of the oracle's spectral neural operator: finite-difference
gradients of every parameter and of the input, the spectral transform pair
on band-limited fields, the Hermitian projection, bfloat16 rounding against
its bit-level definition, and the exact linear propagator against the HOS
oracle at M = 1."""
import math
import zlib

import numpy as np
import pytest

from oracle import Grid, hos
from oracle import fno


def _tiny(in_channels=2):
    cfg = fno.FnoConfig(n=16, channels=6, layers=2, p_modes=4, q_modes=3, hidden=8, in_channels=in_channels)
    rng = np.random.default_rng(0)
    P = fno.init_params(cfg, rng)
    for k in P:  # non-trivial biases and a non-negligible output layer
        if k.startswith(("b", "c")):
            P[k] = 0.1 * rng.standard_normal(P[k].shape)
    P["Q2"] *= 10
    x = rng.standard_normal((2, in_channels, 16, 16))
    t = rng.standard_normal((2, 2, 16, 16))
    return cfg, P, x, t


def _loss(P, x, t, cfg):
    y, _ = fno.forward(P, x, cfg)
    return fno.loss(y, t)[0]


@pytest.mark.parametrize("name", ["W0", "b0", "W1", "b1", "R1", "W2", "R2", "Q1", "c1", "Q2", "c2"])
def test_gradients_match_finite_differences(name):
    cfg, P, x, t = _tiny()
    y, cache = fno.forward(P, x, cfg)
    _, gy = fno.loss(y, t)
    G = fno.backward(P, cache, gy, cfg)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    arr = P[name]
    idxs = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(4)]
    h = 1e-6
    for idx in idxs:
        parts = [1.0, 1j] if np.iscomplexobj(arr) else [1.0]
        for part in parts:
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name][idx] += h * part
            Pm[name][idx] -= h * part
            fd = (_loss(Pp, x, t, cfg) - _loss(Pm, x, t, cfg)) / (2 * h)
            an = G[name][idx].real if part == 1.0 else G[name][idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, idx, part, fd, an)


@pytest.mark.parametrize("in_channels", [2, 4])
def test_input_gradient_matches_finite_differences(in_channels):
    cfg, P, x, t = _tiny(in_channels)
    y, cache = fno.forward(P, x, cfg)
    _, gy = fno.loss(y, t)
    G = fno.backward(P, cache, gy, cfg)
    rng = np.random.default_rng(5)
    G0 = G["W0"]
    assert G0.shape == (6, in_channels) and G["x"].shape == x.shape
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (_loss(P, xp, t, cfg) - _loss(P, xm, t, cfg)) / (2 * h)
        assert abs(fd - G["x"][idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_spectral_pair_is_exact_on_band_limited_fields():
    cfg = fno.FnoConfig(n=32, channels=3, layers=1, p_modes=6, q_modes=5)
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((2, 11, 6, 3)) + 1j * rng.standard_normal((2, 11, 6, 3))
    Y = fno.hermitian_p0(Y, cfg)
    u = fno.spec_inverse(Y, cfg)
    # direct sum of c_p Re(Y e^{ik.x})
    _, _, qs = fno.retained(cfg)
    x = np.arange(32) * 2 * math.pi / 32
    X, Yg = np.meshgrid(x, x)  # X along axis 1 (p), Yg along axis 0 (q)
    ref = np.zeros((2, 3, 32, 32))
    for a, q in enumerate(qs):
        for p in range(6):
            c = 1.0 if p == 0 else 2.0
            ph = np.exp(1j * (p * X + q * Yg))
            ref += c * np.real(Y[:, a, p, :][:, :, None, None] * ph[None, None])
    assert np.abs(u - ref).max() < 1e-12
    assert np.abs(fno.spec_forward(u, cfg) - Y).max() < 1e-13


def test_hermitian_projection_is_an_orthogonal_projection():
    cfg = fno.FnoConfig(n=16, channels=2, layers=1, p_modes=4, q_modes=3)
    rng = np.random.default_rng(2)
    a = rng.standard_normal((2, 7, 4, 2)) + 1j * rng.standard_normal((2, 7, 4, 2))
    b = rng.standard_normal((2, 7, 4, 2)) + 1j * rng.standard_normal((2, 7, 4, 2))
    Pa, Pb = fno.hermitian_p0(a, cfg), fno.hermitian_p0(b, cfg)
    assert np.allclose(fno.hermitian_p0(Pa, cfg), Pa)
    assert abs(np.sum(np.real(np.conj(Pa) * b)) - np.sum(np.real(np.conj(a) * Pb))) < 1e-12


def test_bf16_rounding_definition():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-3, 65504.0])
    got = fno.to_bf16(vals)
    # bfloat16 keeps 8 significant bits; ties go to even
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2 ** -7 and got[3] == -2.5
    assert abs(got[4] - 3.0e-3) / 3.0e-3 < 2 ** -8 and got[5] == 65536.0


@pytest.mark.parametrize("depth", [-1.0, 2.0])
def test_linear_propagator_equals_m1_hos(depth):
    """At order M = 1 the HOS step is the linear problem, so a finely stepped
    M = 1 run pins the closed-form propagator (finite depth: k tanh(kh) in
    place of k)."""
    LAM = 2 * math.pi
    g = Grid(nx=32, ny=16, lx=32 * LAM / 6.4, ly=16 * LAM / 6.4, depth=depth, order_m=1)
    rng = np.random.default_rng(3)
    eh = (rng.standard_normal((16, 17)) + 1j * rng.standard_normal((16, 17))) * g.nyquist_mask() * 1e-2
    ph = (rng.standard_normal((16, 17)) + 1j * rng.standard_normal((16, 17))) * g.nyquist_mask() * 1e-2
    eh[0, 0] = 0
    for q in range(1, 8):
        eh[16 - q, 0] = np.conj(eh[q, 0])
        ph[16 - q, 0] = np.conj(ph[q, 0])
    ph[0, 0] = ph[0, 0].real
    tau = 10 * LAM / 64
    e1, p1 = hos.run(g, eh, ph, tau / 400, 400)
    _, _, K = g.kvec()
    kt = K * np.tanh(K * depth) if depth > 0 else K
    e2, p2 = fno.linear_propagator(eh, ph, kt, 1.0, tau)
    assert np.abs(e1 - e2).max() < 1e-9 and np.abs(p1 - p2).max() < 1e-9
