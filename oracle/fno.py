"""Spectral neural operator (Fourier neural operator) of the surrogate,
FP64 with a hand-written backward pass.  Test infrastructure only.

Nothing in the paper covers this part; it implements the learned surrogate
of the build's specification: lift (2 -> C channels, pointwise), L Fourier
layers v <- gelu(W v + b + K(v)), projection C -> 2C -> 2 (gelu between).
K(v) is the spectral convolution: v_hat = rfft2(v)/N^2 on the retained
modes S = {p in [0, P), q in [-Q, Q]} (p along the half-spectrum axis x),
per-mode complex channel mixing y_hat_o = sum_i v_hat_i R_io, a projection of
the p = 0 column onto Hermitian symmetry (pairs (q, -q) averaged with
conjugation, q = 0 real part), then v(x) = sum_S c_p Re(y_hat e^{ik.x}),
c_0 = 1, c_{p>0} = 2.  gelu is the tanh form.

Quantisation points: with bf16=True every GEMM input (activations and
weights, forward and backward) is rounded to bfloat16 (round to nearest
even), exactly where the GPU kernels round; accumulation stays FP64 here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def to_bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (via float32, round to nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def cbf16(z: np.ndarray) -> np.ndarray:
    return to_bf16(z.real) + 1j * to_bf16(z.imag)


_K = math.sqrt(2.0 / math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(_K * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    t = np.tanh(_K * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * _K * (1.0 + 3 * 0.044715 * z * z)


@dataclass
class FnoConfig:
    n: int = 256          # grid points per axis
    channels: int = 64
    layers: int = 8
    p_modes: int = 32     # p in [0, p_modes)
    q_modes: int = 31     # q in [-q_modes, q_modes]
    hidden: int = 128     # projection width (2 C)
    in_channels: int = 2  # network input: (eta, phis), or with the linearly propagated pair (4)


def retained(cfg: FnoConfig):
    """(q index into [0, n), p) of the retained modes, q-major order: q runs
    0..Q then -Q..-1 (index n-Q..n-1)."""
    qs = list(range(0, cfg.q_modes + 1)) + list(range(-cfg.q_modes, 0))
    return np.array([q % cfg.n for q in qs]), np.arange(cfg.p_modes), np.array(qs)


def init_params(cfg: FnoConfig, rng: np.random.Generator) -> dict:
    C, H = cfg.channels, cfg.hidden
    nq = 2 * cfg.q_modes + 1
    P = {"W0": rng.standard_normal((C, cfg.in_channels)) / math.sqrt(cfg.in_channels), "b0": np.zeros(C),
         "Q1": rng.standard_normal((H, C)) / math.sqrt(C), "c1": np.zeros(H),
         "Q2": rng.standard_normal((2, H)) / math.sqrt(H) * 0.1, "c2": np.zeros(2)}
    for l in range(cfg.layers):
        P[f"W{l + 1}"] = rng.standard_normal((C, C)) / math.sqrt(C)
        P[f"b{l + 1}"] = np.zeros(C)
        s = 1.0 / (C * C)
        P[f"R{l + 1}"] = s * (rng.uniform(-1, 1, (nq, cfg.p_modes, C, C))
                              + 1j * rng.uniform(-1, 1, (nq, cfg.p_modes, C, C)))
    return P


def hermitian_p0(a: np.ndarray, cfg: FnoConfig) -> np.ndarray:
    """Projection of the p = 0 column (axis -3 = q index in retained order,
    axis -2 = p) onto Hermitian symmetry; self-adjoint."""
    out = a.copy()
    Q = cfg.q_modes
    col = a[..., :, 0, :]  # [..., nq, C]
    new = col.copy()
    new[..., 0, :] = col[..., 0, :].real
    for q in range(1, Q + 1):
        iq, jq = q, 2 * Q + 1 - q  # +q and -q positions
        avg = 0.5 * (col[..., iq, :] + np.conj(col[..., jq, :]))
        new[..., iq, :] = avg
        new[..., jq, :] = np.conj(avg)
    out[..., :, 0, :] = new
    return out


def spec_forward(u: np.ndarray, cfg: FnoConfig) -> np.ndarray:
    """u [B, C, n, n] -> retained half-spectrum [B, nq, P, C] (rfft2 / n^2)."""
    qi, _, _ = retained(cfg)
    U = np.fft.rfft2(u) / (cfg.n * cfg.n)  # [B, C, n, n/2+1]
    S = U[:, :, qi, :cfg.p_modes]          # [B, C, nq, P]
    return np.transpose(S, (0, 2, 3, 1))


def spec_inverse(Y: np.ndarray, cfg: FnoConfig) -> np.ndarray:
    """[B, nq, P, C] retained modes (Hermitian p = 0 column assumed) ->
    sum_S c_p Re(Y e^{ik.x}) on the grid [B, C, n, n]."""
    qi, _, _ = retained(cfg)
    B, _, _, C = Y.shape
    big = np.zeros((B, C, cfg.n, cfg.n // 2 + 1), dtype=np.complex128)
    big[:, :, qi, :cfg.p_modes] = np.transpose(Y, (0, 3, 1, 2))
    return np.fft.irfft2(big, s=(cfg.n, cfg.n)) * (cfg.n * cfg.n)


def _cp(cfg):
    c = np.full(cfg.p_modes, 2.0)
    c[0] = 1.0
    return c


def _quant(bf16: bool):
    """The rounding applied to every GEMM input: BF16 (nearest even) or none."""
    if bf16:
        return to_bf16, cbf16
    return (lambda a: a), (lambda a: a)


def layer_forward(P: dict, l: int, v: np.ndarray, cfg: FnoConfig, bf16: bool = False):
    """Fourier layer l on its input v [B, C, n, n]: the pre-activation
    z = W_l v + b_l + (inverse transform of R_l times the retained modes of
    v); returns (z, retained modes of v)."""
    q, qc = _quant(bf16)
    Uh = spec_forward(v, cfg)                                   # [B, nq, P, C]
    Yh = np.einsum("bqpi,qpio->bqpo", qc(Uh), qc(P[f"R{l}"]))
    Yh = hermitian_p0(Yh, cfg)
    s = spec_inverse(Yh, cfg)
    z = np.einsum("oi,bixy->boxy", q(P[f"W{l}"]), q(v)) + P[f"b{l}"][None, :, None, None] + s
    return z, Uh


def forward(P: dict, x: np.ndarray, cfg: FnoConfig, bf16: bool = False):
    """x [B, in_channels, n, n] -> y [B, 2, n, n]; returns (y, cache)."""
    q, _ = _quant(bf16)
    cache = {"x": x}
    v = np.einsum("oi,bixy->boxy", q(P["W0"]), q(x)) + P["b0"][None, :, None, None]
    cache["v0"] = v
    for l in range(1, cfg.layers + 1):
        z, Uh = layer_forward(P, l, v, cfg, bf16)
        cache[f"u{l}"] = v
        cache[f"U{l}"] = Uh
        cache[f"z{l}"] = z
        v = gelu(z)
    cache["vL"] = v
    z1 = np.einsum("oi,bixy->boxy", q(P["Q1"]), q(v)) + P["c1"][None, :, None, None]
    h = gelu(z1)
    y = np.einsum("oi,bixy->boxy", q(P["Q2"]), q(h)) + P["c2"][None, :, None, None]
    cache["zq"] = z1
    cache["h"] = h
    return y, cache


def loss(y: np.ndarray, t: np.ndarray):
    """Mean over (sample, channel) of ||y - t||^2 / ||t||^2; returns (L, dL/dy)."""
    B = y.shape[0]
    d = y - t
    den = np.sum(t * t, axis=(2, 3), keepdims=True)
    L = float(np.mean(np.sum(d * d, axis=(2, 3), keepdims=True) / den))
    g = 2.0 * d / den / (B * 2)
    return L, g


def head_backward(P: dict, gy: np.ndarray, h: np.ndarray, zq: np.ndarray, vL: np.ndarray, bf16: bool = False):
    """Projection (Q1, c1, GELU, Q2, c2) backward from dL/dy: returns the
    head's parameter gradients, dL/dzq and dL/dv_L."""
    q, _ = _quant(bf16)
    G = {}
    G["Q2"] = np.einsum("boxy,bixy->oi", q(gy), q(h))
    G["c2"] = gy.sum(axis=(0, 2, 3))
    gh = np.einsum("oi,boxy->bixy", q(P["Q2"]), q(gy))
    gz1 = gh * gelu_grad(zq)
    G["Q1"] = np.einsum("boxy,bixy->oi", q(gz1), q(vL))
    G["c1"] = gz1.sum(axis=(0, 2, 3))
    gv = np.einsum("oi,boxy->bixy", q(P["Q1"]), q(gz1))
    return G, gz1, gv


def layer_backward(P: dict, l: int, u: np.ndarray, Uh: np.ndarray, gz: np.ndarray, cfg: FnoConfig,
                   bf16: bool = False):
    """Fourier layer l backward from dL/dz (its input u and retained modes Uh
    from the forward pass): returns the gradients of W_l, b_l, R_l and dL/du."""
    q, qc = _quant(bf16)
    cp = _cp(cfg)
    G = {}
    G[f"W{l}"] = np.einsum("boxy,bixy->oi", q(gz), q(u))
    G[f"b{l}"] = gz.sum(axis=(0, 2, 3))
    gu = np.einsum("oi,boxy->bixy", q(P[f"W{l}"]), q(gz))
    # spectral branch: gY = P(c_p n^2 rfft2(gz)/n^2) on S
    gY = spec_forward(gz, cfg) * (cfg.n * cfg.n) * cp[None, None, :, None]
    gY = hermitian_p0(gY, cfg)
    G[f"R{l}"] = np.einsum("bqpi,bqpo->qpio", np.conj(qc(Uh)), qc(gY))
    gU = np.einsum("bqpo,qpio->bqpi", qc(gY), np.conj(qc(P[f"R{l}"])))
    # adjoint of u -> rfft2(u)/n^2 on S: (1/n^2) Re sum_S gU e^{ik.x}
    stored = hermitian_p0(gU / cp[None, None, :, None], cfg)
    gu = gu + spec_inverse(stored, cfg) / (cfg.n * cfg.n)
    return G, gu


def lift_backward(P: dict, gv0: np.ndarray, x: np.ndarray, bf16: bool = False):
    """Lift (W0, b0) backward from dL/dv_0: its gradients and dL/dx."""
    q, _ = _quant(bf16)
    G = {}
    G["W0"] = np.einsum("boxy,bixy->oi", q(gv0), q(x))
    G["b0"] = gv0.sum(axis=(0, 2, 3))
    G["x"] = np.einsum("oi,boxy->bixy", q(P["W0"]), q(gv0))
    return G


def backward(P: dict, cache: dict, gy: np.ndarray, cfg: FnoConfig, bf16: bool = False) -> dict:
    G, _, gv = head_backward(P, gy, cache["h"], cache["zq"], cache["vL"], bf16)
    for l in range(cfg.layers, 0, -1):
        gz = gv * gelu_grad(cache[f"z{l}"])
        Gl, gv = layer_backward(P, l, cache[f"u{l}"], cache[f"U{l}"], gz, cfg, bf16)
        G.update(Gl)
    G.update(lift_backward(P, gv, cache["x"], bf16))
    return G


def linear_propagator(eta_hat, phis_hat, kmag, g: float, tau: float):
    """Exact solution over time tau of the linear deep-water problem (the
    M = 1 evolution eta_t = k phis, phis_t = -g eta), mode by mode:
    eta  <- cos(w tau) eta + (k/w) sin(w tau) phis,
    phis <- cos(w tau) phis - (g/w) sin(w tau) eta,  w = sqrt(g k);
    k = 0: eta unchanged, phis <- phis - g tau eta."""
    w = np.sqrt(g * kmag)
    c, s = np.cos(w * tau), np.sin(w * tau)
    safe = np.where(w > 0, w, 1.0)
    a = np.where(w > 0, kmag * s / safe, 0.0)
    b = np.where(w > 0, g * s / safe, g * tau)
    return c * eta_hat + a * phis_hat, c * phis_hat - b * eta_hat
