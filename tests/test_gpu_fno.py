"""GPU parity of the surrogate network (spectral neural operator) against the
FP64 oracle with the same BF16 quantisation points: the matrix-core GEMM,
forward pass, loss, every parameter gradient and the input gradient
(relative L2 <= 1e-4 per tensor, 5e-4 for the gradients fed by FP32
transforms: the two sides then differ only in FP32 vs FP64 accumulation and
in BF16 rounding decisions near ties), and the Adam update."""
import numpy as np

import c18
import pytest
import torch

from oracle import fno as F

pytestmark = pytest.mark.gpu
TOL = 1e-4
# Gradients of the spectral weights and of the input: their BF16 factors
# come out of FP32 transforms of whole fields, whose error is relative to the
# field's norm, so a low-amplitude value carries a larger relative error and
# flips its BF16 rounding against the FP64 side (a 2^-8 change of one term
# of a short sum) more often.
TOL_R = 5e-4


def rel(a, b):
    """Relative L2 error.  The network's max-abs measure is not bounded at
    the same level: where the two sides' FP32 and FP64 activations straddle
    a bfloat16 rounding boundary, one GEMM input differs by one bfloat16 unit
    (2^-8 relative), a local error that the L2 measure averages and the
    max-abs measure does not (measured up to 1.7e-3 of the largest output
    with 4 channels, 3e-4 at the full size)."""
    return c18.rel_l2(a, b)


@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (70, 130, 45), (1, 257, 3), (200, 33, 300), (96, 132, 100)])
def test_gemm_bf16_matches_rounded_fp64(gpu_lib, M, N, K):
    from paper_2005_12716_amd import lib
    rng = np.random.default_rng(M * 1000 + N + K)
    a = rng.standard_normal((M, K)).astype(np.float32)
    b = rng.standard_normal((K, N)).astype(np.float32)
    c = lib.gemm_bf16(torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")).cpu().numpy()
    ref = F.to_bf16(a) @ F.to_bf16(b)
    # FP32 accumulation of K products of bf16 values
    assert np.abs(c - ref).max() <= 1e-6 * K * np.abs(F.to_bf16(a)).max() * np.abs(F.to_bf16(b)).max() * 4
    assert rel(c, ref) < 1e-6


def _setup(lib, cfg, B, seed):
    rng = np.random.default_rng(seed)
    P = F.init_params(cfg, rng)
    # non-zero biases so that their gradients and their use are exercised
    for k in list(P):
        if k[0] in "bc":
            P[k] = 0.1 * rng.standard_normal(P[k].shape)
    desc = lib.fno_desc(cfg.n, cfg.channels, cfg.layers, cfg.p_modes, cfg.q_modes, cfg.hidden, max_batch=B,
                        in_channels=cfg.in_channels)
    vec = lib.fno_pack(desc, P)
    P32 = lib.fno_unpack(desc, vec)  # the FP32 values both sides use
    x = rng.standard_normal((B, cfg.in_channels, cfg.n, cfg.n)).astype(np.float32)
    return desc, vec, P32, x


SMALL = [F.FnoConfig(n=64, channels=8, layers=2, p_modes=8, q_modes=7, hidden=16),
         F.FnoConfig(n=128, channels=6, layers=3, p_modes=5, q_modes=9, hidden=10),
         F.FnoConfig(n=64, channels=12, layers=2, p_modes=6, q_modes=10, hidden=20, in_channels=4),
         F.FnoConfig(n=1024, channels=4, layers=1, p_modes=8, q_modes=7, hidden=8)]


@pytest.mark.parametrize("cfg", SMALL, ids=["n64c8", "n128c6", "n64c12in4", "n1024c4"])
def test_fno_forward_backward_parity(gpu_lib, cfg):
    from paper_2005_12716_amd import lib
    B = 2
    desc, vec, P, x = _setup(lib, cfg, B, 11)
    net = lib.Fno(desc, vec)
    xd = torch.tensor(x, device="cuda")
    y = net.forward(xd).cpu().numpy()
    yr, cache = F.forward(P, x.astype(np.float64), cfg, bf16=True)
    assert rel(y, yr) < TOL
    assert y.shape == (B, 2, cfg.n, cfg.n)
    t = np.random.default_rng(5).standard_normal(y.shape).astype(np.float32)
    Lg, gy = net.loss(torch.tensor(y, device="cuda"), torch.tensor(t, device="cuda"))
    Lr, gyr = F.loss(y.astype(np.float64), t.astype(np.float64))
    assert abs(Lg - Lr) <= 1e-5 * Lr
    assert rel(gy.cpu().numpy(), gyr) < 1e-5
    # backward from the oracle's own upstream gradient
    gx = net.backward(xd, torch.tensor(gyr.astype(np.float32), device="cuda"), want_gx=True).cpu().numpy()
    G = F.backward(P, cache, gyr.astype(np.float32).astype(np.float64), cfg, bf16=True)
    Gg = lib.fno_unpack(desc, net.get(1))
    for name, _ in lib.fno_names(desc):
        assert rel(Gg[name], G[name]) < (TOL_R if name.startswith("R") else TOL), name
    assert rel(gx, G["x"]) < TOL_R
    net.close()


# Channel counts 32, 64 and 128 at batches up to 8 take the small-batch
# spectral mixing (vector ALUs, one wavefront per mode); batch 3 runs the
# batch-4 form with one sample masked.
MIX_SMALL = [(F.FnoConfig(n=64, channels=32, layers=2, p_modes=8, q_modes=7, hidden=16), 1),
             (F.FnoConfig(n=64, channels=128, layers=1, p_modes=6, q_modes=5, hidden=16), 3),
             (F.FnoConfig(n=64, channels=64, layers=1, p_modes=5, q_modes=4, hidden=8, in_channels=4), 8)]


@pytest.mark.parametrize("cfg,B", MIX_SMALL, ids=["c32b1", "c128b3", "c64b8"])
def test_fno_forward_parity_small_batch_mixing(gpu_lib, cfg, B):
    from paper_2005_12716_amd import lib
    desc, vec, P, x = _setup(lib, cfg, B, 13)
    net = lib.Fno(desc, vec)
    y = net.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    yr, _ = F.forward(P, x.astype(np.float64), cfg, bf16=True)
    assert rel(y, yr) < TOL
    # each sample as computed alone
    for b in range(B):
        yb = net.forward(torch.tensor(x[b:b + 1], device="cuda")).cpu().numpy()
        assert rel(yb[0], yr[b]) < TOL
    net.close()


def test_fno_adam_step_and_bf16_refresh(gpu_lib):
    from paper_2005_12716_amd import lib
    cfg = SMALL[0]
    desc, vec, P, x = _setup(lib, cfg, 2, 3)
    net = lib.Fno(desc, vec)
    xd = torch.tensor(x, device="cuda")
    t = torch.tensor(np.random.default_rng(9).standard_normal(x.shape).astype(np.float32), device="cuda")
    lr = 1e-3
    L0 = net.train_step(xd, t, lr)
    g = net.get(1).astype(np.float64)
    w1 = net.get(0).astype(np.float64)
    # first Adam step: m = (1-b1) g, v = (1-b2) g^2, bias-corrected -> g / (|g| + eps)
    step = w1 - vec.astype(np.float64)
    expect = -lr * g / (np.abs(g) + 1e-8)
    assert np.abs(step - expect).max() < 1e-6
    m = net.get(2)
    assert np.allclose(m, 0.1 * g, rtol=1e-6, atol=1e-12)
    # the BF16 copy follows the masters: same output as a fresh handle on w1
    y1 = net.forward(xd).cpu().numpy()
    other = lib.Fno(desc, w1.astype(np.float32))
    assert np.array_equal(other.forward(xd).cpu().numpy(), y1)
    # and a few steps reduce the loss on a fixed batch
    losses = [net.train_step(xd, t, lr) for _ in range(5)]
    assert losses[-1] < L0
    other.close()
    net.close()


# At the full size the two sides' activations differ by ~1e-5 relative
# (FP32 vs FP64 through 8 layers), which flips the BF16 rounding of a
# fraction p ~ 1e-5 / 2^-8 of the GEMM inputs by one BF16 unit (2^-8): a sum
# over many such products then differs by ~ sqrt(p) 2^-8 ~ 2e-4 relative (a
# few times that for the long reductions of the weight gradients, and
# growing with the number of layers a gradient has crossed: 4e-4 at the
# projection, 1.8e-3 at the first layer in the measured case).
TOL_FULL_GRAD = 5e-3


def test_fno_full_size_forward_backward_parity(gpu_lib):
    """The surrogate configuration (256^2, 64 channels, 8 layers, p < 32,
    |q| <= 31, projection width 128) with one sample: forward output and the
    gradients of a few layers against the oracle."""
    from paper_2005_12716_amd import lib
    cfg = F.FnoConfig()
    desc, vec, P, x = _setup(lib, cfg, 1, 21)
    net = lib.Fno(desc, vec)
    xd = torch.tensor(x, device="cuda")
    y = net.forward(xd).cpu().numpy()
    yr, cache = F.forward(P, x.astype(np.float64), cfg, bf16=True)
    print("full-size forward error", rel(y, yr))
    assert rel(y, yr) < TOL
    gy = np.random.default_rng(2).standard_normal(y.shape).astype(np.float32)
    net.backward(xd, torch.tensor(gy, device="cuda"))
    G = F.backward(P, cache, gy.astype(np.float64), cfg, bf16=True)
    Gg = lib.fno_unpack(desc, net.get(1))
    errs = {name: rel(Gg[name], G[name]) for name in ["Q2", "c2", "Q1", "W8", "R8", "b8", "R1", "W1", "W0", "b0"]}
    print("full-size gradient errors", errs)
    for name, e in errs.items():
        assert e < TOL_FULL_GRAD, name
    net.close()


def test_fno_full_size_layer_by_layer_parity(gpu_lib):
    """The surrogate configuration with one sample, each layer checked on the
    GPU's own inputs: the oracle takes the activations the GPU stored in its
    forward pass and the upstream gradients its backward pass traced, so both
    sides round the same FP32 values to BF16 at every GEMM input and differ
    only in accumulation (FP32 against FP64) and in the FP32 transforms of the
    spectral branch.  Each layer's pre-activation, every parameter gradient,
    the gradient each layer passes down and the input gradient: relative L2
    within 1e-4 (the pre-activations under both measures)."""
    from paper_2005_12716_amd import lib
    cfg = F.FnoConfig()
    desc, vec, P, x = _setup(lib, cfg, 1, 21)
    net = lib.Fno(desc, vec)
    trace = torch.empty(net.trace_floats(), dtype=torch.float32, device="cuda")
    net.set_trace(trace)
    xd = torch.tensor(x, device="cuda")
    net.forward(xd)
    A = net.activations(1)
    gy = np.random.default_rng(2).standard_normal((1, 2, cfg.n, cfg.n)).astype(np.float32)
    gx = net.backward(xd, torch.tensor(gy, device="cuda"), want_gx=True).cpu().numpy()
    Gg = lib.fno_unpack(desc, net.get(1))
    T = trace.cpu().numpy()
    net.set_trace(None)
    C, H, n, L = cfg.channels, cfg.hidden, cfg.n, cfg.layers
    blk = C * n * n
    gz = [T[l * blk:(l + 1) * blk].reshape(1, C, n, n).astype(np.float64) for l in range(L)]
    gv0 = T[L * blk:(L + 1) * blk].reshape(1, C, n, n).astype(np.float64)
    gzq = T[(L + 1) * blk:(L + 1) * blk + H * n * n].reshape(1, H, n, n)
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    errs = {}
    Gh, gz1, gvL = F.head_backward(P, f64(gy), f64(A["h"]), f64(A["zq"]), f64(A["v"][L]), bf16=True)
    errs["dL/dzq"] = rel(gzq, gz1)
    for k, val in Gh.items():
        errs[k] = rel(Gg[k], val)
    errs[f"dL/dz{L} from the head"] = rel(gz[L - 1], gvL * F.gelu_grad(f64(A["z"][L - 1])))
    for l in range(L, 0, -1):
        u = f64(A["v"][l - 1])
        z, Uh = F.layer_forward(P, l, u, cfg, bf16=True)
        errs[f"z{l}"] = c18.both(A["z"][l - 1], z)
        errs[f"v{l} = gelu(z{l})"] = c18.both(A["v"][l], F.gelu(f64(A["z"][l - 1])))
        Gl, gu = F.layer_backward(P, l, u, Uh, gz[l - 1], cfg, bf16=True)
        for k, val in Gl.items():
            errs[k] = rel(Gg[k], val)
        if l > 1:
            errs[f"dL/dz{l - 1} from layer {l}"] = rel(gz[l - 2], gu * F.gelu_grad(f64(A["z"][l - 2])))
        else:
            errs["dL/dv0 from layer 1"] = rel(gv0, gu)
    Gx = F.lift_backward(P, gv0, f64(x), bf16=True)
    for k in ("W0", "b0"):
        errs[k] = rel(Gg[k], Gx[k])
    errs["x"] = rel(gx, Gx["x"])
    print("layer-by-layer errors", {k: f"{v:.2e}" for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not v < 1e-4}
    assert not bad, bad
    net.close()
