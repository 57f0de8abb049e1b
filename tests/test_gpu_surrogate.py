"""GPU checks of the surrogate rollout: network input features and the exact
linear propagation against the oracle, the training target, and the
advance loop's decisions (judged calls keep the HOS state bit for bit, guards
catch non-finite and energy-violating states, cool-down after a fallback,
the residual enters with its stated scaling)."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import Grid, hos, fno as F

pytestmark = pytest.mark.gpu
LAM = 2 * math.pi
N = 64
S = 5


def _realisation(lib, depth=-1.0, seed=7):
    lx = N * LAM / 6.4
    d = lib.hos_desc(3, N, N, lx, lx, depth, order_m=3, dt=LAM / 64)
    eh, ph = lib.sea_spectrum(d, kind=0, hs=0.02 * LAM, kp=1.0, gamma=3.3,
                              phases=synth.mode_phases(seed, N, N // 2 + 1))
    return d, eh, ph


def _net(lib, seed=1, in_channels=2):
    desc = lib.fno_desc(N, 8, 2, 8, 7, 16, max_batch=1, in_channels=in_channels)
    return desc, lib.fno_init(desc, seed)


def _sur(lib, depth=-1.0, in_channels=2, **kw):
    d, eh, ph = _realisation(lib, depth)
    h = lib.Hos(d, eh, ph)
    desc, vec = _net(lib, in_channels=in_channels)
    net = lib.Fno(desc, vec)
    sig = 0.02 * LAM / 4
    sd = lib.surrogate_desc(stride_s=S, sigma_eta=sig, sigma_phi=sig, rho=0.05, **kw)
    return d, eh, ph, h, desc, vec, net, lib.Surrogate(h, net, sd), sd


def _close(*objs):
    for o in objs:
        o.close()


def _grid(d):
    return Grid(nx=d.nx, ny=d.ny, lx=d.lx, ly=d.ly, depth=d.depth, order_m=3)


def _lin(d, eh, ph, tau):
    g = _grid(d)
    _, _, K = g.kvec()
    kt = K * np.tanh(K * d.depth) if d.depth > 0 else K
    return F.linear_propagator(eh, ph, kt, d.g, tau)


@pytest.mark.parametrize("depth", [-1.0, 1.5])
def test_features_and_linear_propagation(gpu_lib, depth):
    from paper_2005_12716_amd import lib
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, depth)
    x, lin = sur.features()
    x, lin = x.cpu().numpy(), lin.cpu().numpy()
    g = _grid(d)
    e_phys, p_phys, _ = h.state(lib.PHYSICAL)
    sig = sd.sigma_eta
    assert np.abs(x[0] - e_phys / sig).max() <= 1e-6 * np.abs(e_phys / sig).max()
    assert np.abs(x[1] - p_phys / sig).max() <= 1e-6 * np.abs(p_phys / sig).max()
    le, lp = _lin(d, eh, ph, S * d.dt)
    for got, ref in ((lin[0], g.to_phys(le, (N, N)) / sig), (lin[1], g.to_phys(lp, (N, N)) / sig)):
        assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()
    # the target of a pair is (x_next - lin) / rho, elementwise
    h.step(S)
    xn, _ = sur.features(want_lin=False)
    t = sur.target(xn, torch.tensor(lin, device="cuda")).cpu().numpy()
    ref = (xn.cpu().numpy() - lin) * np.float32(1.0 / sd.rho)
    assert np.allclose(t, ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())
    _close(sur, net, h)


def _hos_ref(lib, d, eh, ph, nsteps):
    ref = lib.Hos(d, eh, ph)
    ref.step(nsteps)
    out = ref.state()
    ref.close()
    return out


@pytest.mark.parametrize("in_channels", [2, 4])
def test_judged_calls_keep_the_hos_state(gpu_lib, in_channels):
    """tol = 0 and A = 1: every call is judged and falls back, so the rollout
    is the plain HOS run bit for bit."""
    from paper_2005_12716_amd import lib
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, tol=0.0, audit_every=1, cooldown=0, in_channels=in_channels)
    st = sur.advance(3)
    assert st["audits"] == 3 and st["fallbacks"] == 3 and st["surrogate_calls"] == 3 and st["hos_calls"] == 0
    assert st["max_audit_err"] > 0
    e, p, t = h.state()
    er, pr, tr = _hos_ref(lib, d, eh, ph, 3 * S)
    assert np.array_equal(e, er) and np.array_equal(p, pr) and t == tr
    _close(sur, net, h)


def test_cooldown_after_fallback(gpu_lib):
    from paper_2005_12716_amd import lib
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, tol=0.0, audit_every=1, cooldown=2)
    st = sur.advance(5)
    assert st["surrogate_calls"] == 2 and st["hos_calls"] == 3 and st["fallbacks"] == 2
    e, p, t = h.state()
    er, pr, tr = _hos_ref(lib, d, eh, ph, 5 * S)
    assert np.array_equal(e, er) and np.array_equal(p, pr)
    _close(sur, net, h)


def test_nan_weights_trip_the_guard(gpu_lib):
    from paper_2005_12716_amd import lib
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, tol=1.0, audit_every=1000, cooldown=0)
    bad = vec.copy()
    bad[0] = np.nan
    net.set(bad)
    st = sur.advance(2)
    assert st["guard_trips"] == 2 and st["fallbacks"] == 2 and st["audits"] == 2
    e, p, t = h.state()
    er, pr, tr = _hos_ref(lib, d, eh, ph, 2 * S)
    assert np.array_equal(e, er) and np.array_equal(p, pr)
    _close(sur, net, h)


def test_probation_judges_calls_until_they_pass(gpu_lib):
    """A network that never passes (tol = 0) is judged on every call under
    probation even with a long audit period, so the rollout keeps the HOS state
    throughout; with tol = inf the first `probation` calls are judged and the
    rest run unaudited between the A-th ones."""
    from paper_2005_12716_amd import lib
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, tol=0.0, audit_every=1000, cooldown=0, probation=2)
    st = sur.advance(4)
    assert st["audits"] == 4 and st["fallbacks"] == 4
    e, p, t = h.state()
    er, pr, tr = _hos_ref(lib, d, eh, ph, 4 * S)
    assert np.array_equal(e, er) and np.array_equal(p, pr)
    _close(sur, net, h)
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, tol=1e30, audit_every=3, cooldown=0, probation=2)
    st = sur.advance(7)
    # judged: calls 1, 2 (probation), then every 3rd network call: 3, 6
    assert st["audits"] == 4 and st["fallbacks"] == 0
    _close(sur, net, h)


def test_energy_guard(gpu_lib):
    from paper_2005_12716_amd import lib
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, tol=1.0, audit_every=1000, cooldown=0, energy_tol=1e-14)
    st = sur.advance(1)
    assert st["guard_trips"] == 1 and st["fallbacks"] == 1
    _close(sur, net, h)


def _with_output(lib, vec, desc, c2):
    P = lib.fno_unpack(desc, vec)
    P["Q2"] = np.zeros_like(P["Q2"])
    P["c2"] = np.array(c2, dtype=np.float64)
    return lib.fno_pack(desc, P)


@pytest.mark.parametrize("depth,in_channels", [(-1.0, 2), (1.5, 2), (-1.0, 4)])
def test_network_call_is_linear_plus_scaled_residual(gpu_lib, depth, in_channels):
    """Zero projection weights make the network output the constant c2: the
    state becomes Lin(X) plus rho sigma c2 in the k = 0 modes, with the mean
    of eta kept (mass)."""
    from paper_2005_12716_amd import lib
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, depth, in_channels, tol=1.0, audit_every=1000, cooldown=0,
                                                 probation=0, drift_tol=0.0)
    net.set(_with_output(lib, vec, desc, [0.75, -0.5]))
    st = sur.advance(2)
    assert st["surrogate_calls"] == 2 and st["audits"] == 0
    e, p, t = h.state()
    er, pr = eh, ph
    for _ in range(2):
        er, pr = _lin(d, er, pr, S * d.dt)
        pr = pr.copy()
        pr[0, 0] += sd.rho * sd.sigma_phi * (-0.5)
    assert np.abs(e - er).max() <= 1e-13 * np.abs(er).max()
    assert np.abs(p - pr).max() <= 1e-13 * np.abs(pr).max()
    assert abs(t - 2 * S * d.dt) < 1e-12
    _close(sur, net, h)


def test_network_call_over_the_integrating_factor_base(gpu_lib):
    """With the coarse integrating-factor RK4 base and a constant network
    output the state becomes the oracle's integrating-factor step plus the
    scaled residual in the k = 0 mode of phis (eta's mean kept)."""
    from paper_2005_12716_amd import lib
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, -1.0, 4, tol=1.0, audit_every=1000, cooldown=0, probation=0,
                                                 base_substeps=1, drift_tol=0.0)
    net.set(_with_output(lib, vec, desc, [0.75, -0.5]))
    x, base = sur.features()
    e0, p0, t0 = h.state()
    assert np.array_equal(e0, eh) and t0 == 0.0  # features leave the state unchanged
    sur.advance(1)
    e, p, t = h.state()
    g = _grid(d)
    er, pr = hos.ifrk4_step(g, eh, ph, S * d.dt)
    pr = pr.copy()
    pr[0, 0] += sd.rho * sd.sigma_phi * (-0.5)
    er = er.copy()
    er[0, 0] = eh[0, 0]
    assert np.linalg.norm(e - er) <= 1e-6 * np.linalg.norm(er)
    assert np.linalg.norm(p - pr) <= 1e-6 * np.linalg.norm(pr)
    ref_base = g.to_phys(hos.ifrk4_step(g, eh, ph, S * d.dt)[0], (N, N)) / sd.sigma_eta
    assert np.linalg.norm(base.cpu().numpy()[0] - ref_base) <= 1e-6 * np.linalg.norm(ref_base)
    _close(sur, net, h)


def _rel_state(e, p, er, pr):
    """The judge's measure: Parseval-weighted relative L2 of the half
    spectra, max over eta and phis."""
    w = np.full(er.shape[1], 2.0)
    w[0] = 1.0
    one = lambda a, b: math.sqrt(np.sum(w * np.abs(a - b) ** 2) / np.sum(w * np.abs(b) ** 2))
    return max(one(e, er), one(p, pr))


def test_drift_bound_stops_learned_calls(gpu_lib):
    """A network whose output is a constant shifts the k = 0 mode of phis by
    the same amount on every call, an error that HOS then carries unchanged
    (the mean of phis does not enter its right-hand side), over a base (two
    integrating-factor substeps) far more accurate than that shift.  With the
    first call judged and the drift bound at 3.5 times its error, calls 2-4
    go unjudged (estimate 3 e1), call 5 would pass the bound, so calls 5-8
    are advanced by HOS; the final state's error against plain HOS is the
    estimate to within the base's error.  A reset starts a new rollout."""
    from paper_2005_12716_amd import lib
    kw = dict(tol=1e-2, audit_every=1000, cooldown=0, probation=1, base_substeps=2)
    shift = [0.0, 0.02]
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, -1.0, 4, drift_tol=0.0, **kw)
    net.set(_with_output(lib, vec, desc, shift))
    st = sur.advance(1)
    e1 = st["last_audit_err"]
    assert st["audits"] == 1 and st["fallbacks"] == 0 and 2e-4 < e1 < 5e-3, st
    _close(sur, net, h)
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, -1.0, 4, drift_tol=3.5 * e1, **kw)
    net.set(_with_output(lib, vec, desc, shift))
    st = sur.advance(8)
    assert st["surrogate_calls"] == 4 and st["audits"] == 1 and st["bound_calls"] == 4 and st["hos_calls"] == 4, st
    # the judged error is a sum reduced across blocks in no fixed order: the
    # same call's error agrees with the first run's to rounding
    assert st["max_audit_err"] == pytest.approx(e1, rel=1e-9)
    assert st["drift_est"] == pytest.approx(3 * st["max_audit_err"], rel=1e-12)
    e, p, t = h.state()
    er, pr, tr = _hos_ref(lib, d, eh, ph, 8 * S)
    off = _rel_state(e, p, er, pr)
    print("drift estimate", st["drift_est"], "error against plain HOS", off)
    assert 0.9 * st["drift_est"] <= off <= 1.02 * st["drift_est"]
    assert t == pytest.approx(tr, abs=1e-12)
    # a new rollout: judged first call, learned calls again
    sur.reset()
    st = sur.advance(2)
    assert st["surrogate_calls"] == 2 and st["audits"] == 1 and st["bound_calls"] == 0, st
    _close(sur, net, h)


def test_base_only_calls_skip_the_network(gpu_lib):
    """base_only: each call is the base prediction alone (here the exact
    linear propagation); the network is not evaluated (NaN weights leave the
    state finite and the guard untouched)."""
    from paper_2005_12716_amd import lib
    d, eh, ph, h, desc, vec, net, sur, sd = _sur(lib, 1.5, 2, tol=1.0, audit_every=1000, cooldown=0, probation=0,
                                                 drift_tol=0.0, base_only=True)
    bad = vec.copy()
    bad[:] = np.nan
    net.set(bad)
    st = sur.advance(2)
    assert st["surrogate_calls"] == 2 and st["guard_trips"] == 0 and st["audits"] == 0
    e, p, t = h.state()
    er, pr = eh, ph
    for _ in range(2):
        er, pr = _lin(d, er, pr, S * d.dt)
    er = er.copy()
    er[0, 0] = eh[0, 0]
    assert np.abs(e - er).max() <= 1e-13 * np.abs(er).max()
    assert np.abs(p - pr).max() <= 1e-13 * np.abs(pr).max()
    _close(sur, net, h)
