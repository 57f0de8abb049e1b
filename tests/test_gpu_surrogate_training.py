"""What the trained network gains over the method without it: a small
network trained on the GPU (forward, backward and Adam in the HIP library)
on HOS trajectories the library generates, judged by HOS on held-out seas
against the exact linear propagator alone (the same calls with the network
not evaluated).  Small grid (64^2 over 5 peak wavelengths, the
resolution of the 256^2 / 20 wavelength surrogate configuration) so the test
runs in seconds."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("in_channels", [2, 4])
def test_trained_network_beats_linear_propagation(gpu_lib, in_channels):
    from paper_2005_12716_amd import lib, train as T
    desc = lib.fno_desc(64, 16, 4, 12, 11, 32, max_batch=8, in_channels=in_channels)
    vec0 = lib.fno_init(desc, 0)
    net = lib.Fno(desc, vec0)
    scales = T.default_scales(5)
    store = T.Pairs(32 * 20, 64, in_channels)
    T.generate(net, scales, range(1000, 1032), 100, 5.0, store)
    assert store.count == 640
    hist = T.train(net, store, 600, 8, 2e-3, seed=1)
    assert np.mean(hist[-50:]) < 0.5 * np.mean(hist[:20])
    errs = T.one_call_errors(net, scales, range(3000, 3004), 5, 5.0)
    e_net, e_lin = errs["network"].mean(), errs["base_only"].mean()
    print(f"in_channels {in_channels} one-call relative error: network {e_net:.3e}, linear only {e_lin:.3e}, "
          f"loss {np.mean(hist[:20]):.3e} -> {np.mean(hist[-50:]):.3e}")
    assert np.isfinite(e_net) and e_net < e_lin
    net.close()


def test_trained_rollout_stays_within_the_bound(gpu_lib):
    """A rollout of the learned configuration's length (200 steps: 20 calls of
    10 steps) with a trained network over the two-substep base, judged every
    4th call with the drift bound at the judge's tolerance: the final state
    stays within 1e-3 of plain HOS on every held-out sea, the estimate bounds
    the measured error to a factor of two, and the base-only rollout is
    held to the same bars."""
    pytest.importorskip("torch")
    from paper_2005_12716_amd import lib, train as T
    desc = lib.fno_desc(64, 16, 4, 12, 11, 32, max_batch=8, in_channels=4)
    vec0 = lib.fno_init(desc, 0)
    net = lib.Fno(desc, vec0)
    scales = T.default_scales(10, 2)
    store = T.Pairs(32 * 20, 64, 4)
    T.generate(net, scales, range(1000, 1032), 200, 5.0, store)
    T.train(net, store, 600, 8, 2e-3, seed=1)
    del store
    seeds = range(3000, 3003)
    roll = T.rollout(net, scales, seeds, 20, 5.0, tol=1e-3, audit_every=4, cooldown=4)
    base = T.rollout(net, scales, seeds, 20, 5.0, tol=1e-3, audit_every=4, cooldown=4, base_only=True)
    for name, rr in (("network", roll), ("base only", base)):
        for r in rr:
            print(name, {k: r[k] for k in ("seed", "surrogate_calls", "hos_calls", "bound_calls", "audits",
                                           "fallbacks", "max_audit_err", "drift_est", "offline_err")})
            assert r["calls"] == 20 and r["offline_err"] <= 1e-3, (name, r)
            # every unjudged call adds the largest judged error to the
            # estimate; the accumulated error stays within twice that (the
            # unjudged calls' own errors are only sampled by the judged ones)
            assert r["offline_err"] <= 2 * r["drift_est"] + 1e-12, (name, r)
    net.close()
