"""What the trained network gains over the method without it: a small
network trained on the GPU (forward, backward and Adam in the HIP library)
on HOS trajectories the library generates, judged by HOS on held-out seas
against the exact linear propagator alone (the same rollout with a network
whose output is zero).  Small grid (64^2 over 5 peak wavelengths, the
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
    zero = lib.Fno(desc, T.zero_output(desc, vec0))
    errs = T.one_call_errors(net, scales, range(3000, 3004), 5, 5.0, zero)
    e_net, e_lin = errs["network"].mean(), errs["base_only"].mean()
    print(f"in_channels {in_channels} one-call relative error: network {e_net:.3e}, linear only {e_lin:.3e}, "
          f"loss {np.mean(hist[:20]):.3e} -> {np.mean(hist[-50:]):.3e}")
    assert np.isfinite(e_net) and e_net < e_lin
    zero.close()
    net.close()
