"""What the trained surrogate gains over the exact kernel alone: on the 2000
held-out 64x64 test scans (config-4-style sampling, seed 6), the committed
network with its exact judge and fallback reproduces the exact final maps to
<= 1% mean relative L2 error and finishes sooner than the exact batched
kernel.  Maps it rejects are the exact maps, bit for bit."""
import os
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_TEST = 2000
SPOT_TOL = 0.02


@pytest.fixture(scope="module")
def setup():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_00294_amd as dd
    from paper_2507_00294_amd import surrogate as sg
    from paper_2507_00294_amd import workloads as wl

    assert os.path.exists(sg.DEFAULT_WEIGHTS), "trained weights are part of the package"
    net = dd.UNet(0)
    sg.load_weights(net)
    scans = [dd.Scan(**s.kwargs()) for s in wl.surrogate_scans(N_TEST, seed=6)]
    return dd, sg, net, scans


def _median_time(f, reps=3):
    import torch

    ts = []
    out = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = f()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return out, float(np.median(ts))


def test_surrogate_gain_on_test_set(setup):
    dd, sg, net, scans = setup
    exact_maps = lambda: sg.exact_final_maps(scans, "mixed")
    exact_maps()  # builds the scans' device tables
    net.predict(scans, SPOT_TOL, "mixed")  # builds the surrogate input tables
    exact, t_exact = _median_time(exact_maps)
    (psi, fb), t_sur = _median_time(lambda: net.predict(scans, SPOT_TOL, "mixed"))
    err = sg.rel_l2(psi, exact)
    print(f"\nexact {t_exact * 1e3:.1f} ms, surrogate {t_sur * 1e3:.1f} ms "
          f"(x{t_exact / t_sur:.2f}); rel L2 mean {err.mean():.4f} p95 "
          f"{np.percentile(err, 95):.4f} max {err.max():.4f}; fallback {fb.mean():.3f}")
    assert err.mean() <= 0.01
    assert fb.mean() < 0.25
    assert t_sur < t_exact
    # rejected maps are the exact kernel's
    ex = exact.cpu().numpy()
    ps = psi.cpu().numpy()
    for k in np.flatnonzero(fb)[:50]:
        assert np.array_equal(ps[k], ex[k])


def test_network_alone_is_accurate(setup):
    """Without the judge the network's own error is already near the target:
    the fallback only trims the tail."""
    dd, sg, net, scans = setup
    exact = sg.exact_final_maps(scans, "mixed")
    raw, fb = net.predict(scans, 1e300, "mixed")
    assert fb.sum() == 0
    err = sg.rel_l2(raw, exact)
    assert err.mean() <= 0.012
    assert np.percentile(err, 50) <= 0.01
