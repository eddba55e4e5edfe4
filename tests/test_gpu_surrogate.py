"""Learned surrogate on the GPU: the BF16-MFMA U-Net forward pass and
gradients against the CPU float64 reference network, the input and target
definitions, and an end-to-end training run of the library's own kernels."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_00294_amd as dd

    dd.load_library()
    return dd


def test_forward_and_gradients_match_reference(dd):
    import torch

    from oracle import unet_ref

    net = dd.UNet(seed=3)
    assert net.num_params == unet_ref.num_params()
    p = net.params()
    p[-1] = 0.3
    net.set_params(p)
    rng = np.random.default_rng(7)
    x = rng.random((2, 64, 64, 3)).astype(np.float32)
    t = rng.normal(size=(2, 64, 64)).astype(np.float32)
    y = net.forward(torch.tensor(x, device="cuda"))
    loss, dy = net.mse(y, torch.tensor(t, device="cuda"))
    net.backward(dy)
    g = net.grads()
    ref_loss, ref_y, ref_g = unet_ref.loss_and_grad(p.astype(np.float64), x, t)
    y = y.cpu().numpy()
    # BF16 operands (8-bit mantissa) with FP32 accumulation
    assert np.linalg.norm(y - ref_y) <= 2e-2 * np.linalg.norm(ref_y)
    assert abs(loss - ref_loss) <= 2e-2 * ref_loss
    for name, s in unet_ref.layer_slices():
        gn = np.linalg.norm(ref_g[s])
        if gn == 0:
            continue
        err = np.linalg.norm(g[s] - ref_g[s]) / gn
        assert err <= 6e-2, (name, err)
    # the gradient points the same way overall
    cos = float(np.dot(g, ref_g) / (np.linalg.norm(g) * np.linalg.norm(ref_g)))
    assert cos > 0.999


def test_inputs_and_targets(dd):
    import torch

    from paper_2507_00294_amd import workloads as wl

    specs = wl.surrogate_scans(3, seed=11)
    scans = [dd.Scan(**s.kwargs()) for s in specs]
    x = dd.surrogate_inputs(scans).cpu().numpy()
    for k, (spec, s) in enumerate(zip(specs, scans)):
        v = s.visits()
        first = np.full(64 * 64, -1)
        for j, pid in enumerate(v):
            if first[pid] < 0:
                first[pid] = j
        assert np.allclose(x[k, :, :, 0].ravel(), first / v.size, rtol=0, atol=1e-7)
        kap = spec.D_m2s * spec.dwell_s / spec.pitch_m ** 2
        assert np.allclose(x[k, :, :, 1], (math.log10(kap) + 1) / 3, atol=1e-6)
        assert np.allclose(x[k, :, :, 2], (spec.sigma_m / spec.pitch_m - 0.6) / 0.4, atol=1e-6)
    outs = dd.batch_solve(scans, dd.Q_FINAL_AT_PROBES, "fp64")
    psi = torch.stack([o.view(64, 64) for o in outs])
    t = dd.surrogate_targets(scans, psi).cpu().numpy()
    for k, spec in enumerate(specs):
        hat = psi[k].cpu().numpy() * 4 * math.pi * spec.D_m2s / spec.Q0_us
        assert np.allclose(t[k], np.log(hat), rtol=0, atol=2e-5)


def test_training_reduces_loss(dd):
    from paper_2507_00294_amd import surrogate as sg
    from paper_2507_00294_amd import workloads as wl

    x, t = sg.generate(wl.surrogate_scans(256, seed=12))
    net = dd.UNet(seed=0)
    sg.init_head(net, t)
    hist = sg.train(net, x, t, steps=120, batch=16, lr=2e-3, log_every=40, warmup=20)
    assert hist[-1][1] < 0.5 * hist[0][1], hist
    assert all(np.isfinite(l) for _, l in hist)


def test_predict_fallback_is_exact(dd):
    """With spot_tol = 0 every map is rejected and computed exactly; scans
    outside the training range always fall back."""
    import torch

    from paper_2507_00294_amd import workloads as wl

    net = dd.UNet(seed=0)
    specs = wl.surrogate_scans(4, seed=13)
    scans = [dd.Scan(**s.kwargs()) for s in specs]
    psi, fb = net.predict(scans, spot_tol=0.0, precision="mixed")
    assert fb.tolist() == [1, 1, 1, 1]
    outs = dd.batch_solve(scans, dd.Q_FINAL_AT_PROBES, "mixed")
    for k, o in enumerate(outs):
        assert np.array_equal(psi[k].cpu().numpy().ravel(), o.cpu().numpy())
    odd = dd.Scan(64, 64, "raster", D_m2s=1e-9)  # kappa far outside the training range
    psi2, fb2 = net.predict([odd], spot_tol=1.0, precision="mixed")
    assert fb2.tolist() == [1]
