"""Pins for the CPU float64 reference of the surrogate network: its autograd
gradient against central finite differences, and its parameter layout."""
import numpy as np
import pytest
import torch


def test_layout_matches_library_count():
    from oracle import unet_ref

    # 14 convolutions (weights + biases) and the 33-value head
    assert unet_ref.num_params() == 1_946_881
    sl = unet_ref.layer_slices()
    assert sl[-1][1].stop == unet_ref.num_params()


@pytest.mark.parametrize("seed", [0, 1])
def test_reference_gradient_against_finite_differences(seed):
    from oracle import unet_ref

    rng = np.random.default_rng(seed)
    n = unet_ref.num_params()
    p = np.zeros(n)
    for name, s in unet_ref.layer_slices():
        if name.endswith(".w"):
            fan_in = (s.stop - s.start) // (unet_ref.CONVS[int(name[4:-2])][1])
            p[s] = rng.normal(0, np.sqrt(2.0 / fan_in), s.stop - s.start)
        elif name == "head":
            p[s] = rng.normal(0, 0.2, 33)
        else:
            p[s] = rng.normal(0, 0.05, s.stop - s.start)
    x = rng.random((1, 16, 16, 3))
    t = rng.normal(size=(1, 16, 16))
    _, _, g = unet_ref.loss_and_grad(p, x, t)
    # a few parameters from several layers, central differences in float64
    picks = [unet_ref.layer_slices()[k][1].start + 3 for k in (0, 5, 14, 20, 27)]
    picks.append(n - 1)  # head bias
    for i in picks:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _, _ = unet_ref.loss_and_grad(pp, x, t)
        lm, _, _ = unet_ref.loss_and_grad(pm, x, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])
