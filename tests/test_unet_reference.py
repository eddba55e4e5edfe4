"""Pins for the CPU float64 reference of the surrogate network: its autograd
gradient against central finite differences, its loss against a direct
evaluation, and its parameter layout."""
import numpy as np
import pytest
import torch


def test_layout_matches_library_count():
    from oracle import unet_ref

    # 14 convolutions (weights + biases) and the 33-value head
    assert unet_ref.num_params() == 1_947_457
    sl = unet_ref.layer_slices()
    assert sl[-1][1].stop == unet_ref.num_params()


def _objective(unet_ref, p, x, own, t, anchor):
    y = unet_ref.forward(torch.tensor(p), torch.tensor(x))
    own_t, t_t = torch.tensor(own), torch.tensor(t)
    return float(unet_ref.rel_l2_loss(y, own_t, t_t) + anchor * unet_ref.anchor_term(y, own_t, t_t))


@pytest.mark.parametrize("seed,anchor", [(0, 0.0), (1, 1.0)])
def test_reference_gradient_against_finite_differences(seed, anchor):
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
    x = rng.random((1, 16, 16, unet_ref.CIN))
    own = rng.random((1, 16, 16))
    t = own + rng.random((1, 16, 16)) + 0.5
    _, _, g, _ = unet_ref.loss_and_grad(p, x, own, t, anchor=anchor)
    # a few parameters from several layers, central differences in float64
    picks = [unet_ref.layer_slices()[k][1].start + 3 for k in (0, 5, 14, 20, 27)]
    picks.append(n - 1)  # head bias
    for i in picks:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp = _objective(unet_ref, pp, x, own, t, anchor)
        lm = _objective(unet_ref, pm, x, own, t, anchor)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_loss_is_mean_squared_relative_l2():
    from oracle import unet_ref

    rng = np.random.default_rng(3)
    y = rng.normal(size=(3, 8, 8))
    own = rng.random((3, 8, 8))
    t = own + rng.random((3, 8, 8))
    got = float(unet_ref.rel_l2_loss(torch.tensor(y), torch.tensor(own), torch.tensor(t)))
    want = np.mean([np.sum((own[b] + np.exp(y[b]) - t[b]) ** 2) / np.sum(t[b] ** 2)
                    for b in range(3)])
    assert got == pytest.approx(want, rel=1e-14)
    # an exact prediction has zero loss and zero anchor term
    ye = torch.tensor(np.log(t - own))
    assert float(unet_ref.rel_l2_loss(ye, torch.tensor(own), torch.tensor(t))) < 1e-28
    assert float(unet_ref.anchor_term(ye, torch.tensor(own), torch.tensor(t))) < 1e-28
    # the anchor term weighs pixel i by (r_i / t_i)^2
    y0 = torch.zeros(1, 1, 2, dtype=torch.float64)
    own2 = torch.tensor([[[1.0, 0.0]]], dtype=torch.float64)
    t2 = torch.tensor([[[2.0, 4.0]]], dtype=torch.float64)
    want2 = 0.5 * ((0.5 ** 2) * (0 - np.log(1.0)) ** 2 + 1.0 * (0 - np.log(4.0)) ** 2)
    assert float(unet_ref.anchor_term(y0, own2, t2)) == pytest.approx(want2, rel=1e-12)


def test_bf16_reference_without_rounding_is_the_network_and_its_autograd():
    """The BF16 reference with rounding switched off computes the float64
    network (forward) and, through its hand-written backward (convolution
    adjoints, pooling, upsampling and concatenation routing, head), the
    autograd gradient of forward(p, x) . dy; with rounding on it differs only
    at BF16 level."""
    import torch

    from oracle import unet_ref as R

    rng = np.random.default_rng(11)
    p = torch.tensor(rng.normal(0, 0.05, R.num_params()))
    x = torch.tensor(rng.random((2, 16, 16, R.CIN)))
    dy = torch.tensor(rng.normal(0, 1, (2, 16, 16)))
    y0, st0 = R.forward_bf16(p, x, rounding=False)
    y64 = R.forward(p, x)
    assert float((y0 - y64).abs().max()) <= 1e-13 * float(y64.abs().max())
    g0 = R.backward_bf16(p, st0, dy)
    pa = p.clone().requires_grad_(True)
    (R.forward(pa, x) * dy).sum().backward()
    for name, s in R.layer_slices():
        ref = pa.grad[s]
        assert float((g0[s] - ref).abs().max()) <= 1e-11 * float(ref.abs().max()), name
    yb, stb = R.forward_bf16(p, x)
    gb = R.backward_bf16(p, stb, dy)
    assert 1e-6 < float((yb - y64).abs().max() / y64.abs().max()) < 1e-2
    for name, s in R.layer_slices():
        ref = pa.grad[s]
        err = float((gb[s] - ref).abs().max() / ref.abs().max())
        assert err < 5e-2, (name, err)
    # the rounding itself: BF16 keeps 8 significant bits, ties to even
    v = torch.tensor([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 3.0 * 2 ** -100])
    assert R.bf16(v).tolist() == [1.0, 1.0, 1.0 + 4 * 2 ** -8, 1.0, 3.0 * 2 ** -100]


def test_elementwise_bounds_see_a_wrong_tap_or_border():
    """The element-wise bound of the GPU comparison (5e-3 of max |y|) is far
    below what a mistake confined to one tap or to one layer's border
    handling does to the reference's own output."""
    import torch
    import torch.nn.functional as F

    from oracle import unet_ref as R

    rng = np.random.default_rng(13)
    p = torch.tensor(rng.normal(0, 0.08, R.num_params()))
    x = torch.tensor(rng.random((1, 16, 16, R.CIN)))
    y, _ = R.forward_bf16(p, x)
    scale = float(y.abs().max())
    off = 0
    offs = []
    for ci, co in R.CONVS:
        offs.append(off)
        off += 9 * ci * co + co
    # one tap (the centre of layer 9) zeroed
    q = p.clone()
    ci, co = R.CONVS[9]
    q[offs[9] + 4 * ci * co: offs[9] + 5 * ci * co] = 0
    assert float((R.forward_bf16(q, x)[0] - y).abs().max()) > 10 * 5e-3 * scale
    # border pixels of the input replicated instead of zero padded, first layer
    real_conv2d = F.conv2d
    calls = []

    def replicate_first(inp, w, b=None, padding=0):
        calls.append(1)
        if len(calls) == 1:
            return real_conv2d(F.pad(inp, (1, 1, 1, 1), mode="replicate"), w, b)
        return real_conv2d(inp, w, b, padding=padding)

    R.F.conv2d = replicate_first
    try:
        y2, _ = R.forward_bf16(p, x)
    finally:
        R.F.conv2d = real_conv2d
    d = (y2 - y).abs()[0]
    assert float(d[[0, -1], :].max()) > 5e-3 * scale or float(d[:, [0, -1]].max()) > 5e-3 * scale
