"""CPU float64 reference of the surrogate network (test infrastructure only).

TEST INFRASTRUCTURE: used only by the tests to check the GPU surrogate's
forward pass and gradients.  It shares no code with the GPU library.

The network is defined by its parameter layout (one flat vector):

* per 3x3 convolution, in forward order: weights W[k][co] with
  k = (3 ky + kx) ci + c, then bias[co];
* then the 1x1 head: 32 weights, 1 bias.

Forward order (each convolution followed by SiLU):

* encoder: two convolutions per level (3->32, 32->32 | 32->64, 64->64 |
  64->128, 128->128 | 128->256, 256->256), 2x2 average pooling between levels;
* decoder: nearest 2x upsampling, concatenation [upsampled, skip] on channels,
  two convolutions per level (384->128, 128->128 | 192->64, 64->64 |
  96->32, 32->32);
* head: y = sum_c a_c w_c + b.

Written with plain PyTorch CPU operations in float64 (convolution,
pooling, interpolation, autograd); any input side divisible by 8 works.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

CONVS = [(3, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128), (128, 256), (256, 256),
         (384, 128), (128, 128), (192, 64), (64, 64), (96, 32), (32, 32)]


def num_params() -> int:
    return sum(9 * ci * co + co for ci, co in CONVS) + 33


def unpack(p: torch.Tensor):
    """Split the flat vector into (conv weight [co][ci][3][3], bias) pairs and the head."""
    layers, off = [], 0
    for ci, co in CONVS:
        w = p[off: off + 9 * ci * co].reshape(3, 3, ci, co)  # [ky][kx][c][co]
        off += 9 * ci * co
        b = p[off: off + co]
        off += co
        layers.append((w.permute(3, 2, 0, 1), b))
    head_w, head_b = p[off: off + 32], p[off + 32]
    return layers, head_w, head_b


def forward(p: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """x [B][H][W][3] -> y [B][H][W] (float64)."""
    layers, hw, hb = unpack(p)
    h = x.permute(0, 3, 1, 2)

    def conv(k, t):
        w, b = layers[k]
        return F.silu(F.conv2d(t, w, b, padding=1))

    s1 = conv(1, conv(0, h))
    s2 = conv(3, conv(2, F.avg_pool2d(s1, 2)))
    s3 = conv(5, conv(4, F.avg_pool2d(s2, 2)))
    m = conv(7, conv(6, F.avg_pool2d(s3, 2)))
    d3 = conv(9, conv(8, torch.cat([F.interpolate(m, scale_factor=2, mode="nearest"), s3], 1)))
    d2 = conv(11, conv(10, torch.cat([F.interpolate(d3, scale_factor=2, mode="nearest"), s2], 1)))
    d1 = conv(13, conv(12, torch.cat([F.interpolate(d2, scale_factor=2, mode="nearest"), s1], 1)))
    return (d1 * hw[None, :, None, None]).sum(1) + hb


def loss_and_grad(params: np.ndarray, x: np.ndarray, t: np.ndarray):
    """Mean squared error of forward(params, x) against t and its gradient."""
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    y = forward(p, torch.tensor(np.asarray(x, dtype=np.float64)))
    loss = ((y - torch.tensor(np.asarray(t, dtype=np.float64))) ** 2).mean()
    loss.backward()
    return float(loss.detach()), y.detach().numpy(), p.grad.numpy()


def layer_slices():
    """(name, slice) of every parameter group in the flat vector."""
    out, off = [], 0
    for k, (ci, co) in enumerate(CONVS):
        out.append((f"conv{k}.w", slice(off, off + 9 * ci * co)))
        off += 9 * ci * co
        out.append((f"conv{k}.b", slice(off, off + co)))
        off += co
    out.append(("head", slice(off, off + 33)))
    return out
