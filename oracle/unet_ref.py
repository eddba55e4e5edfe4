"""CPU float64 reference of the surrogate network (test infrastructure only).

TEST INFRASTRUCTURE: used only by the tests to check the GPU surrogate's
forward pass and gradients.  It shares no code with the GPU library.

The network is defined by its parameter layout (one flat vector):

* per 3x3 convolution, in forward order: weights W[k][co] with
  k = (3 ky + kx) ci + c, then bias[co];
* then the 1x1 head: 32 weights, 1 bias.

Forward order (each convolution followed by SiLU):

* encoder: two convolutions per level (5->32, 32->32 | 32->64, 64->64 |
  64->128, 128->128 | 128->256, 256->256), 2x2 average pooling between levels;
* decoder: nearest 2x upsampling, concatenation [upsampled, skip] on channels,
  two convolutions per level (384->128, 128->128 | 192->64, 64->64 |
  96->32, 32->32);
* head: y = sum_c a_c w_c + b.

The loss of a batch of maps with own-visit terms O and targets t is the mean
over maps of |O + exp(y) - t|^2 / |t|^2 (the squared relative L2 error of the
prediction O + exp(y)); the training objective adds, per map, the anchor
term (anchor / n) sum_i (r_i / t_i)^2 (y_i - ln r_i)^2, r_i = max(t_i - O_i,
1e-6 t_i), n pixels per map.

Written with plain PyTorch CPU operations in float64 (convolution,
pooling, interpolation, autograd); any input side divisible by 8 works.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

CIN = 5  # input channels per probe
CONVS = [(CIN, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128), (128, 256), (256, 256),
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
    """x [B][H][W][CIN] -> y [B][H][W] (float64)."""
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


def rel_l2_loss(y: torch.Tensor, own: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    """Mean over maps of |own + exp(y) - t|^2 / |t|^2."""
    d = (own + torch.exp(y) - t).flatten(1)
    return ((d * d).sum(1) / (t.flatten(1) ** 2).sum(1)).mean()


def anchor_term(y: torch.Tensor, own: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    """Mean over maps of (1/n) sum_i (r_i/t_i)^2 (y_i - ln r_i)^2."""
    r = torch.maximum(t - own, 1e-6 * t)
    return (((r / t) ** 2 * (y - torch.log(r)) ** 2).flatten(1).mean(1)).mean()


def loss_and_grad(params: np.ndarray, x: np.ndarray, own: np.ndarray, t: np.ndarray,
                  anchor: float = 1.0):
    """rel_l2_loss of forward(params, x), the network output y, and the
    gradients of rel_l2_loss + anchor * anchor_term with respect to the
    parameters and to y."""
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    y = forward(p, torch.tensor(np.asarray(x, dtype=np.float64)))
    y.retain_grad()
    own_t = torch.tensor(np.asarray(own, dtype=np.float64))
    t_t = torch.tensor(np.asarray(t, dtype=np.float64))
    loss = rel_l2_loss(y, own_t, t_t)
    (loss + anchor * anchor_term(y, own_t, t_t)).backward()
    return float(loss.detach()), y.detach().numpy(), p.grad.numpy(), y.grad.numpy()


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
