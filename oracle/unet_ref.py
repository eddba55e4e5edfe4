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


# ---------------------------------------------------------------------------
# The same network with its operands rounded to BF16 where the GPU kernels
# round them, for element-wise comparison.  Every product of a convolution
# (forward, data gradient, weight gradient) takes BF16-rounded operands and is
# accumulated here in float64; stored activations and 2x2 averages are
# rounded to BF16; pre-activations, gradients, biases and the head stay in
# float64.  The rounding points:
#   forward   conv l: z = conv(bf16(input), bf16(W)) + b, stored A = bf16(silu(z));
#             the first input is bf16(x); pooling p = bf16(mean of 4 stored values);
#             decoder inputs are [upsample(stored coarse), stored skip];
#             the head reads silu(z_13) unrounded: y = sum_c silu(z_13)_c w_c + b_h;
#   backward  dA_13 = dy w (head), the head weight gradient sums dy bf16-stored A_13;
#             per conv: dZ = dA silu'(z), bias gradient sum dZ, weight gradient
#             sum bf16(input) bf16(dZ), data gradient conv^T(bf16(dZ), bf16(W));
#             the adjoints of pooling, upsampling and concatenation are exact.

def bf16(t: torch.Tensor) -> torch.Tensor:
    """Nearest BF16 value (ties to even) of the single-precision rounding of t,
    as float64 (the kernels round FP32 values to BF16)."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _no_rounding(t: torch.Tensor) -> torch.Tensor:
    return t


def forward_bf16(p: torch.Tensor, x: torch.Tensor, rounding: bool = True):
    """y [B][H][W] and the cache of forward_bf16's intermediate values.  With
    rounding=False no value is rounded (then y equals forward(p, x))."""
    bf16 = globals()["bf16"] if rounding else _no_rounding
    layers, hw, hb = unpack(p)
    wb = [(bf16(w), b) for w, b in layers]
    cache = {}

    def conv(k, inp):
        w, b = wb[k]
        z = F.conv2d(inp, w, b, padding=1)
        cache[k] = (inp, z)
        return z

    def act(z):
        return bf16(F.silu(z))

    def pool(a):
        return bf16(F.avg_pool2d(a, 2))

    def up(t):
        return F.interpolate(t, scale_factor=2, mode="nearest")

    A = {}
    A[0] = act(conv(0, bf16(x.permute(0, 3, 1, 2))))
    A[1] = act(conv(1, A[0]))
    A[2] = act(conv(2, pool(A[1])))
    A[3] = act(conv(3, A[2]))
    A[4] = act(conv(4, pool(A[3])))
    A[5] = act(conv(5, A[4]))
    A[6] = act(conv(6, pool(A[5])))
    A[7] = act(conv(7, A[6]))
    A[8] = act(conv(8, torch.cat([up(A[7]), A[5]], 1)))
    A[9] = act(conv(9, A[8]))
    A[10] = act(conv(10, torch.cat([up(A[9]), A[3]], 1)))
    A[11] = act(conv(11, A[10]))
    A[12] = act(conv(12, torch.cat([up(A[11]), A[1]], 1)))
    z13 = conv(13, A[12])
    A[13] = bf16(F.silu(z13))
    y = (F.silu(z13) * hw[None, :, None, None]).sum(1) + hb
    return y, (cache, A, rounding)


def backward_bf16(p: torch.Tensor, state, dy: torch.Tensor) -> torch.Tensor:
    """Gradient of the parameters (flat vector) for output gradient dy, with
    the rounding points of the kernels (see above); without rounding (state of
    forward_bf16(..., rounding=False)) the gradient of forward(p, x) . dy."""
    from torch.nn.grad import conv2d_input, conv2d_weight

    layers, hw, _ = unpack(p)
    cache, A, rounding = state
    bf16 = globals()["bf16"] if rounding else _no_rounding
    grads = {}

    def conv_bwd(k, dA, want_dx=True):
        inp, z = cache[k]
        s = torch.sigmoid(z)
        dZ = dA * s * (1 + z * (1 - s))
        dZb = bf16(dZ)
        w = layers[k][0]
        grads[k] = (conv2d_weight(inp, w.shape, dZb, padding=1), dZ.sum((0, 2, 3)))
        return conv2d_input(inp.shape, bf16(w), dZb, padding=1) if want_dx else None

    def split_up(d, c1):  # gradient of [upsample(coarse), skip] -> (coarse, skip)
        du = d[:, :c1]
        return (du[:, :, 0::2, 0::2] + du[:, :, 0::2, 1::2] + du[:, :, 1::2, 0::2] +
                du[:, :, 1::2, 1::2]), d[:, c1:]

    def pool_bwd(dp):
        return dp.repeat_interleave(2, 2).repeat_interleave(2, 3) / 4

    g_head = torch.zeros(33, dtype=torch.float64)
    g_head[:32] = (dy[:, None] * A[13]).sum((0, 2, 3))
    g_head[32] = dy.sum()
    d = conv_bwd(13, dy[:, None] * hw[None, :, None, None])
    d11, ds1 = split_up(conv_bwd(12, d), 64)
    d9, ds2 = split_up(conv_bwd(10, conv_bwd(11, d11)), 128)
    d7, ds3 = split_up(conv_bwd(8, conv_bwd(9, d9)), 256)
    ds3 = ds3 + pool_bwd(conv_bwd(6, conv_bwd(7, d7)))
    ds2 = ds2 + pool_bwd(conv_bwd(4, conv_bwd(5, ds3)))
    ds1 = ds1 + pool_bwd(conv_bwd(2, conv_bwd(3, ds2)))
    conv_bwd(0, conv_bwd(1, ds1), want_dx=False)
    parts = []
    for k in range(len(CONVS)):
        gw, gb = grads[k]
        parts += [gw.permute(2, 3, 1, 0).reshape(-1), gb]  # [ky][kx][c][co], then bias
    parts.append(g_head)
    return torch.cat(parts)


def loss_dy(y: np.ndarray, own: np.ndarray, t: np.ndarray, anchor: float = 1.0):
    """rel_l2_loss and its gradient plus the anchor term's with respect to y
    (float64, autograd on the definitions above), evaluated at the given y."""
    yt = torch.tensor(np.asarray(y, dtype=np.float64), requires_grad=True)
    own_t = torch.tensor(np.asarray(own, dtype=np.float64))
    t_t = torch.tensor(np.asarray(t, dtype=np.float64))
    loss = rel_l2_loss(yt, own_t, t_t)
    (loss + anchor * anchor_term(yt, own_t, t_t)).backward()
    return float(loss.detach()), yt.grad.numpy()
