"""Plain PyTorch CPU reference of the warm-start network (FP64).

TEST INFRASTRUCTURE ONLY: imported by tests/ and nothing else. It shares no
code with the GPU library.

The network is not in the paper; it is the learned initial guess of the
Poisson solve (Eq. poi) described in the C header: a 3D U-Net with four
levels of 16, 32, 64, 128 channels, two 3x3x3 convolutions + ReLU per level,
2x2x2 stride-2 convolutions + ReLU down, 2x2x2 stride-2 transposed
convolutions up (no activation), skip connections by concatenation
(upsampled tensor first), and a linear 1x1x1 head, trained with the mean
squared error.

The flat parameter vector is read in the documented layout: per layer W then
b, W[tap][cin][cout] with tap = 9 dz + 3 dy + dx (offsets -1..1) for the
3x3x3 convolutions and tap = 4 pz + 2 py + px for the stride-2 ones; the head
is w[16], b[1]. The first layer reads 8 channels, channel 0 being the input.

With bf16=True the forward reproduces the storage precision of the GPU path
(weights of the convolutions and every stored activation rounded to bfloat16,
round to nearest even; biases, the head and all arithmetic in FP64). The
rounding is applied as a straight-through step (value rounded, derivative
one), so gradients are those of the FP64 network at the rounded values.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def layer_table(base: int = 16):
    """(kind, cin, cout) per layer in parameter order."""
    c = [base, 2 * base, 4 * base, 8 * base]
    t = [("conv3", 8, c[0]), ("conv3", c[0], c[0])]
    for lv in (1, 2, 3):
        t.append(("down", c[lv - 1], c[lv]))
        t.append(("conv3", c[lv], c[lv]))
        t.append(("conv3", c[lv], c[lv]))
    for lv in (2, 1, 0):
        t.append(("up", c[lv + 1], c[lv]))
        t.append(("conv3", 2 * c[lv], c[lv]))
        t.append(("conv3", c[lv], c[lv]))
    return t


def n_params(base: int = 16) -> int:
    n = 0
    for kind, cin, cout in layer_table(base):
        n += (27 if kind == "conv3" else 8) * cin * cout + cout
    return n + base + 1


def layer_weight(flat: torch.Tensor, kind: str, cin: int, cout: int) -> torch.Tensor:
    """W[tap][cin][cout] (tap = 9 kz + 3 ky + kx, or 4 kz + 2 ky + kx) in
    torch's layout: [cout][cin][kz][ky][kx] for conv3d, [cin][cout][kz][ky][kx]
    for conv_transpose3d."""
    k = 3 if kind == "conv3" else 2
    w = flat.reshape(k, k, k, cin, cout)
    return w.permute(3, 4, 0, 1, 2) if kind == "up" else w.permute(4, 3, 0, 1, 2)


def unpack(p: torch.Tensor, base: int = 16):
    """Split the flat vector into (kind, torch-layout weight, bias) per layer
    and the head weights."""
    out = []
    o = 0
    for kind, cin, cout in layer_table(base):
        taps = 27 if kind == "conv3" else 8
        w = layer_weight(p[o:o + taps * cin * cout], kind, cin, cout)
        o += taps * cin * cout
        b = p[o:o + cout]
        o += cout
        out.append((kind, w, b))
    hw = p[o:o + base]
    hb = p[o + base:o + base + 1]
    assert o + base + 1 == p.numel()
    return out, hw, hb


def _round_bf16(t: torch.Tensor) -> torch.Tensor:
    return t + (t.to(torch.bfloat16).to(t.dtype) - t).detach()


class _RoundGrad(torch.autograd.Function):
    """Identity whose backward rounds the incoming gradient to bfloat16 (the
    storage precision of the gradient that the GPU's matrix products read)."""

    @staticmethod
    def forward(ctx, t):
        return t.view_as(t)

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.bfloat16).to(g.dtype)


def conv3(x, w, b):
    """3x3x3 convolution, zero padding, stride 1 (cross-correlation: output
    voxel v reads input voxel v + offset)."""
    return F.conv3d(x, w, b, stride=1, padding=1)


def down(x, w, b):
    """2x2x2 convolution of stride 2: output voxel v reads input 2v + p."""
    return F.conv3d(x, w, b, stride=2)


def up(x, w, b):
    """2x2x2 transposed convolution of stride 2: input voxel v feeds output
    voxel 2v + p with weight W[p]."""
    return F.conv_transpose3d(x, w, b, stride=2)


def forward(p: torch.Tensor, x: torch.Tensor, base: int = 16, bf16: bool = False,
            bf16_grad: bool = False) -> torch.Tensor:
    """x: [B][D][H][W] -> y: [B][D][H][W]. With bf16_grad the gradient that
    reaches each convolution (after the ReLU mask, not the one of its bias)
    is rounded to bfloat16 as well."""
    layers, hw, hb = unpack(p, base)
    r = _round_bf16 if bf16 else (lambda t: t)
    B, D, H, W = x.shape
    t = torch.cat([x.to(p.dtype)[:, None], torch.zeros(B, 7, D, H, W, dtype=p.dtype)], dim=1)
    t = r(t)
    it = iter(layers)

    def apply(kind, w, b, inp, relu):
        wq = r(w)
        f = {"conv3": conv3, "down": down, "up": up}[kind]
        if bf16_grad:
            y = _RoundGrad.apply(f(inp, wq, None)) + b.view(1, -1, 1, 1, 1)
        else:
            y = f(inp, wq, b)
        if relu:
            y = torch.relu(y)
        return r(y)

    def nxt():
        return next(it)

    # encoder
    k, w, b = nxt(); t = apply(k, w, b, t, True)
    k, w, b = nxt(); s0 = apply(k, w, b, t, True)
    k, w, b = nxt(); t = apply(k, w, b, s0, True)
    k, w, b = nxt(); t = apply(k, w, b, t, True)
    k, w, b = nxt(); s1 = apply(k, w, b, t, True)
    k, w, b = nxt(); t = apply(k, w, b, s1, True)
    k, w, b = nxt(); t = apply(k, w, b, t, True)
    k, w, b = nxt(); s2 = apply(k, w, b, t, True)
    k, w, b = nxt(); t = apply(k, w, b, s2, True)
    k, w, b = nxt(); t = apply(k, w, b, t, True)
    k, w, b = nxt(); t = apply(k, w, b, t, True)
    # decoder
    for skip in (s2, s1, s0):
        k, w, b = nxt(); t = apply(k, w, b, t, False)
        k, w, b = nxt(); t = apply(k, w, b, torch.cat([t, skip], dim=1), True)
        k, w, b = nxt(); t = apply(k, w, b, t, True)
    y = torch.einsum("bcdhw,c->bdhw", t, hw) + hb[0]
    return y


def loss_and_grad(p_np: np.ndarray, x_np: np.ndarray, target_np: np.ndarray, base: int = 16, bf16: bool = False,
                  bf16_grad: bool = False):
    """Mean squared error and its gradient with respect to the flat
    parameters (autograd in FP64)."""
    p = torch.tensor(np.asarray(p_np, np.float64), requires_grad=True)
    x = torch.tensor(np.asarray(x_np, np.float64))
    tg = torch.tensor(np.asarray(target_np, np.float64))
    y = forward(p, x, base, bf16, bf16_grad)
    loss = ((y - tg) ** 2).mean()
    loss.backward()
    return float(loss.detach()), p.grad.numpy().copy(), y.detach().numpy()


def forward_np(p_np: np.ndarray, x_np: np.ndarray, base: int = 16, bf16: bool = False) -> np.ndarray:
    with torch.no_grad():
        return forward(torch.tensor(np.asarray(p_np, np.float64)), torch.tensor(np.asarray(x_np, np.float64)), base,
                       bf16).numpy()
