"""FP64 CPU oracle of the flexible lightweight U-Net ("Ours-FL") -- TEST
INFRASTRUCTURE ONLY.

Only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never touches it.

Section III replaces the fixed-noise residual network by a U-Net with 4
encoders and 4 decoders, skip connections, 3x3 depthwise separable
convolutions throughout, stride-2 depthwise separable convolutions to
downsample, 2x2 deconvolutions to upsample, and an FFDNet-style noise-level
map as an extra input plane.  The block details are only drawn in a figure;
the structure written here is a reading whose operation count is within
1.2 % of Table 3's 4.52 G at 512 x 512:

  z      = Concatenate(first-stage estimate, y, sigma map) / 255   (2C + 1 planes)
  DS(ci -> co, s): depthwise 3x3 (stride s, zero padding 1) + affine + ReLU,
                   then pointwise 1x1 ci -> co + affine + ReLU
  encoder level i = 0..3:  e_i = DS(c -> w_i, 1)(x);  x = DS(w_i -> w_{i+1}, 2)(e_i)
  decoder level i = 3..0:  x = ReLU(deconv2x2(x) + bias)[crop to e_i] + e_i;
                           x = DS(w_i -> w_i, 1)(x)
  F      = pointwise 1x1 w_0 -> C + bias
  x_hat  = first-stage estimate + 255 F

with widths w = (32, 64, 128, 256, 256).  "affine" is a per-channel bias, or
an inference-mode batch normalisation after it.  A stride-2 convolution of an
H x W map gives ceil(H/2) x ceil(W/2); the 2x2 deconvolution (stride 2, no
overlap) doubles that and is cropped back to the skip's size.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (32, 64, 128, 256, 256)


def depthwise3x3(x, weight, stride=1):
    """x: (C, H, W); weight: (C, 3, 3).  Zero-padded per-channel 3x3
    cross-correlation sampled at stride s: out[c, y, x] = sum over dy, dx of
    weight[c, dy + 1, dx + 1] * x[c, s y + dy, s x + dx]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(weight, np.float64)
    C, H, W = x.shape
    Ho, Wo = -(-H // stride), -(-W // stride)
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    out = np.zeros((C, Ho, Wo))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            out += w[:, ky, kx][:, None, None] * patch
    return out


def pointwise(x, weight):
    """1x1 convolution: weight (Cout, Cin)."""
    return np.tensordot(np.asarray(weight, np.float64), np.asarray(x, np.float64), axes=(1, 0))


def deconv2x2(x, weight):
    """Transposed 2x2 convolution, stride 2 (PyTorch layout weight (Cin,
    Cout, 2, 2)): out[o, 2y + a, 2x + b] = sum over i of x[i, y, x] *
    weight[i, o, a, b]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(weight, np.float64)
    _, H, W = x.shape
    out = np.zeros((w.shape[1], 2 * H, 2 * W))
    for a in range(2):
        for b in range(2):
            out[:, a::2, b::2] = np.tensordot(w[:, :, a, b], x, axes=(0, 0))
    return out


def affine(x, L, prefix=""):
    """+ bias, then the optional inference-mode batch normalisation."""
    b = L.get(prefix + "bias")
    if b is not None:
        x = x + np.asarray(b, np.float64)[:, None, None]
    g = L.get(prefix + "gamma")
    if g is not None:
        m = np.asarray(L[prefix + "mean"], np.float64)[:, None, None]
        v = np.asarray(L[prefix + "var"], np.float64)[:, None, None]
        x = (np.asarray(g, np.float64)[:, None, None] * (x - m) / np.sqrt(v + float(L[prefix + "eps"]))
             + np.asarray(L[prefix + "beta"], np.float64)[:, None, None])
    return x


def ds_block(x, L, stride):
    """Depthwise separable block: L has dw (C,3,3), dw_bias..., pw (Co,C),
    pw_bias, optional pw_gamma/beta/mean/var/eps."""
    x = np.maximum(affine(depthwise3x3(x, L["dw"], stride), L, "dw_"), 0.0)
    return np.maximum(affine(pointwise(x, L["pw"]), L, "pw_"), 0.0)


def residual(z, net):
    """F(z) for z (2C + 1, H, W); net: dict with lists enc[4], down[4],
    up[4], dec[4] (index = level) and out."""
    x = np.asarray(z, np.float64)
    skips = []
    for i in range(4):
        x = ds_block(x, net["enc"][i], 1)
        skips.append(x)
        x = ds_block(x, net["down"][i], 2)
    for i in range(3, -1, -1):
        U = net["up"][i]
        u = np.maximum(deconv2x2(x, U["weight"]) + np.asarray(U["bias"], np.float64)[:, None, None], 0.0)
        e = skips[i]
        x = u[:, :e.shape[1], :e.shape[2]] + e
        x = ds_block(x, net["dec"][i], 1)
    O = net["out"]
    return pointwise(x, O["weight"]) + np.asarray(O["bias"], np.float64)[:, None, None]


def restore(basic, noisy, sigma, net):
    """x_hat = basic + 255 F(Concatenate(basic, noisy, sigma map) / 255),
    same layout as ``basic`` (HxW or HxWxC), FP64."""
    b = np.asarray(basic, np.float64)
    y = np.asarray(noisy, np.float64)
    grey = b.ndim == 2
    if grey:
        b, y = b[:, :, None], y[:, :, None]
    H, W = b.shape[:2]
    z = np.concatenate([np.moveaxis(b, 2, 0), np.moveaxis(y, 2, 0), np.full((1, H, W), float(sigma))]) / 255.0
    out = np.moveaxis(np.moveaxis(b, 2, 0) + 255.0 * residual(z, net), 0, 2)
    return out[:, :, 0] if grey else out


def macs(channels: int, h: int, w: int, widths=WIDTHS) -> float:
    """Multiply-adds of F on an h x w image, counted per output sample:
    9 per depthwise tap, cin per pointwise output, cin per deconvolution
    output."""
    tot = 0.0
    c, hh, ww = 2 * channels + 1, h, w
    dims = []
    for i in range(4):
        tot += (9 * c + c * widths[i]) * hh * ww
        dims.append((hh, ww))
        hh, ww = -(-hh // 2), -(-ww // 2)
        tot += (9 * widths[i] + widths[i] * widths[i + 1]) * hh * ww
        c = widths[i + 1]
    for i in range(3, -1, -1):
        hh, ww = 2 * hh, 2 * ww
        tot += widths[i + 1] * widths[i] * hh * ww
        hh, ww = dims[i]
        tot += (9 * widths[i] + widths[i] * widths[i]) * hh * ww
    tot += widths[0] * channels * h * w
    return tot
