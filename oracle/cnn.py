"""FP64 CPU oracle of the residual CNN behind the first stage -- TEST
INFRASTRUCTURE ONLY.

Only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never touches it.

Section II combines the non-local estimate with a small residual network:
the network sees z = Concatenate(BM3D(y), y) (eq. (3)) and the restored
image is F(z) + BM3D(y) (the bracket of the loss, eq. (2)).  F follows
DnCNN with 3x3 convolutions and K layers (K = 10 or 16):

  layer 1        conv 3x3, 2C -> 64 features, + bias, ReLU
  layers 2..K-1  conv 3x3, 64 -> 64, + bias, batch normalisation, ReLU
  layer K        conv 3x3, 64 -> C, + bias

Convolutions are cross-correlations with zero padding of one pixel on every
side (the output has the input's size), as in DnCNN.  Batch normalisation is
its inference form with stored statistics:
gamma * (x - mean) / sqrt(var + eps) + beta.  Images enter on the [0, 1]
scale (the [0, 255] values divided by 255) and the residual is scaled back:
x_hat = BM3D(y) + 255 F(z).  Any per-layer bias or normalisation can be
absent (None).
"""
from __future__ import annotations

import numpy as np


def conv3x3(x, weight, bias=None):
    """x: (Cin, H, W); weight: (Cout, Cin, 3, 3).  Zero-padded 3x3
    cross-correlation: out[o, y, x] = bias[o] + sum over i, dy, dx in {-1,0,1}
    of weight[o, i, dy + 1, dx + 1] * x[i, y + dy, x + dx]."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(weight, dtype=np.float64)
    cin, H, W = x.shape
    assert w.shape[1:] == (cin, 3, 3)
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    out = np.zeros((w.shape[0], H, W))
    for ky in range(3):
        for kx in range(3):
            out += np.tensordot(w[:, :, ky, kx], xp[:, ky:ky + H, kx:kx + W], axes=(1, 0))
    if bias is not None:
        out += np.asarray(bias, dtype=np.float64)[:, None, None]
    return out


def batch_norm(x, gamma, beta, mean, var, eps):
    """Inference-mode batch normalisation over the channel axis 0."""
    g = np.asarray(gamma, np.float64)[:, None, None]
    b = np.asarray(beta, np.float64)[:, None, None]
    m = np.asarray(mean, np.float64)[:, None, None]
    v = np.asarray(var, np.float64)[:, None, None]
    return g * (x - m) / np.sqrt(v + float(eps)) + b


def residual(z, layers):
    """F(z) for z of shape (2C, H, W); ``layers`` is the list of K dicts with
    keys weight, bias, and (optional) gamma, beta, mean, var, eps."""
    a = np.asarray(z, dtype=np.float64)
    for k, L in enumerate(layers):
        a = conv3x3(a, L["weight"], L.get("bias"))
        if L.get("gamma") is not None:
            a = batch_norm(a, L["gamma"], L["beta"], L["mean"], L["var"], L["eps"])
        if k < len(layers) - 1:
            a = np.maximum(a, 0.0)
    return a


def restore(basic, noisy, layers):
    """x_hat = BM3D(y) + 255 F(Concatenate(BM3D(y), y) / 255).
    basic: HxW or HxWxC float (the first-stage estimate on [0, 255]);
    noisy: same shape, the observation.  Returns the same layout, FP64."""
    b = np.asarray(basic, dtype=np.float64)
    y = np.asarray(noisy, dtype=np.float64)
    grey = b.ndim == 2
    if grey:
        b, y = b[:, :, None], y[:, :, None]
    z = np.concatenate([np.moveaxis(b, 2, 0), np.moveaxis(y, 2, 0)]) / 255.0
    out = np.moveaxis(b, 2, 0) + 255.0 * residual(z, layers)
    out = np.moveaxis(out, 0, 2)
    return out[:, :, 0] if grey else out


def macs(layers: int, channels: int, h: int, w: int, features: int = 64) -> int:
    """Multiply-accumulates of F on an h x w image: 9 per (input channel,
    output channel) pair per pixel and layer."""
    per_px = 9 * (2 * channels * features + (layers - 2) * features * features
                  + features * channels)
    return per_px * h * w
