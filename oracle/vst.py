"""FP64 CPU oracle of the variance-stabilising wrapper -- TEST
INFRASTRUCTURE ONLY.

Only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never touches it.

The paper's observation model (eq. (1), y = x + n with n approximately
white Gaussian) holds for raw sensor data after a variance-stabilising
transform (Introduction).  For Poisson-Gaussian raw data
z = alpha p + n, p ~ Poisson(x / alpha), n ~ N(mu, sigma^2), the standard
choice is the generalised Anscombe transform (Murtagh, Starck and Bijaoui),
with the closed-form approximation of its exact unbiased inverse (Makitalo
and Foi):

  f(z)  = (2 / alpha) sqrt(max(alpha z + 3/8 alpha^2 + sigma^2 - alpha mu, 0))
  I(D)  = D^2/4 + sqrt(3/2)/4 D^-1 - 11/8 D^-2 + 5/8 sqrt(3/2) D^-3 - 1/8
          - (sigma / alpha)^2
  x_hat = alpha max(I(D), 0) + mu     for D >= 2 sqrt(3/8), else mu

f maps the data to unit-variance noise; I inverts the expectation of f (not
f itself), so that denoising in the stabilised domain gives an unbiased
estimate.  (The Anscombe part of I vanishes exactly at D = 2 sqrt(3/8) =
f(0) for sigma = 0, where the estimate is 0.)

The wrapper puts the stabilised image on the denoisers' 8-bit scale:
u = clip(rint(scale f(z) + offset), 0, 255), whose noise level is
sqrt(scale^2 + 1/12) (unit variance times scale^2, plus the rounding); the
estimate comes back as D = (u_hat - offset) / scale.  Because the 8-bit code
is an integer decided by floating point, ``forward_u8_f32`` evaluates it in
the kernel's FP32 operation order (no fused multiply-adds); every other
function here is FP64.
"""
from __future__ import annotations

import math

import numpy as np

SQ32 = math.sqrt(1.5)
D0 = 2.0 * math.sqrt(3.0 / 8.0)  # f(0) of the plain Anscombe transform


def forward(z, alpha: float, sigma: float, mu: float = 0.0):
    """Generalised Anscombe transform, FP64."""
    z = np.asarray(z, np.float64)
    return (2.0 / alpha) * np.sqrt(np.maximum(alpha * z + 0.375 * alpha * alpha + sigma * sigma - alpha * mu, 0.0))


def algebraic_inverse(D, alpha: float, sigma: float, mu: float = 0.0):
    """The inverse of f itself on its range: f(algebraic_inverse(D)) = D."""
    D = np.asarray(D, np.float64)
    return (alpha * alpha * D * D / 4.0 - 0.375 * alpha * alpha - sigma * sigma + alpha * mu) / alpha


def unbiased_inverse(D, alpha: float, sigma: float, mu: float = 0.0):
    """Closed-form approximation of the exact unbiased inverse, FP64."""
    D = np.asarray(D, np.float64)
    s = sigma / alpha
    Dc = np.maximum(D, D0)
    I = (Dc * Dc / 4.0 + SQ32 / 4.0 / Dc - 11.0 / 8.0 / (Dc * Dc) + 5.0 / 8.0 * SQ32 / (Dc * Dc * Dc) - 0.125
         - s * s)
    return np.where(D >= D0, alpha * np.maximum(I, 0.0) + mu, mu)


def constants(alpha: float, sigma: float, mu: float, scale: float):
    """FP32 constants of the 8-bit forward map: a = alpha, c = 3/8 alpha^2 +
    sigma^2 - alpha mu, k = 2 scale / alpha (computed in FP64, rounded)."""
    return (np.float32(alpha), np.float32(0.375 * alpha * alpha + sigma * sigma - alpha * mu),
            np.float32(2.0 * scale / alpha))


def forward_u8_f32(z, alpha: float, sigma: float, mu: float, scale: float, offset: float):
    """u = clip(rint(k sqrt(max(a z + c, 0)) + offset), 0, 255) in FP32, one
    rounding per operation in this order."""
    a, c, k = constants(alpha, sigma, mu, scale)
    z = np.asarray(z, np.float32)
    t = np.maximum(a * z + c, np.float32(0.0))  # a z rounded, then + c rounded
    u = k * np.sqrt(t) + np.float32(offset)
    return np.clip(np.rint(u), 0, 255).astype(np.uint8)


def noise_level(scale: float) -> float:
    """Noise standard deviation of the 8-bit stabilised image."""
    return math.sqrt(scale * scale + 1.0 / 12.0)


def restore_from_u8(u_hat, alpha: float, sigma: float, mu: float, scale: float, offset: float):
    """x_hat from a denoised stabilised image on the 8-bit scale, FP64."""
    D = (np.asarray(u_hat, np.float64) - offset) / scale
    return unbiased_inverse(D, alpha, sigma, mu)
