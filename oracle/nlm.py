"""FP64 CPU oracle of the NL-means first stage -- TEST INFRASTRUCTURE ONLY.

Only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never touches it.

The paper offers NL-means as the alternative non-local first stage (the
NLM-G column of Table 3 and the "Ours-FL (NLM)" results, Section III); it
gives none of its internals, so this follows the published pixelwise
NL-means of Buades, Coll and Morel that it cites:

  u_hat(p) = sum_q w(p, q) u(q) / sum_q w(p, q),   q in the search window of p
  d2(p, q) = mean over the patch offsets k and the channels c of
             (u_c(p + k) - u_c(q + k))^2
  w(p, q)  = exp(-max(d2(p, q) - 2 sigma^2, 0) / h^2)   for q != p
  w(p, p)  = max over q != p of w(p, q)

with a (2f+1)^2 patch, a (2r+1)^2 search window clipped to the image, patch
pixels outside the image read from its symmetric extension, and (f, r, h)
from the published sigma table (params_default).  Every weight is evaluated
relative to the smallest exponent E_min of the window (a common factor, so
the ratio is unchanged); the centre weight is then exactly 1 and no sum
underflows.
"""
from __future__ import annotations

import math

import numpy as np

# (sigma upper bound, patch radius f, search radius r, h / sigma): grey, colour
_GREY = ((15.0, 1, 10, 0.40), (30.0, 2, 10, 0.40), (45.0, 3, 17, 0.35), (75.0, 4, 17, 0.35),
         (math.inf, 5, 17, 0.30))
_COLOUR = ((25.0, 1, 10, 0.55), (55.0, 2, 17, 0.40), (math.inf, 3, 17, 0.35))


def params_default(sigma: float, channels: int):
    """(f, r, h) of the published NL-means parameter table for this sigma."""
    if not sigma > 0:
        raise ValueError("sigma must be positive")
    for top, f, r, k in (_GREY if channels == 1 else _COLOUR):
        if sigma <= top:
            return f, r, k * sigma
    raise AssertionError


def _planes(img):
    a = np.asarray(img, dtype=np.float64)
    if a.ndim == 2:
        return a[None], 1
    return np.moveaxis(a, 2, 0), a.shape[2]


def _offsets(r):
    return [(dy, dx) for dy in range(-r, r + 1) for dx in range(-r, r + 1) if (dy, dx) != (0, 0)]


def _exponent(u, pad, g, sigma, f, dy, dx):
    """max(d2(p, p + o) - 2 sigma^2, 0) for every pixel p, +inf where p + o
    lies outside the image (o = (dy, dx))."""
    C, H, W = u.shape
    d2 = np.zeros((H, W))
    for ky in range(-f, f + 1):
        for kx in range(-f, f + 1):
            a = pad[:, g + ky:g + ky + H, g + kx:g + kx + W]
            b = pad[:, g + dy + ky:g + dy + ky + H, g + dx + kx:g + dx + kx + W]
            d2 += ((a - b) ** 2).sum(axis=0)
    d2 /= C * (2 * f + 1) ** 2
    e = np.maximum(d2 - 2.0 * sigma * sigma, 0.0)
    yy, xx = np.mgrid[0:H, 0:W]
    inside = (yy + dy >= 0) & (yy + dy < H) & (xx + dx >= 0) & (xx + dx < W)
    return np.where(inside, e, np.inf)


def exponents(img, sigma: float, f: int, r: int):
    """E[o, y, x] = max(d2(p, p + o) - 2 sigma^2, 0) for every search offset o
    = (dy, dx) in [-r, r]^2 except (0, 0), row-major; +inf where p + o lies
    outside the image.  Also returns the offsets.  (Small images only: it
    holds every offset at once.)"""
    u, _ = _planes(img)
    g = f + r
    pad = np.pad(u, ((0, 0), (g, g), (g, g)), mode="symmetric")
    offs = _offsets(r)
    return np.stack([_exponent(u, pad, g, sigma, f, dy, dx) for dy, dx in offs]), offs


def nlm(img, sigma: float, f: int | None = None, r: int | None = None, h: float | None = None):
    """NL-means estimate (FP64, same layout as the input: HxW or HxWxC, on the
    [0, 255] scale, unclipped)."""
    u, C = _planes(img)
    _, H, W = u.shape
    df, dr, dh = params_default(sigma, C)
    f = df if f is None else f
    r = dr if r is None else r
    h = dh if h is None else h
    if not h > 0:
        raise ValueError("h must be positive")
    g = f + r
    pad = np.pad(u, ((0, 0), (g, g), (g, g)), mode="symmetric")
    offs = _offsets(r)
    # first pass: the smallest exponent of each window (+inf only where the
    # window holds p alone); second pass: the weights relative to it
    Emin = np.full((H, W), np.inf)
    for dy, dx in offs:
        Emin = np.minimum(Emin, _exponent(u, pad, g, sigma, f, dy, dx))
    num = u.copy()        # the centre, weight exp(-(E_min - E_min)/h^2) = 1
    den = np.ones((H, W))
    for dy, dx in offs:
        E = _exponent(u, pad, g, sigma, f, dy, dx)
        w = np.where(np.isfinite(E), np.exp(-(E - Emin) / (h * h)), 0.0)  # 0 outside
        num += w * pad[:, g + dy:g + dy + H, g + dx:g + dx + W]
        den += w
    out = num / den
    return out[0] if C == 1 else np.moveaxis(out, 0, 2)
