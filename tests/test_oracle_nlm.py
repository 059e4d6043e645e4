"""Pins of the FP64 NL-means oracle (no GPU): the definition brute-forced in
pure Python on tiny images (unnormalised weights, the centre weight taken
literally as the largest other weight, an independently written symmetric
extension), and closed forms -- a constant image is returned unchanged, and
where every weight is 1 (h huge, or sigma so large that every d2 <= 2 sigma^2)
the estimate is the plain mean over the clipped search window, computed with
scipy's 2-D convolution."""
import math

import numpy as np
import pytest
from scipy.signal import convolve2d

from oracle import nlm as O


def reflect(t, n):
    """Index of the symmetric extension (edge sample repeated), any distance."""
    t = t % (2 * n)
    return t if t < n else 2 * n - 1 - t


def brute(img, sigma, f, r, h):
    a = np.asarray(img, dtype=np.float64)
    if a.ndim == 2:
        a = a[:, :, None]
    H, W, C = a.shape
    P = (2 * f + 1) ** 2
    out = np.zeros_like(a)
    for y in range(H):
        for x in range(W):
            ws, vs = [], []
            for qy in range(max(0, y - r), min(H, y + r + 1)):
                for qx in range(max(0, x - r), min(W, x + r + 1)):
                    if (qy, qx) == (y, x):
                        continue
                    d2 = 0.0
                    for ky in range(-f, f + 1):
                        for kx in range(-f, f + 1):
                            for c in range(C):
                                pa = a[reflect(y + ky, H), reflect(x + kx, W), c]
                                pb = a[reflect(qy + ky, H), reflect(qx + kx, W), c]
                                d2 += (pa - pb) ** 2
                    d2 /= C * P
                    ws.append(math.exp(-max(d2 - 2 * sigma * sigma, 0.0) / (h * h)))
                    vs.append(a[qy, qx])
            wc = max(ws) if ws else 1.0
            num = wc * a[y, x] + sum(w * v for w, v in zip(ws, vs))
            out[y, x] = num / (wc + sum(ws))
    return out[:, :, 0] if np.asarray(img).ndim == 2 else out


@pytest.mark.parametrize("shape,sigma,f,r,h", [
    ((7, 9), 20.0, 1, 2, 12.0),
    ((6, 5, 3), 15.0, 1, 3, 9.0),      # window wider than the image
    ((5, 6), 25.0, 2, 2, 14.0),        # patches reflected over two edges
    ((8, 8), 5.0, 1, 3, 6.0),          # small sigma: the clamp rarely bites
])
def test_matches_brute_force(shape, sigma, f, r, h):
    rng = np.random.default_rng(7)
    img = rng.integers(0, 256, shape).astype(np.uint8)
    got = O.nlm(img, sigma, f=f, r=r, h=h)
    want = brute(img, sigma, f, r, h)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)


def test_exponents_brute_force():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, (6, 7)).astype(np.uint8)
    E, offs = O.exponents(img, 10.0, 1, 2)
    a = img.astype(np.float64)
    for i, (dy, dx) in enumerate(offs):
        for y in range(6):
            for x in range(7):
                qy, qx = y + dy, x + dx
                if not (0 <= qy < 6 and 0 <= qx < 7):
                    assert math.isinf(E[i, y, x])
                    continue
                d2 = sum((a[reflect(y + ky, 6), reflect(x + kx, 7)] - a[reflect(qy + ky, 6), reflect(qx + kx, 7)]) ** 2
                         for ky in range(-1, 2) for kx in range(-1, 2)) / 9
                assert abs(E[i, y, x] - max(d2 - 200.0, 0.0)) < 1e-9


@pytest.mark.parametrize("c", [1, 3])
def test_constant_image(c):
    img = np.full((20, 23) if c == 1 else (20, 23, 3), 137, np.uint8)
    out = O.nlm(img, 25.0)
    assert np.array_equal(out, img.astype(np.float64))


def window_mean(img, r):
    a = np.asarray(img, dtype=np.float64)
    k = np.ones((2 * r + 1, 2 * r + 1))
    cnt = convolve2d(np.ones(a.shape[:2]), k, mode="same")
    if a.ndim == 2:
        return convolve2d(a, k, mode="same") / cnt
    return np.stack([convolve2d(a[:, :, ch], k, mode="same") / cnt for ch in range(a.shape[2])], 2)


@pytest.mark.parametrize("c", [1, 3])
def test_huge_h_is_window_mean(c):
    rng = np.random.default_rng(11 + c)
    img = rng.integers(0, 256, (17, 21) if c == 1 else (17, 21, 3)).astype(np.uint8)
    out = O.nlm(img, 20.0, f=1, r=3, h=1e9)
    np.testing.assert_allclose(out, window_mean(img, 3), rtol=0, atol=1e-9)


def test_large_sigma_clamps_every_exponent():
    # every d2 <= 100 < 2 sigma^2: all weights are exp(0) = 1 whatever h is;
    # a sign error in the sigma term would make them differ
    rng = np.random.default_rng(5)
    img = rng.integers(0, 11, (15, 16)).astype(np.uint8)
    out = O.nlm(img, 100.0, f=1, r=4, h=0.5)
    np.testing.assert_allclose(out, window_mean(img, 4), rtol=0, atol=1e-9)
    # with a small sigma the same image is not averaged uniformly
    assert np.abs(O.nlm(img, 1.0, f=1, r=4, h=0.5) - window_mean(img, 4)).max() > 0.1


def test_params_table_shape():
    # the table covers every positive sigma, grows with it and keeps h > 0
    last = (0, 0)
    for s in np.linspace(0.5, 120, 60):
        f, r, h = O.params_default(float(s), 1)
        assert (f, r) >= last and h > 0
        last = (f, r)
    with pytest.raises(ValueError):
        O.params_default(0.0, 1)
