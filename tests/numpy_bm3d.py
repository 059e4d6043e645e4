"""A second, independent FP64 BM3D written with numpy/scipy, used only to pin
the C oracle on tiny images.  It shares no code with the oracle: transforms
come from scipy.fft / scipy.linalg.hadamard / numpy.kaiser, matching is
vectorised brute force with numpy.lexsort, aggregation uses numpy.add.at.
The method and every reading are the same as the oracle's (two-step BM3D,
8x8 patches, stride 3, opponent colour with luminance grouping)."""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg
from numpy.lib.stride_tricks import sliding_window_view

PATCH, STRIDE = 8, 3
OPP = np.array([[1, 1, 1] / np.sqrt(3.0),
                [1, 0, -1] / np.sqrt(2.0),
                [1, -2, 1] / np.sqrt(6.0)])


def grid(length):
    last = length - PATCH
    p = list(range(0, last + 1, STRIDE))
    if p[-1] != last:
        p.append(last)
    return np.array(p)


def window(i, length, S):
    npos = length - PATCH + 1
    if npos <= S:
        return 0, npos
    return min(max(i - S // 2, 0), npos - S), S


def all_patches(plane):
    h, w = plane.shape
    return sliding_window_view(plane, (PATCH, PATCH)).reshape(h - 7, w - 7, 64)


def match(lum, S, nmax, tau, P=None, shape=None):
    if P is None:
        lum = np.asarray(lum, np.float64)
        h, w = lum.shape
        P = all_patches(lum)
    else:
        h, w = shape
    rows, cols = grid(h), grid(w)
    idx = np.full((len(rows) * len(cols), nmax), -1, np.int32)
    cnt = np.zeros(len(rows) * len(cols), np.int32)
    r = 0
    for ry in rows:
        for rx in cols:
            wy, ny = window(ry, h, S)
            wx, nx = window(rx, w, S)
            cand = P[wy:wy + ny, wx:wx + nx]
            d = ((cand - P[ry, rx]) ** 2).sum(-1)
            yy, xx = np.mgrid[wy:wy + ny, wx:wx + nx]
            gi = (yy * w + xx).ravel()
            d = d.ravel()
            keep = (gi != ry * w + rx) & (d <= 64.0 * tau)
            d, gi = d[keep], gi[keep]
            order = np.lexsort((gi, d))
            m = min(1 + len(order), nmax)
            n = 1 << (m.bit_length() - 1)
            idx[r, 0] = ry * w + rx
            idx[r, 1:n] = gi[order[:n - 1]]
            cnt[r] = n
            r += 1
    return idx, cnt


# bior1.5 through its synthesis bank (the oracle builds it from the analysis
# side): box lowpass at offsets 0, 1 and the highpass g[j] = (-1)^j lo[1-j],
# lo the 10-tap spline lowpass at offsets -4..5; three periodic levels.
BIOR_LO = np.array([3, -3, -22, 22, 128, 128, 22, -22, -3, 3]) * np.sqrt(2.0) / 256.0


def _synthesis_level(n):
    """n x n operator taking [a (n/2), d (n/2)] to a periodic signal of length n."""
    S = np.zeros((n, n))
    for k in range(n // 2):
        S[(2 * k) % n, k] += 1 / np.sqrt(2.0)
        S[(2 * k + 1) % n, k] += 1 / np.sqrt(2.0)
        for j in range(-4, 6):
            S[(2 * k + j) % n, n // 2 + k] += (-1.0) ** j * BIOR_LO[(1 - j) + 4]
    return S


def bior15_pair():
    """(F, I): forward matrix with unit-norm rows (coefficients [a3, d3, d2,
    d1]) and its inverse, from the multilevel synthesis operator."""
    S = np.zeros((8, 8))
    for c in range(8):
        e = np.zeros(8)
        e[c] = 1.0
        a2 = _synthesis_level(2) @ e[0:2]                          # a3, d3 -> a2
        a1 = _synthesis_level(4) @ np.concatenate([a2, e[2:4]])    # a2, d2 -> a1
        S[:, c] = _synthesis_level(8) @ np.concatenate([a1, e[4:8]])  # a1, d1 -> x
    F = np.linalg.inv(S)
    F /= np.linalg.norm(F, axis=1, keepdims=True)
    return F, np.linalg.inv(F)


def t2d(group, transform):
    if transform == 0:
        return scipy.fft.dctn(group, type=2, norm="ortho", axes=(-2, -1))
    F, _ = bior15_pair()
    return np.einsum("au,...uv,bv->...ab", F, group, F)


def it2d(spec, transform):
    if transform == 0:
        return scipy.fft.idctn(spec, type=2, norm="ortho", axes=(-2, -1))
    _, I = bior15_pair()
    return np.einsum("ua,...ab,vb->...uv", I, spec, I)


def t3d(group, transform=0):
    n = group.shape[0]
    H = scipy.linalg.hadamard(n) / np.sqrt(n)
    return np.tensordot(H, t2d(group, transform), axes=(1, 0))


def it3d(spec, transform=0):
    n = spec.shape[0]
    H = scipy.linalg.hadamard(n) / np.sqrt(n)
    g2 = np.tensordot(H.T, spec, axes=(1, 0))
    return it2d(g2, transform)


def match_prefiltered(lum, S, nmax, tau, thr2d, transform):
    """Grouping on 2-D spectra of the patches hard-thresholded at thr2d
    (vectorised: all patch spectra at once, then brute-force windows)."""
    lum = np.asarray(lum, np.float64)
    h, w = lum.shape
    P = t2d(sliding_window_view(lum, (PATCH, PATCH)), transform)
    P = np.where(np.abs(P) > thr2d, P, 0.0).reshape(h - 7, w - 7, 64)
    return match(None, S, nmax, tau, P=P, shape=(h, w))


def filt(noisy, basic, sigma, step, idx, cnt, lam=2.7, beta=2.0, transform=0):
    c, h, w = noisy.shape
    kw = np.kaiser(PATCH, beta)
    K = np.outer(kw, kw)
    num = np.zeros_like(noisy)
    den = np.zeros_like(noisy)
    for r in range(len(cnt)):
        n = cnt[r]
        ys, xs = idx[r, :n] // w, idx[r, :n] % w
        for k in range(c):
            G = np.stack([noisy[k, y:y + 8, x:x + 8] for y, x in zip(ys, xs)])
            xf = transform if step == 1 else 0  # step 2 always uses the DCT
            S = t3d(G, xf)
            if step == 1:
                keep = np.abs(S) > lam * sigma
                S = np.where(keep, S, 0.0)
                nk = int(keep.sum())
                wt = 1.0 / nk if nk else 1.0
            else:
                B = t3d(np.stack([basic[k, y:y + 8, x:x + 8] for y, x in zip(ys, xs)]))
                den_w = B * B + sigma * sigma
                W = np.where(den_w > 0, B * B / np.where(den_w > 0, den_w, 1.0), 1.0)
                S = W * S
                # the Wiener weight 1/sum W^2, capped at 2^10
                wt = 1.0 / max(float((W * W).sum()), 2.0 ** -10)
            E = it3d(S, xf)
            for m, (y, x) in enumerate(zip(ys, xs)):
                num[k, y:y + 8, x:x + 8] += wt * K * E[m]
                den[k, y:y + 8, x:x + 8] += wt * K
    return num, den


def denoise(img, sigma, S_ht=16, S_wie=16, n_ht=16, n_wie=32, tau_ht=2500.0, tau_wie=400.0,
            lam=2.7, beta=2.0, transform=0, lam2d=0.0):
    img = np.asarray(img)
    if img.ndim == 2:
        Z = img[None].astype(np.float64)
        L1 = img.astype(np.float64)
    else:
        Z = np.einsum("kc,hwc->khw", OPP, img.astype(np.float64))
        s = img.astype(np.int64).sum(-1)
        L1 = np.floor((s + 1) / 3.0)
    if lam2d > 0:
        sl = sigma if img.ndim == 2 else sigma / np.sqrt(3.0)  # noise of the matching luminance
        i1, c1 = match_prefiltered(L1, S_ht, n_ht, tau_ht, lam2d * sl, transform)
    else:
        i1, c1 = match(L1, S_ht, n_ht, tau_ht)
    num, den = filt(Z, None, sigma, 1, i1, c1, lam, beta, transform)
    B = num / den
    L2 = B[0] if img.ndim == 2 else B[0] / np.sqrt(3.0)
    i2, c2 = match(L2, S_wie, n_wie, tau_wie)
    num, den = filt(Z, B, sigma, 2, i2, c2, lam, beta)
    E = num / den
    if img.ndim == 2:
        return E[0], B, (i1, c1, i2, c2)
    return np.einsum("kc,khw->hwc", OPP, E), B, (i1, c1, i2, c2)
