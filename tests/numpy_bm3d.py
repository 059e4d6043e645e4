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


def match(lum, S, nmax, tau):
    lum = np.asarray(lum, np.float64)
    h, w = lum.shape
    P = all_patches(lum)
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


def t3d(group):
    n = group.shape[0]
    H = scipy.linalg.hadamard(n) / np.sqrt(n)
    s2 = scipy.fft.dctn(group, type=2, norm="ortho", axes=(1, 2))
    return np.tensordot(H, s2, axes=(1, 0))


def it3d(spec):
    n = spec.shape[0]
    H = scipy.linalg.hadamard(n) / np.sqrt(n)
    g2 = np.tensordot(H.T, spec, axes=(1, 0))
    return scipy.fft.idctn(g2, type=2, norm="ortho", axes=(1, 2))


def filt(noisy, basic, sigma, step, idx, cnt, lam=2.7, beta=2.0):
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
            S = t3d(G)
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
            E = it3d(S)
            for m, (y, x) in enumerate(zip(ys, xs)):
                num[k, y:y + 8, x:x + 8] += wt * K * E[m]
                den[k, y:y + 8, x:x + 8] += wt * K
    return num, den


def denoise(img, sigma, S_ht=16, S_wie=16, n_ht=16, n_wie=32, tau_ht=2500.0, tau_wie=400.0,
            lam=2.7, beta=2.0):
    img = np.asarray(img)
    if img.ndim == 2:
        Z = img[None].astype(np.float64)
        L1 = img.astype(np.float64)
    else:
        Z = np.einsum("kc,hwc->khw", OPP, img.astype(np.float64))
        s = img.astype(np.int64).sum(-1)
        L1 = np.floor((s + 1) / 3.0)
    i1, c1 = match(L1, S_ht, n_ht, tau_ht)
    num, den = filt(Z, None, sigma, 1, i1, c1, lam, beta)
    B = num / den
    L2 = B[0] if img.ndim == 2 else B[0] / np.sqrt(3.0)
    i2, c2 = match(L2, S_wie, n_wie, tau_wie)
    num, den = filt(Z, B, sigma, 2, i2, c2, lam, beta)
    E = num / den
    if img.ndim == 2:
        return E[0], B, (i1, c1, i2, c2)
    return np.einsum("kc,khw->hwc", OPP, E), B, (i1, c1, i2, c2)
