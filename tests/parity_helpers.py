"""Helpers shared by the GPU parity tests: running the HIP stages through the
binding, and deciding which pixels a floating-point threshold decision near
its boundary may legitimately change (compare what is unique, check the rest).

Tolerances (derived from the arithmetic, not tuned):
  * HT_MARGIN: the FP32 3-D spectrum is a chain of 64-term, 16/32-term and
    64-term products of values |x| <= 441 with |basis| <= 0.25; a worst-case
    rounding bound of the chain is ~0.02 in coefficient units.  Both sides
    report each group's number of kept coefficients; a group whose counts
    differ must have an oracle coefficient within HT_MARGIN of lambda*sigma
    (a legitimate near-tie), and the pixels it aggregates into are excluded.
  * D_REL: an FP32 sum of 64 squared differences has relative error below
    66 * 2^-24 ~ 4e-6; step-2 selections are checked as valid top-n sets
    under a 1e-5 relative tolerance.
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

HT_MARGIN = 0.05
D_REL = 1e-5
FP32_TOL = 1e-3  # max |difference| on the [0,255] scale for the FP32 form


def patch_cover(idx, cnt, refs, h, w):
    """Pixels covered by the member patches of the selected references."""
    m = np.zeros((h, w), bool)
    for r in np.nonzero(refs)[0]:
        for g in idx[r, :cnt[r]]:
            y, x = divmod(int(g), w)
            m[y:y + 8, x:x + 8] = True
    return m


def groups_touching(idx, cnt, mask, h, w):
    """References whose group has a member patch overlapping mask."""
    box = sliding_window_view(mask, (8, 8)).any(axis=(2, 3))  # [h-7, w-7]
    flat = box.reshape(-1)
    pos = idx.copy()
    pos[pos < 0] = 0
    ys, xs = pos // w, pos % w
    hit = flat[ys * (w - 7) + xs]
    valid = np.arange(idx.shape[1])[None, :] < cnt[:, None]
    return (hit & valid).any(axis=1)


def kaiser_den(wsum, beta):
    """Aggregation denominator from per-position weight sums (FP64):
    den[k, y, x] = sum over u, v < 8 of wsum[k, y-u, x-v] K[u] K[v], with K
    numpy's Kaiser window.  The filters report weights this way; summing
    w K(u) K(v) over the 64 pixels of every aggregated patch gives the same
    denominator."""
    K = np.kaiser(8, beta)
    ws = np.asarray(wsum, np.float64)
    _, h, w = ws.shape
    den = np.zeros_like(ws)
    for u in range(8):
        for v in range(8):
            den[:, u:, v:] += K[u] * K[v] * ws[:, :h - u, :w - v]
    return den


# fixed-point accumulators: value = integer * 2^-frac (num: 28, wsum: 40 bits)
FRAC = {"num": 28, "wsum": 40}


def from_fix(a, buffer):
    """Real values (float64) of int64 fixed-point accumulators."""
    return np.asarray(a).astype(np.float64) * 2.0 ** -FRAC[buffer]


def to_fix(a, buffer):
    """Nearest fixed-point integers of real values."""
    return np.rint(np.asarray(a, np.float64) * 2.0 ** FRAC[buffer]).astype(np.int64)


def oracle_params(sigma, S=32):
    """The oracle's parameters for a noise level, with the values the HIP
    path receives: lambda = 2.7 rounded to FP32, as in bm3d_params.  Some
    spectral coefficients (the 2-D mean of a group, along any Walsh row) are
    exact multiples of 1/32, and so is lambda*sigma at these noise levels:
    an exact tie is not kept (strict >).  With lambda as the FP32 value the
    FP64 oracle's threshold sits just above the tie, as the exact rule
    says; with lambda = 2.7 in FP64 its rounding would keep some of them."""
    import oracle
    p = oracle.Params.for_sigma(sigma, S)
    p.lambda_ht = float(np.float32(p.lambda_ht))
    return p


def anchored_masks(idx1, cnt1, flips, idx2, cnt2, h, w):
    """Pixels an FP32 run may legitimately change: those aggregated from the
    step-1 groups whose threshold decision differs (a near-tie), and then
    every pixel of a step-2 group that reads one of them (through the basic
    estimate).  Returns (step-1 mask, final mask)."""
    m1 = patch_cover(idx1, cnt1, flips, h, w)
    t2 = groups_touching(idx2, cnt2, m1, h, w)
    return m1, patch_cover(idx2, cnt2, t2, h, w)


def all_patches(plane):
    h, w = plane.shape
    return sliding_window_view(np.asarray(plane, np.float64), (8, 8)).reshape(h - 7, w - 7, 64)


def window(i, length, S):
    npos = length - 7
    if npos <= S:
        return 0, npos
    return min(max(i - S // 2, 0), npos - S), S


def check_topn_valid(lum, ref_yx, S, nmax, tau, gpu_idx_row, gpu_cnt, P=None):
    """Is the GPU group a valid ordered top-n of the exact (float64) distances
    on the same input, up to FP32 rounding of the distances?  Returns a string
    describing the first violation, or None."""
    h, w = lum.shape
    if P is None:
        P = all_patches(lum)
    ry, rx = ref_yx
    wy, ny = window(ry, h, S)
    wx, nx = window(rx, w, S)
    d = ((P[wy:wy + ny, wx:wx + nx] - P[ry, rx]) ** 2).sum(-1).ravel()
    yy, xx = np.mgrid[wy:wy + ny, wx:wx + nx]
    gi = (yy * w + xx).ravel()
    tol = D_REL * d + 1e-6
    not_ref = gi != ry * w + rx
    T = 64.0 * tau
    surely = not_ref & (d + tol < T) if np.isfinite(T) else not_ref
    maybe = not_ref & (d - tol <= T) if np.isfinite(T) else not_ref
    lo, hi = int(surely.sum()), int(maybe.sum())
    ok_n = {1 << (min(1 + k, nmax).bit_length() - 1) for k in range(lo, hi + 1)}
    if gpu_cnt not in ok_n:
        return "group size %d not in %s" % (gpu_cnt, sorted(ok_n))
    row = list(gpu_idx_row[:gpu_cnt])
    if row[0] != ry * w + rx:
        return "slot 0 is not the reference"
    if any(v != -1 for v in gpu_idx_row[gpu_cnt:]):
        return "unused slots not -1"
    pos = {int(g): k for k, g in enumerate(gi)}
    members = row[1:]
    if len(set(members)) != len(members):
        return "duplicate members"
    for g in members:
        if g not in pos or not maybe[pos[g]]:
            return "member %d not a candidate" % g
    dm = np.array([d[pos[g]] for g in members])
    tm = np.array([tol[pos[g]] for g in members])
    if len(dm) > 1 and np.any(dm[1:] + tm[1:] + tm[:-1] < dm[:-1]):
        return "members out of order"
    if len(dm):
        chosen = np.zeros(len(d), bool)
        chosen[[pos[g] for g in members]] = True
        rest = surely & ~chosen
        if np.any(d[rest] + tol[rest] < dm[-1] - tm[-1]):
            return "a closer candidate was left out"
    return None
