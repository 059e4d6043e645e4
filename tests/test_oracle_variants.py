"""Pins of the oracle's variants of the published method (CPU): the bior1.5
step-1 transform and the prefiltered step-1 matching of the high-noise
profile.  Each pin checks the oracle against something other than itself:
the defining conditions of the bior1.5 filters, an independent synthesis-side
construction of its matrix, brute-force matching on spectra computed with
scipy or plain matrix products, exact identities (sigma = 0, no threshold),
and the second numpy implementation on whole denoises."""
import numpy as np
import pytest
import scipy.fft

import numpy_bm3d as nb
import oracle
from paper_2403_03488_amd import synth

oracle.set_threads(4)


def test_bior15_taps_follow_from_their_conditions():
    # 10 taps symmetric about 1/2 (offsets -4..5): biorthogonal to the box
    # lowpass [1, 1]/sqrt2 (sum_k lo[k] box[k - 2n] = delta_n) and five zeros
    # at pi (sum_k (-1)^k k^p lo[k] = 0, p = 0..4) fix them uniquely
    offs = np.arange(-4, 6)
    tap = lambda o: (o if o >= 1 else 1 - o) - 1  # shared tap of offsets o and 1 - o
    A, b = [], []
    for n in (-2, -1, 0, 1, 2):
        row = np.zeros(5)
        for o in offs:
            if o in (2 * n, 2 * n + 1):
                row[tap(o)] += 1 / np.sqrt(2.0)
        A.append(row)
        b.append(1.0 if n == 0 else 0.0)
    for p in range(5):
        row = np.zeros(5)
        for o in offs:
            row[tap(o)] += (-1.0) ** o * float(o) ** p
        A.append(row)
        b.append(0.0)
    t, res, rank, _ = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)
    assert rank == 5 and res.sum() < 1e-24
    np.testing.assert_allclose(oracle.bior15_filters(), [t[tap(o)] for o in offs], atol=1e-15)


def test_bior15_matrix_is_the_normalised_inverse_of_its_synthesis_bank():
    F, I = oracle.bior15_matrix()
    Fs, Is = nb.bior15_pair()  # built from the synthesis side
    np.testing.assert_allclose(F, Fs, atol=1e-12)
    np.testing.assert_allclose(I, Is, atol=1e-12)
    np.testing.assert_allclose(F @ I, np.eye(8), atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(F, axis=1), 1.0, atol=1e-14)


def test_bior15_structure():
    F, I = oracle.bior15_matrix()
    # constants go to the coarsest approximation only, both ways
    np.testing.assert_allclose(F @ np.ones(8), np.sqrt(8.0) * np.eye(8)[0], atol=1e-14)
    np.testing.assert_allclose(I[:, 0], np.full(8, 1 / np.sqrt(8.0)), atol=1e-14)
    # the finest details are Haar differences of neighbouring pixels
    for k in range(4):
        e = np.zeros(8)
        e[2 * k], e[2 * k + 1] = 1 / np.sqrt(2.0), -1 / np.sqrt(2.0)
        np.testing.assert_allclose(np.abs(F[4 + k]), np.abs(e), atol=1e-14)
    # biorthogonal, not orthogonal: the inverse is not the transpose
    assert np.abs(F @ F.T - np.eye(8)).max() > 0.05


@pytest.mark.parametrize("n", [1, 4, 16])
def test_bior_transform3d_roundtrip_and_library(n):
    rng = np.random.default_rng(n)
    g = rng.uniform(0, 255, (n, 8, 8))
    s = oracle.transform3d(g, transform=oracle.T_BIOR15)
    np.testing.assert_allclose(oracle.transform3d(s, inverse=True, transform=oracle.T_BIOR15), g, atol=1e-10)
    np.testing.assert_allclose(s, nb.t3d(g, 1), atol=1e-10)
    # the DCT path is unchanged: scipy's orthonormal DCT-II
    np.testing.assert_allclose(oracle.transform3d(g), nb.t3d(g, 0), atol=1e-10)


def bruteforce_prefiltered(lum, S, nmax, tau, thr, transform, want_dist=False):
    """Literal definition with scipy/matrix spectra and Python sorting."""
    h, w = lum.shape
    if transform == oracle.T_DCT:
        spec = lambda p: scipy.fft.dctn(p, type=2, norm="ortho")
    else:
        F, _ = nb.bior15_pair()
        spec = lambda p: F @ p @ F.T
    co = {}
    for y in range(h - 7):
        for x in range(w - 7):
            c = spec(lum[y:y + 8, x:x + 8].astype(np.float64))
            co[y, x] = np.where(np.abs(c) > thr, c, 0.0)
    rows, cols = nb.grid(h), nb.grid(w)
    out_i, out_c = [], []
    for ry in rows:
        for rx in cols:
            wy, ny = nb.window(ry, h, S)
            wx, nx = nb.window(rx, w, S)
            cand = []
            for qy in range(wy, wy + ny):
                for qx in range(wx, wx + nx):
                    if (qy, qx) == (ry, rx):
                        continue
                    d = float(((co[ry, rx] - co[qy, qx]) ** 2).sum())
                    if d <= 64 * tau:
                        cand.append((d, qy * w + qx))
            cand.sort()
            m = min(1 + len(cand), nmax)
            n = 1 << (m.bit_length() - 1)
            row = [ry * w + rx] + [g for _, g in cand[:n - 1]]
            out_i.append(row + [-1] * (nmax - len(row)))
            out_c.append(n)
            if want_dist:
                dists.append(dict((g, d) for d, g in cand))
    if want_dist:
        return np.array(out_i, np.int32), np.array(out_c, np.int32), dists
    return np.array(out_i, np.int32), np.array(out_c, np.int32)


dists = []


def same_up_to_rounding_ties(oi, oc, bi, bc, bd, tol=1e-9):
    """Groups equal, except that members whose distances agree to rounding
    (exact ties in exact arithmetic: thresholded spectra often keep only
    the mean, a multiple of 1/8) may come in either order."""
    np.testing.assert_array_equal(oc, bc)
    for r in range(len(oc)):
        if np.array_equal(oi[r], bi[r]):
            continue
        d = bd[r]
        mine = [d[g] for g in oi[r, 1:oc[r]]]
        theirs = [d[g] for g in bi[r, 1:bc[r]]]
        assert all(g in d for g in oi[r, 1:oc[r]]), r
        np.testing.assert_allclose(sorted(mine), sorted(theirs), rtol=tol, atol=tol)
        np.testing.assert_allclose(mine, sorted(mine), rtol=tol, atol=tol)


@pytest.mark.parametrize("transform", [oracle.T_DCT, oracle.T_BIOR15])
@pytest.mark.parametrize("kind", ["random", "duplicates"])
def test_match_prefiltered_bruteforce(transform, kind):
    rng = np.random.default_rng(3 + transform)
    if kind == "random":
        lum = rng.integers(0, 256, (20, 23)).astype(np.uint8)
    else:  # repeated tiles: exact distance ties, broken by the lower index
        tile = rng.integers(0, 256, (5, 6))
        lum = np.tile(tile, (5, 4))[:22, :21].astype(np.uint8)
    # thresholds that are not multiples of 1/8: for integer pixels some
    # spectral coefficients are exact multiples of 1/8 (the mean, and the
    # Haar-type products of bior1.5), and a coefficient exactly at the
    # threshold is decided by rounding, differently by each implementation
    for thr, tau in ((60.3, np.inf), (0.0, 1500.0), (150.7, 400.0)):
        oi, oc = oracle.match_prefiltered(lum, 8, 16, tau, thr, transform)
        dists.clear()
        bi, bc, bd = bruteforce_prefiltered(lum, 8, 16, tau, thr, transform, want_dist=True)
        same_up_to_rounding_ties(oi, oc, bi, bc, bd)
        assert np.mean(np.all(oi == bi, axis=1)) > 0.8


@pytest.mark.parametrize("transform", [oracle.T_DCT, oracle.T_BIOR15])
def test_prefilter_threshold_is_strict_at_exact_ties(transform):
    # An 8x8 block of 100 at the corner of an image of 101.  The corner patch
    # is flat: its only nonzero coefficient is the 2-D mean term, exactly
    # 8 * 100 = 800 for both transforms (their first basis row is constant
    # 1/sqrt(8)).  Its neighbours hold some 101s, so their mean terms lie in
    # (800, 808].  At threshold 800 the corner's spectrum vanishes (800 is not
    # > 800) and every other patch is at least 800^2 away: with 64 tau = 6400
    # the corner reference groups alone.  Just below the tie its mean term is
    # kept and the neighbours come within 8^2 + (small AC) of it.
    lum = np.full((24, 24), 101, np.uint8)
    lum[:8, :8] = 100
    idx, cnt = oracle.match_prefiltered(lum, 16, 16, 100.0, 800.0, transform)
    assert idx[0, 0] == 0
    assert cnt[0] == 1
    idx2, cnt2 = oracle.match_prefiltered(lum, 16, 16, 100.0, 800.0 - 1e-6, transform)
    assert idx2[0, 0] == 0
    assert cnt2[0] == 16


def test_prefilter_without_threshold_is_plain_matching():
    # the orthonormal DCT keeps distances: with nothing thresholded the
    # spectral distance is the pixel SSD, so the groups hold the same
    # distances as the integer matcher's (members of equal SSD may swap)
    lum = synth.small_gray().noisy
    oi, oc = oracle.match_prefiltered(lum, 16, 16, 2500.0, -1.0, oracle.T_DCT)
    ui, uc = oracle.match_u8(lum, 16, 16, 2500.0)
    np.testing.assert_array_equal(oc, uc)
    P = nb.all_patches(lum.astype(np.float64))
    w = lum.shape[1]
    for r in range(len(oc)):
        ref = P[ui[r, 0] // w, ui[r, 0] % w]
        dist = lambda row: sorted(float(((P[g // w, g % w] - ref) ** 2).sum()) for g in row[1:oc[r]])
        assert dist(oi[r]) == dist(ui[r])


def test_bior_sigma_zero_is_identity():
    s = synth.small_gray()
    p = oracle.Params(16, 16, 16, 32, 2.7, 2500.0, 400.0, 2.0, oracle.T_BIOR15, 2.0)
    out = oracle.denoise(s.noisy, 0.0, p)
    np.testing.assert_allclose(out, s.noisy.astype(np.float64), atol=1e-9)


def test_bior_singleton_groups_are_patchwise_hard_thresholding():
    # tau = 0 and a noise-free-distinct image: every group is its reference
    # alone, so step 1 is per-patch 2-D bior1.5 hard thresholding with weight
    # 1/N_kept and the Kaiser window
    rng = np.random.default_rng(11)
    img = rng.integers(0, 256, (19, 22)).astype(np.uint8)
    sigma = 20.0
    p = oracle.Params(8, 8, 16, 32, 2.7, 0.0, 0.0, 2.0, oracle.T_BIOR15, 0.0)
    _, inter = oracle.denoise(img, sigma, p, want_intermediates=True)
    assert np.all(inter["cnt1"] == 1)
    F, I = nb.bior15_pair()
    K = np.outer(np.kaiser(8, 2.0), np.kaiser(8, 2.0))
    num = np.zeros(img.shape)
    den = np.zeros(img.shape)
    for ry in nb.grid(19):
        for rx in nb.grid(22):
            c = F @ img[ry:ry + 8, rx:rx + 8].astype(np.float64) @ F.T
            keep = np.abs(c) > float(np.float64(2.7) * sigma)
            wt = 1.0 / keep.sum() if keep.any() else 1.0
            num[ry:ry + 8, rx:rx + 8] += wt * K * (I @ np.where(keep, c, 0.0) @ I.T)
            den[ry:ry + 8, rx:rx + 8] += wt * K
    np.testing.assert_allclose(inter["basic"][0], num / den, atol=1e-9)


@pytest.mark.parametrize("colour", [False, True])
@pytest.mark.parametrize("transform,lam2d", [(1, 0.0), (0, 2.0), (1, 2.0)])
def test_variants_match_the_numpy_implementation(colour, transform, lam2d):
    # sigma 49.7: the prefilter threshold 2 sigma is not a multiple of 1/8,
    # so no coefficient of integer patches sits exactly on it (such ties
    # would be decided by each implementation's rounding)
    sigma = 49.7
    if colour:
        s = synth.colour_481x321(h=22, w=25, sigma=sigma)
    else:
        s = synth.small_gray(h=24, w=27, sigma=sigma)
    p = oracle.Params(16, 16, 16, 32, 2.7, 5000.0, 3500.0, 2.0, transform, lam2d)
    out, inter = oracle.denoise(s.noisy, sigma, p, want_intermediates=True)
    ref, basic, groups = nb.denoise(s.noisy, sigma, tau_ht=5000.0, tau_wie=3500.0, transform=transform,
                                    lam2d=lam2d)
    np.testing.assert_array_equal(inter["idx1"], groups[0])
    np.testing.assert_allclose(inter["basic"], basic, atol=1e-9)
    np.testing.assert_allclose(out, ref, atol=1e-9)
