"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: step-1 grouping bit-exact; FP32 forms within 1e-3 on the [0,255] scale
wherever the result is uniquely defined (pixels reached by a hard-threshold
decision within rounding distance of lambda*sigma are excluded and counted);
step-2 groups valid ordered top-n sets of the exact distances up to FP32
rounding; BF16/FP16 transform forms within 0.05 dB PSNR of the FP32 form."""
import math

import numpy as np
import pytest

import oracle
import parity_helpers as ph
from paper_2403_03488_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

oracle.set_threads(8)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03488_amd import bm3d
    return bm3d


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gparams(B, sigma, S, xform=0, **kw):
    p = B.params_default(sigma, search_ht=S, search_wie=S, xform=xform)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def oparams(p):
    return oracle.Params(p.search_ht, p.search_wie, p.n_ht, p.n_wie, float(p.lambda_ht),
                         float(p.tau_ht), float(p.tau_wie), float(p.kaiser_beta))


def log(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ prep ---

@pytest.mark.parametrize("shape", [(64, 64), (37, 53, 3), (8, 8), (9, 100, 3)])
def test_prepare(B, shape):
    img = np.random.default_rng(1).integers(0, 256, shape).astype(np.uint8)
    c = 1 if len(shape) == 2 else 3
    h, w = shape[:2]
    planar = torch.empty((c, h, w), dtype=torch.float32, device="cuda")
    lum = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    B.prepare(dev(img), planar, lum)
    op, ol = oracle.prepare(img)
    np.testing.assert_array_equal(host(lum), ol)
    np.testing.assert_allclose(host(planar), op, atol=1e-4)


# ---------------------------------------------------------- step-1 match ---

def match1_cases():
    yield "small_gray", synth.small_gray().noisy, 16, 2500.0, 16
    for s in (15, 25, 50):
        yield "gray512_s%d" % s, synth.gray_512(sigma=s).noisy, 32, (5000.0 if s > 40 else 2500.0), 16
    rng = np.random.default_rng(7)
    yield "ragged_37x53", rng.integers(0, 256, (37, 53)).astype(np.uint8), 32, 2500.0, 16
    yield "tiny_8x8", rng.integers(0, 256, (8, 8)).astype(np.uint8), 32, np.inf, 16
    yield "thin_9x100", rng.integers(0, 256, (9, 100)).astype(np.uint8), 16, np.inf, 32
    yield "low_entropy", rng.integers(0, 3, (70, 90)).astype(np.uint8), 32, np.inf, 32
    yield "constant", np.full((50, 61), 200, np.uint8), 32, 2500.0, 16
    yield "tau0", rng.integers(0, 256, (40, 40)).astype(np.uint8), 8, 0.0, 16
    yield "saturated", np.clip(rng.normal(250, 20, (64, 80)), 0, 255).astype(np.uint8), 32, 400.0, 32


@pytest.mark.parametrize("case", list(match1_cases()), ids=lambda c: c[0])
def test_match1_bit_exact(B, case):
    name, lum, S, tau, nmax = case
    log("match1 %s %s S=%d tau=%s n=%d" % (name, lum.shape, S, tau, nmax))
    h, w = lum.shape
    p = gparams(B, 25.0, S, n_ht=nmax, tau_ht=tau)
    R = B.num_refs(h, w)
    idx = torch.full((R, nmax), -7, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(R, dtype=torch.int32, device="cuda")
    B.block_match(dev(lum), 1, p, idx, cnt)
    oi, oc = oracle.match_u8(lum, S, nmax, float(p.tau_ht))
    gi, gc = host(idx), host(cnt)
    np.testing.assert_array_equal(gc, oc)
    np.testing.assert_array_equal(gi, oi)


# --------------------------------------------------------- step-1 filter ---

def filter1_compare(B, img, sigma, S, xform=0):
    c = 1 if img.ndim == 2 else 3
    h, w = img.shape[:2]
    p = gparams(B, sigma, S, xform=xform)
    op = oparams(p)
    planar, lum = oracle.prepare(img)
    oi, oc = oracle.match_u8(lum, S, p.n_ht, float(p.tau_ht))
    onum, oden, margin, onk = oracle.collab_filter(planar, None, sigma, 1, oi, oc, op, want_margin=True)
    num = torch.zeros((c, h, w), dtype=torch.float32, device="cuda")
    wsum = torch.zeros((c, h, w), dtype=torch.float32, device="cuda")
    gnk = torch.full((c, len(oc)), -1, dtype=torch.int32, device="cuda")
    p.debug_nkept = gnk.data_ptr()
    B.collab_filter(dev(planar.astype(np.float32)), None, sigma, 1, dev(oi), dev(oc), p, num, wsum)
    basic = torch.empty((c, h, w), dtype=torch.float32, device="cuda")
    B.aggregate(num, wsum, False, p, basic)
    gws = host(wsum)
    # weights sit at patch corners only
    assert not gws[:, h - 7:, :].any() and not gws[:, :, w - 7:].any()
    gden = ph.kaiser_den(gws, p.kaiser_beta)
    flips = (host(gnk) != onk).any(axis=0)
    # every threshold decision that differs must sit within rounding of lambda*sigma
    assert np.all(margin[flips] < ph.HT_MARGIN), margin[flips]
    taint = ph.patch_cover(oi, oc, flips, h, w)
    ok = ~taint
    gb, ob = host(basic), onum / oden
    err = np.abs(gb - ob)[:, ok]
    log("filter1 %s: groups with a differing threshold decision %d of %d (%.3f%% px), "
        "max|basic diff| %.2e (rest), %.2e (all)" %
        (img.shape, flips.sum(), len(flips), 100 * taint.mean(), err.max(), np.abs(gb - ob).max()))
    return err, taint, gden, oden, ok


@pytest.mark.parametrize("which", ["small_gray", "gray512", "colour"])
def test_filter1_fp32(B, which):
    if which == "small_gray":
        s = synth.small_gray()
        err, taint, gden, oden, ok = filter1_compare(B, s.noisy, 25.0, 16)
    elif which == "gray512":
        s = synth.gray_512()
        err, taint, gden, oden, ok = filter1_compare(B, s.noisy, 25.0, 32)
    else:
        s = synth.colour_481x321()
        err, taint, gden, oden, ok = filter1_compare(B, s.noisy, 25.0, 32)
    assert err.max() <= ph.FP32_TOL
    assert taint.mean() < 0.05
    np.testing.assert_allclose(gden[:, ok], oden[:, ok], rtol=1e-5)


# ---------------------------------------------------------- step-2 match ---

@pytest.mark.parametrize("which", ["small_gray", "gray512"])
def test_match2_valid_topn(B, which):
    s = synth.small_gray() if which == "small_gray" else synth.gray_512()
    S = 16 if which == "small_gray" else 32
    p = gparams(B, 25.0, S)
    _, inter = oracle.denoise(s.noisy, 25.0, oparams(p), want_intermediates=True)
    lum32 = inter["basic"][0].astype(np.float32)
    h, w = lum32.shape
    R = B.num_refs(h, w)
    idx = torch.full((R, 32), -7, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(R, dtype=torch.int32, device="cuda")
    B.block_match(dev(lum32), 2, p, idx, cnt)
    gi, gc = host(idx), host(cnt)
    oi, oc = oracle.match_f64(lum32.astype(np.float64), S, 32, float(p.tau_wie))
    same = np.all(gi == oi, axis=1)
    log("match2 %s: identical groups %.3f%%" % (which, 100 * same.mean()))
    rows, cols = oracle.ref_positions(h), oracle.ref_positions(w)
    P = ph.all_patches(lum32)
    check = np.nonzero(~same)[0]
    rng = np.random.default_rng(0)
    sample = rng.choice(R, size=min(R, 1500), replace=False)
    for r in np.unique(np.concatenate([check, sample])):
        ry, rx = rows[r // len(cols)], cols[r % len(cols)]
        why = ph.check_topn_valid(lum32, (ry, rx), S, 32, float(p.tau_wie), gi[r], gc[r], P)
        assert why is None, "ref %d: %s" % (r, why)
    assert same.mean() > 0.95


# --------------------------------------------------------- step-2 filter ---

@pytest.mark.parametrize("which", ["small_gray", "gray512", "colour"])
def test_filter2_fp32(B, which):
    if which == "small_gray":
        s, S = synth.small_gray(), 16
    elif which == "gray512":
        s, S = synth.gray_512(), 32
    else:
        s, S = synth.colour_481x321(), 32
    img = s.noisy
    p = gparams(B, 25.0, S)
    op = oparams(p)
    _, inter = oracle.denoise(img, 25.0, op, want_intermediates=True)
    planar, _ = oracle.prepare(img)
    basic32 = inter["basic"].astype(np.float32)
    oi, oc = inter["idx2"], inter["cnt2"]
    onum, oden = oracle.collab_filter(planar, basic32.astype(np.float64), 25.0, 2, oi, oc, op)
    c, h, w = planar.shape
    num = torch.zeros((c, h, w), dtype=torch.float32, device="cuda")
    wsum = torch.zeros((c, h, w), dtype=torch.float32, device="cuda")
    B.collab_filter(dev(planar.astype(np.float32)), dev(basic32), 25.0, 2, dev(oi), dev(oc), p, num, wsum)
    est = torch.empty((c, h, w), dtype=torch.float32, device="cuda")
    B.aggregate(num, wsum, False, p, est)
    g, o = host(est), onum / oden
    np.testing.assert_allclose(ph.kaiser_den(host(wsum), p.kaiser_beta), oden, rtol=1e-5)
    log("filter2 %s: max|diff| %.2e" % (which, np.abs(g - o).max()))
    assert np.abs(g - o).max() <= ph.FP32_TOL


# -------------------------------------------------------------- aggregate ---

@pytest.mark.parametrize("c", [1, 3])
def test_aggregate(B, c):
    # shapes that leave partial 16 x 64 aggregation tiles in both directions
    rng = np.random.default_rng(c)
    num = rng.uniform(-100, 300, (c, 33, 147)).astype(np.float32)
    wsum = rng.uniform(0.05, 1, (c, 33, 147)).astype(np.float32)
    p = gparams(B, 25.0, 16)
    den = ph.kaiser_den(wsum, p.kaiser_beta)
    gnum, gws = dev(num), dev(wsum)
    out = torch.empty((33, 147, c) if c == 3 else (c, 33, 147), dtype=torch.float32, device="cuda")
    B.aggregate(gnum, gws, True, p, out)
    ref = oracle.aggregate(num.astype(np.float64), den, True)
    # FP32 denominator (two 8-term FMA chains) and division: relative error ~1e-6
    np.testing.assert_allclose(host(out).reshape(ref.shape), ref, rtol=1e-5, atol=1e-4)
    basic = torch.empty((c, 33, 147), dtype=torch.float32, device="cuda")
    B.aggregate(gnum, gws, False, p, basic)
    np.testing.assert_allclose(host(basic), oracle.aggregate(num.astype(np.float64), den, False),
                               rtol=1e-5, atol=1e-4)
    lum = torch.empty((33, 147), dtype=torch.float32, device="cuda")
    B.luminance(basic, lum)
    np.testing.assert_allclose(host(lum), oracle.luminance(host(basic).astype(np.float64)), atol=1e-4)


# ------------------------------------------------------ whole path, anchored ---

def gpu_chain_with_idx2(B, img, sigma, p, idx2, cnt2):
    """HIP stages end to end, except that the step-2 groups are the oracle's."""
    c = 1 if img.ndim == 2 else 3
    h, w = img.shape[:2]
    R = B.num_refs(h, w)
    gnk = torch.full((c, R), -1, dtype=torch.int32, device="cuda")
    p = p.copy()
    p.debug_nkept = gnk.data_ptr()
    planar = torch.empty((c, h, w), dtype=torch.float32, device="cuda")
    lum = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    B.prepare(dev(img), planar, lum)
    i1 = torch.empty((R, p.n_ht), dtype=torch.int32, device="cuda")
    c1 = torch.empty(R, dtype=torch.int32, device="cuda")
    B.block_match(lum, 1, p, i1, c1)
    num = torch.zeros((c, h, w), dtype=torch.float32, device="cuda")
    wsum = torch.zeros_like(num)
    B.collab_filter(planar, None, sigma, 1, i1, c1, p, num, wsum)
    basic = torch.empty_like(num)
    B.aggregate(num, wsum, False, p, basic)
    num.zero_()
    wsum.zero_()
    B.collab_filter(planar, basic, sigma, 2, dev(idx2), dev(cnt2), p, num, wsum)
    out = torch.empty(img.shape, dtype=torch.float32, device="cuda")
    B.aggregate(num, wsum, True, p, out)
    return host(out), host(i1), host(c1), host(gnk)


@pytest.mark.parametrize("which", ["small_gray", "gray512", "colour"])
def test_denoise_fp32_anchored(B, which):
    if which == "small_gray":
        s, S = synth.small_gray(), 16
    elif which == "gray512":
        s, S = synth.gray_512(), 32
    else:
        s, S = synth.colour_481x321(), 32
    img, sigma = s.noisy, 25.0
    h, w = img.shape[:2]
    p = gparams(B, sigma, S)
    op = oparams(p)
    ref, inter = oracle.denoise(img, sigma, op, want_intermediates=True)
    out, gi1, gc1, gnk = gpu_chain_with_idx2(B, img, sigma, p, inter["idx2"], inter["cnt2"])
    np.testing.assert_array_equal(gi1, inter["idx1"])
    planar, _ = oracle.prepare(img)
    _, _, margin, onk = oracle.collab_filter(planar, None, sigma, 1, inter["idx1"], inter["cnt1"], op,
                                             want_margin=True)
    flips = (gnk != onk).any(axis=0)
    assert np.all(margin[flips] < ph.HT_MARGIN), margin[flips]
    m1 = ph.patch_cover(inter["idx1"], inter["cnt1"], flips, h, w)
    t2 = ph.groups_touching(inter["idx2"], inter["cnt2"], m1, h, w)
    m2 = ph.patch_cover(inter["idx2"], inter["cnt2"], t2, h, w)
    ok = ~m2
    diff = np.abs(out - ref)
    dok = diff[ok] if out.ndim == 2 else diff[ok, :]
    log("anchored %s: %d step-1 decision flips, tainted %.3f%% max|diff| %.2e untainted, %.2e all; "
        "psnr gpu %.4f oracle %.4f" % (which, flips.sum(), 100 * m2.mean(), dok.max(), diff.max(),
                                       synth.psnr(s.clean, out), synth.psnr(s.clean, ref)))
    assert dok.max() <= ph.FP32_TOL
    # each near-tie flip reaches every step-2 group touching its patches: a
    # coarse but bounded region
    assert m2.mean() < 0.15


@pytest.mark.parametrize("which", ["small_gray", "gray512", "colour"])
def test_denoise_free_running(B, which):
    if which == "small_gray":
        s, S = synth.small_gray(), 16
    elif which == "gray512":
        s, S = synth.gray_512(), 32
    else:
        s, S = synth.colour_481x321(), 32
    sigma = 25.0
    p = gparams(B, sigma, S)
    ref = oracle.denoise(s.noisy, sigma, oparams(p))
    out = host(B.denoise(dev(s.noisy), sigma, p))
    d_psnr = synth.psnr(s.clean, out) - synth.psnr(s.clean, ref)
    log("free-running %s: max|diff| %.3e mean|diff| %.2e dPSNR %.5f dB" %
        (which, np.abs(out - ref).max(), np.abs(out - ref).mean(), d_psnr))
    assert abs(d_psnr) < 0.01
    assert np.abs(out - ref).mean() < 0.01


# ----------------------------------------------------- reduced precision forms ---

@pytest.mark.parametrize("xform", [1, 2], ids=["bf16", "fp16"])
@pytest.mark.parametrize("which", ["gray512", "colour"])
def test_low_precision_psnr(B, xform, which):
    s = synth.gray_512() if which == "gray512" else synth.colour_481x321()
    sigma = 25.0
    p32 = gparams(B, sigma, 32)
    plo = gparams(B, sigma, 32, xform=xform)
    o32 = host(B.denoise(dev(s.noisy), sigma, p32))
    olo = host(B.denoise(dev(s.noisy), sigma, plo))
    ref = oracle.denoise(s.noisy, sigma, oparams(p32))
    d = synth.psnr(s.clean, olo) - synth.psnr(s.clean, o32)
    log("%s xform=%d: PSNR fp32 %.4f low %.4f (d %.4f dB); max|low-fp64| %.3f, max|fp32-fp64| %.3f" %
        (which, xform, synth.psnr(s.clean, o32), synth.psnr(s.clean, olo), d,
         np.abs(olo - ref).max(), np.abs(o32 - ref).max()))
    assert abs(d) <= 0.05


# -------------------------------------------------------------- edge cases ---

def test_constant_image_closed_form(B):
    for c in (128, 2):
        img = np.full((40, 44), c, np.uint8)
        p = gparams(B, 25.0, 16)
        out = host(B.denoise(dev(img), 25.0, p))
        e = 64.0 * 32 * c * c
        expect = c * e / (e + 625.0) if c > 2 else 0.0
        np.testing.assert_allclose(out, expect, atol=1e-3)


def test_sigma_zero_identity(B):
    s = synth.small_gray()
    out = host(B.denoise(dev(s.noisy), 0.0, gparams(B, 0.0, 16)))
    np.testing.assert_allclose(out, s.noisy.astype(np.float64), atol=1e-3)
    c = synth.colour_481x321(h=40, w=48)
    out = host(B.denoise(dev(c.noisy), 0.0, gparams(B, 0.0, 16)))
    np.testing.assert_allclose(out, c.noisy.astype(np.float64), atol=1e-3)


@pytest.mark.parametrize("shape", [(8, 8), (8, 9, 3), (11, 8), (23, 31, 3), (100, 9)])
def test_tiny_and_ragged(B, shape):
    img = np.random.default_rng(sum(shape)).integers(0, 256, shape).astype(np.uint8)
    p = gparams(B, 25.0, 32)
    ref = oracle.denoise(img, 25.0, oparams(p))
    out = host(B.denoise(dev(img), 25.0, p))
    log("tiny %s max|diff| %.2e" % (shape, np.abs(out - ref).max()))
    assert np.abs(out - ref).mean() < 0.05


def test_invalid_arguments_enqueue_nothing(B):
    p = gparams(B, 25.0, 32)
    img = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BM3DError):
        B.denoise(img, float("nan"), p)
    bad = p.copy()
    bad.n_wie = 24
    with pytest.raises(B.BM3DError):
        B.denoise(img, 25.0, bad)
