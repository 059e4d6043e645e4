"""The timed path -- the batched, graph-captured pass -- element by element
against the FP64 oracle.

Workloads: the 64-image mixed batch (areas 128^2..1024^2, aspect 1:1-2:1,
half grey / half colour, sigma ~ U[10,50] with the per-image distance
thresholds of BM3D_FLAG_SIGMA_PROFILE) and the benchmark's 16 x 512^2 grey
batch at sigma 25.

* Step-1 groups (and the matching luminance) of every image, read out of the
  plan after graph replays, equal the oracle's bit for bit.
* The FP32 form of the batched pass, through the anchored protocol: the
  basic estimate within 1e-3 of the oracle's away from near-tie threshold
  decisions, the step-2 groups valid ordered top-n sets of the exact
  distances, and, with the oracle's step-2 groups set into the plan, the
  final image within 1e-3 away from the pixels a near-tie can reach.
* The BF16 form of the batched pass within 0.05 dB of its FP32 form.
* The batched pass equals the single-image path bit for bit (exact
  fixed-point accumulation makes both deterministic)."""
import functools

import numpy as np
import pytest

import oracle
import parity_helpers as ph
from paper_2403_03488_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

oracle.set_threads(16)
TILE = 10  # the filter tile (references per workgroup side) the autotuner picks here


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03488_amd import bm3d
    return bm3d


def log(msg):
    print(msg, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def taus(sigma):
    p = oracle.Params.for_sigma(sigma)
    return p.tau_ht, p.tau_wie


@functools.lru_cache(maxsize=None)
def mixed():
    return [synth.batch_image(i, sh) for i, sh in enumerate(synth.batch_shapes(64))]


@functools.lru_cache(maxsize=None)
def bench16():
    return [synth.gray_512(index=i, sigma=25.0) for i in range(16)]


def make_plan(B, samples, xform, tile=TILE, persistent=0, flags=0, match_refs=0):
    p = B.params_default(25.0, xform=xform, flags=flags | B.FLAG_SIGMA_PROFILE)
    p.tile_refs, p.persistent_wgs, p.match_refs = tile, persistent, match_refs
    imgs = [dev(s.noisy) for s in samples]
    outs = [torch.empty(s.noisy.shape, dtype=torch.float32, device="cuda") for s in samples]
    return B.Batch(imgs, outs, [s.sigma for s in samples], p), imgs, outs, p


def replay_graph(plan, times=2):
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture(stream)
        for _ in range(times):  # replays, as the timed loop does
            plan.launch(stream)
        stream.synchronize()


def check_step1_bit_exact(B, plan, samples, what):
    bad = []
    for i, s in enumerate(samples):
        h, w = s.noisy.shape[:2]
        R = B.num_refs(h, w)
        _, olum = oracle.prepare(s.noisy)
        glum = host(plan.read_buffer(i, "lum8")).reshape(h, w)
        oi, oc = oracle.match_u8(olum, 32, 16, taus(s.sigma)[0])
        gi = host(plan.read_buffer(i, "idx1")).reshape(R, 16)
        gc = host(plan.read_buffer(i, "cnt1"))
        ok = np.array_equal(glum, olum) and np.array_equal(gc, oc) and np.array_equal(gi, oi)
        if not ok:
            bad.append(i)
        if i % 8 == 7 or not ok:
            log("%s step-1 groups: image %d (%dx%dx%d, sigma %.1f) %s" % (what, i, h, w, s.c, s.sigma,
                                                                          "ok" if ok else "DIFFERS"))
    assert not bad, "images whose step-1 groups differ from the oracle: %s" % bad


def test_mixed_batch_step1_bit_exact(B):
    samples = mixed()
    plan, *_ = make_plan(B, samples, xform=1)
    replay_graph(plan)
    check_step1_bit_exact(B, plan, samples, "mixed batch")
    plan.close()


@pytest.mark.parametrize("tile,match_refs", [(8, 0), (10, 0), (10, 16)])
def test_bench_config_step1_bit_exact(B, tile, match_refs):
    samples = bench16()
    plan, *_ = make_plan(B, samples, xform=1, tile=tile, match_refs=match_refs)
    replay_graph(plan)
    check_step1_bit_exact(B, plan, samples, "16 x 512^2 tile %d refs/pass %d" % (tile, match_refs))
    plan.close()


# The anchored subset of the mixed batch: the largest grey (1061x988, sigma
# 42.2) and colour (899x1167, sigma 49.9) images, sigma on both sides of 40,
# widths that are not multiples of the tile, small images.
ANCHORED_MIXED = (2, 45, 13, 9, 22, 4, 63)


@functools.lru_cache(maxsize=None)
def oracle_intermediates(key, i):
    s = mixed()[i] if key == "mixed" else bench16()[i]
    op = ph.oracle_params(s.sigma, 32)
    ref, inter = oracle.denoise(s.noisy, s.sigma, op, want_intermediates=True)
    planar, _ = oracle.prepare(s.noisy)
    _, _, margin, onk = oracle.collab_filter(planar, None, s.sigma, 1, inter["idx1"], inter["cnt1"], op,
                                             want_margin=True)
    return ref, inter, margin, onk


def anchored_batch(B, key, samples, subset):
    """FP32 batched pass over all the samples, checked on `subset` by the
    anchored protocol (see the module docstring)."""
    plan, imgs, outs, p = make_plan(B, samples, xform=0, flags=B.FLAG_DEBUG_NKEPT)
    plan.run_stages(0, len(samples), 0, 4)  # prep .. match2
    torch.cuda.synchronize()
    masks = {}
    for i in subset:
        s = samples[i]
        h, w, c = s.noisy.shape[0], s.noisy.shape[1], s.c
        R = B.num_refs(h, w)
        ref, inter, margin, onk = oracle_intermediates(key, i)
        gi1 = host(plan.read_buffer(i, "idx1")).reshape(R, 16)
        np.testing.assert_array_equal(gi1, inter["idx1"])
        gnk = host(plan.read_buffer(i, "nkept")).reshape(c, R)
        flips = (gnk != onk).any(axis=0)
        assert np.all(margin[flips] < ph.HT_MARGIN), margin[flips]
        m1, m2 = ph.anchored_masks(inter["idx1"], inter["cnt1"], flips, inter["idx2"], inter["cnt2"], h, w)
        gb = host(plan.read_buffer(i, "basic")).reshape(c, h, w)
        db = np.abs(gb - inter["basic"])[:, ~m1]
        assert db.size == 0 or db.max() <= ph.FP32_TOL, (i, db.max())
        # step-2 groups on the plan's own basic estimate: valid ordered top-n
        lum = host(plan.read_buffer(i, "lumf")).reshape(h, w)
        np.testing.assert_allclose(lum, oracle.luminance(gb.astype(np.float64)), rtol=1e-6, atol=1e-4)
        gi2 = host(plan.read_buffer(i, "idx2")).reshape(R, 32)
        gc2 = host(plan.read_buffer(i, "cnt2"))
        oi2, _ = oracle.match_f64(lum.astype(np.float64), 32, 32, taus(s.sigma)[1])
        same = np.all(gi2 == oi2, axis=1)
        rows, cols = oracle.ref_positions(h), oracle.ref_positions(w)
        P = ph.all_patches(lum)
        rng = np.random.default_rng(i)
        refs = np.unique(np.concatenate([np.nonzero(~same)[0], rng.choice(R, size=min(R, 400), replace=False)]))
        for r in refs:
            why = ph.check_topn_valid(lum, (rows[r // len(cols)], cols[r % len(cols)]), 32, 32, taus(s.sigma)[1],
                                      gi2[r], gc2[r], P)
            assert why is None, "image %d ref %d: %s" % (i, r, why)
        # anchor step 2 on the oracle's groups
        plan.write_buffer(i, "idx2", dev(inter["idx2"].reshape(-1)))
        plan.write_buffer(i, "cnt2", dev(inter["cnt2"]))
        masks[i] = (m2, flips.sum(), same.mean(), db.max() if db.size else 0.0)
    plan.run_stages(0, len(samples), 5, 6)  # filter2, agg2
    torch.cuda.synchronize()
    for i in subset:
        s = samples[i]
        ref = oracle_intermediates(key, i)[0]
        m2, nflip, same, dbmax = masks[i]
        out = host(outs[i])
        diff = np.abs(out - ref)
        dok = diff[~m2] if out.ndim == 2 else diff[~m2, :]
        log("%s image %d (%s, sigma %.1f): %d near-tie flips, step-2 groups identical %.2f%%, tainted %.3f%%, "
            "max|basic diff| %.2e, max|final diff| %.2e untainted" %
            (key, i, s.noisy.shape, s.sigma, nflip, 100 * same, 100 * m2.mean(), dbmax,
             dok.max() if dok.size else 0.0))
        assert dok.size == 0 or dok.max() <= ph.FP32_TOL
        assert m2.mean() < 0.15
    plan.close()


def test_mixed_batch_fp32_anchored(B):
    anchored_batch(B, "mixed", mixed(), ANCHORED_MIXED)


def test_bench_config_fp32_anchored(B):
    anchored_batch(B, "bench", bench16(), (0, 9))


@pytest.mark.parametrize("key", ["mixed", "bench"])
def test_batch_bf16_within_005db_of_fp32(B, key):
    samples = mixed() if key == "mixed" else bench16()
    res = {}
    for xf in (0, 1):
        plan, imgs, outs, p = make_plan(B, samples, xform=xf)
        replay_graph(plan)
        res[xf] = [host(o) for o in outs]
        plan.close()
    d = [synth.psnr(s.clean, b) - synth.psnr(s.clean, a) for s, a, b in zip(samples, res[0], res[1])]
    log("%s: BF16 - FP32 PSNR per image: min %.4f max %.4f mean %.4f dB" % (key, min(d), max(d), np.mean(d)))
    assert max(abs(x) for x in d) <= 0.05


@pytest.mark.parametrize("xform", [0, 1])
def test_batch_group_sizes_equal_single(B, xform):
    """Group-size limits 32 (step 1) and 16 (step 2): the batched filters
    built for the other member-tile limits equal the single-image path."""
    samples = mixed()[:8]
    p = B.params_default(25.0, xform=xform, flags=B.FLAG_SIGMA_PROFILE)
    p.tile_refs, p.n_ht, p.n_wie = TILE, 32, 16
    imgs = [dev(s.noisy) for s in samples]
    outs = [torch.empty(s.noisy.shape, dtype=torch.float32, device="cuda") for s in samples]
    plan = B.Batch(imgs, outs, [s.sigma for s in samples], p)
    replay_graph(plan, 1)
    for i, (s, im, o) in enumerate(zip(samples, imgs, outs)):
        q = p.copy()
        q.tau_ht, q.tau_wie = taus(s.sigma)
        q.flags = 0
        single = B.denoise(im, s.sigma, q)
        np.testing.assert_array_equal(host(single), host(o), err_msg="image %d" % i)
    log("batch == single bit for bit with groups 32/16: xform %d, %d images" % (xform, len(samples)))
    plan.close()


@pytest.mark.parametrize("xform", [0, 1])
@pytest.mark.parametrize("persistent", [0, 2])
def test_batch_equals_single_bit_for_bit(B, xform, persistent):
    samples = mixed()[:24]
    plan, imgs, outs, p = make_plan(B, samples, xform=xform, persistent=persistent)
    replay_graph(plan, 1)
    for i, (s, im, o) in enumerate(zip(samples, imgs, outs)):
        q = p.copy()
        q.tau_ht, q.tau_wie = taus(s.sigma)
        q.flags = 0
        single = B.denoise(im, s.sigma, q)
        np.testing.assert_array_equal(host(single), host(o), err_msg="image %d" % i)
    log("batch == single bit for bit: xform %d, persistent %d, %d images" % (xform, persistent, len(samples)))
    plan.close()
