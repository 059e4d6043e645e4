"""Batched pass, graph capture, serving loop and autotuner on the GPU.

Batched and single-image paths run the same device code.  Two runs of the
same image can still differ: tiles add their partial sums into the shared
num/den with FP32 atomics, so the basic estimate varies in its last bits
with the order of those additions, and step-2 grouping, which has many
near-ties in flat regions, may then pick another equally valid group for a
few references.  Runs are therefore compared with the free-running bar:
mean |diff| <= 2e-3, max |diff| <= 2 and PSNR equal to 5e-3 dB."""
import json
import os

import numpy as np
import pytest

from paper_2403_03488_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-3


def same_result(a, b, clean=None):
    a = a.float().cpu().numpy() if hasattr(a, "cpu") else a
    b = b.float().cpu().numpy() if hasattr(b, "cpu") else b
    d = np.abs(a - b)
    ok = d.mean() <= 2e-3 and d.max() <= 2.0
    if clean is not None:
        ok = ok and abs(synth.psnr(clean, a) - synth.psnr(clean, b)) <= 5e-3
    return ok, float(d.max()), float(d.mean())


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03488_amd import bm3d
    return bm3d


def log(msg):
    print(msg, flush=True)


def mixed_batch(n=10, seed=0):
    """Uneven sizes, grey and colour, different sigmas (reduced-size stand-ins
    for the 64-image batch, so the single-image comparison stays quick)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h, w = int(rng.integers(8, 200)), int(rng.integers(8, 260))
        c = 1 if i % 2 == 0 else 3
        sigma = float(rng.uniform(10, 50))
        r = np.random.default_rng(100 + i)
        clean = synth.smooth_texture_image(r, h, w) if c == 1 else synth.mixed_colour_image(r, h, w)
        out.append(synth.Sample(clean, synth.add_awgn_u8(clean, sigma, r), sigma))
    return out


@pytest.mark.parametrize("xform", [0, 1])
@pytest.mark.parametrize("persistent", [0, 2])
def test_batch_equals_single(B, xform, persistent):
    samples = mixed_batch()
    p = B.params_default(25.0, xform=xform, persistent_wgs=persistent, flags=B.FLAG_SIGMA_PROFILE)
    imgs = [torch.from_numpy(s.noisy).cuda() for s in samples]
    outs = [torch.empty(s.noisy.shape, dtype=torch.float32, device="cuda") for s in samples]
    plan = B.Batch(imgs, outs, [s.sigma for s in samples], p)
    plan.run()
    worst, worst_mean, all_ok = 0.0, 0.0, True
    for s, im, o in zip(samples, imgs, outs):
        q = p.copy()
        ps = B.params_default(s.sigma, xform=xform)
        q.tau_ht, q.tau_wie = ps.tau_ht, ps.tau_wie  # sigma-dependent profile per image
        single = B.denoise(im, s.sigma, q)
        torch.cuda.synchronize()
        ok, mx, mn = same_result(single, o, s.clean)
        all_ok &= ok
        worst, worst_mean = max(worst, mx), max(worst_mean, mn)
    log("batch vs single xform=%d persistent=%d: max|diff| %.2e, worst mean|diff| %.2e" %
        (xform, persistent, worst, worst_mean))
    assert all_ok
    plan.close()


def test_sigma_profile_flag_selects_tau_per_image(B):
    s = synth.gray_512(sigma=50.0, h=96, w=96)
    img = torch.from_numpy(s.noisy).cuda()
    flagged = B.denoise(img, 50.0, B.params_default(25.0, flags=B.FLAG_SIGMA_PROFILE))
    explicit = B.denoise(img, 50.0, B.params_default(50.0))
    other = B.denoise(img, 50.0, B.params_default(25.0))
    torch.cuda.synchronize()
    assert same_result(flagged, explicit, s.clean)[0]
    assert float((flagged - other).abs().mean()) > 0.05


def test_graph_replays_match_eager(B):
    samples = mixed_batch(6, seed=3)
    p = B.params_default(25.0, xform=1)
    imgs = [torch.from_numpy(s.noisy).cuda() for s in samples]
    outs = [torch.empty(s.noisy.shape, dtype=torch.float32, device="cuda") for s in samples]
    plan = B.Batch(imgs, outs, [s.sigma for s in samples], p)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.run(stream)
        stream.synchronize()
        eager = [o.clone() for o in outs]
        plan.capture(stream)
        for rep in range(3):
            for o in outs:
                o.fill_(-1.0)  # ordinary eager work between replays
            stream.synchronize()
            plan.launch(stream)
            stream.synchronize()
            res = [same_result(a, b, smp.clean) for a, b, smp in zip(eager, outs, samples)]
            log("graph replay %d: max|diff| vs eager %.2e" % (rep, max(r[1] for r in res)))
            assert all(r[0] for r in res)
        # re-bound inputs take effect in the next replay without re-capture
        other = mixed_batch(6, seed=3)
        rng = np.random.default_rng(9)
        new_img = torch.from_numpy(synth.add_awgn_u8(other[0].clean, other[0].sigma, rng)).cuda()
        new_out = torch.empty(other[0].noisy.shape, dtype=torch.float32, device="cuda")
        plan.set_io(0, new_img, new_out, stream)
        plan.launch(stream)
        stream.synchronize()
        q = B.params_default(25.0, xform=1)
        ref = B.denoise(new_img, samples[0].sigma, q, stream=stream)
        stream.synchronize()
        assert same_result(ref, new_out, other[0].clean)[0]
    plan.close()


def make_requests(specs, canvases):
    from paper_2403_03488_amd import serve
    reqs = []
    for sp in specs:
        clean = synth.crop_clean(canvases, sp)
        noisy = synth.add_awgn_u8(clean, sp["sigma"], np.random.default_rng(sp["noise_seed"]))
        reqs.append(serve.Request(sp["rid"], sp["arrival"], torch.from_numpy(noisy).pin_memory(),
                                  sp["sigma"]))
    return reqs


@pytest.fixture(scope="module")
def canvases():
    return synth.serving_canvases(768, seed=77)


def test_serving_alone_equals_mix(B, canvases):
    from paper_2403_03488_amd import serve
    specs = synth.serving_specs(12, rate=400.0, max_side=768, seed=5)
    p = B.params_default(25.0, xform=1, flags=B.FLAG_SIGMA_PROFILE)
    # the request alone
    alone = make_requests([dict(specs[5], arrival=0.0)], canvases)
    serve.ServingLoop(p, max_slots=8, keep_outputs=True).run(alone)
    # the same request inside a mix of overlapping arrivals
    mix = make_requests(specs, canvases)
    loop = serve.ServingLoop(p, max_slots=8, keep_outputs=True)
    loop.run(mix)
    torch.cuda.synchronize()
    clean5 = synth.crop_clean(canvases, specs[5])
    ok, d, dm = same_result(alone[0].out, mix[5].out, clean5)
    shared = sum(1 for n in loop.tick_sizes if n > 1)
    log("serving: alone vs mix max|diff| %.2e mean %.2e; %d ticks, %d with >1 request, max %d per tick" %
        (d, dm, loop.ticks, shared, max(loop.tick_sizes)))
    assert ok
    assert shared > 0  # requests really were batched together
    # and each result matches the plain single-image path
    for r, sp in zip(mix, specs):
        ref = B.denoise(r.host_img.cuda(), r.sigma, p)
        torch.cuda.synchronize()
        assert same_result(ref, r.out, synth.crop_clean(canvases, sp))[0]


def test_serving_admission_respects_budget(B, canvases):
    from paper_2403_03488_amd import serve
    specs = synth.serving_specs(10, rate=1000.0, max_side=768, seed=6)
    p = B.params_default(25.0, xform=1, flags=B.FLAG_SIGMA_PROFILE)
    reqs = make_requests(specs, canvases)
    biggest = max(serve.footprint(r.h, r.w, r.c, p) for r in reqs)
    budget = int(biggest * 1.5)  # at most one large request in flight at a time
    loop = serve.ServingLoop(p, max_slots=8, hbm_budget=budget)
    loop.run(reqs)
    assert loop.peak_used <= budget
    assert all(np.isfinite(r.done) for r in reqs)
    stats = serve.summarize(reqs)
    log("budgeted serving: peak %.1f MB of %.1f MB; p50 %.2f ms p99 %.2f ms" %
        (loop.peak_used / 1e6, budget / 1e6, stats["p50_ms"], stats["p99_ms"]))
    # a request that can never fit is refused up front
    with pytest.raises(ValueError):
        serve.ServingLoop(p, max_slots=4, hbm_budget=biggest // 2).run(reqs[:1] + [max(
            reqs, key=lambda r: serve.footprint(r.h, r.w, r.c, p))])


def test_autotune_cache_roundtrip(B, tmp_path):
    path = str(tmp_path / "tune.json")
    p = B.params_default(25.0, xform=1)
    q = B.autotune(p, path)
    assert q.tile_refs >= 2 and q.persistent_wgs >= 0
    data = json.load(open(path))
    assert len(data) == 1
    key, (tile, wgs, ms) = next(iter(data.items()))
    assert "gfx" in key and tile == q.tile_refs and wgs == q.persistent_wgs and ms > 0
    r = B.autotune(p, path)  # served from the cache
    assert (r.tile_refs, r.persistent_wgs) == (q.tile_refs, q.persistent_wgs)
