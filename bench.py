#!/usr/bin/env python3
"""Throughput of the two-step BM3D stage on one MI355X.

Workload: 512x512 grey images (piecewise-smooth gradients + rotated
textures, seeded synthetic stand-ins for the paper's 512x512 test images),
AWGN sigma = 25, 8x8 patches, 32x32 search, stride 3, group sizes 16/32.
A step denoises one batch of images through the batched, graph-captured
pass (int8 matrix-core matching, BF16 transforms by default); inputs are
resident in HBM before timing starts.

Prints ONE JSON line: value = denoised MP/s over the whole job, the
dominant kernel's roofline (time from HIP events on the launch stream), the
single-image latency p50/p99, the FP32-form comparison, and the FP64 oracle
timed on the host cores as the CPU baseline.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "bf16": 2.5e15, "fp16": 2.5e15, "fp32_mfma": 157.3e12, "int8": 5.0e15,
    # vector FP32 without packed instructions: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
    "fp32_valu": 78.6e12,
    # vector lane operations: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
    "valu_ops": 39.3e12,
}
XF = {"fp32": 0, "bf16": 1, "fp16": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def work_models(h, w, S, cnt1, cnt2, c=1):
    """Algorithmic work per stage for one image, in the separable form of the
    method (the unit each kernel's roofline fraction is computed from):
    matching = one multiply-add per pixel pair of every window candidate
    (int8 cross terms in step 1, FP32 direct differences in step 2), i.e.
    S^2 * 64 per reference; filters = the 3-D transforms with the 2-D DCT as
    8-point row and column passes, at the actual group sizes n:
    2048 n + 128 n^2 multiply-adds per group and channel in step 1 (forward
    and inverse), 3 (1024 n + 64 n^2) in step 2 (noisy and basic forward,
    inverse).  Everything is returned in operations (2 per multiply-add)."""
    def wlen(L):
        return min(S, L - 7)
    cands = len(cnt1) * wlen(h) * wlen(w)
    n1 = cnt1.astype(np.float64)
    n2 = cnt2.astype(np.float64)
    return {
        "match1": 2.0 * cands * 64,
        "filter1": 2.0 * c * float(np.sum(2048 * n1 + 128 * n1 * n1)),
        "match2": 2.0 * cands * 64,
        "filter2": 2.0 * c * float(np.sum(3 * (1024 * n2 + 64 * n2 * n2))),
    }


def mfma_issued(cnt1, cnt2, c=1):
    """Dense matrix-core operations the filters issue: each 2-D DCT is one
    64 x 64 product per patch, each Walsh-Hadamard product runs on 16 x 16
    tiles (groups of up to 16 members in one tile, 32 in two).  Not the
    algorithmic work: the separable count above is."""
    def per_group(n, srcs):
        nt = np.where(n > 16, 32.0, 16.0)  # members padded to whole tiles
        return srcs * (2 * 64 * 64 * nt + 2 * 64 * nt * nt) + (2 * 64 * 64 * nt + 2 * 64 * nt * nt)
    return {"filter1": c * float(np.sum(per_group(cnt1.astype(np.float64), 1))),
            "filter2": c * float(np.sum(per_group(cnt2.astype(np.float64), 2)))}


# The sources each kernel family is compiled from: a counter record counts
# only while these are unchanged.
FAMILY_SOURCES = {"bm3d": "bm3d_*", "cnn": "cnn.hip"}


def source_sha(family):
    import glob
    import hashlib
    src = "".join(open(f).read() for f in sorted(glob.glob(os.path.join(
        ROOT, "paper_2403_03488_amd", "csrc", FAMILY_SOURCES[family]))))
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def measured_traffic(kernel, images, tile, family="bm3d", match_refs=8):
    """HBM bytes per launch of `kernel` from the committed counter runs
    (profiles/hbm_traffic_*.json), if they were taken on the current sources
    of its kernel family with the settings that shape its accesses (the
    filter tile for the filters, the references per step-1 matching pass for
    match1); None otherwise."""
    import glob
    sha = source_sha(family)
    for path in glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.json")):
        rec = json.load(open(path))
        if kernel.startswith("filter") and rec.get("tile_refs") != tile:
            continue
        if kernel == "match1" and rec.get("match_refs", 8) != match_refs:
            continue
        if (rec.get("family", "bm3d") == family and rec.get("source_sha") == sha
                and kernel in rec.get("kernels", {})):
            k = rec["kernels"][kernel]
            return images * (k["fetch_bytes_per_image"] + k["write_bytes_per_image"])
    return None


def calibration_copy(torch):
    """A 256 MiB device-to-device copy: the reference the byte counters of
    the profiled kernels are scaled by."""
    src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def single_image_checks(torch, bm3d, synth, p, imgs, outs, samples, sigma, H, W, B):
    """Single-image latency (plain path) and the FP32 comparison on image 0."""
    ws = torch.empty(bm3d.workspace_size(H, W, 1, p), dtype=torch.uint8, device="cuda")
    lat = []
    for i in range(30):
        torch.cuda.synchronize()
        t = time.perf_counter()
        bm3d.denoise(imgs[i % B], sigma, p, out=outs[0], workspace=ws)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
    lat_ms = sorted(1e3 * x for x in lat[5:])
    p32 = bm3d.params_default(sigma, xform=0, tile_refs=p.tile_refs)
    ws32 = torch.empty(bm3d.workspace_size(H, W, 1, p32), dtype=torch.uint8, device="cuda")
    o32 = bm3d.denoise(imgs[0], sigma, p32, workspace=ws32)
    olo = bm3d.denoise(imgs[0], sigma, p, workspace=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(10):
        bm3d.denoise(imgs[i % B], sigma, p32, out=outs[1], workspace=ws32)
    torch.cuda.synchronize()
    fp32_single = 10 * H * W / 1e6 / (time.perf_counter() - t)
    clean0 = samples[0].clean
    psnr32 = synth.psnr(clean0, o32.cpu().numpy())
    psnrlo = synth.psnr(clean0, olo.cpu().numpy())

    return lat_ms, fp32_single, psnr32, psnrlo


def stage_times(torch, bm3d, plan, B, stream):
    """Per-stage kernel time (ms) with HIP events on the launch stream.  After
    one full pass the matching/filter stages can be re-run on valid data (the
    filters only add into num/den); the stages that reset or rewrite state
    (prep + zero-fill, agg1 + zero-fill, agg2) are timed last."""
    plan.run(stream)
    stage_ms = {}
    for st in (1, 2, 4, 5, 0, 3, 6):
        name = bm3d.STAGES[st]
        reps = 5
        plan.run_stages(0, B, st, st, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.run_stages(0, B, st, st, stream)
        e1.record(stream)
        e1.synchronize()
        stage_ms[name] = e0.elapsed_time(e1) / reps
    return stage_ms


def cpu_baseline(args, samples, sigma, S, H, W):
    """The FP64 C oracle on the host cores, on whole 512x512 images: first on
    one thread, then on every core the host reports (OpenMP over reference
    rows); about args.cpu_seconds of work in all."""
    import oracle
    op = oracle.Params.for_sigma(sigma, S)
    host = os.cpu_count() or 1
    res = {}
    for threads in (1, host):
        oracle.set_threads(threads)
        n, t0 = 0, time.perf_counter()
        while True:
            oracle.denoise(samples[n % len(samples)].noisy, sigma, op)
            n += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds / 2 or n >= 4 * len(samples):
                break
        res[threads] = (n * H * W / 1e6 / el, n, el)
        log("cpu baseline: %.4f MP/s on %d thread(s) (%d images, %.1f s)" % (res[threads][0], threads, n, el))
    v, n, el = res[host]
    v1, n1, el1 = res[1]
    return {"value": v, "unit": "MP/s", "cores": host, "kind": "oracle",
            "sample": "%d x 512x512 grey sigma=25 images, FP64 C oracle on all %d host cores (OpenMP), %.1f s"
                      % (n, host, el),
            "host_cores": host, "cpu_model": cpu_model(),
            "single_thread": {"value": v1, "unit": "MP/s", "cores": 1,
                              "sample": "%d x 512x512 grey image(s), one thread, %.1f s" % (n1, el1)}}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def tuned_params(args, bm3d, sigma, flags=0):
    p = bm3d.params_default(sigma, xform=XF[args.xform], flags=flags)
    if not args.no_autotune and not (args.tile and args.persistent >= 0):
        t0 = time.time()
        q = bm3d.autotune(p, None)
        p.tile_refs, p.persistent_wgs, p.match_refs = q.tile_refs, q.persistent_wgs, q.match_refs
        log("autotune: tile %d refs, persistent %d WG/CU, step-1 matching %d refs per pass (%.1fs)" % (
            p.tile_refs, p.persistent_wgs, p.match_refs, time.time() - t0))
    if args.tile:
        p.tile_refs = args.tile
    if args.persistent >= 0:
        p.persistent_wgs = args.persistent
    if args.match_refs:
        p.match_refs = args.match_refs
    return p


def nlm_ops_per_candidate(f, c):
    """Lane operations per pixel and search candidate of NL-means in the
    separable form: per channel a difference and a fused square-add, 2f adds
    for the horizontal and 2f for the vertical patch sum, the exponent
    (scale, clamp, difference to the running minimum, multiply, exponential),
    the running minimum, and per channel plus the denominator one
    multiply-add."""
    return 2 * c + 4 * f + 5 + 1 + (c + 1)


def run_nlm(args):
    """NL-means first stage: 16 x 512^2 grey, sigma 25, one batched launch per step."""
    import torch
    from paper_2403_03488_amd import bm3d, synth
    assert torch.cuda.is_available(), "no GPU"
    sigma, H, W, B = 25.0, 512, 512, args.batch
    samples = [synth.gray_512(index=i, sigma=sigma) for i in range(B)]
    imgs = [torch.from_numpy(s.noisy).cuda() for s in samples]
    outs = [torch.empty((H, W), dtype=torch.float32, device="cuda") for _ in range(B)]
    p = bm3d.nlm_params_default(sigma, 1)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    for _ in range(args.warmup):
        bm3d.nlm_batch(imgs, sigma, p, outs, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        bm3d.nlm_batch(imgs, sigma, p, outs, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ms_launch = e0.elapsed_time(e1) / args.steps
    mp = B * H * W / 1e6
    log("nlm batched: %.3f ms/step, %.1f MP/s" % (dt * 1e3, mp / dt))
    f, r = p.patch_radius, p.search_radius
    # candidates inside the image for every pixel (clipped windows)
    span = lambda n: sum(min(n - 1, i + r) - max(0, i - r) + 1 for i in range(n))
    cand = span(H) * span(W) - H * W
    work = B * cand * nlm_ops_per_candidate(f, 1)
    achieved = work / (ms_launch * 1e-3)
    ps = [synth.psnr(s.clean, o.cpu().numpy()) for s, o in zip(samples, outs)]
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import nlm as onlm
        crop = samples[0].noisy[:192, :192]
        n, t1 = 0, time.perf_counter()
        while True:
            onlm.nlm(crop, sigma)
            n += 1
            el = time.perf_counter() - t1
            if el >= min(args.cpu_seconds, 10.0):
                break
        cpu = {"value": n * crop.size / 1e6 / el, "unit": "MP/s", "cores": 1, "kind": "oracle",
               "sample": "%d x 192x192 crop of a 512x512 grey sigma=25 image, FP64 numpy oracle, %.1f s"
                         % (n, el)}
    res = {
        "metric": "denoised MP/s (NL-means first stage, sigma=25)", "value": mp / dt, "unit": "MP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512x512 grey, sigma=25, 5x5 patches, 21x21 windows, h=10, batch of %d "
                               "images per launch" % B, "batch": B, "patch_radius": f, "search_radius": r,
                   "h": p.h},
        "roofline": {"bound": "alu", "kernel": "nlm", "achieved": achieved / 1e12,
                     "peak": PEAK["valu_ops"] / 1e12, "unit": "TOP/s",
                     "frac": achieved / PEAK["valu_ops"], "traffic": None, "ms_per_launch": ms_launch,
                     "work_per_launch": work},
        "psnr_db": {"mean": float(np.mean(ps)), "min": float(np.min(ps))},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def run_cnn(args):
    """Residual network behind the first stage (K = 10, colour, Table 3's
    512 x 512 case): 16 images per call, one launch per layer."""
    import torch
    from paper_2403_03488_amd import bm3d, synth
    assert torch.cuda.is_available(), "no GPU"
    K, C, H, W, B = 10, 3, 512, 512, args.batch
    layers = synth.cnn_layers(K, C, seed=1)
    net = bm3d.Cnn(layers, C)
    samples = [synth.colour_481x321(index=i) for i in range(B)]
    rng = np.random.default_rng(0)
    basics, noisys = [], []
    for s in samples:
        # 512 x 512 from the 481 x 321 colour family, tiled by reflection
        cl = np.pad(s.clean, ((0, H - s.clean.shape[0]), (0, W - s.clean.shape[1]), (0, 0)), mode="reflect")
        ny = np.pad(s.noisy, ((0, H - s.noisy.shape[0]), (0, W - s.noisy.shape[1]), (0, 0)), mode="reflect")
        basics.append(torch.from_numpy((cl + rng.normal(0, 3, cl.shape)).astype(np.float32)).cuda())
        noisys.append(torch.from_numpy(np.ascontiguousarray(ny)).cuda())
    outs = [torch.empty((H, W, C), dtype=torch.float32, device="cuda") for _ in range(B)]
    if args.calibrate_copy:
        calibration_copy(torch)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    for _ in range(args.warmup):
        net.restore(basics, noisys, outs, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.restore(basics, noisys, outs, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the dominant kernel: the 64 -> 64 layers, K - 2 launches per pass
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        net.restore(basics, noisys, outs, stream=stream, layers=(1, K - 1))
    e1.record(stream)
    torch.cuda.synchronize()
    ms_hidden = e0.elapsed_time(e1) / (args.steps * (K - 2))
    net.restore(basics, noisys, outs, stream=stream)
    torch.cuda.synchronize()
    mp = B * H * W / 1e6
    flops_pass = 2 * B * ocnn_macs(K, C, H, W)
    flops_hidden = 2 * B * H * W * 9 * 64 * 64
    achieved = flops_hidden / (ms_hidden * 1e-3)
    log("cnn K=%d: %.3f ms/step (%d images), %.1f MP/s, %.1f TFLOP/s whole pass; hidden layer %.3f ms, "
        "%.1f TFLOP/s" % (K, dt * 1e3, B, mp / dt, flops_pass / dt / 1e12, ms_hidden, achieved / 1e12))
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import cnn as ocnn
        b0, y0 = basics[0][:128, :128].cpu().numpy(), noisys[0][:128, :128].cpu().numpy()
        n, t1 = 0, time.perf_counter()
        while True:
            ocnn.restore(b0, y0, layers)
            n += 1
            el = time.perf_counter() - t1
            if el >= min(args.cpu_seconds, 10.0):
                break
        cpu = {"value": n * 128 * 128 / 1e6 / el, "unit": "MP/s", "cores": blas_threads(),
               "kind": "oracle",
               "sample": "%d x 128x128 colour crop, K=10, FP64 numpy oracle (BLAS tensordot), %.1f s" % (n, el)}
    res = {
        "metric": "restored MP/s (residual network x_hat = BM3D(y) + F(z), K=10, colour)", "value": mp / dt,
        "unit": "MP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (seeded random weights; trained weights not available)",
        "config": {"workload": "512x512 colour, K=10 (2C->64, 8 x 64->64 with batch norm, 64->C), batch of %d "
                               "images per call" % B, "batch": B, "layers": K,
                   "gflop_per_image": flops_pass / B / 1e9},
        "roofline": {"bound": "mfma", "kernel": "k_conv<1,4,false> (64->64 layer)", "achieved": achieved / 1e12,
                     "peak": PEAK["bf16"] / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK["bf16"],
                     "traffic": measured_traffic("hidden", B, 0, "cnn"), "ms_per_launch": ms_hidden,
                     "work_per_launch": flops_hidden},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def unet_bytes(C, H, W, widths=(32, 64, 128, 256, 256)):
    """Compulsory HBM bytes of one U-Net pass on one image: every launch
    reads its input maps once and writes its output once (bf16 maps padded
    to 8-channel words; FP32 estimate and output, uint8 observation)."""
    hs, ws = [H], [W]
    for _ in range(4):
        hs.append((hs[-1] + 1) // 2)
        ws.append((ws[-1] + 1) // 2)
    px = [h * w for h, w in zip(hs, ws)]
    m = lambda lv, ch: px[lv] * 2 * 8 * ((ch + 7) // 8)  # one bf16 map
    cin = 2 * C + 1
    tot = px[0] * (4 * C + C) + m(0, cin)               # z packed: images in, one map out
    tot += 2 * m(0, cin)                                # first depthwise
    tot += m(0, cin) + m(0, widths[0])                  # its pointwise
    for i in range(4):
        if i > 0:
            tot += 2 * m(i, widths[i]) + 2 * m(i, widths[i])  # encoder depthwise + pointwise
        tot += m(i, widths[i]) + m(i + 1, widths[i])          # stride-2 depthwise
        tot += m(i + 1, widths[i]) + m(i + 1, widths[i + 1])  # its pointwise
    for i in range(4):
        tot += m(i + 1, widths[i + 1]) + 2 * m(i, widths[i])  # deconvolution: input, skip, output
        tot += 4 * m(i, widths[i])                            # decoder depthwise + pointwise
    tot += m(0, widths[0]) + px[0] * 8 * C                    # output layer: map, estimate, result
    return tot


def unet_macs(C, H, W, widths=(32, 64, 128, 256, 256)):
    """Multiply-adds of the U-Net on one image: 9 per depthwise output, cin
    per pointwise and deconvolution output."""
    hs, ws = [H], [W]
    for _ in range(4):
        hs.append((hs[-1] + 1) // 2)
        ws.append((ws[-1] + 1) // 2)
    px = [h * w for h, w in zip(hs, ws)]
    c, tot = 2 * C + 1, 0
    for i in range(4):
        tot += px[i] * (9 * c + c * widths[i]) + px[i + 1] * (9 * widths[i] + widths[i] * widths[i + 1])
        c = widths[i + 1]
    for i in range(4):
        tot += 4 * px[i + 1] * widths[i + 1] * widths[i] + px[i] * (9 * widths[i] + widths[i] ** 2)
    return tot + px[0] * widths[0] * C


def run_unet(args):
    """Flexible U-Net behind the first stage (colour, Table 3's 512 x 512
    case): 16 images per call, 30 launches per pass."""
    import torch
    from paper_2403_03488_amd import bm3d, synth
    assert torch.cuda.is_available(), "no GPU"
    C, H, W, B, sigma = 3, 512, 512, args.batch, 25.0
    weights = synth.unet_net(C, seed=1)
    net = bm3d.Unet(weights, C)
    rng = np.random.default_rng(0)
    basics, noisys = [], []
    for i in range(B):
        s = synth.colour_481x321(index=i)
        cl = np.pad(s.clean, ((0, H - s.clean.shape[0]), (0, W - s.clean.shape[1]), (0, 0)), mode="reflect")
        ny = np.pad(s.noisy, ((0, H - s.noisy.shape[0]), (0, W - s.noisy.shape[1]), (0, 0)), mode="reflect")
        basics.append(torch.from_numpy((cl + rng.normal(0, 3, cl.shape)).astype(np.float32)).cuda())
        noisys.append(torch.from_numpy(np.ascontiguousarray(ny)).cuda())
    outs = [torch.empty((H, W, C), dtype=torch.float32, device="cuda") for _ in range(B)]
    if args.calibrate_copy:
        calibration_copy(torch)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    for _ in range(args.warmup):
        net.restore(basics, noisys, sigma, outs, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        net.restore(basics, noisys, sigma, outs, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ms_pass = e0.elapsed_time(e1) / args.steps
    mp = B * H * W / 1e6
    flops = 2 * B * unet_macs(C, H, W)
    traffic = B * unet_bytes(C, H, W)
    log("unet: %.3f ms/step (%d images), %.1f MP/s, %.1f TFLOP/s, %.2f TB/s compulsory" % (
        dt * 1e3, B, mp / dt, flops / dt / 1e12, traffic / (ms_pass * 1e-3) / 1e12))
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import unet as ounet
        b0, y0 = basics[0][:256, :256].cpu().numpy(), noisys[0][:256, :256].cpu().numpy()
        n, t1 = 0, time.perf_counter()
        while True:
            ounet.restore(b0, y0, sigma, weights)
            n += 1
            el = time.perf_counter() - t1
            if el >= min(args.cpu_seconds, 10.0):
                break
        cpu = {"value": n * 256 * 256 / 1e6 / el, "unit": "MP/s", "cores": blas_threads(), "kind": "oracle",
               "sample": "%d x 256x256 colour crop, FP64 numpy oracle (BLAS tensordot), %.1f s" % (n, el)}
    res = {
        "metric": "restored MP/s (flexible U-Net x_hat = BM3D(y) + F(z, sigma), colour)", "value": mp / dt,
        "unit": "MP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (seeded random weights; trained weights not available)",
        "config": {"workload": "512x512 colour, sigma=25, widths 32/64/128/256/256, batch of %d images per call"
                               % B, "batch": B, "gflop_per_image": flops / B / 1e9},
        "roofline": {"bound": "hbm", "kernel": "whole pass (30 launches, stream-ordered)",
                     "achieved": traffic / (ms_pass * 1e-3) / 1e9, "peak": PEAK["hbm_GBps"], "unit": "GB/s",
                     "frac": traffic / (ms_pass * 1e-3) / 1e9 / PEAK["hbm_GBps"], "traffic": None,
                     "ms_per_launch": ms_pass,
                     "work_per_launch": traffic},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def run_vst(args):
    """Variance-stabilising wrapper: 16 raw Poisson-Gaussian 512 x 512 grey
    images (alpha 1.5, sigma 2, up to 150 counts); per step the forward map
    over the batch, the batched BM3D pass (captured graph) at the 8-bit
    noise level, and the unbiased inverse."""
    import torch
    from paper_2403_03488_amd import bm3d, synth
    assert torch.cuda.is_available(), "no GPU"
    H, W, B, alpha, sigma, peak = 512, 512, args.batch, 1.5, 2.0, 150.0
    rng = np.random.default_rng(0)
    raw = np.empty((B, H, W), np.float32)
    for i in range(B):
        x = synth.gray_512(index=i).clean.astype(np.float64) / 255.0 * peak
        raw[i] = alpha * rng.poisson(x / alpha) + rng.normal(0.0, sigma, x.shape)
    fmax = 2.0 / alpha * math.sqrt(max(alpha * float(raw.max()) + 0.375 * alpha * alpha + sigma * sigma, 0.0))
    g = bm3d.GatParams(alpha, sigma, 0.0, 235.0 / fmax, 10.0)
    sig = bm3d.gat_noise_level(g.scale)
    zd = torch.from_numpy(raw).cuda()
    u = torch.empty((B, H, W), dtype=torch.uint8, device="cuda")
    d = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
    xh = torch.empty_like(d)
    p = tuned_params(args, bm3d, sig, 0)
    plan = bm3d.Batch([u[i] for i in range(B)], [d[i] for i in range(B)], [sig] * B, p)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    if args.calibrate_copy:
        calibration_copy(torch)
    bm3d.gat_forward(zd, g, out=u, stream=stream)
    torch.cuda.synchronize()
    plan.capture(stream)

    def step():
        bm3d.gat_forward(zd, g, out=u, stream=stream)
        plan.launch(stream)
        bm3d.gat_inverse(d, g, out=xh, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the wrapper's own kernels, timed alone with HIP events on their stream
    reps = 50
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(stream)
    for _ in range(reps):
        bm3d.gat_forward(zd, g, out=u, stream=stream)
    e1.record(stream)
    for _ in range(reps):
        bm3d.gat_inverse(d, g, out=xh, stream=stream)
    e2.record(stream)
    torch.cuda.synchronize()
    ms_f, ms_i = e0.elapsed_time(e1) / reps, e1.elapsed_time(e2) / reps
    n = B * H * W
    bytes_f, bytes_i = 5 * n, 8 * n  # float in + u8 out; float in + float out
    mp = n / 1e6
    x = np.stack([synth.gray_512(index=i).clean.astype(np.float64) / 255.0 * peak for i in range(B)])
    rmse = lambda a: float(np.sqrt(np.mean((a - x) ** 2)))
    out = xh.cpu().numpy().astype(np.float64)
    log("vst: %.3f ms/step (%d images), %.1f MP/s; forward %.1f us (%.0f GB/s), inverse %.1f us (%.0f GB/s); "
        "rmse raw %.2f -> %.2f" % (dt * 1e3, B, mp / dt, ms_f * 1e3, bytes_f / ms_f / 1e6, ms_i * 1e3,
                                    bytes_i / ms_i / 1e6, rmse(raw), rmse(out)))
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import vst as ovst
        n_cpu, t1 = 0, time.perf_counter()
        while True:
            uu = ovst.forward_u8_f32(raw[0], alpha, sigma, 0.0, g.scale, g.offset)
            ovst.restore_from_u8(uu.astype(np.float64), alpha, sigma, 0.0, g.scale, g.offset)
            n_cpu += 1
            el = time.perf_counter() - t1
            if el >= min(args.cpu_seconds, 5.0):
                break
        cpu = {"value": n_cpu * H * W / 1e6 / el, "unit": "MP/s", "cores": 1, "kind": "oracle",
               "sample": "%d x one 512x512 image through the oracle's forward map and inverse (the BM3D "
                         "step excluded), numpy, %.1f s" % (n_cpu, el)}
    res = {
        "metric": "restored MP/s (raw Poisson-Gaussian: GAT, BM3D, unbiased inverse)", "value": mp / dt,
        "unit": "MP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16+int8",
        "data": "synthetic",
        "config": {"workload": "16 raw 512x512 grey images, alpha=1.5, sigma=2, up to 150 counts; BM3D at the "
                               "8-bit noise level %.2f" % sig, "batch": B, "alpha": alpha, "sigma": sigma,
                   "scale": g.scale, "offset": g.offset},
        "roofline": {"bound": "hbm", "kernel": "k_inverse (unbiased inverse)", "achieved": bytes_i / ms_i / 1e6,
                     "peak": PEAK["hbm_GBps"], "unit": "GB/s", "frac": bytes_i / ms_i / 1e6 / PEAK["hbm_GBps"],
                     "traffic": None, "ms_per_launch": ms_i, "work_per_launch": bytes_i,
                     "forward": {"ms_per_launch": ms_f, "achieved": bytes_f / ms_f / 1e6}},
        "rmse": {"raw": rmse(raw), "restored": rmse(out)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def run_pipeline(args):
    """The method of Section II end to end: BM3D (batched, graph-captured)
    on 16 noisy colour 512 x 512 images (sigma 25), then the K = 10 residual
    network on its estimate and the observation."""
    import torch
    from paper_2403_03488_amd import bm3d, synth
    assert torch.cuda.is_available(), "no GPU"
    K, C, H, W, B, sigma = 10, 3, 512, 512, args.batch, 25.0
    rng = np.random.default_rng(0)
    imgs = []
    for i in range(B):
        s = synth.colour_481x321(index=i, sigma=sigma)
        cl = np.pad(s.clean, ((0, H - s.clean.shape[0]), (0, W - s.clean.shape[1]), (0, 0)), mode="reflect")
        imgs.append(torch.from_numpy(synth.add_awgn_u8(cl.astype(np.float64), sigma, rng)).cuda())
    basic = [torch.empty((H, W, C), dtype=torch.float32, device="cuda") for _ in range(B)]
    outs = [torch.empty((H, W, C), dtype=torch.float32, device="cuda") for _ in range(B)]
    p = tuned_params(args, bm3d, sigma, 0)
    plan = bm3d.Batch(imgs, basic, [sigma] * B, p)
    net = bm3d.Cnn(synth.cnn_layers(K, C, seed=1), C)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    torch.cuda.synchronize()
    plan.capture(stream)

    def step():
        plan.launch(stream)
        net.restore(basic, imgs, outs, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    for _ in range(args.steps):
        plan.launch(stream)
    ev[1].record(stream)
    for _ in range(args.steps):
        net.restore(basic, imgs, outs, stream=stream)
    ev[2].record(stream)
    torch.cuda.synchronize()
    ms_bm3d, ms_cnn = ev[0].elapsed_time(ev[1]) / args.steps, ev[1].elapsed_time(ev[2]) / args.steps
    mp = B * H * W / 1e6
    log("pipeline: %.3f ms/step (%d colour images): BM3D %.3f ms, network %.3f ms; %.1f MP/s, %.3f ms per image" % (
        dt * 1e3, B, ms_bm3d, ms_cnn, mp / dt, dt * 1e3 / B))
    res = {
        "metric": "restored MP/s (BM3D then the K=10 residual network, colour, sigma=25)", "value": mp / dt,
        "unit": "MP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+int8",
        "data": "synthetic (seeded random network weights)",
        "config": {"workload": "16 noisy 512x512 colour images, sigma=25: batched BM3D pass, then K=10 network",
                   "batch": B, "layers": K},
        "stages_ms": {"bm3d": ms_bm3d, "network": ms_cnn}, "ms_per_image": dt * 1e3 / B,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def blas_threads():
    """Threads of the BLAS numpy's tensordot runs on."""
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        return 1


def ocnn_macs(K, C, H, W, F=64):
    """Multiply-adds of the network on one H x W image (9 per input/output
    channel pair, pixel and layer)."""
    return 9 * H * W * (2 * C * F + (K - 2) * F * F + F * C)


def measure_batch64(args, steps=None, warmup=None):
    """The mixed batch: 64 images of areas 128^2..1024^2 (aspect 1:1-2:1),
    half grey / half colour, sigma ~ U[10,50], one captured graph per step.
    Returns the measurement as a dict."""
    import torch
    from paper_2403_03488_amd import bm3d, synth
    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    shapes = synth.batch_shapes(64)
    log("generating the 64-image mixed batch")
    samples = [synth.batch_image(i, sh) for i, sh in enumerate(shapes)]
    imgs = [torch.from_numpy(s.noisy).cuda() for s in samples]
    outs = [torch.empty(s.noisy.shape, dtype=torch.float32, device="cuda") for s in samples]
    p = tuned_params(args, bm3d, 25.0, bm3d.FLAG_SIGMA_PROFILE)
    plan = bm3d.Batch(imgs, outs, [s.sigma for s in samples], p)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    torch.cuda.synchronize()
    plan.capture(stream)
    for _ in range(warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.launch(stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    mp = sum(s.h * s.w for s in samples) / 1e6
    cmp = sum(s.h * s.w * s.c for s in samples) / 1e6
    log("mixed batch %s: %.3f ms/step, %.1f MP/s" % (args.xform, dt * 1e3, mp / dt))
    stage_ms = stage_times(torch, bm3d, plan, len(samples), stream)
    plan.launch(stream)
    torch.cuda.synchronize()
    ps = [synth.psnr(s.clean, o.cpu().numpy()) for s, o in zip(samples, outs)]
    plan.close()
    return {"MPps": mp / dt, "ms_per_step": dt * 1e3, "steps": steps, "megapixels": mp,
            "channel_megapixels": cmp, "channel_MPps": cmp / dt, "stages_ms": stage_ms,
            "tile_refs": p.tile_refs, "persistent_wgs": p.persistent_wgs, "match_refs": p.match_refs,
            "psnr_db": {"mean": float(np.mean(ps)), "min": float(np.min(ps))},
            "workload": "64 images, areas 128^2-1024^2, aspect 1:1-2:1, half grey / half colour, "
                        "sigma U[10,50], one graph-captured batched pass per step"}


def measure_highsigma(args, steps=None, warmup=None):
    """The published method's high-noise variants on the headline batch shape:
    16 x 512^2 grey at sigma = 50 with the bior1.5 step-1 transform and step-1
    grouping on 2-D spectra hard-thresholded at 2 sigma, beside the default
    profile (DCT, grouping on the noisy pixels) on the same images and
    settings.  Returns the measurement as a dict."""
    import torch
    from paper_2403_03488_amd import bm3d, synth
    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    sigma, H, W, B = 50.0, 512, 512, args.batch
    log("generating %d synthetic %dx%d images at sigma %.0f" % (B, H, W, sigma))
    samples = [synth.gray_512(index=i, sigma=sigma) for i in range(B)]
    imgs = [torch.from_numpy(s.noisy).cuda() for s in samples]
    outs = [torch.empty((H, W), dtype=torch.float32, device="cuda") for _ in range(B)]
    base = tuned_params(args, bm3d, sigma)
    res = {}
    for name, lam2d, xf in (("variant", 2.0, bm3d.T_BIOR15), ("default", 0.0, bm3d.T_DCT)):
        p = bm3d.params_default(sigma, xform=XF[args.xform])
        p.tile_refs, p.persistent_wgs, p.match_refs = base.tile_refs, base.persistent_wgs, base.match_refs
        p.lambda_2d, p.transform_ht = lam2d, xf
        plan = bm3d.Batch(imgs, outs, [sigma] * B, p)
        stream = torch.cuda.Stream()
        torch.cuda.set_stream(stream)
        torch.cuda.synchronize()
        plan.capture(stream)
        for _ in range(warmup):
            plan.launch(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.launch(stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        stage_ms = stage_times(torch, bm3d, plan, B, stream)
        plan.launch(stream)
        torch.cuda.synchronize()
        ps = [synth.psnr(s.clean, o.cpu().numpy()) for s, o in zip(samples, outs)]
        plan.close()
        res[name] = {"MPps": B * H * W / 1e6 / dt, "ms_per_step": dt * 1e3, "stages_ms": stage_ms,
                     "psnr_db_mean": float(np.mean(ps))}
        log("sigma 50 %s profile: %.3f ms/step, %.1f MP/s, PSNR %.3f dB; stages %s" % (
            name, dt * 1e3, res[name]["MPps"], res[name]["psnr_db_mean"],
            ", ".join("%s %.3f" % kv for kv in stage_ms.items())))
    v = res["variant"]
    return {"MPps": v["MPps"], "ms_per_step": v["ms_per_step"], "steps": steps, "stages_ms": v["stages_ms"],
            "psnr_db_mean": v["psnr_db_mean"], "default_profile": res["default"],
            "tile_refs": base.tile_refs, "persistent_wgs": base.persistent_wgs,
            "workload": "%d x 512x512 grey, sigma=50, bior1.5 step-1 transform, step-1 grouping on 2-D "
                        "spectra thresholded at 2 sigma (match1 time includes the spectra), S=32, "
                        "N1=16, N2=32, stride 3, graph-captured batched pass" % B}


def run_highsigma(args):
    import torch
    assert torch.cuda.is_available(), "no GPU"
    m = measure_highsigma(args)
    res = {
        "metric": "denoised MP/s (both BM3D steps, sigma=50, high-noise variants)", "value": m["MPps"],
        "unit": "MP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.xform + "+fp32", "data": "synthetic",
        "config": {"workload": m["workload"], "batch": args.batch, "xform": args.xform,
                   "tile_refs": m["tile_refs"], "persistent_wgs": m["persistent_wgs"]},
        "stages_ms": m["stages_ms"], "psnr_db_mean": m["psnr_db_mean"],
        "default_profile": m["default_profile"],
    }
    print(json.dumps(res), flush=True)


def run_batch64(args):
    import torch
    assert torch.cuda.is_available(), "no GPU"
    m = measure_batch64(args)
    res = {
        "metric": "denoised MP/s (64-image mixed batch, both BM3D steps)", "value": m["MPps"],
        "unit": "MP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.xform + "+int8", "data": "synthetic",
        "config": {"workload": m["workload"], "megapixels": m["megapixels"],
                   "channel_megapixels": m["channel_megapixels"], "xform": args.xform,
                   "tile_refs": m["tile_refs"], "persistent_wgs": m["persistent_wgs"]},
        "channel_MPps": m["channel_MPps"], "stages_ms": m["stages_ms"], "psnr_db": m["psnr_db"],
    }
    print(json.dumps(res), flush=True)


def measure_serving(args, n=None):
    """Serving: Poisson arrivals at args.load x the measured capacity, sides
    log-uniform 256-4096, 70 % grey, sigma U[5,60], 30 % moire.  The request
    loop (stage-level continuous batching, BF16 transforms + int8 matching)
    against the plain FP32 single-image path serving the same trace one
    request at a time.  Returns the measurement as a dict."""
    import torch
    from paper_2403_03488_amd import bm3d, serve, synth
    n = n or args.requests
    log("building %d serving requests (canvases, noise, pinned inputs)" % n)
    canv = synth.serving_canvases(4096)
    noise = synth.serving_noise(4096)
    specs = synth.serving_specs(n, rate=1.0)  # arrival times in units of 1/rate
    hosts = []
    for sp in specs:
        x = torch.from_numpy(synth.crop_clean(canv, sp)).float()
        x.add_(torch.from_numpy(synth.noise_crop(noise, sp)), alpha=sp["sigma"]).round_().clamp_(0, 255)
        buf = torch.empty(x.shape, dtype=torch.uint8, pin_memory=True)
        buf.copy_(x)
        hosts.append(buf)
    del canv, noise
    mean_mp = sum(sp["h"] * sp["w"] for sp in specs) / 1e6 / n
    log("requests ready: mean %.2f MP" % mean_mp)
    p = tuned_params(args, bm3d, 25.0, bm3d.FLAG_SIGMA_PROFILE)
    p32 = bm3d.params_default(25.0, xform=0, flags=bm3d.FLAG_SIGMA_PROFILE)

    def requests(scale):
        return [serve.Request(sp["rid"], sp["arrival"] * scale, h, sp["sigma"]) for sp, h in zip(specs, hosts)]

    # warm-up and capacity: the first requests all present at t = 0
    m = min(n, args.capacity_requests)
    serve.ServingLoop(p, max_slots=args.slots).run(requests(0.0)[:8])
    torch.cuda.synchronize()
    cap = serve.summarize(serve.ServingLoop(p, max_slots=args.slots).run(requests(0.0)[:m]))
    cap_req = cap["MPps"] / mean_mp
    rate = args.load * cap_req
    log("capacity %.1f MP/s (%.1f req/s); offered load %.2f -> %.2f req/s" % (cap["MPps"], cap_req,
                                                                            args.load, rate))
    loop = serve.ServingLoop(p, max_slots=args.slots)
    rs = loop.run(requests(1.0 / rate))
    st = serve.summarize(rs)
    log("served: %.1f MP/s, p50 %.1f ms, p99 %.1f ms, %d ticks (mean %.1f requests per tick)" % (
        st["MPps"], st["p50_ms"], st["p99_ms"], loop.ticks, np.mean(loop.tick_sizes)))
    base = serve.summarize(serve.serve_one_at_a_time(requests(1.0 / rate), p32))
    log("FP32 single-image path: %.1f MP/s, p50 %.1f ms, p99 %.1f ms" % (base["MPps"], base["p50_ms"],
                                                                        base["p99_ms"]))
    return {"MPps": st["MPps"], "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
            "makespan_s": st["makespan_s"], "capacity_MPps": cap["MPps"], "requests": n, "mean_MP": mean_mp,
            "load": args.load, "rate_req_s": rate, "slots": args.slots, "ticks": loop.ticks,
            "mean_requests_per_tick": float(np.mean(loop.tick_sizes)), "peak_hbm_bytes": loop.peak_used,
            "tile_refs": p.tile_refs, "persistent_wgs": p.persistent_wgs, "match_refs": p.match_refs,
            "fp32_single_image_path": {"MPps": base["MPps"], "p50_ms": base["p50_ms"],
                                       "p99_ms": base["p99_ms"], "makespan_s": base["makespan_s"]},
            "workload": "serving: %d requests, sides log-uniform 256-4096, 70%% grey / 30%% colour, "
                        "sigma U[5,60], 30%% moire, Poisson arrivals at %.1fx the measured capacity"
                        % (n, args.load)}


def run_serving(args):
    import torch
    assert torch.cuda.is_available(), "no GPU"
    m = measure_serving(args)
    res = {
        "metric": "served MP/s with p50/p99 latency (Poisson arrivals at %.1fx capacity)" % args.load,
        "value": m["MPps"], "unit": "MP/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": args.xform + "+int8", "data": "synthetic",
        "config": {"workload": m["workload"], "requests": m["requests"], "mean_MP": m["mean_MP"],
                   "rate_req_s": m["rate_req_s"], "slots": m["slots"], "xform": args.xform,
                   "tile_refs": m["tile_refs"], "persistent_wgs": m["persistent_wgs"]},
        "p50_ms": m["p50_ms"], "p99_ms": m["p99_ms"], "mean_ms": m["mean_ms"],
        "makespan_s": m["makespan_s"], "capacity_MPps": m["capacity_MPps"],
        "ticks": m["ticks"], "mean_requests_per_tick": m["mean_requests_per_tick"],
        "peak_hbm_bytes": m["peak_hbm_bytes"], "fp32_single_image_path": m["fp32_single_image_path"],
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--xform", default="bf16", choices=list(XF))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="force the filter tile side (refs)")
    ap.add_argument("--persistent", type=int, default=-1, help="force workgroups per CU (0 = one per item)")
    ap.add_argument("--match-refs", type=int, default=0, choices=(0, 8, 16),
                    help="force the step-1 references per matching pass (0 = autotuned)")
    ap.add_argument("--quick", action="store_true",
                    help="only the timed batched pass and stage timings (for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--workload", default="grey512", choices=["grey512", "batch64", "serving", "highsigma", "nlm", "cnn", "unet", "vst",
                             "pipeline"],
                    help="grey512: the headline 16 x 512^2 batch (default); batch64: the 64-image "
                         "mixed batch; serving: the request loop against the FP32 single-image path; "
                         "highsigma: the high-noise variants (bior1.5, prefiltered grouping) at sigma=50; "
                         "nlm: the NL-means first stage on the 16 x 512^2 batch")
    ap.add_argument("--requests", type=int, default=2000, help="serving: number of requests")
    ap.add_argument("--default-requests", type=int, default=500,
                    help="requests of the serving trace measured in the default run")
    ap.add_argument("--no-extra", action="store_true",
                    help="default run: skip the mixed-batch, serving and high-noise measurements")
    ap.add_argument("--load", type=float, default=0.7, help="serving: offered load / capacity")
    ap.add_argument("--slots", type=int, default=32, help="serving: requests in flight")
    ap.add_argument("--capacity-requests", type=int, default=300,
                    help="serving: requests in the capacity measurement")
    args = ap.parse_args()
    if args.quick:
        args.no_autotune = args.no_cpu_baseline = True
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "every image is independent, so a batch would shard by image across GPUs",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch64":
        return run_batch64(args)
    if args.workload == "serving":
        return run_serving(args)
    if args.workload == "highsigma":
        return run_highsigma(args)
    if args.workload == "cnn":
        return run_cnn(args)
    if args.workload == "unet":
        return run_unet(args)
    if args.workload == "vst":
        return run_vst(args)
    if args.workload == "pipeline":
        return run_pipeline(args)
    if args.workload == "nlm":
        return run_nlm(args)

    import torch
    from paper_2403_03488_amd import bm3d, synth

    assert torch.cuda.is_available(), "no GPU"
    sigma, S, H, W = 25.0, 32, 512, 512
    B = args.batch
    log("generating %d synthetic %dx%d images" % (B, H, W))
    samples = [synth.gray_512(index=i, sigma=sigma) for i in range(B)]
    imgs = [torch.from_numpy(s.noisy).cuda() for s in samples]
    outs = [torch.empty((H, W), dtype=torch.float32, device="cuda") for _ in range(B)]

    p = tuned_params(args, bm3d, sigma)
    plan = bm3d.Batch(imgs, outs, [sigma] * B, p)
    stream = torch.cuda.Stream()  # graph capture needs a non-default stream
    torch.cuda.set_stream(stream)
    torch.cuda.synchronize()
    plan.capture(stream)

    for _ in range(args.warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch(stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    mp = B * H * W / 1e6
    value = mp / dt
    log("batched %s: %.3f ms/step, %.1f MP/s" % (args.xform, dt * 1e3, value))

    stage_ms = stage_times(torch, bm3d, plan, B, stream)
    log("stage ms: " + ", ".join("%s %.3f" % kv for kv in stage_ms.items()))

    # group sizes of every image (stage entry points, outside the timed region)
    R = bm3d.num_refs(H, W)
    work = {"match1": 0.0, "filter1": 0.0, "match2": 0.0, "filter2": 0.0}
    issued = {"filter1": 0.0, "filter2": 0.0}
    planar = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    lum = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    lumf = torch.empty((H, W), dtype=torch.float32, device="cuda")
    i1 = torch.empty((R, p.n_ht), dtype=torch.int32, device="cuda")
    c1 = torch.empty(R, dtype=torch.int32, device="cuda")
    i2 = torch.empty((R, p.n_wie), dtype=torch.int32, device="cuda")
    c2 = torch.empty(R, dtype=torch.int32, device="cuda")
    num = torch.empty((1, H, W), dtype=torch.int64, device="cuda")
    wsum = torch.empty_like(num)
    basic = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    for im in imgs:
        bm3d.prepare(im, planar, lum)
        bm3d.block_match(lum, 1, p, i1, c1)
        num.zero_()
        wsum.zero_()
        bm3d.collab_filter(planar, None, sigma, 1, i1, c1, p, num, wsum)
        bm3d.aggregate(num, wsum, False, p, basic)
        bm3d.luminance(basic, lumf)
        bm3d.block_match(lumf, 2, p, i2, c2)
        c1h, c2h = c1.cpu().numpy(), c2.cpu().numpy()
        wm = work_models(H, W, S, c1h, c2h)
        for k in work:
            work[k] += wm[k]
        for k, v in mfma_issued(c1h, c2h).items():
            issued[k] += v
    kinds = {"match1": ("mfma", "int8", PEAK["int8"], "TOP/s"),
             "match2": ("alu", "fp32_valu", PEAK["fp32_valu"], "TFLOP/s"),
             "filter1": ("mfma", args.xform, PEAK[args.xform if args.xform != "fp32" else "fp32_mfma"], "TFLOP/s"),
             "filter2": ("mfma", args.xform, PEAK[args.xform if args.xform != "fp32" else "fp32_mfma"], "TFLOP/s")}
    dom = max(work, key=lambda k: stage_ms[k])
    bound, _, peak, unit = kinds[dom]
    achieved = work[dom] / (stage_ms[dom] * 1e-3)
    roof = {"bound": bound, "kernel": dom, "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": unit, "frac": achieved / peak,
            "traffic": (measured_traffic(dom, B, p.tile_refs, match_refs=p.match_refs)
                        if args.xform == "bf16" else None),
            "ms_per_launch": stage_ms[dom], "work_per_launch": work[dom],
            "work_model": {"match1": "S^2 * 64 int8 multiply-adds per reference",
                           "match2": "S^2 * 64 FP32 multiply-adds per reference (direct differences)",
                           "filter1": "separable 3-D transforms at the actual group sizes, 2048n + 128n^2 "
                                      "multiply-adds per group and channel",
                           "filter2": "separable 3-D transforms at the actual group sizes, 3 (1024n + 64n^2) "
                                      "multiply-adds per group and channel"}[dom] + " (2 ops per multiply-add)"}
    if dom in issued:
        roof["mfma_issued"] = {"ops_per_launch": issued[dom],
                               "TOPps": issued[dom] / (stage_ms[dom] * 1e-3) / 1e12,
                               "note": "dense 64x64 DCT products and 16/32-member WHT tiles as executed"}
    per_stage = {k: {"ms": stage_ms[k], "frac": (work[k] / (stage_ms[k] * 1e-3)) / kinds[k][2]}
                 for k in work}
    # pass-level bound: the time each resource needs for the whole pass at its
    # peak (HBM: the compulsory bytes, 13 B per grey pixel); the largest one
    # over the measured pass time
    need_s = {"fp32_valu (step-2 distances)": work["match2"] / PEAK["fp32_valu"],
              "%s matrix cores (transforms)" % args.xform:
                  (work["filter1"] + work["filter2"]) / kinds["filter1"][2],
              "int8 matrix cores (step-1 distances)": work["match1"] / PEAK["int8"],
              "hbm (compulsory bytes)": 13.0 * B * H * W / (PEAK["hbm_GBps"] * 1e9)}
    binding = max(need_s, key=need_s.get)
    pass_bound = {"binding": binding, "us_at_peak": need_s[binding] * 1e6,
                  "us_per_MP_at_peak": need_s[binding] * 1e6 / mp, "frac": need_s[binding] / dt,
                  "all_us_at_peak": {k: v * 1e6 for k, v in need_s.items()}}
    log("roofline %s: %.1f %s of %.0f (%.4f); pass bound %s: %.1f us at peak, %.4f of the pass"
        % (dom, achieved / 1e12, unit, peak / 1e12, achieved / peak, binding, need_s[binding] * 1e6,
           need_s[binding] / dt))

    if args.calibrate_copy:
        calibration_copy(torch)
    lat_ms, fp32_single, psnr32, psnrlo = [float("nan")], float("nan"), float("nan"), float("nan")
    if not args.quick:
        lat_ms, fp32_single, psnr32, psnrlo = single_image_checks(torch, bm3d, synth, p, imgs, outs,
                                                                  samples, sigma, H, W, B)
    plan.close()
    # the mixed 64-image batch and the serving trace, measured in the same run
    mixed = serving = high = None
    if not args.quick and not args.no_extra:
        mixed = measure_batch64(args, steps=10, warmup=2)
        serving = measure_serving(args, n=args.default_requests)
        high = measure_highsigma(args, steps=10, warmup=2)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, samples, sigma, S, H, W)

    res = {
        "metric": "denoised MP/s (both BM3D steps, sigma=25)", "value": value, "unit": "MP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.xform + "+int8", "data": "synthetic",
        "config": {"workload": "512x512 grey, sigma=25, S=32, N1=16, N2=32, stride 3, "
                               "batch of %d images per step, graph-captured batched pass" % B,
                   "batch": B, "xform": args.xform, "tile_refs": p.tile_refs,
                   "persistent_wgs": p.persistent_wgs, "match_refs": p.match_refs},
        "roofline": roof, "stages": per_stage, "pass_bound": pass_bound,
        "latency_ms_single_image": {"p50": float(np.percentile(lat_ms, 50)),
                                    "p99": float(np.percentile(lat_ms, 99))},
        "fp32_single_image_MPps": fp32_single,
        "psnr_db": {"fp32": psnr32, args.xform: psnrlo, "delta": psnrlo - psnr32},
        "mixed_batch": mixed, "serving": serving, "high_noise_variants": high,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
