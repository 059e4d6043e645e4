"""Residual network through the C ABI against the FP64 oracle.

The HIP path stores z and every activation in bfloat16 (round to nearest,
relative error <= 2^-9) and accumulates in FP32; the oracle keeps FP64
throughout, with the same bfloat16-representable weights.  Propagating the
storage rounding through the remaining layers (an FP64 emulation on these
seeded weights) gives max |error| 0.04-0.27 grey levels and an RMS error of
0.3-1.4 % of the residual's RMS for K = 10 and 16; the bar is max |error| <=
0.5 and RMS error <= 3 % of the residual.  A wrong tap, channel or plane
changes the output by the size of the residual itself (several grey
levels)."""
import numpy as np
import pytest

from oracle import cnn as O
from paper_2403_03488_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
MAX_ABS, REL_RMS = 0.5, 0.03


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03488_amd import bm3d
    return bm3d


def log(msg):
    print(msg, flush=True)


def inputs(h, w, c, seed):
    """A first-stage-like estimate (smooth content plus a little noise) and
    its observation."""
    rng = np.random.default_rng(seed)
    clean = synth.mixed_colour_image(rng, h, w) if c == 3 else synth.smooth_texture_image(rng, h, w)
    clean = clean.astype(np.float64)
    noisy = synth.add_awgn_u8(clean, 25.0, rng)
    basic = (clean + rng.normal(0, 3, clean.shape)).astype(np.float32)
    return basic, noisy


def run(B, net, basics, noisys):
    bd = [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in basics]
    nd = [torch.from_numpy(np.ascontiguousarray(y)).cuda() for y in noisys]
    outs = net.restore(bd, nd)
    torch.cuda.synchronize()
    return [o.cpu().numpy().astype(np.float64) for o in outs]


def check(got, basic, noisy, layers, what):
    ref = O.restore(basic, noisy, layers)
    err = got - ref
    F = ref - basic
    rms_e, rms_f = np.sqrt((err ** 2).mean()), np.sqrt((F ** 2).mean())
    log("%s: max|err| %.4f rms err %.4f rms residual %.3f" % (what, np.abs(err).max(), rms_e, rms_f))
    assert np.isfinite(got).all()
    assert np.abs(err).max() <= MAX_ABS
    assert rms_e <= REL_RMS * rms_f


@pytest.mark.parametrize("K,c,h,w", [(10, 3, 96, 160), (10, 3, 100, 150), (10, 1, 37, 75), (16, 3, 64, 96),
                                     (16, 1, 50, 33)])
def test_restore_matches_oracle(B, K, c, h, w):
    layers = synth.cnn_layers(K, c, seed=K + c)
    net = B.Cnn(layers, c)
    basic, noisy = inputs(h, w, c, seed=h + w)
    got = run(B, net, [basic], [noisy])[0]
    check(got, basic, noisy, layers, "K=%d c=%d %dx%d" % (K, c, h, w))


@pytest.mark.parametrize("shape", [(1, 1, 3), (3, 40), (17, 1), (2, 2, 3), (16, 32), (17, 33, 3)])
def test_small_and_degenerate_images(B, shape):
    c = 3 if len(shape) == 3 else 1
    layers = synth.cnn_layers(10, c, seed=3)
    net = B.Cnn(layers, c)
    basic, noisy = inputs(shape[0], shape[1], c, seed=11)
    got = run(B, net, [basic], [noisy])[0]
    check(got, basic, noisy, layers, "shape %s" % (shape,))


def test_minimal_network_without_bias_or_normalisation(B):
    # K = 3, no biases, normalisation on neither layer
    layers = [{"weight": L["weight"]} for L in synth.cnn_layers(3, 3, seed=21)]
    net = B.Cnn(layers, 3)
    basic, noisy = inputs(40, 70, 3, seed=5)
    got = run(B, net, [basic], [noisy])[0]
    check(got, basic, noisy, layers, "K=3 plain")


def test_zero_last_layer_returns_basic_exactly(B):
    layers = synth.cnn_layers(10, 3, seed=4)
    layers[-1] = {"weight": np.zeros_like(layers[-1]["weight"]), "bias": np.zeros(3, np.float32)}
    net = B.Cnn(layers, 3)
    basic, noisy = inputs(45, 67, 3, seed=6)
    got = run(B, net, [basic], [noisy])[0]
    assert np.array_equal(got, basic.astype(np.float64))


def test_batch_equals_single(B):
    layers = synth.cnn_layers(10, 1, seed=7)
    net = B.Cnn(layers, 1)
    pairs = [inputs(70, 90, 1, seed=30 + i) for i in range(4)]
    batched = run(B, net, [p[0] for p in pairs], [p[1] for p in pairs])
    for (b, y), g in zip(pairs, batched):
        assert np.array_equal(run(B, net, [b], [y])[0], g)
    check(batched[2], pairs[2][0], pairs[2][1], layers, "batch image 2")


def test_full_size_batch_sampled(B):
    # 16 colour 512 x 512 images in one call, as timed; the oracle evaluates
    # sampled pixels on crops of radius K around them (clipped to the image):
    # the network's output at a pixel depends on inputs within K pixels only,
    # and zero padding at crop edges reaches at most K - 1 pixels inward
    K, c, n = 10, 3, 16
    layers = synth.cnn_layers(K, c, seed=1)
    net = B.Cnn(layers, c)
    pairs = [inputs(512, 512, c, seed=100 + i) for i in range(n)]
    outs = run(B, net, [p[0] for p in pairs], [p[1] for p in pairs])
    rng = np.random.default_rng(0)
    pts = [(0, 0), (511, 511), (0, 511), (511, 0), (15, 31), (16, 32), (255, 256)]
    pts += [tuple(int(v) for v in rng.integers(0, 512, 2)) for _ in range(9)]
    worst = 0.0
    for i in (0, 7, 15):
        basic, noisy = pairs[i]
        for y, x in pts:
            y0, y1, x0, x1 = max(0, y - K), min(512, y + K + 1), max(0, x - K), min(512, x + K + 1)
            ref = O.restore(basic[y0:y1, x0:x1], noisy[y0:y1, x0:x1], layers)[y - y0, x - x0]
            worst = max(worst, np.abs(outs[i][y, x] - ref).max())
        assert np.isfinite(outs[i]).all()
    log("512x512 x16 sampled: max|err| %.4f" % worst)
    assert worst <= MAX_ABS


def test_split_layers_equal_one_pass(B):
    # layers 0..3 then 4..K-1 through bm3d_cnn_run_layers give the one-call result
    layers = synth.cnn_layers(10, 3, seed=9)
    net = B.Cnn(layers, 3)
    basic, noisy = inputs(33, 65, 3, seed=8)
    bd, nd = [torch.from_numpy(basic).cuda()], [torch.from_numpy(noisy).cuda()]
    whole = net.restore(bd, nd)[0]
    out = [torch.empty_like(whole)]
    net.restore(bd, nd, outs=out, layers=(0, 4))
    net.restore(bd, nd, outs=out, layers=(4, 10))
    torch.cuda.synchronize()
    assert torch.equal(out[0], whole)


def test_errors_are_reported_before_any_launch(B):
    layers = synth.cnn_layers(4, 1, seed=2)
    net = B.Cnn(layers, 1)
    basic, noisy = inputs(20, 30, 1, seed=1)
    bd, nd = [torch.from_numpy(basic).cuda()], [torch.from_numpy(noisy).cuda()]
    small = torch.empty(B.Cnn.workspace_bytes(1, 20, 30) - 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BM3DError):
        net.restore(bd, nd, workspace=small)
    ws = torch.empty(B.Cnn.workspace_bytes(1, 20, 30) + 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BM3DError):
        net.restore(bd, nd, workspace=ws[1:])                  # misaligned
    for rng_ in ((0, 5), (3, 3), (-1, 2)):
        with pytest.raises(B.BM3DError):
            net.restore(bd, nd, layers=rng_)
    with pytest.raises(ValueError):
        net.restore([torch.zeros((20, 30, 3), device="cuda")], [torch.zeros((20, 30, 3), dtype=torch.uint8,
                                                                             device="cuda")])
    torch.cuda.synchronize()
