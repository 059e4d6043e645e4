"""Seeded synthetic inputs for the BM3D stage.

This module draws images and noise only; it holds none of the denoiser's
arithmetic, so both the HIP path and the FP64 oracle can be fed from it.

The paper evaluates on photographic colour sets (Kodak, McMaster, CBSD68,
MIT moire, Urban100, SIDD; Section II and Section IV) that are not available
here.  These generators stand in for them with images of the same shapes
(512x512 and 1600x1200 in Table 3, 481x321 CBSD-like, up to 4048x3044 SIDD)
and the same kinds of content the paper stresses: piecewise-smooth regions,
sharp edges and periodic textures (the moire / Urban100 argument of
Section II).  The observation model is the paper's eq. (1): y = x + n with n
additive white Gaussian noise of known sigma, then quantised to uint8.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ----------------------------------------------------------------- noise ----


def add_awgn_u8(clean: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """y = clip(rint(x + sigma * N(0,1)), 0, 255) as uint8 (eq. (1), quantised)."""
    x = clean.astype(np.float64)
    y = np.rint(x + sigma * rng.standard_normal(x.shape))
    return np.clip(y, 0, 255).astype(np.uint8)


# ------------------------------------------------------------- painters ----


def _grating(h, w, freq, theta, phase):
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    return np.sin(2.0 * math.pi * freq * (xx * math.cos(theta) + yy * math.sin(theta)) + phase)


def rect_grating_image(rng: np.random.Generator, h: int = 64, w: int = 64) -> np.ndarray:
    """Axis-aligned piecewise-constant rectangles plus one 0.2 cycle/px grating."""
    img = np.full((h, w), float(rng.integers(40, 216)))
    for _ in range(8):
        rh, rw = int(rng.integers(8, 33)), int(rng.integers(8, 33))
        y0, x0 = int(rng.integers(0, max(1, h - rh + 1))), int(rng.integers(0, max(1, w - rw + 1)))
        img[y0:y0 + rh, x0:x0 + rw] = float(rng.integers(0, 256))
    gs = min(24, h, w)
    gy, gx = int(rng.integers(0, h - gs + 1)), int(rng.integers(0, w - gs + 1))
    theta, phase = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi)
    img[gy:gy + gs, gx:gx + gs] = 128.0 + 60.0 * _grating(gs, gs, 0.2, theta, phase)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def smooth_texture_image(rng: np.random.Generator, h: int, w: int,
                         n_regions: int = 12, n_textures: int = 6) -> np.ndarray:
    """Voronoi regions with linear gradients, plus rotated sinusoid/checkerboard
    texture patches with periods 3-16 px."""
    seeds = np.stack([rng.uniform(0, h, n_regions), rng.uniform(0, w, n_regions)], 1)
    # nearest seed per pixel, computed in row blocks to bound memory
    label = np.empty((h, w), np.int32)
    xs = np.arange(w, dtype=np.float64)
    dx2 = (xs[:, None] - seeds[None, :, 1]) ** 2                      # [w, k]
    for r0 in range(0, h, 64):
        ys = np.arange(r0, min(h, r0 + 64), dtype=np.float64)
        dy2 = (ys[:, None] - seeds[None, :, 0]) ** 2                  # [rows, k]
        label[r0:r0 + 64] = np.argmin(dy2[:, None, :] + dx2[None, :, :], axis=2)
    img = np.empty((h, w))
    for k in range(n_regions):
        a = rng.uniform(30, 225)
        b, c = rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)
        # gradients are referenced to the region's seed so levels stay in range
        yy, xx = np.nonzero(label == k)
        img[yy, xx] = a + b * (xx.astype(np.float64) - seeds[k, 1]) + c * (yy.astype(np.float64) - seeds[k, 0])
    for _ in range(n_textures):
        th = int(rng.integers(min(h, 48), min(h, 160) + 1))
        tw = int(rng.integers(min(w, 48), min(w, 160) + 1))
        y0, x0 = int(rng.integers(0, h - th + 1)), int(rng.integers(0, w - tw + 1))
        period = rng.uniform(3.0, 16.0)
        amp = rng.uniform(20.0, 60.0)
        theta, phase = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi)
        base = img[y0:y0 + th, x0:x0 + tw].mean()
        if rng.random() < 0.5:
            pat = _grating(th, tw, 1.0 / period, theta, phase)
        else:
            ly, lx = np.mgrid[0:th, 0:tw].astype(np.float64)
            u = lx * math.cos(theta) + ly * math.sin(theta)
            v = -lx * math.sin(theta) + ly * math.cos(theta)
            pat = np.where((np.floor(u / period) + np.floor(v / period)) % 2 == 0, 1.0, -1.0)
        img[y0:y0 + th, x0:x0 + tw] = base + amp * pat
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def mixed_colour_image(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    """Three independent smooth/texture channels correlated by a random
    row-stochastic positive 3x3 mix; returns HWC uint8."""
    ch = [smooth_texture_image(rng, h, w).astype(np.float64) for _ in range(3)]
    m = rng.uniform(0.1, 1.0, (3, 3))
    m /= m.sum(axis=1, keepdims=True)
    rgb = np.einsum("kc,chw->hwk", m, np.stack(ch))
    return np.clip(np.rint(rgb), 0, 255).astype(np.uint8)


def moire_image(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    """2-3 superposed rotated gratings at 0.3-0.5 cycles/px."""
    img = np.full((h, w), 128.0)
    k = int(rng.integers(2, 4))
    for _ in range(k):
        img += (90.0 / k) * _grating(h, w, rng.uniform(0.3, 0.5), rng.uniform(0, math.pi),
                                     rng.uniform(0, 2 * math.pi))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


# --------------------------------------------------------------- configs ----


@dataclass
class Sample:
    clean: np.ndarray      # uint8, HxW or HxWx3
    noisy: np.ndarray      # uint8, same shape
    sigma: float

    @property
    def h(self):
        return self.clean.shape[0]

    @property
    def w(self):
        return self.clean.shape[1]

    @property
    def c(self):
        return 1 if self.clean.ndim == 2 else self.clean.shape[2]


def _rngs(config: int, index: int):
    return (np.random.default_rng(1000 * config + index),
            np.random.default_rng(1000 * config + index + 500))


def small_gray(index: int = 0, sigma: float = 25.0, h: int = 64, w: int = 64) -> Sample:
    """64x64 grey: rectangles + one 0.2 cycle/px grating, sigma=25."""
    r, rn = _rngs(0, index)
    x = rect_grating_image(r, h, w)
    return Sample(x, add_awgn_u8(x, sigma, rn), sigma)


def gray_512(index: int = 0, sigma: float = 25.0, h: int = 512, w: int = 512) -> Sample:
    """512x512 grey piecewise-smooth gradients plus rotated textures."""
    r, rn = _rngs(1, index)
    x = smooth_texture_image(r, h, w)
    return Sample(x, add_awgn_u8(x, sigma, rn), sigma)


def colour_481x321(index: int = 0, sigma: float = 25.0, h: int = 321, w: int = 481) -> Sample:
    """481x321 colour (CBSD-like shape), channels correlated by a random mix."""
    r, rn = _rngs(2, index)
    x = mixed_colour_image(r, h, w)
    return Sample(x, add_awgn_u8(x, sigma, rn), sigma)


def batch_shapes(n: int = 64, seed_config: int = 3):
    """Sizes for the 64-image batch: area in {128^2,256^2,512^2,1024^2},
    aspect r ~ U[1,2], orientation swapped with p=1/2, half grey / half colour,
    sigma ~ U[10,50]."""
    rng = np.random.default_rng(1000 * seed_config + 999)
    out = []
    for i in range(n):
        area = float(rng.choice([128 ** 2, 256 ** 2, 512 ** 2, 1024 ** 2]))
        r = rng.uniform(1.0, 2.0)
        hh, ww = int(round(math.sqrt(area / r))), int(round(math.sqrt(area * r)))
        if rng.random() < 0.5:
            hh, ww = ww, hh
        c = 1 if i % 2 == 0 else 3
        out.append((hh, ww, c, float(rng.uniform(10.0, 50.0))))
    return out


def batch_image(index: int, shape) -> Sample:
    hh, ww, c, sigma = shape
    r, rn = _rngs(3, index)
    x = smooth_texture_image(r, hh, ww) if c == 1 else mixed_colour_image(r, hh, ww)
    return Sample(x, add_awgn_u8(x, sigma, rn), sigma)


def serving_request(index: int, max_side: int = 4096) -> Sample:
    """Serving mix: sides log-uniform in [256, max_side], 70 % grey, sigma ~ U[5,60],
    30 % moire-like content."""
    r, rn = _rngs(4, index)
    lo, hi = math.log(256), math.log(max_side)
    hh, ww = int(round(math.exp(r.uniform(lo, hi)))), int(round(math.exp(r.uniform(lo, hi))))
    c = 1 if r.random() < 0.7 else 3
    sigma = float(r.uniform(5.0, 60.0))
    if r.random() < 0.3:
        planes = [moire_image(r, hh, ww) for _ in range(c)]
    else:
        planes = [smooth_texture_image(r, hh, ww) for _ in range(c)]
    x = planes[0] if c == 1 else np.stack(planes, axis=2)
    return Sample(x, add_awgn_u8(x, sigma, rn), sigma)


# --------------------------------------------------------------- metrics ----


def psnr(ref: np.ndarray, est: np.ndarray) -> float:
    """PSNR on the [0,255] scale; for colour this is the composite PSNR (CPSNR,
    Section II): one MSE over all channels of all pixels."""
    d = ref.astype(np.float64) - est.astype(np.float64)
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0 else 10.0 * math.log10(255.0 ** 2 / mse)


# ---------------------------------------------------------- serving trace ---


def serving_canvases(side: int = 4096, seed: int = 4000):
    """Large seeded canvases that serving requests are cropped from: grey and
    colour piecewise-smooth/texture content, grey and colour moire."""
    r = np.random.default_rng(seed)
    g = smooth_texture_image(r, side, side, n_regions=48, n_textures=96)
    col = mixed_colour_image(r, side, side)
    m = moire_image(r, side, side)
    mc = np.stack([moire_image(r, side, side) for _ in range(3)], axis=2)
    return {"grey": g, "colour": col, "grey_moire": m, "colour_moire": mc}


def serving_specs(n: int, rate: float, max_side: int = 4096, seed: int = 4001):
    """Poisson arrivals at `rate` requests/s; sides log-uniform in
    [256, max_side]; 70 % grey / 30 % colour; sigma ~ U[5, 60]; 30 % moire."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = math.log(256), math.log(max_side)
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        hh = int(round(math.exp(rng.uniform(lo, hi))))
        ww = int(round(math.exp(rng.uniform(lo, hi))))
        colour = rng.random() < 0.3
        moire = rng.random() < 0.3
        kind = ("colour" if colour else "grey") + ("_moire" if moire else "")
        out.append({"rid": i, "arrival": t, "h": hh, "w": ww, "c": 3 if colour else 1,
                    "sigma": float(rng.uniform(5.0, 60.0)), "kind": kind,
                    "y0": int(rng.integers(0, max_side - hh + 1)),
                    "x0": int(rng.integers(0, max_side - ww + 1)), "noise_seed": 10_000 + i})
    return out


def serving_noise(side: int = 4096, seed: int = 4002) -> np.ndarray:
    """One seeded canvas of standard normals [side, side, 3] (float32); each
    serving request takes its noise from a crop of it at its own offset."""
    return np.random.default_rng(seed).standard_normal((side, side, 3), dtype=np.float32)


def noise_crop(noise: np.ndarray, spec) -> np.ndarray:
    """The request's noise: a crop of the noise canvas at an offset drawn
    from its noise seed (shape HxW or HxWx3, float32)."""
    r = np.random.default_rng(spec["noise_seed"])
    side = noise.shape[0]
    y0 = int(r.integers(0, side - spec["h"] + 1))
    x0 = int(r.integers(0, side - spec["w"] + 1))
    n = noise[y0:y0 + spec["h"], x0:x0 + spec["w"]]
    return n[:, :, 0] if spec["c"] == 1 else n


def crop_clean(canvases, spec):
    a = canvases[spec["kind"]]
    return np.ascontiguousarray(a[spec["y0"]:spec["y0"] + spec["h"], spec["x0"]:spec["x0"] + spec["w"]])


# ------------------------------------------------------- network weights ----
# Trained weights of the residual network (WED training, Section II) are not
# available; both the HIP path and the oracle take these seeded stand-ins.


def bf16_representable(a: np.ndarray) -> np.ndarray:
    """float32 copy of `a` whose values are exactly representable in bfloat16
    (round to nearest, ties to even, on the float32 bit pattern)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def cnn_layers(layers: int = 10, channels: int = 3, features: int = 64, seed: int = 0,
               residual_scale: float = 0.02):
    """K layer dicts for the residual network: He-normal 3x3 kernels
    (std sqrt(2 / fan_in)), rounded to bfloat16-representable values so that
    every precision sees the same weights; small biases; inference-mode batch
    normalisation statistics on the middle layers.  The last layer is scaled
    so that the residual is a correction of a few grey levels (std
    residual_scale * sqrt(1 / fan_in))."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(layers):
        cin = 2 * channels if k == 0 else features
        cout = channels if k == layers - 1 else features
        fan_in = 9 * cin
        std = residual_scale * math.sqrt(1.0 / fan_in) if k == layers - 1 else math.sqrt(2.0 / fan_in)
        L = {"weight": bf16_representable(rng.normal(0.0, std, (cout, cin, 3, 3))),
             "bias": rng.normal(0.0, 0.02, cout).astype(np.float32)}
        if 0 < k < layers - 1:
            L.update(gamma=rng.uniform(0.8, 1.2, cout).astype(np.float32),
                     beta=rng.normal(0.0, 0.05, cout).astype(np.float32),
                     mean=rng.normal(0.0, 0.1, cout).astype(np.float32),
                     var=rng.uniform(0.5, 1.5, cout).astype(np.float32),
                     eps=1e-5)
        out.append(L)
    return out


def unet_net(channels: int = 3, seed: int = 0, widths=(32, 64, 128, 256, 256), residual_scale: float = 0.02):
    """Seeded weights of the flexible U-Net: per depthwise separable block a
    depthwise 3x3 kernel (std sqrt(2/9)) with bias and a pointwise kernel
    (std sqrt(2/cin)) with bias and inference-mode batch normalisation; per
    decoder level a 2x2 deconvolution (std sqrt(2/cin)) with bias; a 1x1
    output layer scaled to a small residual.  All kernels are
    bfloat16-representable."""
    rng = np.random.default_rng(seed)
    f32 = lambda a: np.asarray(a, np.float32)

    def block(ci, co):
        return {"dw": bf16_representable(rng.normal(0.0, math.sqrt(2.0 / 9.0), (ci, 3, 3))),
                "dw_bias": f32(rng.normal(0.0, 0.02, ci)),
                "pw": bf16_representable(rng.normal(0.0, math.sqrt(2.0 / ci), (co, ci))),
                "pw_bias": f32(rng.normal(0.0, 0.02, co)),
                "pw_gamma": f32(rng.uniform(0.8, 1.2, co)), "pw_beta": f32(rng.normal(0.0, 0.05, co)),
                "pw_mean": f32(rng.normal(0.0, 0.1, co)), "pw_var": f32(rng.uniform(0.5, 1.5, co)),
                "pw_eps": 1e-5}

    net = {"enc": [], "down": [], "up": [None] * 4, "dec": [None] * 4}
    c = 2 * channels + 1
    for i in range(4):
        net["enc"].append(block(c, widths[i]))
        net["down"].append(block(widths[i], widths[i + 1]))
        c = widths[i + 1]
    for i in range(4):
        net["up"][i] = {"weight": bf16_representable(rng.normal(0.0, math.sqrt(2.0 / widths[i + 1]),
                                                               (widths[i + 1], widths[i], 2, 2))),
                        "bias": f32(rng.normal(0.0, 0.02, widths[i]))}
        net["dec"][i] = block(widths[i], widths[i])
    net["out"] = {"weight": bf16_representable(rng.normal(0.0, residual_scale * math.sqrt(1.0 / widths[0]),
                                                          (channels, widths[0]))),
                  "bias": f32(rng.normal(0.0, 0.02, channels))}
    return net
