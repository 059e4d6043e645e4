"""FP64 CPU oracle of the BM3D stage -- TEST INFRASTRUCTURE ONLY.

Only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never touches it.

The computation lives in plain C (``bm3d_oracle.c``, FP64); this module
compiles it with gcc when needed and wraps it with numpy-facing functions.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bm3d_oracle.c")
_LIB = os.path.join(_HERE, "_bm3d_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle (gcc -O2, OpenMP, no hand-written SIMD)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        vp = ctypes.c_void_p
        ci, cd = ctypes.c_int, ctypes.c_double
        L.orc_ref_positions.argtypes = [ci, vp]
        L.orc_ref_positions.restype = ci
        L.orc_dct_matrix.argtypes = [f64p]
        L.orc_hadamard.argtypes = [ci, f64p]
        L.orc_kaiser.argtypes = [cd, f64p]
        L.orc_opponent.argtypes = [f64p]
        L.orc_transform3d.argtypes = [f64p, ci, f64p, ci]
        L.orc_transform3d_ex.argtypes = [f64p, ci, f64p, ci, ci]
        L.orc_bior15_filters.argtypes = [f64p]
        L.orc_bior15_matrix.argtypes = [f64p, f64p]
        L.orc_match_prefiltered.argtypes = [u8p, ci, ci, ci, ci, cd, cd, ci, i32p, i32p]
        L.orc_prepare.argtypes = [u8p, ci, ci, ci, f64p, u8p]
        L.orc_match_u8.argtypes = [u8p, ci, ci, ci, ci, cd, i32p, i32p]
        L.orc_match_f64.argtypes = [f64p, ci, ci, ci, ci, cd, i32p, i32p]
        L.orc_filter.argtypes = [f64p, vp, ci, ci, ci, cd, ci, i32p, i32p, ci,
                                 vp, f64p, f64p, vp, vp]
        L.orc_aggregate.argtypes = [f64p, f64p, ci, ci, ci, ci, f64p]
        L.orc_luminance_f64.argtypes = [f64p, ci, ci, ci, f64p]
        L.orc_denoise.argtypes = [u8p, ci, ci, ci, cd, vp, f64p, vp, vp, vp, vp, vp]
        L.orc_denoise.restype = ci
        L.orc_set_threads.argtypes = [ci]
        L.orc_get_threads.restype = ci
        _lib = L
    return _lib


class _CParams(ctypes.Structure):
    _fields_ = [("search_ht", ctypes.c_int), ("search_wie", ctypes.c_int),
                ("n_ht", ctypes.c_int), ("n_wie", ctypes.c_int),
                ("lambda_ht", ctypes.c_double), ("tau_ht", ctypes.c_double),
                ("tau_wie", ctypes.c_double), ("kaiser_beta", ctypes.c_double),
                ("transform_ht", ctypes.c_int), ("lambda_2d", ctypes.c_double)]


T_DCT, T_BIOR15 = 0, 1  # step-1 2-D transforms


@dataclass
class Params:
    """Parameters of the two-step method.  tau_* are per-pixel-normalised
    squared-distance thresholds (a candidate passes if SSD <= 64*tau)."""
    search_ht: int = 32
    search_wie: int = 32
    n_ht: int = 16
    n_wie: int = 32
    lambda_ht: float = 2.7
    tau_ht: float = 2500.0
    tau_wie: float = 400.0
    kaiser_beta: float = 2.0
    transform_ht: int = 0     # step-1 2-D transform: T_DCT or T_BIOR15
    lambda_2d: float = 0.0    # > 0: prefiltered step-1 matching (high-noise profile)

    @staticmethod
    def for_sigma(sigma: float, search: int = 32) -> "Params":
        """sigma-dependent distance thresholds (low/high noise profile)."""
        if sigma > 40.0:
            return Params(search, search, 16, 32, 2.7, 5000.0, 3500.0, 2.0)
        return Params(search, search, 16, 32, 2.7, 2500.0, 400.0, 2.0)

    def _c(self):
        return _CParams(self.search_ht, self.search_wie, self.n_ht, self.n_wie,
                        self.lambda_ht, self.tau_ht, self.tau_wie, self.kaiser_beta,
                        self.transform_ht, self.lambda_2d)


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return lib().orc_get_threads()


def ref_positions(length: int) -> np.ndarray:
    n = lib().orc_ref_positions(length, None)
    out = np.zeros(n, np.int32)
    lib().orc_ref_positions(length, out.ctypes.data)
    return out


def num_refs(h: int, w: int) -> int:
    return len(ref_positions(h)) * len(ref_positions(w))


def dct_matrix() -> np.ndarray:
    c = np.zeros(64)
    lib().orc_dct_matrix(c)
    return c.reshape(8, 8)


def hadamard(n: int) -> np.ndarray:
    h = np.zeros(n * n)
    lib().orc_hadamard(n, h)
    return h.reshape(n, n)


def kaiser(beta: float = 2.0) -> np.ndarray:
    k = np.zeros(8)
    lib().orc_kaiser(beta, k)
    return k


def opponent() -> np.ndarray:
    t = np.zeros(9)
    lib().orc_opponent(t)
    return t.reshape(3, 3)


def transform3d(group: np.ndarray, inverse: bool = False, transform: int = T_DCT) -> np.ndarray:
    g = np.ascontiguousarray(group, np.float64)
    n = g.shape[0]
    s = np.zeros_like(g)
    lib().orc_transform3d_ex(g.reshape(-1), n, s.reshape(-1), 1 if inverse else 0, int(transform))
    return s


def bior15_filters() -> np.ndarray:
    """bior1.5 analysis lowpass taps at offsets -4..5."""
    lo = np.zeros(10)
    lib().orc_bior15_filters(lo)
    return lo


def bior15_matrix():
    """(F, I): the 8-point bior1.5 forward matrix F[a, u] (unit-norm rows)
    and its inverse I[u, a]."""
    f, i = np.zeros(64), np.zeros(64)
    lib().orc_bior15_matrix(f, i)
    return f.reshape(8, 8), i.reshape(8, 8)


def match_prefiltered(lum, search: int, nmax: int, tau: float, thr2d: float, transform: int = T_DCT):
    """Step-1 grouping on 2-D spectra hard-thresholded at thr2d."""
    lum = np.ascontiguousarray(lum, np.uint8)
    h, w = lum.shape
    R = num_refs(h, w)
    idx = np.zeros((R, nmax), np.int32)
    cnt = np.zeros(R, np.int32)
    lib().orc_match_prefiltered(lum.reshape(-1), h, w, search, nmax, tau, thr2d, int(transform),
                                idx.reshape(-1), cnt)
    return idx, cnt


def _img_hwc(img):
    a = np.ascontiguousarray(img, np.uint8)
    if a.ndim == 2:
        return a, a.shape[0], a.shape[1], 1
    return a, a.shape[0], a.shape[1], a.shape[2]


def prepare(img):
    a, h, w, c = _img_hwc(img)
    planar = np.zeros((c, h, w))
    lum = np.zeros((h, w), np.uint8)
    lib().orc_prepare(a.reshape(-1), h, w, c, planar.reshape(-1), lum.reshape(-1))
    return planar, lum


def match_u8(lum, search: int, nmax: int, tau: float):
    lum = np.ascontiguousarray(lum, np.uint8)
    h, w = lum.shape
    R = num_refs(h, w)
    idx = np.zeros((R, nmax), np.int32)
    cnt = np.zeros(R, np.int32)
    lib().orc_match_u8(lum.reshape(-1), h, w, search, nmax, tau, idx.reshape(-1), cnt)
    return idx, cnt


def match_f64(lum, search: int, nmax: int, tau: float):
    lum = np.ascontiguousarray(lum, np.float64)
    h, w = lum.shape
    R = num_refs(h, w)
    idx = np.zeros((R, nmax), np.int32)
    cnt = np.zeros(R, np.int32)
    lib().orc_match_f64(lum.reshape(-1), h, w, search, nmax, tau, idx.reshape(-1), cnt)
    return idx, cnt


def collab_filter(noisy_planar, basic_planar, sigma: float, step: int, idx, cnt,
                  params: Params, want_margin: bool = False):
    """Returns (num, den[, margin, nkept]) with num/den planar [c,h,w] (fresh,
    not +=); with want_margin also the per-reference distance of the closest
    coefficient to the hard threshold and N_kept per [channel, reference]."""
    noisy = np.ascontiguousarray(noisy_planar, np.float64)
    c, h, w = noisy.shape
    basic = None if basic_planar is None else np.ascontiguousarray(basic_planar, np.float64)
    idx = np.ascontiguousarray(idx, np.int32)
    cnt = np.ascontiguousarray(cnt, np.int32)
    num = np.zeros((c, h, w))
    den = np.zeros((c, h, w))
    margin = np.zeros(len(cnt)) if want_margin else None
    nkept = np.zeros((c, len(cnt)), np.int32) if want_margin else None
    cp = params._c()
    lib().orc_filter(noisy.reshape(-1), None if basic is None else basic.ctypes.data,
                     h, w, c, sigma, step, idx.reshape(-1), cnt, idx.shape[1],
                     ctypes.addressof(cp), num.reshape(-1), den.reshape(-1),
                     None if margin is None else margin.ctypes.data,
                     None if nkept is None else nkept.ctypes.data)
    return (num, den, margin, nkept) if want_margin else (num, den)


def aggregate(num, den, final_step: bool):
    num = np.ascontiguousarray(num, np.float64)
    den = np.ascontiguousarray(den, np.float64)
    c, h, w = num.shape
    out = np.zeros((h, w, c) if (final_step and c == 3) else (c, h, w))
    lib().orc_aggregate(num.reshape(-1), den.reshape(-1), h, w, c, 1 if final_step else 0,
                        out.reshape(-1))
    return out


def luminance(basic_planar):
    b = np.ascontiguousarray(basic_planar, np.float64)
    c, h, w = b.shape
    out = np.zeros((h, w))
    lib().orc_luminance_f64(b.reshape(-1), h, w, c, out.reshape(-1))
    return out


def denoise(img, sigma: float, params: Params | None = None, want_intermediates: bool = False):
    """Full two-step denoiser.  Returns the FP64 estimate, HxW (grey) or HxWx3,
    on the [0,255] scale, unclipped."""
    a, h, w, c = _img_hwc(img)
    p = params or Params.for_sigma(sigma)
    out = np.zeros((h, w) if c == 1 else (h, w, 3))
    R = num_refs(h, w)
    basic = np.zeros((c, h, w))
    i1 = np.zeros((R, p.n_ht), np.int32)
    c1 = np.zeros(R, np.int32)
    i2 = np.zeros((R, p.n_wie), np.int32)
    c2 = np.zeros(R, np.int32)
    cp = p._c()
    rc = lib().orc_denoise(a.reshape(-1), h, w, c, float(sigma), ctypes.addressof(cp),
                           out.reshape(-1), basic.ctypes.data, i1.ctypes.data, c1.ctypes.data,
                           i2.ctypes.data, c2.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the input")
    if want_intermediates:
        return out, dict(basic=basic, idx1=i1, cnt1=c1, idx2=i2, cnt2=c2)
    return out
