"""Python binding of the C ABI in include/bm3d.h (ctypes).

Argument marshalling only: every step of the denoiser runs in the HIP
library (libbm3d_mi355x.so, built from csrc/).  Device memory and streams
come from PyTorch (ROCm); tensors are passed as raw device pointers.  There
is no fallback: importing this module fails if the library is not built.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbm3d_mi355x.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("HIP library %s is not built (run __graft_entry__.build())" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

XF_FP32, XF_BF16, XF_FP16 = 0, 1, 2
T_DCT, T_BIOR15 = 0, 1  # step-1 2-D transforms
FLAG_DEBUG_SYNC = 1
FLAG_SIGMA_PROFILE = 2
FLAG_DEBUG_NKEPT = 4
STAGES = ("prep", "match1", "filter1", "agg1", "match2", "filter2", "agg2")
# working buffers of a workspace / batched plan (bm3d_buffer), with their
# element types; num and wsum are fixed point with NUM_FRAC_BITS / WSUM_FRAC_BITS
# fractional bits
BUFFERS = ("planar", "lum8", "lumf", "basic", "num", "wsum", "idx1", "cnt1", "idx2", "cnt2", "nkept", "coef")
BUFFER_DTYPES = ("float32", "uint8", "float32", "float32", "int64", "int64", "int32", "int32", "int32", "int32",
                 "int32", "float32")
NUM_FRAC_BITS, WSUM_FRAC_BITS = 28, 40


class Params(ctypes.Structure):
    _fields_ = [("search_ht", ctypes.c_int), ("search_wie", ctypes.c_int),
                ("n_ht", ctypes.c_int), ("n_wie", ctypes.c_int),
                ("lambda_ht", ctypes.c_float), ("tau_ht", ctypes.c_float),
                ("tau_wie", ctypes.c_float), ("kaiser_beta", ctypes.c_float),
                ("xform", ctypes.c_int), ("tile_refs", ctypes.c_int),
                ("persistent_wgs", ctypes.c_int), ("flags", ctypes.c_uint),
                ("debug_nkept", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("lambda_2d", ctypes.c_float), ("transform_ht", ctypes.c_int),
                ("match_refs", ctypes.c_int)]

    def copy(self) -> "Params":
        q = Params()
        ctypes.pointer(q)[0] = self
        return q


class NlmParams(ctypes.Structure):
    _fields_ = [("patch_radius", ctypes.c_int), ("search_radius", ctypes.c_int), ("h", ctypes.c_float)]


class CnnLayer(ctypes.Structure):
    _fields_ = [("weight", ctypes.c_void_p), ("bias", ctypes.c_void_p), ("bn_gamma", ctypes.c_void_p),
                ("bn_beta", ctypes.c_void_p), ("bn_mean", ctypes.c_void_p), ("bn_var", ctypes.c_void_p),
                ("bn_eps", ctypes.c_float)]


class DsBlock(ctypes.Structure):
    _fields_ = ([(k, ctypes.c_void_p) for k in ("dw", "dw_bias", "dw_gamma", "dw_beta", "dw_mean", "dw_var")]
                + [("dw_eps", ctypes.c_float)]
                + [(k, ctypes.c_void_p) for k in ("pw", "pw_bias", "pw_gamma", "pw_beta", "pw_mean", "pw_var")]
                + [("pw_eps", ctypes.c_float)])


class UnetWeights(ctypes.Structure):
    _fields_ = [("enc", DsBlock * 4), ("down", DsBlock * 4), ("dec", DsBlock * 4),
                ("up_weight", ctypes.c_void_p * 4), ("up_bias", ctypes.c_void_p * 4),
                ("out_weight", ctypes.c_void_p), ("out_bias", ctypes.c_void_p)]


class GatParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("sigma", ctypes.c_float), ("mu", ctypes.c_float),
                ("scale", ctypes.c_float), ("offset", ctypes.c_float)]


class ImageDesc(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("out", ctypes.c_void_p), ("h", ctypes.c_int),
                ("w", ctypes.c_int), ("c", ctypes.c_int), ("sigma", ctypes.c_float)]


class Request(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("out", ctypes.c_void_p), ("h", ctypes.c_int),
                ("w", ctypes.c_int), ("c", ctypes.c_int), ("sigma", ctypes.c_float),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("stage", ctypes.c_int)]


_vp, _i, _f, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_size_t
_PP = ctypes.POINTER(Params)
_SIGS = {
    "bm3d_params_default": (_i, [_f, _PP]),
    "bm3d_num_refs": (_i, [_i, _i]),
    "bm3d_workspace_size": (_sz, [_i, _i, _i, _PP]),
    "bm3d_workspace_buffer": (_i, [_i, _i, _i, _PP, _i, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "bm3d_prepare": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "bm3d_block_match": (_i, [_vp, _i, _i, _i, _i, _PP, _vp, _vp, _vp]),
    "bm3d_collab_filter": (_i, [_vp, _vp, _i, _i, _i, _f, _i, _vp, _vp, _PP, _vp, _vp, _vp]),
    "bm3d_aggregate": (_i, [_vp, _vp, _i, _i, _i, _i, _PP, _vp, _vp]),
    "bm3d_luminance": (_i, [_vp, _i, _i, _i, _vp, _vp]),
    "bm3d_denoise": (_i, [_vp, _i, _i, _i, _f, _PP, _vp, _vp]),
    "bm3d_denoise_noalloc": (_i, [_vp, _i, _i, _i, _f, _PP, _vp, _vp]),
    "bm3d_nlm_params_default": (_i, [_f, _i, ctypes.POINTER(NlmParams)]),
    "bm3d_nlm": (_i, [_vp, _i, _i, _i, _f, ctypes.POINTER(NlmParams), _vp, _vp]),
    "bm3d_nlm_batch": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i, _i, _i, _i, _f,
                            ctypes.POINTER(NlmParams), _vp]),
    "bm3d_cnn_create": (_i, [_i, _i, _i, ctypes.POINTER(CnnLayer), ctypes.POINTER(_vp)]),
    "bm3d_cnn_destroy": (_i, [_vp]),
    "bm3d_cnn_workspace_bytes": (_i, [_i, _i, _i, ctypes.POINTER(_sz)]),
    "bm3d_cnn_restore": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i, _i, _i,
                              _vp, _sz, _vp]),
    "bm3d_cnn_run_layers": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i, _i, _i,
                                 _vp, _sz, _i, _i, _vp]),
    "bm3d_unet_create": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(UnetWeights), ctypes.POINTER(_vp)]),
    "bm3d_unet_destroy": (_i, [_vp]),
    "bm3d_unet_workspace_bytes": (_i, [_vp, _i, _i, _i, ctypes.POINTER(_sz)]),
    "bm3d_unet_restore": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i, _i, _i,
                               _f, _vp, _sz, _vp]),
    "bm3d_gat_forward": (_i, [_vp, ctypes.c_longlong, ctypes.POINTER(GatParams), _vp, _vp]),
    "bm3d_gat_inverse": (_i, [_vp, ctypes.c_longlong, ctypes.POINTER(GatParams), _vp, _vp]),
    "bm3d_gat_noise_level": (_f, [_f]),
    "bm3d_vst_denoise": (_i, [_vp, _i, _i, _i, ctypes.POINTER(GatParams), _PP, _vp, _vp, _vp]),
    "bm3d_batch_create": (_i, [ctypes.POINTER(ImageDesc), _i, _PP, ctypes.POINTER(_vp)]),
    "bm3d_batch_device_bytes": (_sz, [_vp]),
    "bm3d_batch_copy_buffer": (_i, [_vp, _i, _i, _vp, _sz, _i, _vp]),
    "bm3d_batch_set_io": (_i, [_vp, _i, _vp, _vp, _vp]),
    "bm3d_batch_run": (_i, [_vp, _vp]),
    "bm3d_batch_capture": (_i, [_vp, _vp]),
    "bm3d_batch_launch": (_i, [_vp, _vp]),
    "bm3d_batch_run_stages": (_i, [_vp, _i, _i, _i, _i, _vp]),
    "bm3d_batch_destroy": (_i, [_vp]),
    "bm3d_autotune": (_i, [_PP, ctypes.c_char_p]),
    "bm3d_server_create": (_i, [_i, _PP, ctypes.POINTER(_vp)]),
    "bm3d_server_tick": (_i, [_vp, ctypes.POINTER(Request), _i, _vp]),
    "bm3d_server_destroy": (_i, [_vp]),
    "bm3d_strerror": (ctypes.c_char_p, [_i]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class BM3DError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, _lib.bm3d_strerror(status).decode(), status))


def _check(status: int, where: str):
    if status != 0:
        raise BM3DError(status, where)


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _ptr(t, dtype=None, name="tensor", numel=None, exact=False):
    """Device pointer of a contiguous tensor of the given dtype; with numel,
    the tensor must hold at least (exact: exactly) that many elements, so a
    kernel never writes past a caller's buffer."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and (t.numel() != numel if exact else t.numel() < numel):
        raise ValueError("%s must have %s%d elements, got %d" % (name, "" if exact else "at least ", numel,
                                                                 t.numel()))
    return t.data_ptr()


def _hwc(img, name="img"):
    if img.dim() == 2:
        return img.shape[0], img.shape[1], 1
    if img.dim() == 3 and img.shape[2] in (1, 3):
        return img.shape[0], img.shape[1], img.shape[2]
    raise ValueError("%s must be [h,w] or [h,w,c] with c in (1, 3), got %s" % (name, tuple(img.shape)))


def params_default(sigma: float, **overrides) -> Params:
    p = Params()
    _check(_lib.bm3d_params_default(float(sigma), ctypes.byref(p)), "bm3d_params_default")
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def num_refs(h: int, w: int) -> int:
    return _lib.bm3d_num_refs(h, w)


def workspace_size(h: int, w: int, c: int, p: Params) -> int:
    return _lib.bm3d_workspace_size(h, w, c, ctypes.byref(p))


def workspace_buffer(h: int, w: int, c: int, p: Params, buffer: str):
    """(byte offset, bytes) of a working buffer inside bm3d_denoise's workspace."""
    off, nb = _sz(), _sz()
    _check(_lib.bm3d_workspace_buffer(h, w, c, ctypes.byref(p), BUFFERS.index(buffer), ctypes.byref(off),
                                      ctypes.byref(nb)), "bm3d_workspace_buffer")
    return off.value, nb.value


def workspace_view(workspace, h: int, w: int, c: int, p: Params, buffer: str):
    """A typed view (1-D tensor) of one working buffer inside a device
    workspace tensor, e.g. the step-1 groups after bm3d_denoise."""
    torch = _torch()
    off, nb = workspace_buffer(h, w, c, p, buffer)
    if off + nb > workspace.numel():
        raise ValueError("workspace too small for %s" % buffer)
    return workspace[off:off + nb].view(getattr(torch, BUFFER_DTYPES[BUFFERS.index(buffer)]))


def strerror(status: int) -> str:
    return _lib.bm3d_strerror(status).decode()


# ------------------------------------------------------------ stage calls ---

def prepare(img, planar, lum, stream=None):
    """img: uint8 [h,w] or [h,w,3]; planar: float32 [c,h,w]; lum: uint8 [h,w]."""
    torch = _torch()
    h, w, c = _hwc(img)
    _check(_lib.bm3d_prepare(_ptr(img, torch.uint8, "img"), h, w, c,
                             _ptr(planar, torch.float32, "planar", c * h * w, True),
                             _ptr(lum, torch.uint8, "lum", h * w, True), _stream(stream)), "bm3d_prepare")


def block_match(src, step: int, p: Params, idx, cnt, stream=None):
    torch = _torch()
    if src.dim() != 2:
        raise ValueError("src must be a [h,w] luminance")
    h, w = src.shape
    is_f32 = 1 if src.dtype == torch.float32 else 0
    R = num_refs(h, w)
    nmax = p.n_ht if step == 1 else p.n_wie
    _check(_lib.bm3d_block_match(_ptr(src, torch.float32 if is_f32 else torch.uint8, "src"), is_f32, h, w, step,
                                 ctypes.byref(p), _ptr(idx, torch.int32, "idx", R * nmax),
                                 _ptr(cnt, torch.int32, "cnt", R), _stream(stream)), "bm3d_block_match")


def collab_filter(noisy, basic, sigma: float, step: int, idx, cnt, p: Params, num, wsum,
                  stream=None):
    """num/wsum: int64 fixed-point accumulators [c,h,w] (added into)."""
    torch = _torch()
    c, h, w = noisy.shape
    R = num_refs(h, w)
    nmax = p.n_ht if step == 1 else p.n_wie
    _check(_lib.bm3d_collab_filter(_ptr(noisy, torch.float32, "noisy"),
                                   _ptr(basic, torch.float32, "basic", c * h * w, True), h, w, c, float(sigma),
                                   step, _ptr(idx, torch.int32, "idx", R * nmax),
                                   _ptr(cnt, torch.int32, "cnt", R), ctypes.byref(p),
                                   _ptr(num, torch.int64, "num", c * h * w, True),
                                   _ptr(wsum, torch.int64, "wsum", c * h * w, True), _stream(stream)),
           "bm3d_collab_filter")


def aggregate(num, wsum, final_step: bool, p: Params, out, stream=None):
    torch = _torch()
    c, h, w = num.shape
    _check(_lib.bm3d_aggregate(_ptr(num, torch.int64, "num"), _ptr(wsum, torch.int64, "wsum", c * h * w, True),
                               h, w, c, 1 if final_step else 0, ctypes.byref(p),
                               _ptr(out, torch.float32, "out", c * h * w, True), _stream(stream)),
           "bm3d_aggregate")


def from_fix(t, buffer: str):
    """Real values (float64) of a fixed-point accumulator tensor ("num" or "wsum")."""
    return t.double() * 2.0 ** -(NUM_FRAC_BITS if buffer == "num" else WSUM_FRAC_BITS)


def luminance(basic, lum, stream=None):
    torch = _torch()
    c, h, w = basic.shape
    _check(_lib.bm3d_luminance(_ptr(basic, torch.float32, "basic"), h, w, c,
                               _ptr(lum, torch.float32, "lum", h * w, True), _stream(stream)), "bm3d_luminance")


def denoise(img, sigma: float, p: Params | None = None, out=None, workspace=None, stream=None):
    """Two-step denoiser on one device image (uint8 [h,w] or [h,w,3]).
    Returns a float32 device tensor of the same shape on the [0,255] scale.
    A workspace tensor passed in holds the working buffers afterwards
    (workspace_view)."""
    torch = _torch()
    h, w, c = _hwc(img)
    p = (p or params_default(sigma)).copy()
    need = workspace_size(h, w, c, p)
    if need == 0:
        raise BM3DError(-1, "bm3d_workspace_size")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=img.device)
    p.workspace = _ptr(workspace, torch.uint8, "workspace")
    p.workspace_bytes = workspace.numel()
    if out is None:
        out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
    _check(_lib.bm3d_denoise(_ptr(img, torch.uint8, "img"), h, w, c, float(sigma),
                             ctypes.byref(p), _ptr(out, torch.float32, "out", h * w * c, True), _stream(stream)),
           "bm3d_denoise")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def denoise_noalloc(img, sigma: float, p: Params | None = None, out=None, stream=None):
    """bm3d_denoise_noalloc: the two-step denoiser with the library's static
    device scratch as workspace (no allocation by the library; calls on one
    GPU must not overlap).  `out` must be given by callers that cannot
    allocate; otherwise a float32 tensor is made here."""
    torch = _torch()
    h, w, c = _hwc(img)
    p = p or params_default(sigma)
    if out is None:
        out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
    _check(_lib.bm3d_denoise_noalloc(_ptr(img, torch.uint8, "img"), h, w, c, float(sigma), ctypes.byref(p),
                                     _ptr(out, torch.float32, "out", h * w * c, True), _stream(stream)),
           "bm3d_denoise_noalloc")
    return out


def nlm_params_default(sigma: float, c: int = 1) -> NlmParams:
    p = NlmParams()
    _check(_lib.bm3d_nlm_params_default(float(sigma), int(c), ctypes.byref(p)), "bm3d_nlm_params_default")
    return p


def nlm(img, sigma: float, p: NlmParams | None = None, out=None, stream=None):
    """NL-means of one device image (uint8 [h,w] or [h,w,3]).  Returns a
    float32 device tensor of the same shape on the [0,255] scale."""
    torch = _torch()
    h, w = img.shape[0], img.shape[1]
    c = 1 if img.dim() == 2 else img.shape[2]
    p = p or nlm_params_default(sigma, c)
    if out is None:
        out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
    _check(_lib.bm3d_nlm(_ptr(img, torch.uint8, "img"), h, w, c, float(sigma), ctypes.byref(p),
                         _ptr(out, torch.float32, "out"), _stream(stream)), "bm3d_nlm")
    return out


def nlm_batch(imgs, sigma: float, p: NlmParams | None = None, outs=None, stream=None):
    """NL-means of up to 64 device images of one shape in one launch.
    Returns the list of float32 outputs."""
    torch = _torch()
    n = len(imgs)
    h, w = imgs[0].shape[0], imgs[0].shape[1]
    c = 1 if imgs[0].dim() == 2 else imgs[0].shape[2]
    p = p or nlm_params_default(sigma, c)
    if outs is None:
        outs = [torch.empty(imgs[0].shape, dtype=torch.float32, device=imgs[0].device) for _ in range(n)]
    for t in imgs:
        if tuple(t.shape) != tuple(imgs[0].shape):
            raise ValueError("nlm_batch: images must share one shape")
    ia = (_vp * n)(*[_ptr(t, torch.uint8, "img") for t in imgs])
    oa = (_vp * n)(*[_ptr(t, torch.float32, "out") for t in outs])
    _check(_lib.bm3d_nlm_batch(ia, oa, n, h, w, c, float(sigma), ctypes.byref(p), _stream(stream)),
           "bm3d_nlm_batch")
    return outs


# ------------------------------------------------------ residual network ---

class Cnn:
    """The residual network of bm3d_cnn_create: ``layers`` is a list of K
    dicts of host arrays (weight [cout][cin][3][3], optional bias and
    gamma/beta/mean/var/eps of batch normalisation).  Weights are copied to
    the current device at construction."""

    def __init__(self, layers, c: int, features: int = 64):
        self.c, self.K = int(c), len(layers)
        keep = []

        def arr(a):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float32)
            keep.append(a)
            return a.ctypes.data

        descs = (CnnLayer * self.K)()
        for k, L in enumerate(layers):
            bn = L.get("gamma") is not None
            descs[k] = CnnLayer(arr(L["weight"]), arr(L.get("bias")), arr(L.get("gamma")), arr(L.get("beta")),
                                arr(L.get("mean")), arr(L.get("var")), float(L.get("eps", 0.0)) if bn else 0.0)
        h = ctypes.c_void_p()
        _check(_lib.bm3d_cnn_create(self.K, self.c, int(features), descs, ctypes.byref(h)), "bm3d_cnn_create")
        self._h = h
        self._ws = None

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.bm3d_cnn_destroy(self._h)
            self._h = None

    @staticmethod
    def workspace_bytes(n: int, h: int, w: int) -> int:
        b = _sz()
        _check(_lib.bm3d_cnn_workspace_bytes(int(n), int(h), int(w), ctypes.byref(b)), "bm3d_cnn_workspace_bytes")
        return b.value

    def restore(self, basics, noisys, outs=None, workspace=None, stream=None, layers=None):
        """x_hat = basic + 255 F(basic, noisy) for up to 64 device images of
        one shape (basic float32, noisy uint8, [h,w] or [h,w,c]).  Returns
        the list of float32 outputs.  ``layers=(first, last)`` runs only
        that range (bm3d_cnn_run_layers)."""
        torch = _torch()
        n = len(basics)
        if n != len(noisys):
            raise ValueError("restore: as many first-stage estimates as observations")
        shape = tuple(basics[0].shape)
        for t in list(basics) + list(noisys):
            if tuple(t.shape) != shape:
                raise ValueError("restore: images must share one shape")
        c = 1 if len(shape) == 2 else shape[2]
        if c != self.c:
            raise ValueError("restore: the network was built for %d channels" % self.c)
        h, w = shape[0], shape[1]
        if outs is None:
            outs = [torch.empty(shape, dtype=torch.float32, device=basics[0].device) for _ in range(n)]
        need = self.workspace_bytes(n, h, w)
        if workspace is None:
            if self._ws is None or self._ws.numel() < need:
                self._ws = torch.empty(need, dtype=torch.uint8, device=basics[0].device)
            workspace = self._ws
        ba = (_vp * n)(*[_ptr(t, torch.float32, "basic") for t in basics])
        na = (_vp * n)(*[_ptr(t, torch.uint8, "noisy") for t in noisys])
        oa = (_vp * n)(*[_ptr(t, torch.float32, "out") for t in outs])
        ws = _ptr(workspace, torch.uint8, "workspace")
        if layers is None:
            _check(_lib.bm3d_cnn_restore(self._h, ba, na, oa, n, h, w, ws, workspace.numel(), _stream(stream)),
                   "bm3d_cnn_restore")
        else:
            _check(_lib.bm3d_cnn_run_layers(self._h, ba, na, oa, n, h, w, ws, workspace.numel(), int(layers[0]),
                                            int(layers[1]), _stream(stream)), "bm3d_cnn_run_layers")
        return outs


def _images(basics, noisys, c, what):
    n = len(basics)
    if n != len(noisys):
        raise ValueError("%s: as many first-stage estimates as observations" % what)
    shape = tuple(basics[0].shape)
    for t in list(basics) + list(noisys):
        if tuple(t.shape) != shape:
            raise ValueError("%s: images must share one shape" % what)
    if (1 if len(shape) == 2 else shape[2]) != c:
        raise ValueError("%s: the network was built for %d channels" % (what, c))
    return n, shape


class Unet:
    """The flexible U-Net of bm3d_unet_create.  ``net`` is a dict of host
    arrays: enc / down / dec lists of 4 depthwise separable blocks (keys dw,
    dw_bias, pw, pw_bias and optional [dw_|pw_]gamma/beta/mean/var/eps),
    up (4 dicts of weight [w_{i+1}][w_i][2][2] and bias) and out (weight
    [C][w_0], bias)."""

    def __init__(self, net, c: int, widths=None):
        self.c = int(c)
        keep = []

        def arr(a):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float32)
            keep.append(a)
            return a.ctypes.data

        def block(L):
            b = DsBlock()
            for pre in ("dw", "pw"):
                setattr(b, pre, arr(L[pre]))
                for k in ("bias", "gamma", "beta", "mean", "var"):
                    setattr(b, pre + "_" + k, arr(L.get(pre + "_" + k)))
                setattr(b, pre + "_eps", float(L.get(pre + "_eps", 0.0)))
            return b

        w = UnetWeights()
        for i in range(4):
            w.enc[i] = block(net["enc"][i])
            w.down[i] = block(net["down"][i])
            w.dec[i] = block(net["dec"][i])
            w.up_weight[i] = arr(net["up"][i]["weight"])
            w.up_bias[i] = arr(net["up"][i].get("bias"))
        w.out_weight = arr(net["out"]["weight"])
        w.out_bias = arr(net["out"].get("bias"))
        wa = None if widths is None else (_i * 5)(*[int(x) for x in widths])
        h = ctypes.c_void_p()
        _check(_lib.bm3d_unet_create(self.c, wa, ctypes.byref(w), ctypes.byref(h)), "bm3d_unet_create")
        self._h = h
        self._ws = None

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.bm3d_unet_destroy(self._h)
            self._h = None

    def workspace_bytes(self, n: int, h: int, w: int) -> int:
        b = _sz()
        _check(_lib.bm3d_unet_workspace_bytes(self._h, int(n), int(h), int(w), ctypes.byref(b)),
               "bm3d_unet_workspace_bytes")
        return b.value

    def restore(self, basics, noisys, sigma: float, outs=None, workspace=None, stream=None):
        """x_hat = basic + 255 F(basic, noisy, sigma) for up to 64 device
        images of one shape.  Returns the list of float32 outputs."""
        torch = _torch()
        n, shape = _images(basics, noisys, self.c, "restore")
        h, w = shape[0], shape[1]
        if outs is None:
            outs = [torch.empty(shape, dtype=torch.float32, device=basics[0].device) for _ in range(n)]
        need = self.workspace_bytes(n, h, w)
        if workspace is None:
            if self._ws is None or self._ws.numel() < need:
                self._ws = torch.empty(need, dtype=torch.uint8, device=basics[0].device)
            workspace = self._ws
        ba = (_vp * n)(*[_ptr(t, torch.float32, "basic") for t in basics])
        na = (_vp * n)(*[_ptr(t, torch.uint8, "noisy") for t in noisys])
        oa = (_vp * n)(*[_ptr(t, torch.float32, "out") for t in outs])
        _check(_lib.bm3d_unet_restore(self._h, ba, na, oa, n, h, w, float(sigma),
                                      _ptr(workspace, torch.uint8, "workspace"), workspace.numel(),
                                      _stream(stream)), "bm3d_unet_restore")
        return outs


# ------------------------------------------------ variance stabilisation ---

def gat_noise_level(scale: float) -> float:
    return float(_lib.bm3d_gat_noise_level(float(scale)))


def gat_forward(raw, g: GatParams, out=None, stream=None):
    """8-bit stabilised code of a device float tensor (any shape)."""
    torch = _torch()
    if out is None:
        out = torch.empty(raw.shape, dtype=torch.uint8, device=raw.device)
    if out.numel() != raw.numel():
        raise ValueError("gat_forward: out must have raw's size")
    _check(_lib.bm3d_gat_forward(_ptr(raw, torch.float32, "raw"), raw.numel(), ctypes.byref(g),
                                 _ptr(out, torch.uint8, "out"), _stream(stream)), "bm3d_gat_forward")
    return out


def gat_inverse(stab, g: GatParams, out=None, stream=None):
    """Unbiased inverse of a denoised 8-bit-scale device float tensor."""
    torch = _torch()
    if out is None:
        out = torch.empty(stab.shape, dtype=torch.float32, device=stab.device)
    if out.numel() != stab.numel():
        raise ValueError("gat_inverse: out must have stab's size")
    _check(_lib.bm3d_gat_inverse(_ptr(stab, torch.float32, "stab"), stab.numel(), ctypes.byref(g),
                                 _ptr(out, torch.float32, "out"), _stream(stream)), "bm3d_gat_inverse")
    return out


def vst_denoise(raw, g: GatParams, p: Params | None = None, out=None, stab=None, workspace=None, stream=None):
    """x_hat of a raw Poisson-Gaussian device image (float [h,w] or
    [h,w,3]): stabilise, BM3D at the 8-bit noise level, unbiased inverse."""
    torch = _torch()
    h, w, c = _hwc(raw, "raw")
    p = (p or params_default(gat_noise_level(g.scale))).copy()
    need = workspace_size(h, w, c, p)
    if need == 0:
        raise BM3DError(-1, "bm3d_workspace_size")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=raw.device)
    p.workspace = workspace.data_ptr()
    p.workspace_bytes = workspace.numel()
    if out is None:
        out = torch.empty(raw.shape, dtype=torch.float32, device=raw.device)
    if stab is None:
        stab = torch.empty(raw.shape, dtype=torch.uint8, device=raw.device)
    _check(_lib.bm3d_vst_denoise(_ptr(raw, torch.float32, "raw"), h, w, c, ctypes.byref(g), ctypes.byref(p),
                                 _ptr(stab, torch.uint8, "stab", h * w * c, True),
                                 _ptr(out, torch.float32, "out", h * w * c, True), _stream(stream)),
           "bm3d_vst_denoise")
    return out


def autotune(p: Params, cache_path: str | None = None) -> Params:
    q = p.copy()
    _check(_lib.bm3d_autotune(ctypes.byref(q), cache_path.encode() if cache_path else None),
           "bm3d_autotune")
    return q


# ---------------------------------------------------------------- batches ---

class Batch:
    """A batched plan over many images of different shapes (bm3d_batch_*)."""

    def __init__(self, images, outs, sigmas, p: Params):
        torch = _torch()
        self.n = len(images)
        self.p = p.copy()
        arr = (ImageDesc * self.n)()
        self.shapes = []
        for i, (im, o, s) in enumerate(zip(images, outs, sigmas)):
            h, w, c = _hwc(im)
            arr[i] = ImageDesc(_ptr(im, torch.uint8, "img"), _ptr(o, torch.float32, "out", h * w * c, True), h, w,
                               c, float(s))
            self.shapes.append((h, w, c))
        # the plan reads and writes these until it is closed or re-bound
        self._keep = [[im, o] for im, o in zip(images, outs)]
        self._h = ctypes.c_void_p()
        _check(_lib.bm3d_batch_create(arr, self.n, ctypes.byref(p), ctypes.byref(self._h)),
               "bm3d_batch_create")

    @property
    def device_bytes(self) -> int:
        return _lib.bm3d_batch_device_bytes(self._h)

    def set_io(self, i: int, img, out, stream=None):
        torch = _torch()
        if not 0 <= i < self.n:
            raise ValueError("image index %d out of range" % i)
        if _hwc(img) != self.shapes[i]:
            raise ValueError("set_io: image %d must keep its shape %s" % (i, self.shapes[i]))
        h, w, c = self.shapes[i]
        _check(_lib.bm3d_batch_set_io(self._h, i, _ptr(img, torch.uint8, "img"),
                                      _ptr(out, torch.float32, "out", h * w * c, True), _stream(stream)),
               "bm3d_batch_set_io")
        self._keep[i] = [img, out]

    def run(self, stream=None):
        _check(_lib.bm3d_batch_run(self._h, _stream(stream)), "bm3d_batch_run")

    def run_stages(self, i0: int, i1: int, first: int, last: int, stream=None):
        _check(_lib.bm3d_batch_run_stages(self._h, i0, i1, first, last, _stream(stream)),
               "bm3d_batch_run_stages")

    def buffer_bytes(self, i: int, buffer: str) -> int:
        h, w, c = self.shapes[i]
        return workspace_buffer(h, w, c, self.p, buffer)[1]

    def read_buffer(self, i: int, buffer: str, stream=None):
        """A device copy (1-D, typed) of image i's working buffer."""
        torch = _torch()
        nb = self.buffer_bytes(i, buffer)
        t = torch.empty(nb, dtype=torch.uint8, device="cuda")
        _check(_lib.bm3d_batch_copy_buffer(self._h, i, BUFFERS.index(buffer), t.data_ptr(), nb, 0,
                                           _stream(stream)), "bm3d_batch_copy_buffer")
        return t.view(getattr(torch, BUFFER_DTYPES[BUFFERS.index(buffer)]))

    def write_buffer(self, i: int, buffer: str, src, stream=None):
        """Sets image i's working buffer from a device tensor of its exact size."""
        torch = _torch()
        dt = getattr(torch, BUFFER_DTYPES[BUFFERS.index(buffer)])
        nb = self.buffer_bytes(i, buffer)
        _check(_lib.bm3d_batch_copy_buffer(self._h, i, BUFFERS.index(buffer),
                                           _ptr(src, dt, buffer, nb // src.element_size(), True), nb, 1,
                                           _stream(stream)), "bm3d_batch_copy_buffer")

    def capture(self, stream=None):
        _check(_lib.bm3d_batch_capture(self._h, _stream(stream)), "bm3d_batch_capture")

    def launch(self, stream=None):
        _check(_lib.bm3d_batch_launch(self._h, _stream(stream)), "bm3d_batch_launch")

    def close(self):
        if self._h:
            _lib.bm3d_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Stage-level continuous batching on the device (bm3d_server_*)."""

    def __init__(self, max_requests: int, p: Params):
        self.max_requests = max_requests
        self._h = ctypes.c_void_p()
        _check(_lib.bm3d_server_create(max_requests, ctypes.byref(p), ctypes.byref(self._h)),
               "bm3d_server_create")

    def tick(self, requests, stream=None):
        """requests: list of Request structures (stage set per request)."""
        arr = (Request * max(1, len(requests)))(*requests)
        _check(_lib.bm3d_server_tick(self._h, arr, len(requests), _stream(stream)),
               "bm3d_server_tick")

    def close(self):
        if self._h:
            _lib.bm3d_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def library_symbols():
    """Names of the entry points this binding binds (all declared in bm3d.h)."""
    return sorted(_SIGS)
