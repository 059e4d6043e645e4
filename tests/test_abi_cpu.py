"""The C ABI on the CPU: the library loads without a GPU, exports every entry
point declared in include/bm3d.h, and rejects invalid arguments on the host
before anything is enqueued (no GPU call is reached)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bm3d.h")


@pytest.fixture(scope="module")
def B():
    lib = os.path.join(ROOT, "paper_2403_03488_amd", "libbm3d_mi355x.so")
    if not os.path.exists(lib):
        from paper_2403_03488_amd import build
        build.build()
    from paper_2403_03488_amd import bm3d
    return bm3d


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bm3d_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bm3d_block_match", "bm3d_collab_filter", "bm3d_aggregate", "bm3d_denoise"):
        assert required in names


def test_every_declared_symbol_is_exported(B):
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(B.library_symbols())


def test_struct_layout_matches_header(B):
    # bm3d_params: 4 ints, 4 floats, 4 ints/unsigned, 2 pointers, size_t, float, 2 ints
    # (padded to the pointers' 8-byte alignment)
    assert ctypes.sizeof(B.Params) == 4 * 4 + 4 * 4 + 4 * 4 + 8 + 8 + 8 + 4 + 4 + 4 + 4
    assert ctypes.sizeof(B.ImageDesc) == 8 + 8 + 3 * 4 + 4


def test_defaults_and_geometry(B):
    p = B.params_default(25.0)
    assert (p.search_ht, p.search_wie, p.n_ht, p.n_wie) == (32, 32, 16, 32)
    assert abs(p.lambda_ht - 2.7) < 1e-6 and p.kaiser_beta == 2.0
    assert (p.tau_ht, p.tau_wie) == (2500.0, 400.0)
    q = B.params_default(50.0)
    assert (q.tau_ht, q.tau_wie) == (5000.0, 3500.0)
    assert B.num_refs(512, 512) == 169 * 169
    assert B.num_refs(321, 481) == 106 * 159
    assert B.num_refs(8, 8) == 1 and B.num_refs(7, 100) == 0
    assert B.workspace_size(512, 512, 1, p) > 512 * 512 * 17
    assert B.workspace_size(4, 512, 1, p) == 0
    assert B.strerror(0) == "ok" and "argument" in B.strerror(-1)


def test_nlm_defaults_and_validation(B):
    assert ctypes.sizeof(B.NlmParams) == 12
    p = B.nlm_params_default(25.0, 1)
    assert (p.patch_radius, p.search_radius) == (2, 10) and abs(p.h - 10.0) < 1e-5
    q = B.nlm_params_default(50.0, 3)
    assert (q.patch_radius, q.search_radius) == (2, 17) and abs(q.h - 20.0) < 1e-5
    L = B._lib
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    ref = ctypes.byref
    assert L.bm3d_nlm_params_default(0.0, 1, ref(B.NlmParams())) == -1
    assert L.bm3d_nlm_params_default(25.0, 2, ref(B.NlmParams())) == -1
    assert L.bm3d_nlm(None, 64, 64, 1, 25.0, ref(p), fake, None) == -1
    assert L.bm3d_nlm(fake, 0, 64, 1, 25.0, ref(p), fake, None) == -1
    assert L.bm3d_nlm(fake, 64, 64, 2, 25.0, ref(p), fake, None) == -1
    assert L.bm3d_nlm(fake, 64, 64, 1, float("nan"), ref(p), fake, None) == -1
    assert L.bm3d_nlm(fake, 64, 64, 1, 25.0, None, fake, None) == -1
    arr = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    assert L.bm3d_nlm_batch(arr, arr, 0, 64, 64, 1, 25.0, ref(p), None) == -1
    assert L.bm3d_nlm_batch(arr, arr, 65, 64, 64, 1, 25.0, ref(p), None) == -1
    assert L.bm3d_nlm_batch(None, arr, 2, 64, 64, 1, 25.0, ref(p), None) == -1
    holes = (ctypes.c_void_p * 2)(0x1000, None)
    assert L.bm3d_nlm_batch(arr, holes, 2, 64, 64, 1, 25.0, ref(p), None) == -1
    assert L.bm3d_nlm_batch(arr, arr, 2, 64, 64, 2, 25.0, ref(p), None) == -1
    for field, val in (("patch_radius", -1), ("patch_radius", 9), ("search_radius", 0),
                       ("search_radius", 25), ("h", 0.0), ("h", float("inf"))):
        bad = B.NlmParams(p.patch_radius, p.search_radius, p.h)
        setattr(bad, field, val)
        assert L.bm3d_nlm(fake, 64, 64, 1, 25.0, ref(bad), fake, None) == -1, field


def test_cnn_validation_on_host(B):
    # every rejected case fails before any device call
    import numpy as np
    from paper_2403_03488_amd import synth
    L = B._lib
    ref = ctypes.byref
    assert ctypes.sizeof(B.CnnLayer) == 7 * 8
    layers = synth.cnn_layers(4, 3)
    keep = []

    def descs(ls):
        arr = (B.CnnLayer * len(ls))()
        for k, d in enumerate(ls):
            ptr = {}
            for key in ("weight", "bias", "gamma", "beta", "mean", "var"):
                a = d.get(key)
                if a is not None:
                    a = np.ascontiguousarray(a, np.float32)
                    keep.append(a)
                ptr[key] = None if a is None else a.ctypes.data
            arr[k] = B.CnnLayer(ptr["weight"], ptr["bias"], ptr["gamma"], ptr["beta"], ptr["mean"],
                                ptr["var"], float(d.get("eps", 0.0)))
        return arr

    h = ctypes.c_void_p()
    good = descs(layers)
    assert L.bm3d_cnn_create(4, 3, 64, good, None) == -1
    assert L.bm3d_cnn_create(4, 3, 64, None, ref(h)) == -1
    assert L.bm3d_cnn_create(2, 3, 64, good, ref(h)) == -1      # fewer than 3 layers
    assert L.bm3d_cnn_create(4, 2, 64, good, ref(h)) == -1      # channels
    assert L.bm3d_cnn_create(4, 3, 32, good, ref(h)) == -2      # only 64 features
    assert L.bm3d_cnn_create(65, 3, 64, good, ref(h)) == -2
    bad = [dict(d) for d in layers]
    w = bad[1]["weight"].copy()
    w[0, 0, 1, 1] = np.nan
    bad[1]["weight"] = w
    assert L.bm3d_cnn_create(4, 3, 64, descs(bad), ref(h)) == -1
    bad = [dict(d) for d in layers]
    bad[2] = dict(bad[2], var=None)                               # partial normalisation
    assert L.bm3d_cnn_create(4, 3, 64, descs(bad), ref(h)) == -1
    bad = [dict(d) for d in layers]
    bad[2] = dict(bad[2], var=-np.ones(64, np.float32))           # var + eps <= 0
    assert L.bm3d_cnn_create(4, 3, 64, descs(bad), ref(h)) == -1
    assert not h.value
    b = ctypes.c_size_t()
    assert L.bm3d_cnn_workspace_bytes(3, 20, 30, ref(b)) == 0 and b.value == 3 * 20 * 30 * 256
    assert L.bm3d_cnn_workspace_bytes(0, 20, 30, ref(b)) == -1
    arr = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    fake = ctypes.c_void_p(0x1000)
    assert L.bm3d_cnn_restore(None, arr, arr, arr, 2, 64, 64, fake, 1 << 30, None) == -1
    assert L.bm3d_cnn_destroy(None) == -1


def test_unet_validation_on_host(B):
    # rejected before any device call; nothing is allocated
    import numpy as np
    from paper_2403_03488_amd import synth
    L = B._lib
    ref = ctypes.byref
    h = ctypes.c_void_p()
    with pytest.raises(B.BM3DError):
        B.Unet(synth.unet_net(3), 2)                                   # channels
    with pytest.raises(B.BM3DError):
        B.Unet(synth.unet_net(3, widths=(32, 64, 128, 256, 512)), 3, widths=(32, 64, 128, 256, 512))
    with pytest.raises(B.BM3DError):
        B.Unet(synth.unet_net(3, widths=(16, 32, 64, 128, 256)), 3, widths=(16, 32, 64, 128, 256))
    bad = synth.unet_net(3)
    bad["dec"][2]["dw"] = bad["dec"][2]["dw"].copy()
    bad["dec"][2]["dw"][0, 0, 0] = np.inf
    with pytest.raises(B.BM3DError):
        B.Unet(bad, 3)
    bad = synth.unet_net(3)
    bad["enc"][1] = dict(bad["enc"][1], pw_var=None)                   # partial normalisation
    with pytest.raises(B.BM3DError):
        B.Unet(bad, 3)
    assert L.bm3d_unet_create(3, None, None, ref(h)) == -1 and not h.value
    b = ctypes.c_size_t()
    assert L.bm3d_unet_workspace_bytes(None, 1, 8, 8, ref(b)) == -1
    arr = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    assert L.bm3d_unet_restore(None, arr, arr, arr, 2, 64, 64, 25.0, ctypes.c_void_p(0x1000), 1 << 30, None) == -1
    assert L.bm3d_unet_destroy(None) == -1


def test_vst_validation_on_host(B):
    L = B._lib
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    for bad in ((0.0, 1.0, 0.0, 10.0, 0.0), (1.0, -1.0, 0.0, 10.0, 0.0), (1.0, 1.0, 0.0, 0.0, 0.0),
                (float("nan"), 1.0, 0.0, 10.0, 0.0), (1.0, 1.0, float("inf"), 10.0, 0.0)):
        g = B.GatParams(*bad)
        assert L.bm3d_gat_forward(fake, 16, ctypes.byref(g), fake, None) == -1, bad
        assert L.bm3d_gat_inverse(fake, 16, ctypes.byref(g), fake, None) == -1, bad
    g = B.GatParams(1.0, 1.0, 0.0, 10.0, 0.0)
    assert L.bm3d_gat_forward(None, 16, ctypes.byref(g), fake, None) == -1
    assert L.bm3d_gat_forward(fake, -1, ctypes.byref(g), fake, None) == -1
    assert L.bm3d_gat_forward(fake, 0, ctypes.byref(g), fake, None) == 0  # nothing to do
    assert L.bm3d_gat_inverse(fake, 16, None, fake, None) == -1
    p = B.params_default(25.0)
    assert L.bm3d_vst_denoise(fake, 0, 64, 1, ctypes.byref(g), ctypes.byref(p), fake, fake, None) == -1
    assert L.bm3d_vst_denoise(fake, 64, 64, 2, ctypes.byref(g), ctypes.byref(p), fake, fake, None) == -1
    # everything the BM3D stage checks is checked before the forward map is
    # enqueued: a too-small image or workspace fails without a launch (a
    # launch here, without a GPU, would report a HIP error instead)
    assert L.bm3d_vst_denoise(fake, 4, 64, 1, ctypes.byref(g), ctypes.byref(p), fake, fake, None) == -1
    assert L.bm3d_vst_denoise(fake, 64, 64, 1, ctypes.byref(g), ctypes.byref(p), fake, fake, None) == -3
    small = p.copy()
    small.workspace, small.workspace_bytes = 0x2000, 100
    assert L.bm3d_vst_denoise(fake, 64, 64, 1, ctypes.byref(g), ctypes.byref(small), fake, fake, None) == -3
    bad = p.copy()
    bad.n_ht = 5
    assert L.bm3d_vst_denoise(fake, 64, 64, 1, ctypes.byref(g), ctypes.byref(bad), fake, fake, None) == -1
    assert abs(L.bm3d_gat_noise_level(6.0) - math.sqrt(36 + 1 / 12)) < 1e-5


def test_host_validation_rejects_before_enqueue(B):
    L = B._lib
    p = B.params_default(25.0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    ref = ctypes.byref
    # bad image sizes / channels / sigma
    assert L.bm3d_denoise(fake, 7, 64, 1, 25.0, ref(p), fake, None) == -1
    assert L.bm3d_denoise(fake, 64, 64, 2, 25.0, ref(p), fake, None) == -1
    assert L.bm3d_denoise(fake, 64, 64, 1, float("nan"), ref(p), fake, None) == -1
    assert L.bm3d_denoise(fake, 64, 64, 1, -1.0, ref(p), fake, None) == -1
    assert L.bm3d_denoise(None, 64, 64, 1, 25.0, ref(p), fake, None) == -1
    # missing workspace
    assert L.bm3d_denoise(fake, 64, 64, 1, 25.0, ref(p), fake, None) == -3
    small = p.copy()
    small.workspace = 0x2000
    small.workspace_bytes = 10
    assert L.bm3d_denoise(fake, 64, 64, 1, 25.0, ref(small), fake, None) == -3
    # invalid parameters
    for field, val in (("n_wie", 24), ("n_ht", 0), ("search_ht", 33), ("search_wie", 0),
                       ("lambda_ht", -1.0), ("tau_wie", float("nan")), ("xform", 7),
                       ("kaiser_beta", float("inf")), ("tile_refs", 17), ("lambda_2d", -1.0),
                       ("lambda_2d", float("nan")), ("transform_ht", 2), ("match_refs", 4),
                       ("match_refs", -8), ("match_refs", 32)):
        q = p.copy()
        setattr(q, field, val)
        assert L.bm3d_denoise(fake, 64, 64, 1, 25.0, ref(q), fake, None) == -1, field
    big = p.copy()
    big.tile_refs = 16  # the largest tile: its region still fits the LDS
    assert L.bm3d_denoise(fake, 64, 64, 1, 25.0, ref(big), fake, None) == -3  # (then: no workspace)
    # a Kaiser window so sharp that the FP32 corner weights approach underflow
    sharp = p.copy()
    sharp.kaiser_beta = 60.0
    assert L.bm3d_denoise(fake, 64, 64, 1, 25.0, ref(sharp), fake, None) == -2
    sharp.kaiser_beta = 50.0  # the largest accepted value passes validation (then the workspace check fails)
    assert L.bm3d_denoise(fake, 64, 64, 1, 25.0, ref(sharp), fake, None) == -3
    # stage entry points
    assert L.bm3d_block_match(fake, 1, 64, 64, 1, ref(p), fake, fake, None) == -1  # step 1 needs uint8
    assert L.bm3d_block_match(fake, 0, 64, 64, 3, ref(p), fake, fake, None) == -1
    pre = p.copy()
    pre.lambda_2d = 50.0  # prefiltered step-1 grouping needs workspace for the spectra
    assert L.bm3d_block_match(fake, 0, 64, 64, 1, ref(pre), fake, fake, None) == -3
    assert L.bm3d_collab_filter(fake, fake, 64, 64, 1, 25.0, 1, fake, fake, ref(p), fake, fake,
                                None) == -1  # step 1 takes no basic estimate
    assert L.bm3d_collab_filter(fake, None, 64, 64, 1, 25.0, 2, fake, fake, ref(p), fake, fake,
                                None) == -1  # step 2 needs one
    assert L.bm3d_aggregate(fake, None, 64, 64, 1, 1, ref(p), fake, None) == -1
    assert L.bm3d_aggregate(fake, fake, 64, 64, 1, 1, None, fake, None) == -1
    assert L.bm3d_prepare(fake, 64, 64, 4, fake, fake, None) == -1
    assert L.bm3d_luminance(None, 64, 64, 1, fake, None) == -1
    # batch plans
    h = ctypes.c_void_p()
    arr = (B.ImageDesc * 1)(B.ImageDesc(0x1000, 0x2000, 64, 64, 2, 25.0))
    assert L.bm3d_batch_create(arr, 1, ref(p), ref(h)) == -1
    assert L.bm3d_batch_create(arr, 0, ref(p), ref(h)) == -1
    assert L.bm3d_batch_run(None, None) == -1
    assert L.bm3d_batch_launch(None, None) == -1
    assert L.bm3d_batch_run_stages(None, 0, 1, 0, 6, None) == -1
    assert L.bm3d_batch_copy_buffer(None, 0, 6, fake, 64, 0, None) == -1


def test_workspace_buffers(B):
    """The workspace carve-up: every buffer 256-byte aligned, in order, no
    overlap, sized from the image and params; the kept-count region only
    with the debug flag."""
    p = B.params_default(25.0)
    h, w, c = 37, 53, 3
    R = B.num_refs(h, w)
    want = {"planar": 4 * c * h * w, "lum8": h * w, "lumf": 4 * h * w, "basic": 4 * c * h * w,
            "num": 8 * c * h * w, "wsum": 8 * c * h * w, "idx1": 4 * R * p.n_ht, "cnt1": 4 * R,
            "idx2": 4 * R * p.n_wie, "cnt2": 4 * R, "nkept": 0, "coef": 0}
    end = 0
    for name in B.BUFFERS:
        off, nb = B.workspace_buffer(h, w, c, p, name)
        assert off % 256 == 0 and off >= end and nb == want[name], name
        end = off + nb
    assert end <= B.workspace_size(h, w, c, p)
    q = B.params_default(25.0, flags=B.FLAG_DEBUG_NKEPT)
    off, nb = B.workspace_buffer(h, w, c, q, "nkept")
    assert nb == 4 * c * R and off + nb <= B.workspace_size(h, w, c, q)
    assert B.workspace_size(h, w, c, q) > B.workspace_size(h, w, c, p)
    v = B.params_default(50.0, lambda_2d=2.0, transform_ht=B.T_BIOR15)
    off, nb = B.workspace_buffer(h, w, c, v, "coef")
    assert nb == 4 * 64 * (h - 7) * (w - 7) and off + nb <= B.workspace_size(h, w, c, v)
    with pytest.raises(B.BM3DError):
        B.workspace_buffer(4, w, c, p, "idx1")
    L = B._lib
    o, n = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.bm3d_workspace_buffer(h, w, c, ctypes.byref(p), 12, ctypes.byref(o), ctypes.byref(n)) == -1
    assert L.bm3d_workspace_buffer(h, w, c, ctypes.byref(p), -1, ctypes.byref(o), ctypes.byref(n)) == -1
    assert L.bm3d_workspace_buffer(h, w, c, ctypes.byref(p), 0, None, ctypes.byref(n)) == -1


def test_binding_refuses_host_tensors(B):
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        B._ptr(torch.zeros(4), None, "x")


def test_binding_checks_sizes_and_dtypes(B, monkeypatch):
    """A wrong dtype or a buffer too small for what the kernel writes is
    refused before the C call (host tensors posing as device tensors: the
    checks run before any pointer is used)."""
    torch = pytest.importorskip("torch")

    class Dev:  # a stand-in with the attributes _ptr reads
        def __init__(self, n, dtype):
            self.t = torch.zeros(n, dtype=dtype)
            self.is_cuda, self.dtype = True, dtype

        def is_contiguous(self):
            return True

        def numel(self):
            return self.t.numel()

        def data_ptr(self):
            return 0x1000

    assert B._ptr(Dev(16, torch.float32), torch.float32, "out", 16, True) == 0x1000
    with pytest.raises(ValueError):
        B._ptr(Dev(15, torch.float32), torch.float32, "out", 16, True)
    with pytest.raises(ValueError):
        B._ptr(Dev(17, torch.float32), torch.float32, "out", 16, True)
    assert B._ptr(Dev(17, torch.int32), torch.int32, "idx", 16) == 0x1000
    with pytest.raises(ValueError):
        B._ptr(Dev(16, torch.float16), torch.float32, "out", 16)


def test_server_validation_on_host(B):
    L = B._lib
    p = B.params_default(25.0)
    h = ctypes.c_void_p()
    assert L.bm3d_server_create(0, ctypes.byref(p), ctypes.byref(h)) == -1
    bad = p.copy()
    bad.n_ht = 3
    assert L.bm3d_server_create(4, ctypes.byref(bad), ctypes.byref(h)) == -1
    assert L.bm3d_server_tick(None, None, 0, None) == -1
    assert L.bm3d_server_destroy(None) == -1


def test_footprint_model(B):
    from paper_2403_03488_amd import serve
    p = B.params_default(25.0)
    f = serve.footprint(4096, 4096, 3, p)
    # planar, basic (2 x 12 B/px), fixed-point num, wsum (2 x 24 B/px), luminances
    # (5 B/px), in+out (15 B/px), groups (16 + 32 indices per reference, ~1
    # reference per 9 px: ~21 B/px)
    assert 105 * 4096 * 4096 < f < 120 * 4096 * 4096
