"""Pins of the FP64 flexible U-Net oracle (no GPU).

The depthwise convolution (stride 1 and 2) and the 2x2 deconvolution are
checked against torch's functional forms and against pure-Python loops; the
whole network against the same network assembled from torch.nn layers
(float64, CPU) on even and odd image sizes (the crop after upsampling); the
residual connection against its closed form; the operation count against
Table 3."""
from pathlib import Path

import numpy as np
import pytest

from oracle import unet as O
from paper_2403_03488_amd import synth

torch = pytest.importorskip("torch")
F = torch.nn.functional


@pytest.mark.parametrize("stride,H,W", [(1, 7, 9), (2, 7, 9), (2, 8, 6), (2, 1, 1)])
def test_depthwise_matches_torch_and_loops(stride, H, W):
    rng = np.random.default_rng(H * W + stride)
    x = rng.normal(size=(5, H, W))
    w = rng.normal(size=(5, 3, 3))
    got = O.depthwise3x3(x, w, stride)
    want = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w)[:, None], stride=stride, padding=1,
                    groups=5)[0].numpy()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    for c in range(5):
        for y in range(got.shape[1]):
            for xx in range(got.shape[2]):
                s = sum(w[c, dy + 1, dx + 1] * x[c, stride * y + dy, stride * xx + dx]
                        for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                        if 0 <= stride * y + dy < H and 0 <= stride * xx + dx < W)
                assert abs(got[c, y, xx] - s) < 1e-12


def test_deconv_matches_torch_and_loops():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(3, 4, 5))
    w = rng.normal(size=(3, 2, 2, 2))
    got = O.deconv2x2(x, w)
    want = F.conv_transpose2d(torch.from_numpy(x)[None], torch.from_numpy(w), stride=2)[0].numpy()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    for o in range(2):
        for Y in range(8):
            for X in range(10):
                s = sum(x[i, Y // 2, X // 2] * w[i, o, Y % 2, X % 2] for i in range(3))
                assert abs(got[o, Y, X] - s) < 1e-12


def bn(L, prefix, co):
    m = torch.nn.BatchNorm2d(co, eps=L[prefix + "eps"]).double().eval()
    m.weight.data = torch.from_numpy(L[prefix + "gamma"].astype(np.float64))
    m.bias.data = torch.from_numpy(L[prefix + "beta"].astype(np.float64))
    m.running_mean = torch.from_numpy(L[prefix + "mean"].astype(np.float64))
    m.running_var = torch.from_numpy(L[prefix + "var"].astype(np.float64))
    return m


class TorchDS(torch.nn.Module):
    def __init__(self, L, stride):
        super().__init__()
        ci, co = L["dw"].shape[0], L["pw"].shape[0]
        self.dw = torch.nn.Conv2d(ci, ci, 3, stride=stride, padding=1, groups=ci).double()
        self.dw.weight.data = torch.from_numpy(L["dw"].astype(np.float64))[:, None]
        self.dw.bias.data = torch.from_numpy(L["dw_bias"].astype(np.float64))
        self.pw = torch.nn.Conv2d(ci, co, 1).double()
        self.pw.weight.data = torch.from_numpy(L["pw"].astype(np.float64))[:, :, None, None]
        self.pw.bias.data = torch.from_numpy(L["pw_bias"].astype(np.float64))
        self.bn = bn(L, "pw_", co)

    def forward(self, x):
        return torch.relu(self.bn(self.pw(torch.relu(self.dw(x)))))


class TorchUNet(torch.nn.Module):
    def __init__(self, net):
        super().__init__()
        self.enc = torch.nn.ModuleList([TorchDS(L, 1) for L in net["enc"]])
        self.down = torch.nn.ModuleList([TorchDS(L, 2) for L in net["down"]])
        self.dec = torch.nn.ModuleList([TorchDS(L, 1) for L in net["dec"]])
        self.up = torch.nn.ModuleList()
        for U in net["up"]:
            m = torch.nn.ConvTranspose2d(U["weight"].shape[0], U["weight"].shape[1], 2, stride=2).double()
            m.weight.data = torch.from_numpy(U["weight"].astype(np.float64))
            m.bias.data = torch.from_numpy(U["bias"].astype(np.float64))
            self.up.append(m)
        o = net["out"]
        self.out = torch.nn.Conv2d(o["weight"].shape[1], o["weight"].shape[0], 1).double()
        self.out.weight.data = torch.from_numpy(o["weight"].astype(np.float64))[:, :, None, None]
        self.out.bias.data = torch.from_numpy(o["bias"].astype(np.float64))

    def forward(self, x):
        skips = []
        for e, d in zip(self.enc, self.down):
            x = e(x)
            skips.append(x)
            x = d(x)
        for i in range(3, -1, -1):
            u = torch.relu(self.up[i](x))
            s = skips[i]
            x = self.dec[i](u[:, :, :s.shape[2], :s.shape[3]] + s)
        return self.out(x)


@pytest.mark.parametrize("C,H,W", [(3, 32, 48), (1, 37, 29), (3, 5, 3)])
def test_network_matches_torch_nn(C, H, W):
    net = synth.unet_net(C, seed=C + H)
    rng = np.random.default_rng(H)
    basic = rng.uniform(0, 255, (H, W, C) if C == 3 else (H, W))
    noisy = np.clip(basic + rng.normal(0, 25, basic.shape), 0, 255)
    got = O.restore(basic, noisy, 25.0, net)
    b3 = basic if C == 3 else basic[:, :, None]
    n3 = noisy if C == 3 else noisy[:, :, None]
    z = np.concatenate([np.moveaxis(b3, 2, 0), np.moveaxis(n3, 2, 0), np.full((1, H, W), 25.0)])[None] / 255.0
    with torch.no_grad():
        Fz = TorchUNet(net).eval()(torch.from_numpy(z))[0].numpy()
    want = np.moveaxis(np.moveaxis(b3, 2, 0) + 255.0 * Fz, 0, 2)
    want = want if C == 3 else want[:, :, 0]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)
    assert np.abs(got - basic).max() > 0.5


def test_zero_output_layer_returns_basic_and_sigma_plane_is_read():
    net = synth.unet_net(3, seed=2)
    rng = np.random.default_rng(3)
    basic = rng.uniform(0, 255, (20, 24, 3))
    noisy = rng.uniform(0, 255, (20, 24, 3))
    a = O.restore(basic, noisy, 10.0, net)
    b = O.restore(basic, noisy, 50.0, net)
    assert np.abs(a - b).max() > 1e-3
    net["out"] = {"weight": np.zeros_like(net["out"]["weight"]), "bias": np.zeros(3, np.float32)}
    assert np.array_equal(O.restore(basic, noisy, 25.0, net), basic)


def test_operation_count_matches_table_3():
    rows = [l.split() for l in Path(__file__).with_name("golden").joinpath("unet_table3_gflops.txt")
            .read_text().splitlines() if l.strip() and not l.startswith("#")]
    for h, w, g in rows:
        got = O.macs(3, int(h), int(w)) / 1e9
        # within 1.5 %: halving every width would be ~70 % off, dropping a
        # level's block ~8 %
        assert abs(got - float(g)) / float(g) < 1.5e-2, (h, w, got, g)
    # the count is the sum over the network's layers (an independent tally)
    net = synth.unet_net(3)
    H = W = 64
    tot, hh, ww, dims = 0, H, W, []
    for i in range(4):
        for L, s in ((net["enc"][i], 1), (net["down"][i], 2)):
            if s == 2:
                hh, ww = (hh + 1) // 2, (ww + 1) // 2
            else:
                dims.append((hh, ww))
            tot += hh * ww * (L["dw"].size + L["pw"].size)
    for i in range(3, -1, -1):
        tot += 4 * hh * ww * net["up"][i]["weight"].size // 4
        hh, ww = dims[i]
        tot += hh * ww * (net["dec"][i]["dw"].size + net["dec"][i]["pw"].size)
    tot += H * W * net["out"]["weight"].size
    assert tot == O.macs(3, H, W)
