"""Pins of the oracle's network evaluation (the stand-in networks of the
weight file; the paper's own figure and weights are unpublished).

Checks: single conv layers against torch.nn.functional.conv2d in float64 (an
independent library routine) on tiny random inputs; closed-form kernels
(centre delta = identity, all-ones 3x3 on a constant map = 9c/6c/4c with zero
padding); the full CNN and U-Net against a float64 torch composition of
conv2d / avg_pool2d / nearest interpolate / cat / relu / softplus built from
the same weights; zero input with zero biases gives softplus(0) = ln 2; bad
weight files are rejected.
"""
import math
import struct

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_2010_01775_amd import synth


@pytest.mark.parametrize("ci,co,k,H,W", [(3, 5, 3, 8, 8), (1, 16, 3, 6, 10), (7, 2, 1, 5, 4), (16, 16, 3, 4, 4)])
def test_conv_vs_torch(orc, ci, co, k, H, W):
    rng = np.random.default_rng(ci * 100 + co)
    w = rng.standard_normal((co, ci, k, k)).astype(np.float32)
    b = rng.standard_normal(co).astype(np.float32)
    x = rng.standard_normal((ci, H, W))
    got = orc.conv2d(w, b, x)
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w.astype(np.float64)),
                   torch.from_numpy(b.astype(np.float64)), padding=k // 2)[0].numpy()
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_conv_closed_forms(orc):
    x = np.random.default_rng(0).standard_normal((1, 7, 9))
    delta = np.zeros((1, 1, 3, 3), np.float32)
    delta[0, 0, 1, 1] = 1
    assert np.array_equal(orc.conv2d(delta, None, x), x)
    ones = np.ones((1, 1, 3, 3), np.float32)
    c = 2.5
    y = orc.conv2d(ones, None, np.full((1, 6, 5), c))[0]
    assert np.all(y[1:-1, 1:-1] == 9 * c)
    assert np.all(y[0, 1:-1] == 6 * c) and np.all(y[-1, 1:-1] == 6 * c)
    assert np.all(y[1:-1, 0] == 6 * c) and np.all(y[1:-1, -1] == 6 * c)
    assert y[0, 0] == y[0, -1] == y[-1, 0] == y[-1, -1] == 4 * c


def _torch_net(ws, bs, arch, D, x):
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    h = torch.from_numpy(x)[:, None]
    if arch == synth.ARCH_CNN:
        for i, (w, b) in enumerate(zip(ws, bs)):
            h = F.conv2d(h, t(w), t(b), padding=1)
            if i + 1 < len(ws):
                h = F.relu(h)
        return F.softplus(h, beta=1, threshold=1e9)[:, 0].numpy()
    skips = []
    for d in range(D):
        if d:
            h = F.avg_pool2d(h, 2)
        h = F.relu(F.conv2d(h, t(ws[2 * d]), t(bs[2 * d]), padding=1))
        h = F.relu(F.conv2d(h, t(ws[2 * d + 1]), t(bs[2 * d + 1]), padding=1))
        skips.append(h)
    li = 2 * D
    for d in range(D - 2, -1, -1):
        h = torch.cat([F.interpolate(h, scale_factor=2, mode="nearest"), skips[d]], 1)
        h = F.relu(F.conv2d(h, t(ws[li]), t(bs[li]), padding=1))
        h = F.relu(F.conv2d(h, t(ws[li + 1]), t(bs[li + 1]), padding=1))
        li += 2
    h = F.conv2d(h, t(ws[li]), t(bs[li]))
    return F.softplus(h, beta=1, threshold=1e9)[:, 0].numpy()


@pytest.mark.parametrize("arch,levels,H,W", [
    (synth.ARCH_CNN, (1, 16, 16, 1), 32, 32),
    (synth.ARCH_UNET, (16, 32, 64, 128), 16, 16),
    (synth.ARCH_UNET, (4, 8, 12), 8, 16),
    (synth.ARCH_UNET, (8,), 4, 4),
])
def test_network_vs_torch(orc, arch, levels, H, W):
    layers = synth.cnn_layers(levels) if arch == synth.ARCH_CNN else synth.unet_layers(levels)
    ws, bs = synth.he_weights(3, layers, random_bias=True)
    D = 0 if arch == synth.ARCH_CNN else len(levels)
    model = synth.pack_model(arch, D, ws, bs)
    x = np.random.default_rng(4).lognormal(0, 1, (3, H, W))
    rc, s = orc.net_forward(model, x)
    assert rc == 0
    ref = _torch_net(ws, bs, arch, D, x)
    assert np.allclose(s, ref, rtol=1e-12, atol=1e-300)


def test_zero_input_gives_ln2(orc):
    for model in (synth.cnn_model(1), synth.unet_model(1)):
        rc, s = orc.net_forward(model, np.zeros((2, 16, 16)))
        assert rc == 0
        assert np.all(s == math.log(2.0))


def test_bad_models(orc):
    good = synth.unet_model(1)
    x = np.zeros((1, 16, 16))
    assert orc.net_forward(b"XXXX" + good[4:], x)[0] == orc.E_ARG
    assert orc.net_forward(good[:-4], x)[0] == orc.E_ARG
    assert orc.net_forward(good + b"\0", x)[0] == orc.E_ARG
    # U-Net levels deeper than the map allows
    assert orc.net_forward(good, np.zeros((1, 4, 4)))[0] == orc.E_ARG
    # wrong skip width: swap two decoder layers
    ws, bs = synth.he_weights(1, synth.unet_layers())
    ws[8], ws[9] = ws[9], ws[8]
    bs[8], bs[9] = bs[9], bs[8]
    assert orc.net_forward(synth.pack_model(synth.ARCH_UNET, 4, ws, bs), x)[0] == orc.E_ARG
    bad_arch = good[:8] + struct.pack("<I", 9) + good[12:]
    assert orc.net_forward(bad_arch, x)[0] == orc.E_ARG


def test_parameter_count():
    ws, bs = synth.he_weights(0, synth.unet_layers())
    assert sum(w.size for w in ws) + sum(b.size for b in bs) == 487009
