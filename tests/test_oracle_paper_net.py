"""Pins of the oracle's paper-style U-Net (Sec. 6.1: masked first
convolution on the five input channels, ELU activations, residual links, a
dilated bottleneck, skip connections).

Checks: the dilated convolution against float64 torch.nn.functional.conv2d
(dilation d, padding d) and a one-tap kernel as an exact shift by d pixels;
the whole network against an independent float64 torch composition
(masked first layer written as conv2d of the masked input and of the mask,
F.elu, residual adds, dilations 2 and 4, avg_pool2d, nearest interpolate,
cat, softplus) on random inputs with sparse masks and random biases; the
layer list of the model file; malformed files rejected.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_2010_01775_amd import synth


@pytest.mark.parametrize("dil,H", [(1, 9), (2, 12), (4, 8)])
def test_conv2d_dilated_vs_torch(orc, dil, H):
    rng = np.random.default_rng(dil)
    w = rng.standard_normal((3, 2, 3, 3)).astype(np.float32)
    b = rng.standard_normal(3).astype(np.float32)
    x = rng.standard_normal((2, H, H + 3))
    got = orc.conv2d_dil(w, b, x, dil)
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w.astype(np.float64)),
                   torch.from_numpy(b.astype(np.float64)), padding=dil, dilation=dil)[0].numpy()
    assert np.abs(got - ref).max() < 1e-12


def test_dilated_one_tap_is_a_shift(orc):
    x = np.random.default_rng(9).standard_normal((1, 10, 11))
    w = np.zeros((1, 1, 3, 3), np.float32)
    w[0, 0, 0, 0] = 1.0                       # the upper-left tap: input at (y - d, x - d)
    for d in (1, 2, 4):
        got = orc.conv2d_dil(w, None, x, d)[0]
        want = np.zeros_like(x[0])
        want[d:, d:] = x[0, :-d, :-d]
        assert np.array_equal(got, want)


def _torch_paper(model_levels, ws, bs, x):
    """The architecture written out in float64 torch ops (its own code)."""
    T = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    Wt, Bt = [T(w) for w in ws], [T(b) for b in bs]
    D = len(model_levels)
    xin = T(x)                                    # [L][5][H][W]
    m = xin[:, 4:5]
    # masked first layer: sum over valid taps rescaled by 9 / S, 0 where S = 0
    acc = F.conv2d(xin * m, Wt[0], None, padding=1)
    S = F.conv2d(m, torch.ones((1, 1, 3, 3), dtype=torch.float64), None, padding=1)
    h = torch.where(S > 0, Bt[0][None, :, None, None] + 9.0 / S.clamp_min(1) * acc, torch.zeros_like(acc))
    li = 0
    skips = []
    for d in range(D):
        if d > 0:
            h = F.avg_pool2d(h, 2)
            h = F.conv2d(h, Wt[li], Bt[li], padding=1)
        a = F.elu(h)
        li += 1
        dils = [2, 4] if d == D - 1 else [1]
        for dl in dils:
            a = F.elu(F.conv2d(a, Wt[li], Bt[li], padding=dl, dilation=dl)) + a
            li += 1
        if d < D - 1:
            skips.append(a)
        h = a
    for d in range(D - 2, -1, -1):
        c = torch.cat([F.interpolate(h, scale_factor=2, mode="nearest"), skips[d]], 1)
        a = F.elu(F.conv2d(c, Wt[li], Bt[li], padding=1))
        h = F.elu(F.conv2d(a, Wt[li + 1], Bt[li + 1], padding=1)) + a
        li += 2
    return F.softplus(F.conv2d(h, Wt[li], Bt[li]))[:, 0].numpy()


@pytest.mark.parametrize("levels,H,W", [((8, 16, 32), 16, 16), ((16, 32, 64), 32, 32), ((4, 8), 8, 16)])
def test_paper_net_vs_torch(orc, levels, H, W):
    rng = np.random.default_rng(sum(levels) + H)
    model = synth.paper_unet_model(7, levels, random_bias=True)
    ws, bs = synth.he_weights(7, synth.paper_unet_layers(levels), True)
    L = 3
    x = rng.gamma(0.5, 1.0, (L, 5, H, W))
    x[:, 4] = (rng.random((L, H, W)) < 0.4).astype(np.float64)
    x[:, :4] *= x[:, 4:5]                      # maps are zero where no photon landed
    x[2, 4] = 0.0                              # an empty leaf
    x[2, :4] = 0.0
    rc, s = orc.net_forward5(model, x)
    assert rc == 0
    ref = _torch_paper(levels, ws, bs, x)
    assert np.max(np.abs(s - ref) / np.abs(ref)) < 1e-12
    # the ELU branch for negative inputs is exercised (not a ReLU in disguise)
    assert np.any(F.conv2d(torch.from_numpy(x[:1]), torch.from_numpy(ws[0].astype(np.float64)), None,
                           padding=1).numpy() < 0)


def test_paper_layer_list():
    assert synth.paper_unet_layers((16, 32, 64)) == [
        (16, 5, 3), (16, 16, 3), (32, 16, 3), (32, 32, 3), (64, 32, 3), (64, 64, 3), (64, 64, 3),
        (32, 96, 3), (32, 32, 3), (16, 48, 3), (16, 16, 3), (1, 16, 1)]


def test_paper_malformed(orc):
    x = np.zeros((1, 5, 8, 8))
    ws, bs = synth.he_weights(3, synth.paper_unet_layers((4, 8)))
    bad = [synth.pack_model(synth.ARCH_PAPER, 2, ws[:-1], bs[:-1]),               # no head
           synth.pack_model(synth.ARCH_PAPER, 3, ws, bs),                         # wrong level count
           synth.pack_model(synth.ARCH_PAPER, 2, [ws[1]] + ws[1:], [bs[1]] + bs[1:])]  # 4-channel input
    for m in bad:
        rc, _ = orc.net_forward5(m, x)
        assert rc == orc.E_ARG
    rc, _ = orc.net_forward(synth.paper_unet_model(3, (4, 8)), np.zeros((1, 8, 8)))
    assert rc == orc.E_ARG                                                    # five-channel only
