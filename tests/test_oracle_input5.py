"""Pins of the oracle's five-channel network input (Sec. 6: raw maps of
iterations t and t-1, their photon counts and the valid-bin mask) and its
masked (partial) first convolution.

Checks: the masked convolution with an all-ones mask against
torch.nn.functional.conv2d (float64), rescaled by 9/S at the border where S
in-map taps remain; an all-zero mask gives zero (no bias); one valid bin
gives bias + 9 * (weights . inputs) on its 3x3 neighbourhood and zero
elsewhere; the input channels on a hand-worked 2x2 map; the whole
five-channel U-Net against a float64 torch composition (masked first layer
written out with conv2d of the masked input and of the mask).
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_2010_01775_amd import synth


def _conv(w, b, x):
    return F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w.astype(np.float64)),
                    None if b is None else torch.from_numpy(b.astype(np.float64)), padding=1)[0].numpy()


def test_pconv_all_ones_mask(orc):
    rng = np.random.default_rng(1)
    w = rng.standard_normal((4, 5, 3, 3)).astype(np.float32)
    b = rng.standard_normal(4).astype(np.float32)
    x = rng.standard_normal((5, 6, 7))
    x[4] = 1.0                                             # mask channel
    got = orc.pconv2d(w, b, x, 4)
    S = _conv(np.ones((1, 1, 3, 3), np.float32), None, np.ones((1, 6, 7)))[0]   # in-map taps: 9/6/4
    want = b[:, None, None] + 9.0 / S * _conv(w, None, x)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)
    assert np.allclose(got[:, 1:-1, 1:-1], _conv(w, b, x)[:, 1:-1, 1:-1], rtol=1e-13, atol=1e-13)


def test_pconv_zero_and_single_mask(orc):
    rng = np.random.default_rng(2)
    w = rng.standard_normal((3, 2, 3, 3)).astype(np.float32)
    b = rng.standard_normal(3).astype(np.float32)
    x = rng.standard_normal((2, 5, 5))
    x[1] = 0.0
    assert np.array_equal(orc.pconv2d(w, b, x, 1), np.zeros((3, 5, 5)))
    y0, x0 = 2, 3
    x[1, y0, x0] = 1.0
    got = orc.pconv2d(w, b, x, 1)
    for yy in range(5):
        for xx in range(5):
            dy, dx = y0 - yy + 1, x0 - xx + 1
            if 0 <= dy < 3 and 0 <= dx < 3:
                want = b + 9.0 * (w[:, :, dy, dx].astype(np.float64) @ x[:, y0, x0])
            else:
                want = np.zeros(3)
            assert np.allclose(got[:, yy, xx], want, rtol=1e-13, atol=1e-13), (yy, xx)


def test_input5_hand_case(orc):
    e_t = np.array([[[2, 0], [6, 0]]], np.uint64)
    e_p = np.zeros((1, 2, 2), np.uint64)                    # an empty previous map
    p_t = np.array([[[1, 0], [3, 0]]], np.uint32)
    p_p = np.array([[[1, 1], [1, 1]]], np.uint32)
    x = orc.input5(e_t, e_p, p_t, p_p)
    assert np.array_equal(x[0, 0], [[1.0, 0.0], [3.0, 0.0]])    # 4 * E / 8
    assert np.array_equal(x[0, 1], np.zeros((2, 2)))
    assert np.array_equal(x[0, 2], [[1.0, 0.0], [3.0, 0.0]])    # 4 * P / 4
    assert np.array_equal(x[0, 3], np.ones((2, 2)))
    assert np.array_equal(x[0, 4], [[1.0, 0.0], [1.0, 0.0]])


def test_input5_stays_binary64(orc):
    """Three equal bins of a 2x2 map: each normalised value is H*W/3 = 4/3,
    which float32 cannot hold (nearest float32 1.3333333730697632); the
    channels are binary64 and keep mean 1 to the last bit."""
    e_t = np.array([[[5, 5], [5, 0]]], np.uint64)
    p_t = np.array([[[7, 7], [7, 0]]], np.uint32)
    x = orc.input5(e_t, e_t, p_t, p_t)
    for c in range(4):
        assert np.array_equal(x[0, c], [[4.0 / 3.0, 4.0 / 3.0], [4.0 / 3.0, 0.0]]), c
        assert float(np.float32(x[0, c, 0, 0])) != x[0, c, 0, 0]
    assert abs(x[0, 0].sum() - 4.0) <= 4 * np.finfo(np.float64).eps


def _torch_unet5(ws, bs, D, x):
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    h = torch.from_numpy(x)
    m = h[:, 4:5]
    S = F.conv2d(m, torch.ones((1, 1, 3, 3), dtype=torch.float64), padding=1)
    a = F.conv2d(h * m, t(ws[0]), None, padding=1)
    h = torch.where(S > 0, t(bs[0])[None, :, None, None] + 9.0 / S.clamp(min=1) * a, torch.zeros_like(a))
    h = F.relu(h)
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


@pytest.mark.parametrize("levels,H", [((8, 16), 8), ((16, 32, 64, 128), 16)])
def test_unet5_vs_torch(orc, levels, H):
    ws, bs = synth.he_weights(9, synth.unet_layers(levels, cin=5), random_bias=True)
    model = synth.pack_model(synth.ARCH_UNET, len(levels), ws, bs)
    rng = np.random.default_rng(3)
    L = 3
    e_t = (rng.random((L, H, H)) < 0.4) * rng.integers(1, 1000, (L, H, H))
    p_t = (e_t > 0).astype(np.uint32) * rng.integers(1, 5, (L, H, H)).astype(np.uint32)
    e_p = rng.integers(0, 1000, (L, H, H))
    p_p = rng.integers(0, 3, (L, H, H)).astype(np.uint32)
    x = orc.input5(e_t.astype(np.uint64), e_p.astype(np.uint64), p_t, p_p)
    rc, s = orc.net_forward5(model, x)
    assert rc == 0
    assert np.allclose(s, _torch_unet5(ws, bs, len(levels), x), rtol=1e-12, atol=1e-14)
    rc, _ = orc.net_forward(model, x[:, 0])               # the one-channel entry rejects it
    assert rc == orc.E_ARG
