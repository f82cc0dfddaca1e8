"""The algorithmic FLOP and byte counts bench.py divides by kernel time
(the roofline figures), checked against sums written out over each
network's layer list with the resolution every layer runs at."""
import os
import sys

import pytest

from paper_2010_01775_amd import synth

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _flops(layers, res):
    return sum(2 * ci * co * k * k * p for (co, ci, k), p in zip(layers, res))


def test_unet_flops_per_leaf():
    L = synth.unet_layers()
    px = 64 * 64
    res = [px, px, px // 4, px // 4, px // 16, px // 16, px // 64, px // 64,
           px // 16, px // 16, px // 4, px // 4, px, px, px]
    assert bench.model_flops_per_leaf(synth.unet_model(1), 64, 64) == _flops(L, res)
    assert abs(_flops(L, res) / 1e6 - 331.61216) < 1e-9


@pytest.mark.parametrize("H,W", [(64, 64), (32, 64), (64, 128)])
def test_paper_net_flops_per_leaf(H, W):
    L = synth.paper_unet_layers()
    px = H * W
    # levels 16 / 32 / 64: two convs at full, two at 1/4, three at 1/16 (the
    # bottleneck), then two at 1/4, two at full, the head at full
    res = [px, px, px // 4, px // 4, px // 16, px // 16, px // 16, px // 4, px // 4, px, px, px]
    assert bench.model_flops_per_leaf(synth.paper_unet_model(1), H, W) == _flops(L, res)


def test_cnn_flops_per_leaf():
    L = synth.cnn_layers()
    assert bench.model_flops_per_leaf(synth.cnn_model(1), 32, 32) == _flops(L, [1024] * 3)


def test_phase_saved_flops():
    """FP32-mode decoder convs skip 5 of 9 taps on their upsampled channels:
    U-Net 16/32/64/128 at 64x64: 128, 64, 32 upsampled channels into 64,
    32, 16 outputs at 16x16, 32x32, 64x64; paper-style 16/32/64: 64 and 32
    into 32 and 16 at 32x32 and 64x64."""
    px = 64 * 64
    want = 2 * 5 * (128 * 64 * px // 16 + 64 * 32 * px // 4 + 32 * 16 * px)
    assert bench.phase_saved_flops_per_leaf(synth.unet_model(1), 64, 64) == want
    want3 = 2 * 5 * (64 * 32 * px // 4 + 32 * 16 * px)
    assert bench.phase_saved_flops_per_leaf(synth.paper_unet_model(1), 64, 64) == want3
    assert bench.phase_saved_flops_per_leaf(synth.cnn_model(1), 32, 32) == 0.0


def test_paper_net_bytes_per_leaf():
    """Every conv reads its input and writes its output once; residual convs
    read their residual too; the first reads 24 B per pixel (two u64 energy
    maps and two u32 count maps); the head writes float32."""
    px = 64 * 64
    e = 2
    q, s = px // 4, px // 16
    want = (24 * px + 16 * px * e                      # masked first conv
            + 2 * 16 * px * e + 16 * px * e            # level 0 second conv (+ residual)
            + 16 * px * e + 32 * q * e                 # pooled conv to 32 channels
            + 2 * 32 * q * e + 32 * q * e              # level 1 second conv
            + 32 * q * e + 64 * s * e                  # pooled conv to 64 channels
            + 2 * (2 * 64 * s * e + 64 * s * e)        # two dilated convs with residuals
            + 64 * s * e + 32 * q * e + 32 * q * e     # decoder level 1: [up(64 @ s), skip 32 @ q]
            + 2 * 32 * q * e + 32 * q * e
            + 32 * q * e + 16 * px * e + 16 * px * e   # decoder level 0: [up(32 @ q), skip 16 @ px]
            + 2 * 16 * px * e + 16 * px * e
            + 16 * px * e + 4 * px)                    # head
    assert bench.model_bytes_per_leaf(synth.paper_unet_model(1), 64, 64, e, 24.0) == want
