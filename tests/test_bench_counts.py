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


def test_stage_bytes_per_unit():
    """Per-stage algorithmic bytes: the uniform batch's splat moves 67.1 MB of
    photons and 50.3 MB of maps; a query of the sampler reads 12 B and writes
    20 B; tables are read once."""
    N, L, H, W, nq = 4096 * 1024, 1024, 64, 64, 1 << 20
    assert bench.stage_bytes("splat", N, L, H, W, nq) == 16 * N + 12 * L * H * W == 117_440_512
    tab = L * H * W * 4 + L * H * (W + 1) * 4 + L * (H + 1) * 4
    assert bench.stage_bytes("sample", N, L, H, W, nq) == 32 * nq + tab
    assert bench.stage_bytes("eval", N, L, H, W, nq) == 20 * nq + 4 * L * H * W
    assert bench.stage_bytes("cdf", N, L, H, W, nq) == 4 * L * H * W + tab + 8 * L
    assert bench.stage_bytes("hier", 50_000_000, 18595, 128, 128, 1) == 16 * 50_000_000 + 4 * 18596


def test_stratified_leaves():
    import numpy as np
    counts = np.array([5, 1, 9, 3, 7, 2, 8, 4, 6, 0])
    pick = bench.stratified_leaves(counts, 4)
    assert list(pick) == sorted(pick) and len(set(pick)) == 4
    assert counts[pick].min() == 0 and counts[pick].max() == 9       # both ends of the count order
    assert list(bench.stratified_leaves(counts, 20)) == list(range(10))
