"""GPU tests of the mixture of experts by leaf photon count
(npg_reconstruct_experts) against the oracle and against the single-network
path: routing counts exact, FP32 densities within the FP32 tolerance of the
FP64 oracle of each leaf's own expert, and every precision bit-identical to
running each expert's leaves through npg_reconstruct_density alone."""
import math

import numpy as np
import pytest
import torch

from paper_2010_01775_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BOUNDS = (100, 500, 1000, 5000)
# counts at, below and above every boundary of the paper's ranges, an empty leaf
COUNTS = [0, 37, 99, 100, 250, 499, 500, 750, 999, 1000, 2500, 4999, 5000, 9000, 64]


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(DEV)


def tf(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _batch(seed, counts, H):
    rng = synth.rng_for(seed)
    L = len(counts)
    mus = synth.unit_vectors(rng, 2 * L).reshape(-1, 2, 3)
    dirs = np.concatenate([synth.two_lobe_mixture(rng, c, mus[i, 0], mus[i, 1]) if c else
                           np.zeros((0, 3), np.float32) for i, c in enumerate(counts)])
    w = synth.photon_weights(rng, dirs.shape[0])
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    return dirs, w, off


def _pdf(s):
    s = s.astype(np.float64)
    L, H, W = s.shape
    return s / s.reshape(L, -1).sum(1)[:, None, None] * H * W / (4 * math.pi)


def _models(npg, ctx, arch="unet"):
    raw = [synth.unet_model(60 + k, random_bias=True) if arch == "unet" else synth.cnn_model(70 + k, random_bias=True)
           for k in range(5)]
    return raw, [npg.Model(ctx, r) for r in raw]


@pytest.mark.parametrize("arch,H", [("unet", 32), ("cnn", 16)])
def test_experts_fp32_parity(ctx, npg, orc, arch, H):
    dirs, w, off = _batch(81, COUNTS, H)
    rc, e, _ = orc.splat(dirs, w, off, H, H)
    assert rc == 0
    raw, models = _models(npg, ctx, arch)
    photons = np.diff(off.astype(np.int64))
    rc, s_ref = orc.experts_forward(raw, photons, BOUNDS, orc.normalize_input(e))
    assert rc == 0
    e_dev = torch.from_numpy(e.view(np.int64)).to(DEV)
    s, counts = npg.reconstruct_experts(ctx, models, t32(off), e_dev, "fp32", BOUNDS)
    assert npg.sync_status(ctx) == 0
    want = np.bincount(orc.expert_of(photons, BOUNDS), minlength=5)
    assert counts == want.tolist()
    s = s.cpu().numpy()
    nz = photons > 0                                   # the empty leaf has no pdf
    p, p_ref = _pdf(s[nz]), _pdf(s_ref[nz])
    rel = np.abs(p - p_ref) / p_ref
    assert rel.max() < 1e-5, rel.max()
    assert np.all(s[~nz] > 0)
    for m in models:
        m.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_experts_equal_separate_runs(ctx, npg, prec):
    """Each leaf's density is, bit for bit, that of its expert's network run
    on that expert's leaves alone (and expert 0 on all leaves if the bounds
    send every leaf there)."""
    H = 32
    dirs, w, off = _batch(82, COUNTS * 2, H)
    e, _ = npg.splat_histograms(ctx, tf(dirs), t32(w), t32(off), H, H, want_count=False)
    raw, models = _models(npg, ctx)
    if prec == "fp8":
        for m in models:
            m.calibrate_fp8(e)
    s, counts = npg.reconstruct_experts(ctx, models, t32(off), e, prec, BOUNDS)
    photons = np.diff(off.astype(np.int64))
    idx = np.searchsorted(np.array(BOUNDS), photons, side="right")
    for k, m in enumerate(models):
        sel = torch.from_numpy(np.nonzero(idx == k)[0]).to(DEV)
        assert counts[k] == sel.numel()
        ref = npg.reconstruct_density(ctx, m, e[sel].contiguous(), prec)
        assert torch.equal(s[sel], ref), k
    s1, c1 = npg.reconstruct_experts(ctx, models[:1], t32(off), e, prec, ())
    assert c1 == [len(photons)]
    assert torch.equal(s1, npg.reconstruct_density(ctx, models[0], e, prec))
    assert npg.sync_status(ctx) == 0
    for m in models:
        m.free()


def test_experts_gather_batches(ctx, npg):
    """Gather batches of a few leaves (the chunk_leaves option bounds them)
    give the same bits as whole-expert batches."""
    H = 16
    dirs, w, off = _batch(83, COUNTS * 3, H)
    e, _ = npg.splat_histograms(ctx, tf(dirs), t32(w), t32(off), H, H, want_count=False)
    raw, models = _models(npg, ctx, "cnn")
    s, counts = npg.reconstruct_experts(ctx, models, t32(off), e, "fp32", BOUNDS)
    ctx.set_option("chunk_leaves", 4)
    try:
        s2, counts2 = npg.reconstruct_experts(ctx, models, t32(off), e, "fp32", BOUNDS)
    finally:
        ctx.set_option("chunk_leaves", 0)
    assert counts == counts2 and torch.equal(s, s2)
    for m in models:
        m.free()


def test_experts_errors(ctx, npg):
    H = 16
    dirs, w, off = _batch(84, [300, 2000], H)
    e, _ = npg.splat_histograms(ctx, tf(dirs), t32(w), t32(off), H, H, want_count=False)
    raw, models = _models(npg, ctx, "cnn")
    for bad in [(100, 100, 1000, 5000), (500, 100, 1000, 5000)]:
        with pytest.raises(npg.NpgError) as ex:
            npg.reconstruct_experts(ctx, models, t32(off), e, "fp32", bad)
        assert ex.value.code == npg.E_ARG
    with pytest.raises(npg.NpgError) as ex:
        npg.reconstruct_experts(ctx, [], t32(off), e, "fp32", ())
    assert ex.value.code == npg.E_ARG
    with pytest.raises(npg.NpgError) as ex:                       # uncalibrated FP8 expert
        npg.reconstruct_experts(ctx, models, t32(off), e, "fp8", BOUNDS)
    assert ex.value.code == npg.E_ARG
    assert npg.sync_status(ctx) == 0
    for m in models:
        m.free()
