"""GPU tests of the paper-style U-Net (five-channel masked first layer, ELU,
residual links, dilated bottleneck) through npg_reconstruct_density5:
FP32 densities within 1e-5 of the FP64 oracle on the tiled path and on the
direct path, at square maps and at the paper's 32x64 and 64x128 shapes (bins that
underflow float32 compared in absolute terms); BF16 error
stated; results independent of chunking and of autotuned tiles; FP8
rejected."""
import numpy as np
import pytest
import torch

from paper_2010_01775_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _maps(orc, seed, counts, H, W):
    """Maps of iterations t and t-1 (the first half of each leaf's photons)."""
    rng = synth.rng_for(seed)
    L = len(counts)
    mus = synth.unit_vectors(rng, 2 * L).reshape(-1, 2, 3)
    dirs = np.concatenate([synth.two_lobe_mixture(rng, c, mus[i, 0], mus[i, 1]) if c else
                           np.zeros((0, 3), np.float32) for i, c in enumerate(counts)])
    w = synth.photon_weights(rng, dirs.shape[0])
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    half = np.array(counts) // 2
    keep = np.concatenate([np.arange(off[i], off[i] + half[i]) for i in range(L)]).astype(np.int64)
    off_p = np.concatenate([[0], np.cumsum(half)]).astype(np.uint32)
    rc, e_t, p_t = orc.splat(dirs, w, off, H, W)
    rc2, e_p, p_p = orc.splat(dirs[keep], w[keep], off_p, H, W)
    assert rc == 0 and rc2 == 0
    return e_t, p_t, e_p, p_p


def _dev(e_t, p_t, e_p, p_p):
    t64 = lambda a: torch.from_numpy(a.view(np.int64)).to(DEV)
    t32 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(DEV)
    return t64(e_t), t32(p_t), t64(e_p), t32(p_p)


@pytest.mark.parametrize("H,W,levels,direct", [(32, 32, (16, 32, 64), False), (32, 64, (16, 32, 64), False),
                                              (64, 128, (16, 32, 64), False), (16, 16, (8, 16), False),
                                              (32, 64, (16, 32, 64), True)])
def test_paper_net_fp32_parity(ctx, npg, orc, H, W, levels, direct):
    counts = [3000, 40, 0, 1500, 7, 2200]
    maps = _maps(orc, 100 + H + W, counts, H, W)
    model = synth.paper_unet_model(101, levels, random_bias=True)
    rc, s_ref = orc.net_forward5(model, orc.input5(maps[0], maps[2], maps[1], maps[3]))
    assert rc == 0
    m = npg.Model(ctx, model)
    if direct:
        ctx.set_option("force_direct", 1)
    try:
        s = npg.reconstruct_density5(ctx, m, *_dev(*maps), "fp32").cpu().numpy()
    finally:
        ctx.set_option("force_direct", 0)
    assert npg.sync_status(ctx) == 0
    _check_fp32(s, s_ref)
    m.free()


def _check_fp32(s, s_ref):
    """1e-5 relative error on every bin with p >= 1e-6 * (leaf max); below
    that, 1e-5 of the threshold, absolute.  The sparse leaves drive some
    densities to 1e-40..1e-100 (softplus of very negative inputs), where the
    float32 output underflows to subnormals or zero."""
    L = s.shape[0]
    thr = np.broadcast_to(1e-6 * s_ref.reshape(L, -1).max(1)[:, None, None], s.shape)
    big = s_ref >= thr
    rel = np.abs(s - s_ref)[big] / s_ref[big]
    assert rel.max() < 1e-5, rel.max()
    assert np.all(np.abs(s - s_ref)[~big] <= 1e-5 * thr[~big])


def test_paper_net_bf16_chunking_autotune(ctx, npg, orc):
    H, W = 32, 64
    counts = [4096] * 6 + [90, 600]
    maps = _maps(orc, 120, counts, H, W)
    model = synth.paper_unet_model(121, random_bias=True)
    rc, s_ref = orc.net_forward5(model, orc.input5(maps[0], maps[2], maps[1], maps[3]))
    m = npg.Model(ctx, model)
    args = _dev(*maps)
    p = npg.reconstruct_density5(ctx, m, *args, "bf16").cpu().numpy().astype(np.float64)
    L = len(counts)
    pn = p / p.reshape(L, -1).sum(1)[:, None, None]
    qn = s_ref / s_ref.reshape(L, -1).sum(1)[:, None, None]
    l1 = np.abs(pn - qn).reshape(L, -1).sum(1)
    print(f"paper-style net bf16 L1 median {np.median(l1):.3e} max {l1.max():.3e}")
    assert l1.max() < 5e-2
    for prec in ("fp32", "bf16"):
        full = npg.reconstruct_density5(ctx, m, *args, prec)
        ctx.set_option("chunk_leaves", 3)
        try:
            part = npg.reconstruct_density5(ctx, m, *args, prec)
        finally:
            ctx.set_option("chunk_leaves", 0)
        assert torch.equal(full, part), prec
        npg.autotune(ctx, m, H, W, prec, probe_leaves=4)
        assert torch.equal(full, npg.reconstruct_density5(ctx, m, *args, prec)), prec
    assert npg.sync_status(ctx) == 0
    m.free()


def test_paper_net_rejections(ctx, npg):
    H = 16
    e = torch.zeros((2, H, H), dtype=torch.int64, device=DEV)
    c = torch.zeros((2, H, H), dtype=torch.int32, device=DEV)
    m = npg.Model(ctx, synth.paper_unet_model(122, (8, 16)))
    for call in (lambda: npg.reconstruct_density5(ctx, m, e, c, e, c, "fp8"),
                 lambda: npg.reconstruct_density(ctx, m, e, "fp32"),
                 lambda: m.calibrate_fp8(e),
                 lambda: npg.reconstruct_density5(ctx, m, e[:, :, :12].contiguous(), c[:, :, :12].contiguous(),
                                                  e[:, :, :12].contiguous(), c[:, :, :12].contiguous(), "fp32")):
        with pytest.raises(npg.NpgError) as ex:
            call()
        assert ex.value.code == npg.E_ARG
    assert npg.sync_status(ctx) == 0
    m.free()


@pytest.mark.parametrize("paper", [False, True])
def test_five_channel_full_size_sampled(ctx, npg, orc, paper):
    """The uniform-batch workload (1024 leaves x 4096 photons, 64x64) in the
    launch configuration bench.py times (autotuned tiles, default chunking):
    iteration t-1 = the first half of each leaf's photons; the maps of both
    iterations bit-exact on every leaf, the densities of sampled leaves
    against the oracle run on those leaves alone."""
    b = synth.uniform_batch()
    L, H, W = b.L, b.H, b.W
    off = b.leaf_off.astype(np.int64)
    half = (off[1:] - off[:-1]) // 2
    perm_p = np.concatenate([np.arange(off[l], off[l] + half[l]) for l in range(L)]).astype(np.uint32)
    off_p = np.concatenate([[0], np.cumsum(half)]).astype(np.uint32)
    tf = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)
    t32 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(DEV)
    e_t, p_t = npg.splat_histograms(ctx, tf(b.dirs), t32(b.w), t32(b.leaf_off), H, W)
    e_p, p_p = npg.splat_histograms(ctx, tf(b.dirs), t32(b.w), t32(off_p), H, W, perm=t32(perm_p))
    rc, e_ref, c_ref = orc.splat(b.dirs, b.w, b.leaf_off, H, W)
    rc2, ep_ref, cp_ref = orc.splat(b.dirs, b.w, off_p, H, W, perm=perm_p)
    assert rc == 0 and rc2 == 0
    assert np.array_equal(e_t.cpu().numpy().view(np.uint64), e_ref)
    assert np.array_equal(p_t.cpu().numpy().view(np.uint32), c_ref)
    assert np.array_equal(e_p.cpu().numpy().view(np.uint64), ep_ref)
    assert np.array_equal(p_p.cpu().numpy().view(np.uint32), cp_ref)
    model = synth.paper_unet_model(1006) if paper else synth.unet5_model(1003)
    m = npg.Model(ctx, model)
    npg.autotune(ctx, m, H, W, "fp32", probe_leaves=1024)
    s = npg.reconstruct_density5(ctx, m, e_t, p_t, e_p, p_p, "fp32").cpu().numpy()
    assert npg.sync_status(ctx) == 0
    pick = np.array([0, 1, 200, 511, 512, 777, 900, 1023])
    rc, s_ref = orc.net_forward5(model, orc.input5(e_ref[pick], ep_ref[pick], c_ref[pick], cp_ref[pick]))
    assert rc == 0
    _check_fp32(s[pick], s_ref)
    m.free()
