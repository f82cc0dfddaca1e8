"""GPU tests of the five-channel network (npg_reconstruct_density5): the
maps and photon counts of iterations t and t-1 and the valid-bin mask feed a
masked first layer; FP32 densities within 1e-5 of the FP64 oracle, BF16 error
stated, results independent of chunking, and the one-/five-channel entry
points reject each other's models."""
import numpy as np
import pytest
import torch

from paper_2010_01775_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(DEV)


def tf(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _iterations(seed, counts, H):
    """Photons of iteration t; iteration t-1 saw the first half of each
    leaf's photons (photon maps accumulate over iterations)."""
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
    return (dirs, w, off), (dirs[keep], w[keep], off_p)


def _maps(orc, it, H):
    rc, e, c = orc.splat(*it, H, H)
    assert rc == 0
    return e, c


def _dev_maps(e, c):
    return torch.from_numpy(e.view(np.int64)).to(DEV), t32(c)


@pytest.mark.parametrize("H,levels", [(32, (16, 32, 64, 128)), (16, (8, 16))])
def test_density5_fp32_parity(ctx, npg, orc, H, levels):
    counts = [3000, 40, 0, 1500, 7, 2200]            # an empty leaf, sparse leaves
    cur, prev = _iterations(90 + H, counts, H)
    e_t, p_t = _maps(orc, cur, H)
    e_p, p_p = _maps(orc, prev, H)
    model = synth.unet5_model(91, levels, random_bias=True)
    rc, s_ref = orc.net_forward5(model, orc.input5(e_t, e_p, p_t, p_p))
    assert rc == 0
    m = npg.Model(ctx, model)
    s = npg.reconstruct_density5(ctx, m, *_dev_maps(e_t, p_t), *_dev_maps(e_p, p_p), "fp32").cpu().numpy()
    assert npg.sync_status(ctx) == 0
    rel = np.abs(s - s_ref) / np.abs(s_ref)
    assert rel.max() < 1e-5, rel.max()
    m.free()


def test_density5_bf16_error_and_chunking(ctx, npg, orc):
    H = 32
    counts = [4096] * 6 + [90, 600]
    cur, prev = _iterations(95, counts, H)
    e_t, p_t = _maps(orc, cur, H)
    e_p, p_p = _maps(orc, prev, H)
    model = synth.unet5_model(96, random_bias=True)
    rc, s_ref = orc.net_forward5(model, orc.input5(e_t, e_p, p_t, p_p))
    m = npg.Model(ctx, model)
    args = (*_dev_maps(e_t, p_t), *_dev_maps(e_p, p_p))
    s = npg.reconstruct_density5(ctx, m, *args, "bf16")
    p = s.cpu().numpy().astype(np.float64)
    L = len(counts)
    pn = p / p.reshape(L, -1).sum(1)[:, None, None]
    qn = s_ref / s_ref.reshape(L, -1).sum(1)[:, None, None]
    l1 = np.abs(pn - qn).reshape(L, -1).sum(1)
    print(f"five-channel bf16 L1 median {np.median(l1):.3e} max {l1.max():.3e}")
    assert l1.max() < 5e-2
    for prec in ("fp32", "bf16"):
        full = npg.reconstruct_density5(ctx, m, *args, prec)
        ctx.set_option("chunk_leaves", 3)
        try:
            part = npg.reconstruct_density5(ctx, m, *args, prec)
        finally:
            ctx.set_option("chunk_leaves", 0)
        assert torch.equal(full, part), prec
        # autotuned tiles and chunk size change no result
        npg.autotune(ctx, m, H, H, prec, probe_leaves=4)
        assert torch.equal(full, npg.reconstruct_density5(ctx, m, *args, prec)), prec
    assert npg.sync_status(ctx) == 0
    m.free()


def test_density5_rejections(ctx, npg):
    H = 16
    e = torch.zeros((2, H, H), dtype=torch.int64, device=DEV)
    c = torch.zeros((2, H, H), dtype=torch.int32, device=DEV)
    m5 = npg.Model(ctx, synth.unet5_model(97, (8, 16)))
    m1 = npg.Model(ctx, synth.unet_model(98, (8, 16)))
    for call in (lambda: npg.reconstruct_density5(ctx, m1, e, c, e, c, "fp32"),
                 lambda: npg.reconstruct_density(ctx, m5, e, "fp32"),
                 lambda: npg.reconstruct_density5(ctx, m5, e, c, e, c, "fp8"),
                 lambda: npg.autotune(ctx, m5, H, H, "fp8", probe_leaves=2),
                 lambda: m5.calibrate_fp8(e)):
        with pytest.raises(npg.NpgError) as ex:
            call()
        assert ex.value.code == npg.E_ARG
    assert npg.sync_status(ctx) == 0
    m5.free()
    m1.free()
