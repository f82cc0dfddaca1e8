"""npg_reconstruct_density_noalloc through the C-ABI: the same densities as
npg_reconstruct_density (bit for bit) on two calls in a row, the second with
a smaller input, with no device memory allocated by the call; a map size whose
one leaf does not fit the static array is rejected."""
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


def _energy(npg, ctx, seed, L, H):
    b = synth.uniform_batch(seed=seed, L=L, per_leaf=3000, H=H, W=H, n_queries=8, model=b"")
    e, _ = npg.splat_histograms(ctx, tf(b.dirs), t32(b.w), t32(b.leaf_off), H, H, want_count=False)
    e[L // 3].zero_()                                   # an empty leaf
    return e


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_equals_reconstruct(npg, prec):
    ctx = npg.Context(0)                                # fresh: its memory accounting starts here
    m = npg.Model(ctx, synth.unet_model(31, random_bias=True))
    # 128x128 in FP32 mode needs ~7.5 MB of activations per leaf: 90 leaves
    # take several chunks of the 255 MiB array; then a smaller call at 64x64
    cases = [(_energy(npg, ctx, 51, 90, 128), 128), (_energy(npg, ctx, 52, 7, 64), 64)]
    outs = [torch.full(e.shape, float("nan"), device=DEV) for e, _ in cases]
    torch.cuda.synchronize()
    held0 = ctx.memory_usage()
    for (e, H), out in zip(cases, outs):
        npg.reconstruct_density_noalloc(ctx, m, e, prec, density=out)
    assert npg.sync_status(ctx) == 0
    assert ctx.memory_usage() == held0, "the no-allocation call grew the library's device memory"
    # again after a warm-up, against the device's free memory
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for (e, H), out in zip(cases, outs):
        npg.reconstruct_density_noalloc(ctx, m, e, prec, density=out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    for (e, H), out in zip(cases, outs):
        ref = npg.reconstruct_density(ctx, m, e, prec)
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref), f"{prec} {tuple(e.shape)} differs from reconstruct_density"
    assert npg.sync_status(ctx) == 0
    m.free()
    ctx.close()


def test_noalloc_rejects_leaf_beyond_array(npg, ctx):
    m = npg.Model(ctx, synth.unet_model(32))
    e = torch.zeros((1, 1024, 1024), dtype=torch.int64, device=DEV)   # ~480 MB of FP32-mode activations
    with pytest.raises(npg.NpgError) as ex:
        npg.reconstruct_density_noalloc(ctx, m, e, "fp32")
    assert ex.value.code == npg.E_BUDGET
    assert npg.sync_status(ctx) == 0
    m.free()
