"""GPU tests of the batched form of the path (fused splat -> network -> CDF,
HIP-graph replay, autotuned tiles) and of the clustered workload at full
size against the oracle on sampled leaves."""
import math

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


def _ragged(seed, counts):
    rng = synth.rng_for(seed)
    L = len(counts)
    mus = synth.unit_vectors(rng, 2 * L).reshape(L, 2, 3)
    dirs = np.concatenate([synth.two_lobe_mixture(rng, c, mus[i, 0], mus[i, 1]) if c else np.zeros((0, 3), np.float32)
                           for i, c in enumerate(counts)])
    w = synth.photon_weights(rng, dirs.shape[0])
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    return dirs, w, off


def _separate(npg, ctx, m, dirs, w, off, H, W, prec, perm=None):
    e, _ = npg.splat_histograms(ctx, dirs, w, off, H, W, perm=perm, want_count=False)
    s = npg.reconstruct_density(ctx, m, e, prec)
    return npg.build_cdf(ctx, s)


def _same(a, b):
    return all(torch.equal(x, y) for x, y in ((a.pdf, b.pdf), (a.marg, b.marg), (a.cond, b.cond), (a.total, b.total)))


@pytest.mark.parametrize("prec,H", [("fp32", 64), ("bf16", 64), ("bf16", 32), ("fp32", 16)])
def test_fused_equals_separate(ctx, npg, prec, H):
    counts = [4096, 0, 17, 33000, 900, 4096, 1, 2500, 70000]
    dirs, w, off = _ragged(H + len(prec), counts)
    perm = np.random.default_rng(0).permutation(len(w)).astype(np.uint32)
    m = npg.Model(ctx, synth.unet_model(3, random_bias=True))
    d, ww, o, p = tf(dirs), t32(w), t32(off), t32(perm)
    ref = _separate(npg, ctx, m, d, ww, o, H, H, prec, perm=p)
    got = npg.reconstruct_fused(ctx, m, d, ww, o, H, H, prec, perm=p)
    assert npg.sync_status(ctx) == 0
    assert _same(ref, got)
    ctx.set_option("chunk_leaves", 2)
    try:
        got2 = npg.reconstruct_fused(ctx, m, d, ww, o, H, H, prec, perm=p)
    finally:
        ctx.set_option("chunk_leaves", 0)
    assert _same(ref, got2)
    m.free()


def test_fused_cnn_single_leaf(ctx, npg, orc):
    b = synth.single_leaf()
    ref = orc.pipeline(b)
    m = npg.Model(ctx, b.model)
    t = npg.reconstruct_fused(ctx, m, tf(b.dirs), t32(b.w), t32(b.leaf_off), b.H, b.W, "fp32")
    rel = np.abs(t.pdf.cpu().numpy() - ref["pdf"]) / ref["pdf"]
    assert rel.max() < 1e-5
    m.free()


def test_fused_graph_replay(npg):
    """Captured and replayed calls equal the eager result on every replay,
    with the program's own eager work and synchronisations in between."""
    ctx = npg.Context(0)
    ctx.set_option("graphs", 1)
    counts = [3000, 12, 0, 5000, 800] * 3
    dirs, w, off = _ragged(5, counts)
    m = npg.Model(ctx, synth.unet_model(4))
    d, ww, o = tf(dirs), t32(w), t32(off)
    ref = _separate(npg, ctx, m, d, ww, o, 64, 64, "bf16")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    L = len(counts)
    out = npg._new_tables(L, 64, 64, DEV)
    for rep in range(5):
        for x in (out.pdf, out.marg, out.cond):
            x.fill_(float("nan"))
        out.total.fill_(-1.0)
        junk = torch.randn(1 << 20, device=DEV)      # unrelated eager work
        junk.mul_(2.0).sum().item()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            npg.reconstruct_fused(ctx, m, d, ww, o, 64, 64, "bf16", out=out, stream=s)
        s.synchronize()
        assert _same(ref, out), f"replay {rep} differs"
    assert npg.sync_status(ctx, stream=s) == 0
    m.free()
    ctx.close()


def test_autotune_keeps_results(ctx, npg):
    model = synth.unet_model(6)
    m = npg.Model(ctx, model)
    b = synth.uniform_batch(seed=7, L=40, per_leaf=1000, H=64, W=64, n_queries=8, model=model)
    e, _ = npg.splat_histograms(ctx, tf(b.dirs), t32(b.w), t32(b.leaf_off), 64, 64)
    before = {p: npg.reconstruct_density(ctx, m, e, p).clone() for p in ("fp32", "bf16")}
    for p in ("fp32", "bf16"):
        tab = npg.autotune(ctx, m, 64, 64, p, probe_leaves=128)
        assert tab and tab[0] in (64, 128) and all(c in (1, 2, 4, 8) for c in tab[1:]), tab
        assert torch.equal(before[p], npg.reconstruct_density(ctx, m, e, p))
    m.free()


def test_clustered_full_size_sampled_leaves(ctx, npg, orc, clustered):
    """5e7 clustered photons, octree (split > 8192, depth <= 6), 128x128 maps,
    U-Net FP32 through the fused path as the benchmark launches it; tables of
    sampled leaves (smallest, median, largest, random) against the oracle."""
    cp = clustered
    pos, dirs, w = tf(cp.pos), tf(cp.dirs), t32(cp.w)
    hier = npg.build_hierarchy(ctx, pos, 8192, 6, max_leaves=65536)
    L = hier["n_leaves"]
    model = synth.unet_model(1002)
    m = npg.Model(ctx, model)
    t = npg.reconstruct_fused(ctx, m, dirs, w, hier["leaf_off"], 128, 128, "fp32", perm=hier["perm"])
    assert npg.sync_status(ctx) == 0
    off = hier["leaf_off"].cpu().numpy().view(np.uint32).astype(np.int64)
    perm = hier["perm"].cpu().numpy().view(np.uint32)
    cnt = np.diff(off)
    rng = np.random.default_rng(0)
    pick = sorted({int(np.argmin(cnt)), int(np.argmax(cnt)), int(np.argsort(cnt)[L // 2]),
                   *rng.integers(0, L, 3).tolist()})
    sel = np.concatenate([perm[off[l]:off[l + 1]] for l in pick])
    soff = np.concatenate([[0], np.cumsum(cnt[pick])]).astype(np.uint32)
    rc, e_ref, _ = orc.splat(cp.dirs[sel], cp.w[sel], soff, 128, 128)
    rc, s_ref = orc.net_forward(model, orc.normalize_input(e_ref))
    rc, pdf_ref, marg_ref, cond_ref, tot_ref = orc.build_cdf(s_ref)
    pdf = t.pdf.cpu().numpy()[pick].astype(np.float64)
    pr = pdf_ref.astype(np.float64)
    # 1e-5 relative on bins with p >= 1e-6 * (leaf max); below that (spiky
    # leaves push some densities to float underflow) 1e-5 of that threshold
    thr = 1e-6 * pr.reshape(len(pick), -1).max(1)[:, None, None]
    big = pr >= thr
    rel = np.abs(pdf - pr)[big] / pr[big]
    small_err = (np.abs(pdf - pr) / thr)[~big]
    print(f"leaves {L}, sampled {pick} counts {cnt[pick].tolist()}, max rel pdf err {rel.max():.2e} "
          f"on {big.sum()} bins; {(~big).sum()} bins below 1e-6 max, max err/threshold "
          f"{small_err.max() if small_err.size else 0:.2e}")
    assert rel.max() < 1e-5
    assert small_err.size == 0 or small_err.max() < 1e-5
    m.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("H,L,arch", [(64, 37, "unet"), (16, 21, "unet"), (128, 5, "unet"), (8, 13, "unet"),
                                      (32, 9, "cnn")])
def test_fused_first_layer_equals_separate(ctx, npg, prec, H, L, arch):
    """The first layer computed inside the second layer's patch staging gives
    the same bits as the stored first-layer activations."""
    model = synth.unet_model(21, random_bias=True) if arch == "unet" else synth.cnn_model(22)
    m = npg.Model(ctx, model)
    b = synth.uniform_batch(seed=31 + H, L=L, per_leaf=3000, H=H, W=H, n_queries=8, model=b"")
    e, _ = npg.splat_histograms(ctx, tf(b.dirs), t32(b.w), t32(b.leaf_off), H, H, want_count=False)
    e[L // 2].zero_()                                # an empty leaf
    if prec == "fp8":
        m.calibrate_fp8(e)
    ctx.set_option("fuse_first", 0)
    try:
        ref = npg.reconstruct_density(ctx, m, e, prec).cpu()
    finally:
        ctx.set_option("fuse_first", 1)
    got = npg.reconstruct_density(ctx, m, e, prec).cpu()
    assert npg.sync_status(ctx) == 0
    assert torch.equal(ref, got)
    m.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("H,L", [(64, 37), (16, 21), (128, 5), (8, 13)])
def test_pooled_outputs_equal_pooled_staging(ctx, npg, prec, H, L):
    """The 2x2 means an encoder level stores beside its output give the next
    level the same bits as pooling that output while staging it (ragged last
    tile, an empty leaf, maps small enough for whole-leaf tiles and for the
    direct path at the deepest levels)."""
    m = npg.Model(ctx, synth.unet_model(23, random_bias=True))
    b = synth.uniform_batch(seed=41 + H, L=L, per_leaf=3000, H=H, W=H, n_queries=8, model=b"")
    e, _ = npg.splat_histograms(ctx, tf(b.dirs), t32(b.w), t32(b.leaf_off), H, H, want_count=False)
    e[L // 3].zero_()
    if prec == "fp8":
        m.calibrate_fp8(e)
    ctx.set_option("pool_outputs", 0)
    try:
        ref = npg.reconstruct_density(ctx, m, e, prec).cpu()
    finally:
        ctx.set_option("pool_outputs", 1)
    got = npg.reconstruct_density(ctx, m, e, prec).cpu()
    assert npg.sync_status(ctx) == 0
    assert torch.equal(ref, got)
    m.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("H,L", [(128, 5), (64, 23), (16, 21)])
def test_every_tile_width_gives_same_bits(ctx, npg, prec, H, L):
    """Every matrix-core tile width (option "tile_cap": at most 64, 128, 256
    or 512 output pixels) gives the bits of the default tiles: in FP32 mode
    the weight ring of 2 or 4 K steps with its peeled last taps, the patch
    staged through registers (one pixel per thread) or straight into LDS,
    the phase-merged decoder tiles and the fused first layer; ragged last
    tile and an empty leaf."""
    m = npg.Model(ctx, synth.unet_model(24, random_bias=True))
    b = synth.uniform_batch(seed=51 + H, L=L, per_leaf=3000, H=H, W=H, n_queries=8, model=b"")
    e, _ = npg.splat_histograms(ctx, tf(b.dirs), t32(b.w), t32(b.leaf_off), H, H, want_count=False)
    e[L // 2].zero_()
    if prec == "fp8":
        m.calibrate_fp8(e)
    ref = npg.reconstruct_density(ctx, m, e, prec).cpu()
    try:
        for cap in (1, 2, 8):
            ctx.set_option("tile_cap", cap)
            got = npg.reconstruct_density(ctx, m, e, prec).cpu()
            assert npg.sync_status(ctx) == 0
            assert torch.equal(ref, got), cap
    finally:
        ctx.set_option("tile_cap", 4)
    m.free()


def test_options_checked(ctx, npg):
    """Context tunables: every documented name is accepted; an unknown name
    or a negative value is an argument error."""
    for name, value in (("graphs", 0), ("chunk_leaves", 0), ("force_direct", 0), ("fuse_first", 1),
                        ("upsample_taps9", 0), ("pool_outputs", 1), ("tile_cap", 4)):
        ctx.set_option(name, value)
    for name, value in (("tile_size", 4), ("tile_cap", -1), ("", 1)):
        with pytest.raises(npg.NpgError) as ei:
            ctx.set_option(name, value)
        assert ei.value.code == npg.E_ARG, (name, value)
