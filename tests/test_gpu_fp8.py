"""GPU tests of the FP8 (OCP e4m3) network path: calibration, the stated
per-leaf L1 and KL error of the pdf against the FP64 oracle, and the
structural identities of the batched path (chunking, fused = separate,
graph replay, a leaf's result independent of its batch)."""
import numpy as np
import pytest
import torch

from paper_2010_01775_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(DEV)


def t64(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(DEV)


def tf(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _energy(ctx, npg, seed, L, H, per_leaf=4096, model=b""):
    b = synth.uniform_batch(seed=seed, L=L, per_leaf=per_leaf, H=H, W=H, n_queries=8, model=model)
    e, _ = npg.splat_histograms(ctx, tf(b.dirs), t32(b.w), t32(b.leaf_off), H, H, want_count=False)
    return b, e


def _calibrated(ctx, npg, model, H, seed=500, L=64):
    m = npg.Model(ctx, model)
    _, e = _energy(ctx, npg, seed, L, H)
    m.calibrate_fp8(e)
    return m


def _errors(s, s_ref):
    L = s.shape[0]
    p = s / s.reshape(L, -1).sum(1)[:, None, None]
    q = s_ref / s_ref.reshape(L, -1).sum(1)[:, None, None]
    l1 = np.abs(p - q).reshape(L, -1).sum(1)
    kl = (q * np.log(q / np.maximum(p, 1e-300))).reshape(L, -1).sum(1)
    return l1, kl


def test_fp8_needs_calibration(ctx, npg):
    m = npg.Model(ctx, synth.unet_model(3))
    e = torch.zeros((2, 64, 64), dtype=torch.int64, device=DEV)
    with pytest.raises(npg.NpgError) as ex:
        npg.reconstruct_density(ctx, m, e, "fp8")
    assert ex.value.code == npg.E_ARG
    with pytest.raises(npg.NpgError):
        m.calibrate_fp8(e[:0])                       # empty calibration batch
    m.free()


@pytest.mark.parametrize("L,H", [(8, 64), (4, 128), (3, 32)])
def test_unet_fp8_error_stated(ctx, npg, orc, L, H):
    """FP8 conv (calibrated on other leaves of the same distribution): per-leaf
    L1 and KL of the pdf against the FP64 oracle."""
    model = synth.unet_model(41)
    m = _calibrated(ctx, npg, model, H)
    b = synth.uniform_batch(seed=13, L=L, per_leaf=4096, H=H, W=H, n_queries=8, model=model)
    rc, e, _ = orc.splat(b.dirs, b.w, b.leaf_off, H, H)
    rc, s_ref = orc.net_forward(model, orc.normalize_input(e))
    s = npg.reconstruct_density(ctx, m, t64(e), "fp8").cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(s)) and np.all(s >= 0)
    # densities may underflow to zero only where the exact one is negligible
    tiny = s_ref < 1e-20 * s_ref.reshape(L, -1).max(1)[:, None, None]
    assert np.all(tiny[s == 0]), "zero density where the oracle's is not negligible"
    l1, kl = _errors(s, s_ref)
    print(f"fp8 {H}x{H}: L1 median {np.median(l1):.3e} max {l1.max():.3e}; "
          f"KL median {np.median(kl):.3e} max {kl.max():.3e}; {(s == 0).sum()} zero bins")
    assert l1.max() < 0.15 and kl.max() < 2e-2
    m.free()


def test_cnn_fp8_single_leaf(ctx, npg, orc):
    """The 3-layer CNN in FP8: the two-tap 16-channel tiles and the direct
    softplus layer reading e4m3 activations."""
    b = synth.single_leaf()
    m = npg.Model(ctx, b.model)
    _, ecal = _energy(ctx, npg, 501, 32, 32)
    m.calibrate_fp8(ecal)
    rc, e, _ = orc.splat(b.dirs, b.w, b.leaf_off, 32, 32)
    rc, s_ref = orc.net_forward(b.model, orc.normalize_input(e))
    s = npg.reconstruct_density(ctx, m, t64(e), "fp8").cpu().numpy().astype(np.float64)
    l1, kl = _errors(s, s_ref)
    print(f"cnn fp8: L1 {l1[0]:.3e} KL {kl[0]:.3e}")
    assert l1.max() < 0.1 and kl.max() < 1e-2
    m.free()


def test_fp8_calibration_deterministic_and_batch_independent(ctx, npg):
    model = synth.unet_model(8)
    m1 = _calibrated(ctx, npg, model, 64)
    m2 = _calibrated(ctx, npg, model, 64)
    _, e = _energy(ctx, npg, 12, 10, 64, per_leaf=1000)
    s1 = npg.reconstruct_density(ctx, m1, e, "fp8").cpu()
    s2 = npg.reconstruct_density(ctx, m2, e, "fp8").cpu()
    assert torch.equal(s1, s2)
    ctx.set_option("chunk_leaves", 3)
    try:
        s3 = npg.reconstruct_density(ctx, m1, e, "fp8").cpu()
    finally:
        ctx.set_option("chunk_leaves", 0)
    s4 = npg.reconstruct_density(ctx, m1, e[4:7].contiguous(), "fp8").cpu()
    assert torch.equal(s1, s3) and torch.equal(s1[4:7], s4)
    m1.free()
    m2.free()


def test_fp8_direct_path_close_to_tiled(ctx, npg):
    """The direct kernels (float weights, e4m3 activations) stay close to
    the tiled path (e4m3 weights)."""
    model = synth.unet_model(9)
    m = _calibrated(ctx, npg, model, 32)
    _, e = _energy(ctx, npg, 14, 4, 32)
    s = npg.reconstruct_density(ctx, m, e, "fp8").cpu().numpy().astype(np.float64)
    ctx.set_option("force_direct", 1)
    try:
        sd = npg.reconstruct_density(ctx, m, e, "fp8").cpu().numpy().astype(np.float64)
    finally:
        ctx.set_option("force_direct", 0)
    l1, _ = _errors(s, sd)
    print(f"fp8 tiled vs direct L1 max {l1.max():.3e}")
    assert l1.max() < 0.15
    m.free()


def test_fp8_fused_equals_separate_and_graph_replay(npg):
    ctx = npg.Context(0)
    model = synth.unet_model(3, random_bias=True)
    m = _calibrated(ctx, npg, model, 64)
    counts = [3000, 12, 0, 5000, 800, 70000, 1]
    rng = synth.rng_for(77)
    mus = synth.unit_vectors(rng, 2 * len(counts)).reshape(-1, 2, 3)
    dirs = np.concatenate([synth.two_lobe_mixture(rng, c, mus[i, 0], mus[i, 1]) if c else np.zeros((0, 3), np.float32)
                           for i, c in enumerate(counts)])
    w = synth.photon_weights(rng, dirs.shape[0])
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    d, ww, o = tf(dirs), t32(w), t32(off)
    e, _ = npg.splat_histograms(ctx, d, ww, o, 64, 64, want_count=False)
    ref = npg.build_cdf(ctx, npg.reconstruct_density(ctx, m, e, "fp8"))
    got = npg.reconstruct_fused(ctx, m, d, ww, o, 64, 64, "fp8")
    same = lambda a, b: all(torch.equal(x, y) for x, y in ((a.pdf, b.pdf), (a.marg, b.marg), (a.cond, b.cond)))
    assert same(ref, got)
    ctx.set_option("graphs", 1)
    s = torch.cuda.Stream()
    out = npg._new_tables(len(counts), 64, 64, DEV)
    for rep in range(3):
        out.pdf.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            npg.reconstruct_fused(ctx, m, d, ww, o, 64, 64, "fp8", out=out, stream=s)
        s.synchronize()
        assert same(ref, out), f"replay {rep}"
    m.free()
    ctx.close()
