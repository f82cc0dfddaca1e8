"""GPU tests of the phase-merged decoder convolutions (FP32 mode).  A 3x3
convolution of a nearest-upsampled input equals, for each output phase (row
and column parity), a 2x2 convolution of the low-resolution input whose taps
are sums of the 3x3 taps; the decoder layers use that form for their
upsampled channels.  Checked: the phase form against the nine-tap form
(option "upsample_taps9") to rounding, on the U-Net (whole-leaf tiles at the
deepest decoder level of 16x16 maps, a ragged leaf count, autotuned tiles)
and on the paper-style network; both against the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_2010_01775_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _energy(orc, seed, counts, H, W):
    rng = synth.rng_for(seed)
    L = len(counts)
    mus = synth.unit_vectors(rng, 2 * L).reshape(-1, 2, 3)
    dirs = np.concatenate([synth.two_lobe_mixture(rng, c, mus[i, 0], mus[i, 1]) for i, c in enumerate(counts)])
    w = synth.photon_weights(rng, dirs.shape[0])
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    rc, e, c = orc.splat(dirs, w, off, H, W)
    assert rc == 0
    return e, c


def _both(ctx, call):
    a = call()
    ctx.set_option("upsample_taps9", 1)
    try:
        b = call()
    finally:
        ctx.set_option("upsample_taps9", 0)
    return a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)


def _close(a, b, tol):
    """Relative on bins with b >= 1e-6 x (leaf max), absolute below: where a
    softplus output is tiny (very negative input), the rounding of the
    merged taps to float32 moves it by a larger relative amount."""
    L = b.shape[0]
    thr = np.broadcast_to(1e-6 * b.reshape(L, -1).max(1)[:, None, None], b.shape)
    big = b >= thr
    assert np.all(np.abs(a - b)[big] <= tol * b[big]), np.max(np.abs(a - b)[big] / b[big])
    assert np.all(np.abs(a - b)[~big] <= tol * thr[~big])


@pytest.mark.parametrize("H,W,L,tune", [(64, 64, 5, False), (16, 16, 6, False), (32, 64, 3, True)])
def test_unet_phase_form(ctx, npg, orc, H, W, L, tune):
    model = synth.unet_model(301 + H, random_bias=True)
    e, _ = _energy(orc, 302 + L, [4096] * (L - 1) + [333], H, W)
    m = npg.Model(ctx, model)
    if tune:
        npg.autotune(ctx, m, H, W, "fp32", probe_leaves=4)
    et = torch.from_numpy(e.view(np.int64)).to(DEV)
    a, b = _both(ctx, lambda: npg.reconstruct_density(ctx, m, et, "fp32"))
    assert npg.sync_status(ctx) == 0
    _close(a, b, 1e-5)          # the two forms differ by rounding only
    rc, s_ref = orc.net_forward(model, orc.normalize_input(e))
    assert rc == 0
    pr = s_ref / s_ref.reshape(L, -1).sum(1)[:, None, None]
    for s in (a, b):
        p = s / s.reshape(L, -1).sum(1)[:, None, None]
        assert np.max(np.abs(p - pr) / pr) < 1e-5
    m.free()


def test_paper_net_phase_form(ctx, npg, orc):
    H, W = 32, 64
    counts = [4096, 800, 4096, 50]
    e, c = _energy(orc, 310, counts, H, W)
    model = synth.paper_unet_model(311, random_bias=True)
    m = npg.Model(ctx, model)
    t64 = lambda x: torch.from_numpy(x.view(np.int64)).to(DEV)
    t32 = lambda x: torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).to(DEV)
    a, b = _both(ctx, lambda: npg.reconstruct_density5(ctx, m, t64(e), t32(c), t64(e), t32(c), "fp32"))
    assert npg.sync_status(ctx) == 0
    _close(a, b, 1e-5)
    rc, s_ref = orc.net_forward5(model, orc.input5(e, e, c, c))
    assert rc == 0
    thr = 1e-6 * s_ref.reshape(len(counts), -1).max(1)[:, None, None]
    big = s_ref >= thr
    assert np.max(np.abs(a - s_ref)[big] / s_ref[big]) < 1e-5
    m.free()
