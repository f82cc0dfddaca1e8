"""GPU tests of the continuous-batching server: every request's result is
the same alone and in a mix of overlapping, merged batches; admission by the
table budget in FIFO order; served sampling equals direct sampling."""
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


@pytest.fixture(scope="module")
def pool():
    """A pool of photons; requests address per-leaf windows of it."""
    b = synth.uniform_batch(seed=77, L=256, per_leaf=4096, H=64, W=64, n_queries=8, model=b"")
    return tf(b.dirs), t32(b.w), b.dirs.shape[0]


def _request(seed, n_pool, L, lo=256, hi=20000):
    rng = np.random.default_rng(seed)
    cnt = rng.integers(lo, hi, L).astype(np.uint32)
    beg = np.array([rng.integers(0, n_pool - c) for c in cnt], np.uint32)
    return beg, cnt


def _tables(npg, L, H, W):
    return npg._new_tables(L, H, W, DEV)


def _alone(npg, srv, dirs, w, beg, cnt, H):
    t = srv.submit_recon(dirs, w, beg, cnt, H, H)
    srv.wait(t)
    out = srv.copy_tables(t, _tables(npg, len(beg), H, H))
    torch.cuda.synchronize()
    srv.release(t)
    return out


def _same(a, b):
    return all(torch.equal(x, y) for x, y in ((a.pdf, b.pdf), (a.marg, b.marg), (a.cond, b.cond), (a.total, b.total)))


@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp8"])
def test_alone_equals_mix(ctx, npg, pool, prec):
    dirs, w, n_pool = pool
    m = npg.Model(ctx, synth.unet_model(9, random_bias=True))
    if prec == "fp8":
        for H in (64, 128):   # calibration is per model; the last one holds for both map sizes
            b = synth.uniform_batch(seed=90, L=16, per_leaf=4096, H=H, W=H, n_queries=8, model=b"")
            e, _ = npg.splat_histograms(ctx, tf(b.dirs), t32(b.w), t32(b.leaf_off), H, H, want_count=False)
        m.calibrate_fp8(e)
    srv = npg.Server(ctx, m, n_slots=2, max_batch_leaves=4096, table_bytes=4 << 30, precision=prec)
    reqs = [(_request(100 + i, n_pool, L), H) for i, (L, H) in
            enumerate([(5, 64), (40, 128), (1, 64), (17, 64), (60, 64), (3, 128), (25, 64), (8, 128), (33, 64)])]
    alone = [_alone(npg, srv, dirs, w, beg, cnt, H) for (beg, cnt), H in reqs]
    # the same requests in a burst, interleaved with sampling requests on
    # already-resident tables: merged batches on overlapping slots
    warm = srv.submit_recon(dirs, w, *_request(1, n_pool, 200), 64, 64)
    srv.wait(warm)
    # two large requests occupy both slots, so the burst queues and merges
    blockers = [srv.submit_recon(dirs, w, *_request(2 + i, n_pool, 1500), 128, 128) for i in range(2)]
    qleaf = t32(np.random.default_rng(0).integers(0, 200, 200000).astype(np.uint32))
    qu = tf(np.random.default_rng(1).random((200000, 2)).astype(np.float32))
    outs = [(torch.empty((200000, 3), device=DEV), torch.empty(200000, device=DEV)) for _ in range(4)]
    tickets = []
    for i, ((beg, cnt), H) in enumerate(reqs):
        tickets.append(srv.submit_recon(dirs, w, beg, cnt, H, H))
        if i % 2 == 0:
            srv.submit_sample(warm, qleaf, qu, *outs[i // 2 % 4])
    for k, ((beg, cnt), H) in enumerate(reqs):
        srv.wait(tickets[k])
        got = srv.copy_tables(tickets[k], _tables(npg, len(beg), H, H))
        torch.cuda.synchronize()
        assert _same(alone[k], got), f"request {k} differs in the mix"
    for b in blockers:
        srv.wait(b)
    st = srv.stats()
    print("serve stats", st)
    assert st["merged_requests"] > 0 and st["max_concurrent"] == 2
    # and the served tables equal the library's own batched path
    beg, cnt = reqs[1][0]
    idx = np.concatenate([np.arange(b, b + c) for b, c in zip(beg, cnt)]).astype(np.uint32)
    off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.uint32)
    direct = npg.reconstruct_fused(ctx, m, dirs, w, t32(off), 128, 128, prec, perm=t32(idx))
    assert _same(alone[1], direct)
    srv.close()
    m.free()


def test_admission_budget_fifo(ctx, npg, pool):
    dirs, w, n_pool = pool
    m = npg.Model(ctx, synth.unet_model(2))
    one = 30 * (64 * 64 * 4 + 65 * 4 + 64 * 65 * 4 + 8) + 4096
    srv = npg.Server(ctx, m, n_slots=2, max_batch_leaves=4096, table_bytes=int(one * 1.5), precision="bf16")
    with pytest.raises(npg.NpgError) as e:
        srv.submit_recon(dirs, w, *_request(3, n_pool, 400), 64, 64)   # can never fit
    assert e.value.code == npg.E_BUDGET
    ts = [srv.submit_recon(dirs, w, *_request(10 + i, n_pool, 30), 64, 64) for i in range(3)]
    srv.wait(ts[0])
    import time
    time.sleep(0.05)
    assert srv.poll(ts[1]) is None and srv.poll(ts[2]) is None    # waiting for table memory
    srv.release(ts[0])
    srv.wait(ts[1])
    assert srv.poll(ts[2]) is None
    srv.release(ts[1])
    srv.wait(ts[2])
    srv.release(ts[2])
    assert srv.stats()["table_bytes_free"] == int(one * 1.5)
    srv.close()
    m.free()


def test_served_sampling_equals_direct(ctx, npg, pool):
    dirs, w, n_pool = pool
    m = npg.Model(ctx, synth.unet_model(4))
    srv = npg.Server(ctx, m, n_slots=3, precision="bf16", table_bytes=1 << 30)
    beg, cnt = _request(5, n_pool, 50)
    t = srv.submit_recon(dirs, w, beg, cnt, 64, 64)
    n = 300000
    leaf = t32(np.random.default_rng(2).integers(0, 50, n).astype(np.uint32))
    u = tf(synth.uniforms(synth.rng_for(3), 2 * n).reshape(n, 2))
    d, p = torch.empty((n, 3), device=DEV), torch.empty(n, device=DEV)
    ts = srv.submit_sample(t, leaf, u, d, p)     # submitted before the tables exist
    srv.wait(ts)
    tabs = srv.copy_tables(t, _tables(npg, 50, 64, 64))
    d2, p2, _ = npg.sample_dirs(ctx, tabs, leaf, u, want_bin=False)
    torch.cuda.synchronize()
    assert torch.equal(d, d2) and torch.equal(p, p2)
    srv.release(ts)
    srv.release(t)
    srv.close()
    m.free()


def test_release_with_queued_sampling(ctx, npg, pool):
    """Releasing a reconstruction while sampling requests against it are
    still queued keeps its tables until they are done."""
    dirs, w, n_pool = pool
    m = npg.Model(ctx, synth.unet_model(4))
    srv = npg.Server(ctx, m, n_slots=1, precision="bf16", table_bytes=1 << 30)
    ref = srv.submit_recon(dirs, w, *_request(6, n_pool, 20), 64, 64)
    n = 100000
    leaf = t32(np.random.default_rng(3).integers(0, 20, n).astype(np.uint32))
    u = tf(synth.uniforms(synth.rng_for(4), 2 * n).reshape(n, 2))
    outs = [(torch.empty((n, 3), device=DEV), torch.empty(n, device=DEV)) for _ in range(3)]
    srv.wait(ref)
    want = srv.copy_tables(ref, _tables(npg, 20, 64, 64))
    d0, p0, _ = npg.sample_dirs(ctx, want, leaf, u, want_bin=False)
    torch.cuda.synchronize()
    t = srv.submit_recon(dirs, w, *_request(6, n_pool, 20), 64, 64)
    ts = [srv.submit_sample(t, leaf, u, *o) for o in outs]
    srv.release(t)
    for k, o in zip(ts, outs):
        srv.wait(k)
        torch.cuda.synchronize()
        assert torch.equal(o[0], d0) and torch.equal(o[1], p0)
        srv.release(k)
    srv.release(ref)
    assert srv.stats()["table_bytes_free"] == 1 << 30
    srv.close()
    m.free()


def test_served_fp32_matches_oracle(ctx, npg, orc, pool):
    """Two FP32 requests (64x64 and 128x128) served in a burst with others,
    so they run in merged batches on overlapping slots; their tables against
    the oracle run on the same photon windows."""
    dirs, w, n_pool = pool
    model = synth.unet_model(12, random_bias=True)
    m = npg.Model(ctx, model)
    srv = npg.Server(ctx, m, n_slots=2, max_batch_leaves=4096, table_bytes=2 << 30, precision="fp32")
    blocker = srv.submit_recon(dirs, w, *_request(40, n_pool, 600), 128, 128)
    reqs = [(_request(41 + i, n_pool, L), H) for i, (L, H) in enumerate([(7, 64), (3, 128), (12, 64), (5, 128)])]
    tickets = [srv.submit_recon(dirs, w, beg, cnt, H, H) for (beg, cnt), H in reqs]
    host_dirs, host_w = dirs.cpu().numpy(), w.cpu().numpy().view(np.uint32)
    for k in (0, 1):
        (beg, cnt), H = reqs[k]
        srv.wait(tickets[k])
        got = srv.copy_tables(tickets[k], _tables(npg, len(beg), H, H))
        torch.cuda.synchronize()
        idx = np.concatenate([np.arange(b, b + c) for b, c in zip(beg, cnt)]).astype(np.uint32)
        off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.uint32)
        rc, e_ref, _ = orc.splat(host_dirs, host_w, off, H, H, perm=idx)
        assert rc == 0
        rc, s_ref = orc.net_forward(model, orc.normalize_input(e_ref))
        assert rc == 0
        rc, pdf_ref, marg_ref, cond_ref, tot_ref = orc.build_cdf(s_ref)
        assert rc == 0
        rel = np.abs(got.pdf.cpu().numpy().astype(np.float64) - pdf_ref) / pdf_ref
        print(f"served fp32 request {k} ({len(beg)} leaves, {H}x{H}): max rel pdf err {rel.max():.2e}")
        assert rel.max() < 1e-5
        for tab, want in ((got.marg, marg_ref), (got.cond, cond_ref)):
            g = tab.cpu().numpy().astype(np.float64)
            assert np.all(np.abs(g - want) <= 1e-5 * np.abs(want) + np.spacing(np.float32(1.0)))
    for t in tickets + [blocker]:
        srv.wait(t)
    assert srv.stats()["merged_requests"] > 0
    srv.close()
    m.free()
