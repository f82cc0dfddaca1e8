"""GPU parity of the octree build: leaf ids, CSR offsets, keys, depths and
the stable permutation are bit-exact against the oracle's recursive build."""
import numpy as np
import pytest
import torch

from paper_2010_01775_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _pts(seed, n, k=4, sig=0.03):
    rng = np.random.default_rng(seed)
    c = rng.random((k, 3))
    p = (c[rng.integers(0, k, n)] + sig * rng.standard_normal((n, 3))).astype(np.float32)
    return np.where((p >= 0) & (p < 1), p, rng.random((n, 3)).astype(np.float32))


def _check(npg, ctx, orc, pos, T, D, ref=None):
    if ref is None:
        rc, ref = orc.build_tree(pos, T, D, max_leaves=max(1, pos.shape[0]))
        assert rc == 0
    out = npg.build_hierarchy(ctx, torch.from_numpy(pos).to(DEV), T, D, max_leaves=max(1, pos.shape[0]))
    L = out["n_leaves"]
    assert L == ref["n_leaves"]
    u = lambda t: t.cpu().numpy().view(np.uint32)
    assert np.array_equal(u(out["leaf_off"]), ref["leaf_off"])
    assert np.array_equal(u(out["perm"]), ref["perm"])
    assert np.array_equal(u(out["leaf_of"]), ref["leaf_of"])
    assert np.array_equal(out["key"].cpu().numpy().view(np.uint64), ref["key"])
    assert np.array_equal(out["depth"].cpu().numpy(), ref["depth"])
    return ref


@pytest.mark.parametrize("seed,n,T,D", [(1, 3000, 50, 5), (2, 20000, 500, 6), (3, 4000, 10, 8),
                                        (4, 100000, 64, 7), (5, 70000, 8192, 6), (6, 5000, 1, 2)])
def test_hierarchy_bit_exact(ctx, npg, orc, seed, n, T, D):
    _check(npg, ctx, orc, _pts(seed, n), T, D)


def test_hierarchy_edges(ctx, npg, orc):
    _check(npg, ctx, orc, np.full((100, 3), 0.3, np.float32), 10, 5)     # one deep leaf
    _check(npg, ctx, orc, _pts(0, 500), 10000, 6)                        # root only
    _check(npg, ctx, orc, _pts(0, 300), 1, 0)                            # Dmax = 0
    p = np.array([[0, 0, 0], [np.nextafter(np.float32(1), 0)] * 3], np.float32)
    _check(npg, ctx, orc, p, 0, 8)                                       # extreme corners
    out = npg.build_hierarchy(ctx, torch.zeros((0, 3), device=DEV), 8, 4, max_leaves=4)
    assert out["n_leaves"] == 0 and out["leaf_off"].cpu().tolist() == [0]


def test_hierarchy_leaf_of_unaligned_output(ctx, npg):
    """leaf_of written into a caller buffer that is not 16-byte aligned."""
    pts = _pts(7, 10003)
    buf = torch.full((pts.shape[0] + 1,), -1, dtype=torch.int32, device=DEV)
    out = npg.build_hierarchy(ctx, torch.from_numpy(pts).to(DEV), 64, 5, leaf_of_out=buf[1:])
    ref = npg.build_hierarchy(ctx, torch.from_numpy(pts).to(DEV), 64, 5)
    assert npg.sync_status(ctx) == 0
    assert buf[0].item() == -1
    assert torch.equal(buf[1:], ref["leaf_of"]) and torch.equal(out["perm"], ref["perm"])


def test_hierarchy_errors(ctx, npg):
    pos = torch.from_numpy(_pts(0, 5000)).to(DEV)
    with pytest.raises(npg.NpgError) as e:
        npg.build_hierarchy(ctx, pos, 10, 6, max_leaves=4)
    assert e.value.code == npg.E_CAPACITY
    bad = _pts(0, 10)
    bad[3, 1] = 1.0
    with pytest.raises(npg.NpgError) as e:
        npg.build_hierarchy(ctx, torch.from_numpy(bad).to(DEV), 4, 3)
    assert e.value.code == npg.E_RANGE
    assert npg.sync_status(ctx) == 0
    with pytest.raises(npg.NpgError) as e:
        npg.build_hierarchy(ctx, pos, 10, 9)
    assert e.value.code == npg.E_ARG


def test_hierarchy_clustered_workload_full_size(ctx, npg, orc, clustered, clustered_tree):
    """5e7 photons in 64 Gaussian clusters, split above 8192, depth cap 6."""
    ref = _check(npg, ctx, orc, clustered.pos, 8192, 6, ref=clustered_tree)
    cnt = np.diff(ref["leaf_off"].astype(np.int64))
    print(f"leaves {ref['n_leaves']}, photons per leaf min {cnt.min()} median {np.median(cnt):.0f} max {cnt.max()}")
    assert 15000 < ref["n_leaves"] < 25000


@pytest.mark.parametrize("seed,n,T,D", [(11, 30000, 500, 6), (12, 5000, 10000, 4), (13, 70001, 64, 7),
                                        (14, 3000, 8, 1), (15, 150000, 1, 8)])
def test_hierarchy_sorted_photons(ctx, npg, orc, seed, n, T, D):
    """The leaf-ordered photons equal the input gathered through the oracle's
    permutation, bit for bit; the permutation and offsets equal the oracle's
    (1-, 2- and 3-byte leaf ids: one, two and three sort passes)."""
    rng = np.random.default_rng(seed)
    pos = _pts(seed, n) if T > 1 else rng.random((n, 3)).astype(np.float32)   # T = 1: > 65536 leaves
    dirs = synth.to_f32_dirs(synth.unit_vectors(rng, n))
    w = synth.photon_weights(rng, n)
    rc, ref = orc.build_tree(pos, T, D, max_leaves=n)
    assert rc == 0
    tf = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)
    out = npg.build_hierarchy_sorted(ctx, tf(pos), tf(dirs), torch.from_numpy(w.view(np.int32)).to(DEV), T, D,
                                     max_leaves=n)
    assert npg.sync_status(ctx) == 0
    assert out["n_leaves"] == ref["n_leaves"]
    u = lambda t: t.cpu().numpy().view(np.uint32)
    assert np.array_equal(u(out["perm"]), ref["perm"])
    assert np.array_equal(u(out["leaf_off"]), ref["leaf_off"])
    assert np.array_equal(out["dirs"].cpu().numpy().view(np.uint32), dirs[ref["perm"]].view(np.uint32))
    assert np.array_equal(u(out["w"]), w[ref["perm"]])


def test_hierarchy_sorted_clustered_maps(ctx, npg, orc, clustered, clustered_tree):
    """The clustered workload: maps splatted from the leaf-ordered photons
    (no permutation) equal the oracle's on every leaf."""
    cp, ref = clustered, clustered_tree
    tf = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)
    out = npg.build_hierarchy_sorted(ctx, tf(cp.pos), tf(cp.dirs), torch.from_numpy(cp.w.view(np.int32)).to(DEV),
                                     8192, 6, max_leaves=65536)
    assert out["n_leaves"] == ref["n_leaves"]
    e, c = npg.splat_histograms(ctx, out["dirs"], out["w"], out["leaf_off"], 128, 128)
    assert npg.sync_status(ctx) == 0
    assert np.array_equal(out["perm"].cpu().numpy().view(np.uint32), ref["perm"])
    rc, e_ref, c_ref = orc.splat(cp.dirs, cp.w, ref["leaf_off"], 128, 128, perm=ref["perm"])
    assert rc == 0
    assert np.array_equal(e.cpu().numpy().view(np.uint64), e_ref)
    assert np.array_equal(c.cpu().numpy().view(np.uint32), c_ref)
