"""GPU tests of the paper's hierarchical grid (npg_mark_valid,
npg_build_kdgrid, npg_locate) against the oracle: valid voxels, leaf CSR,
photon permutation, node count and point location bit-exact on random
inputs with ties, creases and invalid voxels; at the paper's parameters on
clustered photons, every sampled voxel's leaves equal the oracle's for that
voxel alone (voxels are independent) and every photon locates to its own
leaf; empty, degenerate and error cases."""
import numpy as np
import pytest
import torch

from oracle import kdgrid as kg
from paper_2010_01775_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def tf(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _case(seed, n, res, ties=True):
    rng = np.random.default_rng(seed)
    c = rng.random((8, 3))
    p = (c[rng.integers(0, 8, n)] + 0.06 * rng.standard_normal((n, 3))).clip(0, 0.999).astype(np.float32)
    if ties:
        p[:n // 20, 0] = p[0, 0]                          # exact ties on x
        p[n // 20:n // 10, 1] = np.float32(0.5)           # ties on y at a voxel boundary
    nrm = synth.surface_normals(seed + 1, p, n_creases=8, crease_radius=0.3, freq=3.0)
    valid = (rng.random(res ** 3) < 0.75).astype(np.uint8)
    return p, nrm, valid


def _gpu_build(npg, ctx, prm, p, nrm, valid, max_leaves=None):
    return npg.build_kdgrid(ctx, prm, tf(p), None if nrm is None else tf(nrm),
                            None if valid is None else torch.from_numpy(valid).to(DEV), max_leaves=max_leaves)


def _compare(npg, ctx, prm, g, ref, p, queries):
    L = g["n_leaves"]
    assert L == ref.n_leaves
    off = g["leaf_off"].cpu().numpy().view(np.uint32)
    assert np.array_equal(off, ref.leaf_off())
    perm = g["perm"][:int(off[-1])].cpu().numpy().view(np.uint32)
    assert np.array_equal(perm, ref.perm())
    assert g["n_nodes"] == ref.n_nodes()
    for q in (p, queries):
        got = npg.locate(ctx, prm, g, tf(q)).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, kg.locate(ref, q))
    assert npg.sync_status(ctx) == 0


@pytest.mark.parametrize("seed,n,res,T,Vt,D,use_nrm,use_valid", [
    (11, 20000, 4, 60.0, 0.3, 8, True, True),
    (12, 20000, 7, 150.0, 0.45, 8, True, False),
    (13, 30000, 10, 25.0, 2.0, 5, False, True),      # count only, depth cap 5
    (14, 5000, 1, 10.0, 0.2, 16, True, False),       # one voxel, deep trees
    (15, 8000, 3, 1e9, 0.25, 8, True, True),         # variance only
])
def test_kdgrid_parity(ctx, npg, seed, n, res, T, Vt, D, use_nrm, use_valid):
    p, nrm, valid = _case(seed, n, res)
    lo, hi = (-0.05, 0.0, 0.0), (1.0, 1.0, 1.25)
    prm = npg.kdgrid_params(res, lo, hi, T, Vt, D)
    g = _gpu_build(npg, ctx, prm, p, nrm if use_nrm else None, valid if use_valid else None)
    ref = kg.build(p, nrm if use_nrm else None, valid if use_valid else None, res, lo, hi, T, Vt, D)
    assert ref.n_leaves > res ** 3 // 4 or res == 1
    q = np.random.default_rng(seed + 7).random((20000, 3)).astype(np.float32) * 1.3 - 0.1
    q[:50] = p[:50]
    _compare(npg, ctx, prm, g, ref, p, q)
    # cell_root: -1 exactly on invalid or empty voxels
    root = g["cell_root"].cpu().numpy()
    assert set(np.nonzero(root >= 0)[0].tolist()) == set(ref.roots.keys())


def test_mark_valid_parity(ctx, npg):
    rng = np.random.default_rng(21)
    res, lo, hi = 9, (0.0, -1.0, 0.5), (1.0, 1.0, 0.75)
    pts = (rng.random((50000, 3)) * [1.2, 2.4, 0.3] + [-0.1, -1.2, 0.475]).astype(np.float32)
    pts[:9, 0] = np.arange(9, dtype=np.float32) / 9           # points on voxel boundaries
    prm = npg.kdgrid_params(res, lo, hi)
    v = npg.mark_valid(ctx, prm, tf(pts)).cpu().numpy()
    assert np.array_equal(v, kg.mark_valid(pts, res, lo, hi))
    assert npg.sync_status(ctx) == 0


def test_kdgrid_paper_scale_sampled(ctx, npg):
    """Paper parameters (100^3 grid over the unit box, count threshold
    500 sqrt(2), variance 0.5, depth 8) on 4e6 clustered photons with crease
    normals and valid voxels from bounce points: the leaves of sampled voxels
    equal the oracle's build on those voxels' photons alone, and every photon
    locates to the leaf that holds it."""
    cp = synth.clustered_photons(seed=31, n=4_000_000, n_clusters=24, sigma=(0.01, 0.05))
    p = cp.pos
    nrm = synth.surface_normals(32, p)
    prm = npg.kdgrid_params()
    pts = synth.bounce_points(33, p, 300_000)
    valid_t = npg.mark_valid(ctx, prm, tf(pts))
    g = npg.build_kdgrid(ctx, prm, tf(p), tf(nrm), valid_t, max_leaves=1 << 20)
    valid = valid_t.cpu().numpy()
    L = g["n_leaves"]
    off = g["leaf_off"].cpu().numpy().view(np.uint32).astype(np.int64)
    perm = g["perm"][:int(off[-1])].cpu().numpy().view(np.uint32).astype(np.int64)
    cid = kg.cell_ids(p, 100, prm.lo[:], prm.hi[:])
    kept = valid[cid] != 0
    assert off[-1] == kept.sum() and L > 1000
    assert np.array_equal(np.sort(perm), np.nonzero(kept)[0])
    leaf_of = np.full(len(p), kg.NONE, np.uint32)
    leaf_of[perm] = np.repeat(np.arange(L, dtype=np.uint32), np.diff(off))
    got = npg.locate(ctx, prm, g, tf(p)).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, leaf_of)
    # sampled voxels: the densest ones and random ones
    root = g["cell_root"].cpu().numpy()
    vox = np.nonzero(root >= 0)[0]
    counts = np.bincount(cid[kept], minlength=100 ** 3)
    pick = np.unique(np.concatenate([np.argsort(counts)[-6:],
                                     np.random.default_rng(34).choice(vox, 30, replace=False)]))
    for v in pick:
        idx = np.nonzero((cid == v) & kept)[0]
        one = np.zeros(100 ** 3, np.uint8)
        one[v] = 1
        ref = kg.build(p[idx], nrm[idx], one, 100, prm.lo[:], prm.hi[:], prm.split_count, prm.split_var,
                       prm.max_depth)
        first = int(leaf_of[idx].min())                 # the voxel's first leaf
        for k, lf in enumerate(ref.leaves):
            a, b = off[first + k], off[first + k + 1]
            assert np.array_equal(perm[a:b], idx[lf]), (v, k)
        assert off[first + ref.n_leaves] - off[first] == len(idx)
    assert npg.sync_status(ctx) == 0


def test_kdgrid_edge_cases(ctx, npg):
    prm = npg.kdgrid_params(3, (0, 0, 0), (1, 1, 1), 2.0, 0.5, 8)
    g = npg.build_kdgrid(ctx, prm, tf(np.zeros((0, 3))), max_leaves=4)
    assert g["n_leaves"] == 0 and g["n_nodes"] == 0 and int(g["leaf_off"][0]) == 0
    assert bool((g["cell_root"] == -1).all())
    # every photon invalid
    p = np.random.default_rng(41).random((1000, 3)).astype(np.float32)
    g = _gpu_build(npg, ctx, prm, p, None, np.zeros(27, np.uint8), max_leaves=4)
    assert g["n_leaves"] == 0 and int(g["leaf_off"][0]) == 0
    assert np.all(npg.locate(ctx, prm, g, tf(p)).cpu().numpy() == -1)
    # identical positions: nothing below the median, one leaf per voxel
    same = np.tile(np.float32([[0.5, 0.5, 0.5]]), (500, 1))
    g = _gpu_build(npg, ctx, prm, same, None, None)
    assert g["n_leaves"] == 1 and g["n_nodes"] == 1
    # max_depth 0
    prm0 = npg.kdgrid_params(3, (0, 0, 0), (1, 1, 1), 2.0, 0.5, 0)
    g = _gpu_build(npg, ctx, prm0, p, None, None)
    assert g["n_leaves"] == len(np.unique(kg.cell_ids(p, 3, [0, 0, 0], [1, 1, 1])))
    assert npg.sync_status(ctx) == 0


def test_kdgrid_errors(ctx, npg):
    prm = npg.kdgrid_params(3, (0, 0, 0), (1, 1, 1), 2.0, 0.5, 8)
    p = np.random.default_rng(42).random((2000, 3)).astype(np.float32)
    with pytest.raises(npg.NpgError) as e:
        _gpu_build(npg, ctx, prm, p, None, None, max_leaves=10)
    assert e.value.code == npg.E_CAPACITY
    bad = p.copy()
    bad[17, 1] = np.nan
    with pytest.raises(npg.NpgError) as e:
        _gpu_build(npg, ctx, prm, bad, None, None)
    assert e.value.code == npg.E_RANGE
    nrm = np.tile(np.float32([[0, 0, 1]]), (2000, 1))
    nrm[5, 2] = np.inf
    with pytest.raises(npg.NpgError) as e:
        _gpu_build(npg, ctx, prm, p, nrm, None)
    assert e.value.code == npg.E_RANGE
    for badp in (npg.kdgrid_params(0), npg.kdgrid_params(3, (0, 0, 0), (1, 0, 1)),
                 npg.kdgrid_params(3, max_depth=17)):
        with pytest.raises(npg.NpgError) as e:
            _gpu_build(npg, ctx, badp, p, None, None)
        assert e.value.code == npg.E_ARG
    # a query that is not finite: none, and a range status
    g = _gpu_build(npg, ctx, prm, p, None, None)
    out = npg.locate(ctx, prm, g, tf(np.float32([[np.nan, 0.5, 0.5], [0.5, 0.5, 0.5]]))).cpu().numpy()
    assert out[0] == -1 and out[1] >= 0
    assert npg.sync_status(ctx) == npg.E_RANGE
    assert npg.sync_status(ctx) == 0
