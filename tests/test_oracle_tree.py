"""Pins of the oracle's adaptive hierarchy (Sec. 7.1 "Voxel subdivision",
read as a count-threshold octree over the unit box).

Checks, against a brute-force top-down descent written with numpy (each
photon's ancestor cells from floor(p * 2^d), their populations counted with
np.unique), on clustered inputs with several depths: leaf membership, leaf
order (lexicographic order of child-index paths = Morton order), the split
invariants (every split cell holds more than T photons, every leaf holds at
most T or sits at Dmax, no empty leaf), stability of perm, the key/depth of
each leaf, and the edge cases (no photons, one cell, capacity overflow,
positions outside the box).
"""
import numpy as np
import pytest

from paper_2010_01775_amd import synth


def _cluster_points(seed, n, k=4, sig=0.03):
    rng = np.random.default_rng(seed)
    c = rng.random((k, 3))
    lab = rng.integers(0, k, n)
    p = (c[lab] + sig * rng.standard_normal((n, 3))).astype(np.float32)
    p = np.where((p >= 0) & (p < 1), p, rng.random((n, 3)).astype(np.float32))
    return p


def _brute(pos, T, Dmax):
    n = pos.shape[0]
    p = pos.astype(np.float64)
    leaf_d = np.full(n, -1)
    for d in range(Dmax + 1):
        cell = np.floor(p * 2.0 ** d).astype(np.int64)
        _, inv, cnt = np.unique(cell, axis=0, return_inverse=True, return_counts=True)
        c = cnt[inv.ravel()]
        pick = (leaf_d < 0) & ((c <= T) | (d == Dmax))
        leaf_d[pick] = d
    cells = np.floor(p * (2.0 ** leaf_d)[:, None]).astype(np.int64)
    return leaf_d, cells


def _path(d, cell):
    """Child-index path from the root: per level, x | y<<1 | z<<2."""
    out = []
    for lev in range(1, d + 1):
        b = (cell >> (d - lev)) & 1
        out.append(int(b[0] | (b[1] << 1) | (b[2] << 2)))
    return tuple(out) + (-1,) * (21 - d)


@pytest.mark.parametrize("seed,n,T,Dmax", [(1, 3000, 50, 5), (2, 5000, 200, 3), (3, 4000, 10, 8), (4, 20000, 500, 6)])
def test_tree_vs_bruteforce(orc, seed, n, T, Dmax):
    pos = _cluster_points(seed, n)
    rc, t = orc.build_tree(pos, T, Dmax)
    assert rc == 0
    L = t["n_leaves"]
    off = t["leaf_off"].astype(np.int64)
    perm = t["perm"].astype(np.int64)
    assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) > 0)
    assert np.array_equal(np.sort(perm), np.arange(n))
    leaf_d, cells = _brute(pos, T, Dmax)
    # group photons of the brute-force leaves
    keys = {}
    for i in range(n):
        keys.setdefault((int(leaf_d[i]),) + tuple(int(v) for v in cells[i]), []).append(i)
    assert len(keys) == L
    order = sorted(keys, key=lambda k: _path(k[0], np.array(k[1:])))
    for lid, k in enumerate(order):
        members = perm[off[lid]:off[lid + 1]]
        assert list(members) == keys[k]          # same photons, input order (stable)
        assert t["depth"][lid] == k[0]
        assert np.all(t["leaf_of"][members] == lid)
        # key = Morton code of the corner on the 2^21 lattice
        corner = np.array(k[1:], np.int64) << (21 - k[0])
        key = 0
        for b in range(21):
            for a in range(3):
                key |= ((int(corner[a]) >> b) & 1) << (3 * b + a)
        assert int(t["key"][lid]) == key
    assert np.all(np.diff(t["key"].astype(np.float64)) > 0)
    # split invariants
    cnt = np.diff(off)
    assert np.all((cnt <= T) | (t["depth"] == Dmax))
    p64 = pos.astype(np.float64)
    for lid, k in enumerate(order):
        d = k[0]
        if d == 0:
            continue
        parent = np.array(k[1:]) >> 1
        inside = np.all(np.floor(p64 * 2.0 ** (d - 1)).astype(np.int64) == parent, axis=1)
        assert inside.sum() > T


def test_tree_edges(orc):
    rc, t = orc.build_tree(np.zeros((0, 3), np.float32), 8, 4)
    assert rc == 0 and t["n_leaves"] == 0
    same = np.full((100, 3), 0.3, np.float32)
    rc, t = orc.build_tree(same, 10, 5)
    assert rc == 0 and t["n_leaves"] == 1 and t["depth"][0] == 5
    assert np.array_equal(t["perm"], np.arange(100))
    rc, t = orc.build_tree(_cluster_points(0, 500), 10000, 6)
    assert rc == 0 and t["n_leaves"] == 1 and t["depth"][0] == 0 and t["key"][0] == 0
    rc, t = orc.build_tree(_cluster_points(0, 5000), 10, 6, max_leaves=4)
    assert rc == orc.E_CAPACITY
    for bad in (1.0, -1e-9, np.nan):
        p = _cluster_points(0, 10)
        p[3, 1] = bad
        rc, _ = orc.build_tree(p, 4, 3)
        assert rc == orc.E_RANGE
    # Dmax = 0: one root leaf regardless of T
    rc, t = orc.build_tree(_cluster_points(0, 300), 1, 0)
    assert rc == 0 and t["n_leaves"] == 1


def test_clustered_generator_shape():
    cp = synth.clustered_photons(seed=5, n=64_000, n_clusters=8)
    assert cp.pos.dtype == np.float32 and cp.pos.shape == (64_000, 3)
    assert np.all((cp.pos >= 0) & (cp.pos < 1))
    assert np.allclose(np.linalg.norm(cp.dirs, axis=1), 1, atol=1e-6)
    assert cp.w.dtype == np.uint32
