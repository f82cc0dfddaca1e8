"""Pins of the oracle's photon binning (Eq. "photon") and input scaling.

Checks: a hand-binned fixture (tests/golden/splat_small.txt); histogram mass
equals the summed photon weight exactly; counts sum to the leaf's photon
count; invariance to photon order, chunking (accumulate) and leaf order; the
mean-1 normalisation of the raw sampling map.
"""
import os

import numpy as np

from paper_2010_01775_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fixture():
    P, E = [], []
    for l in open(os.path.join(GOLD, "splat_small.txt")):
        t = l.split()
        if not t or t[0] == "#":
            continue
        if t[0] == "P":
            P.append((int(t[1]), float(t[2]), float(t[3]), float(t[4]), int(t[5])))
        else:
            E.append(tuple(int(v) for v in t[1:]))
    return P, E


def test_golden_small(orc):
    P, E = _fixture()
    leaf = np.array([p[0] for p in P])
    dirs = np.array([p[1:4] for p in P], np.float32)
    w = np.array([p[4] for p in P], np.uint32)
    off = np.array([0, (leaf == 0).sum(), len(P)], np.uint32)
    rc, en, ct = orc.splat(dirs, w, off, 8, 8)
    assert rc == 0
    want_e = np.zeros((2, 8, 8), np.uint64)
    want_c = np.zeros((2, 8, 8), np.uint32)
    for l, r, c, e, n in E:
        want_e[l, r, c] = e
        want_c[l, r, c] = n
    assert np.array_equal(en, want_e)
    assert np.array_equal(ct, want_c)


def test_mass_and_count_conservation(orc):
    b = synth.uniform_batch(seed=5, L=16, per_leaf=3000, H=32, W=32, n_queries=8)
    rc, en, ct = orc.splat(b.dirs, b.w, b.leaf_off, b.H, b.W)
    assert rc == 0
    for l in range(b.L):
        s, e = b.leaf_off[l], b.leaf_off[l + 1]
        assert int(en[l].sum(dtype=np.uint64)) == int(b.w[s:e].astype(np.uint64).sum())
        assert int(ct[l].sum()) == e - s


def test_order_chunk_and_perm_invariance(orc):
    b = synth.uniform_batch(seed=6, L=8, per_leaf=2000, H=16, W=32, n_queries=8)
    rc, e0, c0 = orc.splat(b.dirs, b.w, b.leaf_off, b.H, b.W)
    rng = np.random.default_rng(1)
    # (1) photons shuffled within each leaf, read through perm
    perm = np.concatenate([rng.permutation(np.arange(b.leaf_off[l], b.leaf_off[l + 1]))
                           for l in range(b.L)]).astype(np.uint32)
    rc, e1, c1 = orc.splat(b.dirs, b.w, b.leaf_off, b.H, b.W, perm=perm)
    assert np.array_equal(e0, e1) and np.array_equal(c0, c1)
    # (2) two chunks accumulated
    half = b.leaf_off.copy()
    first = b.leaf_off[:-1] + (b.leaf_off[1:] - b.leaf_off[:-1]) // 2
    offa = np.empty(b.L + 1, np.uint32)
    # chunk A: first halves, chunk B: second halves, each as its own CSR
    ia = np.concatenate([np.arange(b.leaf_off[l], first[l]) for l in range(b.L)])
    ib = np.concatenate([np.arange(first[l], b.leaf_off[l + 1]) for l in range(b.L)])
    offa = np.concatenate([[0], np.cumsum(first - b.leaf_off[:-1])]).astype(np.uint32)
    offb = np.concatenate([[0], np.cumsum(b.leaf_off[1:] - first)]).astype(np.uint32)
    rc, e2, c2 = orc.splat(b.dirs[ia], b.w[ia], offa, b.H, b.W)
    rc, e2, c2 = orc.splat(b.dirs[ib], b.w[ib], offb, b.H, b.W, energy=e2, count=c2, accumulate=True)
    assert np.array_equal(e0, e2) and np.array_equal(c0, c2)
    del half
    # (3) leaf order reversed
    rev = np.concatenate([np.arange(b.leaf_off[l], b.leaf_off[l + 1]) for l in range(b.L - 1, -1, -1)])
    offr = np.concatenate([[0], np.cumsum((b.leaf_off[1:] - b.leaf_off[:-1])[::-1])]).astype(np.uint32)
    rc, e3, c3 = orc.splat(b.dirs[rev], b.w[rev], offr, b.H, b.W)
    assert np.array_equal(e0, e3[::-1]) and np.array_equal(c0, c3[::-1])


def test_bins_agree_with_binned_sum(orc):
    """Histogram equals the bincount of per-photon bins (np.add.at)."""
    b = synth.uniform_batch(seed=8, L=4, per_leaf=5000, H=64, W=64, n_queries=8)
    rc, en, ct = orc.splat(b.dirs, b.w, b.leaf_off, b.H, b.W)
    rc, bins = orc.bin_dirs(b.dirs, b.H, b.W)
    leaf = np.repeat(np.arange(b.L), np.diff(b.leaf_off))
    flat = leaf * b.H * b.W + bins
    want_c = np.bincount(flat, minlength=b.L * b.H * b.W)
    want_e = np.zeros(b.L * b.H * b.W, np.uint64)
    np.add.at(want_e, flat, b.w.astype(np.uint64))
    assert np.array_equal(ct.ravel(), want_c)
    assert np.array_equal(en.ravel(), want_e)


def test_empty_leaves_and_nan(orc):
    d = np.array([[1, 0, 0], [np.nan, 0, 0]], np.float32)
    w = np.array([5, 7], np.uint32)
    off = np.array([0, 0, 2, 2], np.uint32)
    rc, en, ct = orc.splat(d, w, off, 4, 4)
    assert rc == orc.E_RANGE
    assert en[0].sum() == 0 and en[2].sum() == 0
    assert int(en[1].sum()) == 5 and int(ct[1].sum()) == 1


def test_normalize_mean_one(orc):
    e = np.zeros((3, 8, 8), np.uint64)
    e[0] = 7                       # uniform -> all ones
    e[1, 2, 3] = 2 ** 40           # a single bin -> H*W there
    e[1, 5, 5] = 2 ** 40
    x = orc.normalize_input(e)
    assert np.all(x[0] == 1.0)
    assert x[1, 2, 3] == 32.0 and x[1, 5, 5] == 32.0 and x[1].sum() == 64.0
    assert np.all(x[2] == 0.0)     # empty leaf -> zero map
    b = synth.uniform_batch(seed=9, L=4, per_leaf=1000, H=32, W=32, n_queries=8)
    rc, en, _ = orc.splat(b.dirs, b.w, b.leaf_off, b.H, b.W)
    x = orc.normalize_input(en)
    assert np.allclose(x.reshape(4, -1).mean(1), 1.0, rtol=1e-13)
    assert np.allclose(x, en.astype(np.float64) * 1024 / en.reshape(4, -1).sum(1)[:, None, None].astype(np.float64), rtol=1e-15)
