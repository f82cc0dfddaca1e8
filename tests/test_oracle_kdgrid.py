"""Pins of the oracle of the paper's hierarchical grid (Sec. 7.1: regular
grid, valid voxels from path bounce points, local KD subdivision by photon
count and normal variance; Sec. 8: 100^3 grid, thresholds, depth <= 8, O(1)
grid plus O(log n) tree lookup).

Checks: the cell rule against exact rational arithmetic; valid voxels on a
hand case; the normal variance on closed forms (equal, opposite, orthogonal
normals) and against the float64 formula; hand-worked splits (even and odd
counts, ties at the median, a degenerate node, the axis rule); the strict
thresholds and the depth limit; and on random inputs, brute-force
invariants: every photon of a valid cell in exactly one leaf, leaves in
cell and depth-first order, each split at the (M // 2)-th smallest
coordinate with exactly the smaller coordinates on the left, every leaf
unsplittable, and point location equal to the unique leaf whose cell and
split constraints hold.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import kdgrid as kg


def test_cell_rule_exact():
    rng = np.random.default_rng(1)
    lo, hi, res = np.float32([-1.5, 0.0, 2.0]), np.float32([2.5, 1.0, 2.75]), 7
    p = (rng.random((4000, 3)) * (hi - lo) * 1.2 + lo - 0.1 * (hi - lo)).astype(np.float32)
    p[:6] = [[-1.5, 0, 2], [2.5, 1, 2.75], [0.5, 0.5, 2.375], [-1.5 + 4 / 7, 1 / 7, 2.0], [9, -9, 0], [0, 0, 0]]
    c = kg.cell_coords(p, res, lo, hi)
    for i in range(len(p)):
        for a in range(3):
            t = (Fraction(float(p[i, a])) - Fraction(float(lo[a]))) * res / (Fraction(float(hi[a])) - Fraction(float(lo[a])))
            exact = min(max(t.numerator // t.denominator, 0), res - 1)
            if abs(float(t) - round(float(t))) > 1e-9:       # away from a cell boundary
                assert c[i, a] == exact, (i, a)
    assert list(c[0]) == [0, 0, 0] and list(c[1]) == [6, 6, 6] and list(c[4]) == [6, 0, 0]
    assert list(kg.cell_coords(np.float32([[0.25, 0.2499999, 1.0]]), 4, [0, 0, 0], [1, 1, 1])[0]) == [1, 0, 3]


def test_mark_valid_hand():
    v = kg.mark_valid(np.float32([[0.1, 0.1, 0.1], [0.9, 0.1, 0.6], [0.12, 0.2, 0.0]]), 2, [0, 0, 0], [1, 1, 1])
    assert list(np.nonzero(v)[0]) == [0, 1 + 2 * 2 * 1]


def test_normal_variance_closed_forms():
    e = np.float32([[0, 0, 1]] * 5)
    assert kg.normal_variance(e) == 0.0
    assert kg.normal_variance(np.float32([[0, 0, 1], [0, 0, -1]])) == 1.0
    assert kg.normal_variance(np.float32([[1, 0, 0], [0, 1, 0]])) == 0.5
    rng = np.random.default_rng(2)
    n = rng.standard_normal((1000, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    m = n.astype(np.float64).mean(0)
    assert abs(kg.normal_variance(n) - (1 - m @ m)) < 1e-5


def _one_cell(xs, ys=None, box_hi=(1.0, 0.5, 0.5)):
    xs = np.asarray(xs, np.float32)
    ys = np.full_like(xs, 0.25) if ys is None else np.asarray(ys, np.float32)
    return np.stack([xs, ys, np.full_like(xs, 0.25)], 1), [0, 0, 0], list(box_hi)


@pytest.mark.parametrize("xs,leaves", [
    ([0.1, 0.5, 0.3, 0.9], [[0, 2], [1, 3]]),           # even: s = 2nd smallest (0-based) = 0.5
    ([0.5, 0.1, 0.4, 0.2, 0.3], [[1, 3], [0, 2, 4]]),   # odd: s = 0.3
    ([0.5, 0.5, 0.5, 0.7], [[0, 1, 2, 3]]),             # ties: nothing below the median, no split
    ([0.2, 0.5, 0.5, 0.5], [[0], [1, 2, 3]]),           # ties at the median go right
])
def test_hand_splits(xs, leaves):
    p, lo, hi = _one_cell(xs)
    g = kg.build(p, None, None, 1, lo, hi, split_count=1.5, split_var=2.0, max_depth=1)
    assert [list(x) for x in g.leaves] == leaves


def test_axis_rule_and_depth():
    # unit cube cell: equal extents -> x first; the children are 0.5 x 1 x 1 -> y next
    rng = np.random.default_rng(3)
    p = rng.random((64, 3)).astype(np.float32)
    g = kg.build(p, None, None, 1, [0, 0, 0], [1, 1, 1], split_count=1.0, split_var=2.0, max_depth=2)
    t = g.roots[0]
    assert t[0] == "split" and t[1] == 0
    assert t[3][0] == "split" and t[3][1] == 1 and t[4][1] == 1
    assert g.n_leaves == 4 and set(g.leaf_depth) == {2}
    assert [len(x) for x in g.leaves] == [16, 16, 16, 16]
    g0 = kg.build(p, None, None, 1, [0, 0, 0], [1, 1, 1], 1.0, 2.0, max_depth=0)
    assert g0.n_leaves == 1


def test_strict_thresholds():
    p, lo, hi = _one_cell([0.1, 0.2, 0.3, 0.4])
    assert kg.build(p, None, None, 1, lo, hi, 4.0, 2.0, 8).n_leaves == 1     # M = 4 is not > 4
    assert kg.build(p, None, None, 1, lo, hi, 3.99, 2.0, 8).n_leaves == 2
    # variance alone: opposite normals split a 2-photon node, equal ones do not
    p2, lo, hi = _one_cell([0.1, 0.7])
    nn = np.float32([[0, 0, 1], [0, 0, -1]])
    assert kg.build(p2, nn, None, 1, lo, hi, 1e9, 0.5, 8).n_leaves == 2
    assert kg.build(p2, np.float32([[0, 0, 1]] * 2), None, 1, lo, hi, 1e9, 0.5, 8).n_leaves == 1
    # orthogonal normals: V = 0.5 exactly, not > 0.5
    assert kg.build(p2, np.float32([[1, 0, 0], [0, 1, 0]]), None, 1, lo, hi, 1e9, 0.5, 8).n_leaves == 1


def _random_case(seed, n=3000, res=4):
    rng = np.random.default_rng(seed)
    c = rng.random((6, 3))
    p = (c[rng.integers(0, 6, n)] + 0.08 * rng.standard_normal((n, 3))).clip(0, 0.999).astype(np.float32)
    p[:50, 0] = p[0, 0]                      # exact ties along x
    nrm = np.where((p[:, 0] + p[:, 1] < 0.9)[:, None], [0, 0, 1], [1, 0, 0]).astype(np.float64)
    nrm += 0.3 * rng.standard_normal((n, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    valid = (rng.random(res ** 3) < 0.7).astype(np.uint8)
    return p, nrm, valid, res


@pytest.mark.parametrize("seed,T,Vt", [(4, 40.0, 0.35), (7, 100.0, 0.3)])
def test_brute_force_invariants(seed, T, Vt):
    p, nrm, valid, res = _random_case(seed)
    lo, hi = [0, 0, 0], [1, 1, 1]
    D = 8
    g = kg.build(p, nrm, valid, res, lo, hi, T, Vt, D)
    # the variance criterion acts here (more leaves than by counts alone)
    assert g.n_leaves > kg.build(p, None, valid, res, lo, hi, T, Vt, D).n_leaves
    assert max(g.leaf_depth) == D
    cid = kg.cell_ids(p, res, lo, hi)
    kept = np.nonzero(valid[cid])[0]
    perm = g.perm()
    assert sorted(perm.tolist()) == kept.tolist()                      # each kept photon once
    assert np.all(np.diff(g.leaf_cell) >= 0)                           # cells ascending
    cons = kg.leaf_constraints(g)
    for k, idx in enumerate(g.leaves):
        assert np.all(np.diff(idx) > 0)                                # ascending indices
        assert np.all(cid[idx] == g.leaf_cell[k])
        for a, s, left in cons[k][1]:
            x = kg._canon(p[idx, a])
            assert np.all(x < s) if left else np.all(x >= s)
        M = len(idx)
        V = kg.normal_variance(nrm[idx])
        if g.leaf_depth[k] < D and M >= 2 and (M > T or V > Vt):       # then it must be degenerate
            box = g.leaf_box[k]
            ext = box[1] - box[0]
            a = 0
            if ext[1] > ext[a]:
                a = 1
            if ext[2] > ext[a]:
                a = 2
            x = np.sort(kg._canon(p[idx, a]))
            assert np.all(x[: M // 2 + 1] == x[0])
    # every split: s = the (M // 2)-th smallest of the parent's coordinates
    def check(t):
        if t[0] == "leaf":
            return list(g.leaves[t[1]])
        li, ri = check(t[3]), check(t[4])
        allx = np.sort(kg._canon(p[li + ri, t[1]]))
        assert allx[len(allx) // 2] == t[2]
        assert np.sum(allx < t[2]) == len(li)
        return li + ri
    for t in g.roots.values():
        check(t)
    # depth-first order: each subtree's leaves are consecutive, left first
    assert np.array_equal(g.leaf_off()[-1], len(kept))
    # point location: own photons, then random queries against brute force
    loc = kg.locate(g, p)
    lof = np.full(len(p), kg.NONE, np.uint32)
    for k, idx in enumerate(g.leaves):
        lof[idx] = k
    assert np.array_equal(loc, lof)
    rng = np.random.default_rng(seed + 100)
    q = rng.random((3000, 3)).astype(np.float32)
    ql = kg.locate(g, q)
    qc = kg.cell_ids(q, res, lo, hi)
    for i in range(len(q)):
        hit = [k for k in range(g.n_leaves) if cons[k][0] == qc[i] and
               all((q[i, a] < s) == left for a, s, left in cons[k][1])]
        assert ([ql[i]] if ql[i] != kg.NONE else []) == hit


def test_empty_and_invalid():
    g = kg.build(np.zeros((0, 3), np.float32), None, None, 3, [0, 0, 0], [1, 1, 1], 10, 0.5, 8)
    assert g.n_leaves == 0 and len(g.perm()) == 0
    p = np.float32([[0.1, 0.1, 0.1], [0.9, 0.9, 0.9]])
    v = np.zeros(8, np.uint8)
    v[7] = 1
    g = kg.build(p, None, v, 2, [0, 0, 0], [1, 1, 1], 10, 0.5, 8)
    assert [list(x) for x in g.leaves] == [[1]]
    assert list(kg.locate(g, p)) == [kg.NONE, 0]
    with pytest.raises(ValueError):
        kg.build(np.float32([[np.nan, 0, 0]]), None, None, 2, [0, 0, 0], [1, 1, 1], 10, 0.5, 8)
