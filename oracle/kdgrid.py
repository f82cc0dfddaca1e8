"""Plain numpy oracle of the paper's hierarchical grid (Sec. 7.1 and the
path-guiding implementation details of Sec. 8): a regular grid over the
scene box, voxels marked valid by the bounce points of camera paths, and
each valid voxel split into a local binary KD tree while its photon count
or the variance of its photons' surface normals exceeds a threshold; the
split plane is the median photon position along the longest axis of the
voxel.  Point location walks the grid cell and then the local tree.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the GPU path; both consume the same seeded inputs.

Readings (the paper leaves these open; the GPU library takes the same):
  * cell of a point: floor((p - lo) * (res / (hi - lo))) per axis in float64,
    clamped to [0, res-1]; cell id = ix + res * (iy + res * iz);
  * "middle of photon positions along an axis": the median, the
    (M // 2)-th smallest coordinate (0-based) of the node's M photons, on
    the longest axis of the node's box (ties: the lower axis index); photons
    with a coordinate below it go left, the rest right (-0 counts as +0); a
    node whose left side would be empty stays a leaf;
  * node box: the cell box [lo + i * step, lo + (i+1) * step] with
    step = (hi - lo) / res in float64, cut at the split coordinate;
  * normal variance: V = 1 - |mean normal|^2 (the total variance of unit
    vectors), from integer sums of the normals quantised as
    rint(clamp(n, -1, 1) * 2^20), in float64 as
    1 - ((Sx*Sx + Sy*Sy) + Sz*Sz) / ((M*M) * 2^40);
  * a node splits if depth < max_depth, M >= 2 and (M > split_count or
    V > split_var);
  * leaves are numbered cell by cell in ascending cell id and, inside a
    cell, depth first with the left child first; the photons of a leaf are
    listed in ascending photon index.
"""
from __future__ import annotations

import numpy as np

NONE = 0xFFFFFFFF          # "no leaf" from point location
QSCALE = 2.0 ** 20         # normal quantisation step 2^-20


def _params(res, lo, hi):
    lo = np.asarray(lo, np.float32).astype(np.float64)
    hi = np.asarray(hi, np.float32).astype(np.float64)
    if not (1 <= res <= 1024) or np.any(~(hi > lo)):
        raise ValueError("bad grid")
    return lo, hi


def cell_coords(p, res, lo, hi):
    """Integer cell coordinates [n][3] of float32 points (reading above)."""
    lo, hi = _params(res, lo, hi)
    invr = float(res) / (hi - lo)
    t = (np.asarray(p, np.float32).astype(np.float64) - lo) * invr
    return np.clip(np.floor(t), 0, res - 1).astype(np.int64)


def cell_ids(p, res, lo, hi):
    c = cell_coords(p, res, lo, hi)
    return c[:, 0] + res * (c[:, 1] + res * c[:, 2])


def mark_valid(points, res, lo, hi):
    """Valid voxels: every cell holding at least one bounce point of the
    camera paths (Sec. 7.1, valid voxels).  Returns uint8 [res^3]."""
    v = np.zeros(res ** 3, np.uint8)
    if len(points):
        v[cell_ids(points, res, lo, hi)] = 1
    return v


def normal_variance(nrm):
    """V = 1 - |mean normal|^2 from quantised integer sums (reading above)."""
    q = np.rint(np.clip(np.asarray(nrm, np.float32).astype(np.float64), -1.0, 1.0) * QSCALE).astype(np.int64)
    s = q.sum(axis=0).astype(np.float64)
    m = float(q.shape[0])
    return 1.0 - ((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]) / ((m * m) * (QSCALE * QSCALE))


def _canon(x):
    x = np.asarray(x, np.float32).copy()
    x[x == 0] = np.float32(0.0)
    return x


class KDGrid:
    """The built hierarchy: leaves (CSR over photon indices) plus, per valid
    non-empty cell, a nested tree ('leaf', id, box) | ('split', axis, s, L, R, box)."""

    def __init__(self, res, lo, hi):
        self.res, self.lo, self.hi = res, np.float32(lo), np.float32(hi)
        self.roots = {}
        self.leaves = []          # photon index arrays
        self.leaf_cell = []
        self.leaf_depth = []
        self.leaf_box = []

    @property
    def n_leaves(self):
        return len(self.leaves)

    def leaf_off(self):
        return np.concatenate([[0], np.cumsum([len(x) for x in self.leaves])]).astype(np.uint32)

    def perm(self):
        return (np.concatenate(self.leaves) if self.leaves else np.zeros(0)).astype(np.uint32)

    def n_nodes(self):
        def cnt(t):
            return 1 if t[0] == "leaf" else 1 + cnt(t[3]) + cnt(t[4])
        return sum(cnt(t) for t in self.roots.values())


def build(pos, normal, valid, res, lo, hi, split_count, split_var, max_depth):
    """The hierarchy over photons pos [n][3] (float32), normals [n][3] or
    None (no variance criterion), valid [res^3] uint8 or None (all valid)."""
    lo64, hi64 = _params(res, lo, hi)
    pos = np.asarray(pos, np.float32)
    if not np.all(np.isfinite(pos)):
        raise ValueError("non-finite position")
    g = KDGrid(res, lo, hi)
    cid = cell_ids(pos, res, lo, hi) if len(pos) else np.zeros(0, np.int64)
    keep = np.ones(len(pos), bool) if valid is None else np.asarray(valid)[cid] != 0
    if normal is not None and not np.all(np.isfinite(np.asarray(normal)[keep])):
        raise ValueError("non-finite normal of a photon in a valid voxel")
    step = (hi64 - lo64) / float(res)
    idx_all = np.nonzero(keep)[0]
    order = np.argsort(cid[idx_all], kind="stable")
    idx_sorted = idx_all[order]
    cells, starts = np.unique(cid[idx_sorted], return_index=True)
    ends = np.append(starts[1:], len(idx_sorted))

    def rec(idx, box, depth, cell):
        M = len(idx)
        V = normal_variance(normal[idx]) if normal is not None else 0.0
        if depth < max_depth and M >= 2 and (float(M) > split_count or V > split_var):
            ext = box[1] - box[0]
            a = 0
            if ext[1] > ext[a]:
                a = 1
            if ext[2] > ext[a]:
                a = 2
            x = _canon(pos[idx, a])
            s = np.sort(x)[M // 2]
            lm = x < s
            if lm.any():
                bl, br = box.copy(), box.copy()
                bl[1, a] = float(s)
                br[0, a] = float(s)
                left = rec(idx[lm], bl, depth + 1, cell)
                right = rec(idx[~lm], br, depth + 1, cell)
                return ("split", a, s, left, right, box)
        g.leaves.append(np.asarray(idx, np.int64))
        g.leaf_cell.append(cell)
        g.leaf_depth.append(depth)
        g.leaf_box.append(box)
        return ("leaf", len(g.leaves) - 1, box)

    for c, a, b in zip(cells, starts, ends):
        ijk = np.array([c % res, (c // res) % res, c // (res * res)], np.float64)
        box = np.stack([lo64 + ijk * step, lo64 + (ijk + 1) * step])
        g.roots[int(c)] = rec(idx_sorted[a:b], box, 0, int(c))
    return g


def locate(g: KDGrid, q):
    """Leaf id of each query point (NONE outside valid non-empty cells)."""
    q = np.asarray(q, np.float32)
    out = np.full(len(q), NONE, np.uint32)
    if not len(q):
        return out
    cid = cell_ids(q, g.res, g.lo, g.hi)
    qc = _canon(q.reshape(-1)).reshape(q.shape)
    for i in range(len(q)):
        t = g.roots.get(int(cid[i]))
        if t is None:
            continue
        while t[0] == "split":
            t = t[3] if qc[i, t[1]] < t[2] else t[4]
        out[i] = t[1]
    return out


def leaf_constraints(g: KDGrid):
    """Per leaf: its cell and the list of (axis, s, goes_left) on the path
    from the root (for brute-force point location)."""
    cons = [None] * g.n_leaves

    def walk(t, path, cell):
        if t[0] == "leaf":
            cons[t[1]] = (cell, list(path))
            return
        walk(t[3], path + [(t[1], t[2], True)], cell)
        walk(t[4], path + [(t[1], t[2], False)], cell)

    for c, t in g.roots.items():
        walk(t, [], c)
    return cons
