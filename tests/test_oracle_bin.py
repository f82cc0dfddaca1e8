"""Pins of the oracle's direction -> bin rule (equal-area cylindrical map,
Sec. 5 "Spherical function representation").

The rule is checked against: hand-derived bins of axis, pole and boundary
directions (tests/golden/axis_bins.txt); numpy's float64 arctan2/floor away
from bin boundaries; exact boundary rays; the equal-area property (uniform
directions fill rows and columns uniformly) and the closed-form z-marginal of
a vMF lobe (tests/golden/vmf_rows.txt).
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_2010_01775_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_axis_and_boundary_golden(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "axis_bins.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) >= 12
    for H, W, x, y, z, iz, ip in rows:
        H, W, iz, ip = int(H), int(W), int(iz), int(ip)
        d = np.array([[float(x), float(y), float(z)]], np.float32)
        rc, b = orc.bin_dirs(d, H, W)
        assert rc == 0
        assert b[0] == iz * W + ip, (H, W, x, y, z, b[0], iz * W + ip)


def test_boundary_table(orc):
    for W in (4, 8, 32, 64, 128, 1024):
        ex, ey = orc.boundaries(W)
        t = 2 * np.pi * np.arange(W) / W
        assert np.max(np.abs(ex - np.cos(t))) < 1e-7
        assert np.max(np.abs(ey - np.sin(t))) < 1e-7
        q = W // 4
        # axes exact
        assert (ex[0], ey[0]) == (1.0, 0.0)
        assert (ex[q], ey[q]) == (0.0, 1.0)
        assert (ex[2 * q], ey[2 * q]) == (-1.0, 0.0)
        assert (ex[3 * q], ey[3 * q]) == (0.0, -1.0)
        # strictly increasing azimuth of the rounded rays
        ang = np.mod(np.arctan2(ey.astype(np.float64), ex.astype(np.float64)), 2 * np.pi)
        assert np.all(np.diff(ang) > 0)
        # float32 rounding of cos/sin is far from a rounding midpoint
        c64 = np.cos(t[:q])
        c32 = c64.astype(np.float32).astype(np.float64)
        ulp = np.spacing(np.abs(c64).astype(np.float32)).astype(np.float64)
        nz = np.abs(c64) > 0
        dist_mid = np.abs(np.abs(c64 - c32) - ulp / 2)
        assert np.all(dist_mid[nz] > 2.0 ** -50 * np.abs(c64[nz]))
    # a coarse map's rays are a subset of a fine map's rays
    e4 = orc.boundaries(64)
    e10 = orc.boundaries(1024)
    assert np.array_equal(e4[0], e10[0][::16]) and np.array_equal(e4[1], e10[1][::16])


@pytest.mark.parametrize("H,W", [(4, 4), (32, 32), (64, 64), (32, 128), (128, 128), (1024, 1024)])
def test_matches_atan2_away_from_boundaries(orc, H, W):
    rng = np.random.default_rng(7)
    d = synth.to_f32_dirs(rng.standard_normal((20000, 3)))
    x, y, z = (d[:, i].astype(np.float64) for i in range(3))
    phi = np.mod(np.arctan2(y, x), 2 * np.pi)
    fphi = phi * W / (2 * np.pi)
    fz = (z + 1.0) * H / 2.0
    far = (np.abs(fphi - np.round(fphi)) > 1e-4) & (np.abs(fz - np.round(fz)) > 1e-4)
    want = np.minimum(np.floor(fz), H - 1).astype(np.int64) * W + np.floor(fphi).astype(np.int64)
    rc, got = orc.bin_dirs(d, H, W)
    assert rc == 0
    assert far.sum() > 15000
    assert np.array_equal(got[far], want[far])


@pytest.mark.parametrize("W", [8, 64, 128])
def test_exact_boundary_rays(orc, W):
    ex, ey = orc.boundaries(W)
    H = 8
    b = np.arange(W)
    # the ray itself, and a dyadic multiple of it, is in the sector it opens
    for s in (1.0, 0.5, 4.0):
        d = np.stack([ex * s, ey * s, np.zeros(W, np.float32)], 1).astype(np.float32)
        rc, got = orc.bin_dirs(d, H, W)
        assert np.array_equal(got % W, b)
    # rotate by +-1e-5 rad: inside sector b, or inside sector b-1
    for eps, want in ((1e-5, b), (-1e-5, (b - 1) % W)):
        a = np.arctan2(ey.astype(np.float64), ex.astype(np.float64)) + eps
        d = np.stack([np.cos(a), np.sin(a), np.zeros(W)], 1).astype(np.float32)
        rc, got = orc.bin_dirs(d, H, W)
        assert np.array_equal(got % W, want)


def test_row_boundaries_exact(orc):
    for H in (4, 32, 128, 1024):
        b = np.arange(1, H)
        zb = (-1.0 + 2.0 * b / H).astype(np.float32)
        d = np.stack([np.ones(H - 1), np.zeros(H - 1), zb], 1).astype(np.float32)
        rc, got = orc.bin_dirs(d, H, 4)
        assert np.array_equal(got // 4, b)
        zm = np.nextafter(zb, np.float32(-2.0))
        d[:, 2] = zm
        rc, got = orc.bin_dirs(d, H, 4)
        assert np.array_equal(got // 4, b - 1)
    # outside [-1, 1]: clamped to the end rows
    d = np.array([[0, 0, 1.5], [0, 0, -3.0]], np.float32)
    rc, got = orc.bin_dirs(d, 16, 16)
    assert list(got // 16) == [15, 0]


def test_nonfinite_is_range_error(orc):
    d = np.array([[1, 0, 0], [np.nan, 0, 0], [0, np.inf, 0]], np.float32)
    rc, got = orc.bin_dirs(d, 8, 8)
    assert rc == orc.E_RANGE
    assert got[1] == -1 and got[2] == -1 and got[0] == 4 * 8


def test_bad_sizes(orc):
    d = np.zeros((1, 3), np.float32)
    for H, W in ((3, 8), (8, 6), (2, 8), (2048, 8), (8, 0)):
        rc, _ = orc.bin_dirs(d, H, W)
        assert rc == orc.E_ARG


def test_equal_area_uniform_sphere(orc):
    """Archimedes: uniform directions fill the z rows and phi columns uniformly."""
    rng = synth.rng_for(11)
    n = 400_000
    d = synth.to_f32_dirs(synth.unit_vectors(rng, n))
    H = W = 32
    rc, b = orc.bin_dirs(d, H, W)
    counts = np.bincount(b, minlength=H * W).reshape(H, W)
    for marg in (counts.sum(1), counts.sum(0)):
        p = stats.chisquare(marg).pvalue
        assert p > 1e-4, p
    assert stats.chisquare(counts.ravel()).pvalue > 1e-4


def test_vmf_row_marginal_closed_form(orc):
    """Rows of a vMF lobe about +z follow the closed-form z-CDF; phi uniform."""
    gold = {}
    for l in open(os.path.join(GOLD, "vmf_rows.txt")):
        if l[0] == "#":
            continue
        k, H, b, m = l.split()
        gold.setdefault((float(k), int(H)), {})[int(b)] = float(m)
    rng = synth.rng_for(12)
    n = 200_000
    for (k, H), masses in gold.items():
        exp = np.array([masses[b] for b in range(H)])
        assert abs(exp.sum() - 1) < 1e-12
        d = synth.to_f32_dirs(synth.vmf_directions(rng, np.tile([0.0, 0.0, 1.0], (n, 1)), np.full(n, k)))
        rc, b = orc.bin_dirs(d, H, 16)
        rows = np.bincount(b // 16, minlength=H)
        keep = exp * n >= 5
        obs = np.append(rows[keep], rows[~keep].sum())
        e = np.append(exp[keep], exp[~keep].sum()) * n
        if e[-1] == 0:
            obs, e = obs[:-1], e[:-1]
        assert stats.chisquare(obs, e * obs.sum() / e.sum()).pvalue > 1e-4
        cols = np.bincount(b % 16, minlength=16)
        assert stats.chisquare(cols).pvalue > 1e-4
    # the printed values of the closed form
    assert math.isclose(gold[(200.0, 32)][31], 0.99999627334682806, rel_tol=1e-12)
    assert math.isclose(gold[(20.0, 32)][31], 1 - math.exp(-1.25), rel_tol=1e-12)
