"""Pins of the oracle's pdf/CDF tables (Eq. "energy_target"; environment-map
style inversion, Sec. 7.3) and of its sampler and pdf evaluation.

Checks: a uniform density gives pdf 1/(4 pi) and linear tables; every pdf
integrates to one over the sphere; tables are monotone with exact end points
and their differences reproduce the row masses and conditional masses
(numpy cumsum in float64 as the independent routine); zero rows get a
uniform conditional; an all-zero leaf is an error; samples of a one-hot map
land in its bin; chi-square of sampled bins against p; the mean of 1/pdf is
4 pi (unbiasedness); a uniform map gives uniform z; the in-bin offsets are
uniform; eval_pdf agrees with the sampler's pdf; a hand-worked 4x4 case.
"""
import math

import numpy as np
from scipy import stats

from paper_2010_01775_amd import synth


def test_uniform_density(orc):
    H, W = 8, 16
    s = np.full((2, H, W), 0.7)
    rc, pdf, marg, cond, tot = orc.build_cdf(s)
    assert rc == 0
    assert np.allclose(pdf, 1 / (4 * math.pi), rtol=1e-7)
    assert np.array_equal(marg[0], (np.arange(H + 1) / H).astype(np.float32))
    assert np.array_equal(cond[0, 3], (np.arange(W + 1) / W).astype(np.float32))
    assert np.allclose(tot, 0.7 * H * W)


def test_tables_against_cumsum(orc):
    s = synth.random_density(3, 6, 32, 64, zero_frac=0.3).astype(np.float64)
    s[2, 5, :] = 0.0                    # an empty row
    s[4, :, :] = 0.0
    s[4, 7, 9] = 3.0                    # a one-hot leaf
    rc, pdf, marg, cond, tot = orc.build_cdf(s)
    assert rc == 0
    L, H, W = s.shape
    S = s.reshape(L, -1).sum(1)
    p = s / S[:, None, None]
    # pdf integrates to one
    assert np.allclose(pdf.reshape(L, -1).astype(np.float64).sum(1) * 4 * math.pi / (H * W), 1, atol=1e-6)
    assert np.allclose(tot, S, rtol=1e-15)
    m = p.sum(2)
    M = np.concatenate([np.zeros((L, 1)), np.cumsum(m, 1)], 1)
    M[:, -1] = 1.0
    assert np.allclose(marg, M, atol=1e-7)
    assert np.all(np.diff(marg, axis=1) >= 0) and np.all(marg[:, 0] == 0) and np.all(marg[:, -1] == 1)
    assert np.all(np.diff(cond, axis=2) >= 0) and np.all(cond[:, :, 0] == 0) and np.all(cond[:, :, -1] == 1)
    Cr = np.concatenate([np.zeros((L, H, 1)), np.cumsum(p, 2)], 2)
    nz = m > 0
    Cn = np.where(nz[:, :, None], Cr / np.where(nz, m, 1)[:, :, None], np.arange(W + 1) / W)
    Cn[:, :, -1] = 1
    assert np.allclose(cond, Cn, atol=1e-7)
    assert np.array_equal(cond[2, 5], (np.arange(W + 1) / W).astype(np.float32))
    assert np.allclose(pdf, p * H * W / (4 * math.pi), rtol=1e-6)


def test_zero_leaf_is_error(orc):
    s = np.ones((3, 4, 4))
    s[1] = 0
    rc, pdf, marg, cond, tot = orc.build_cdf(s)
    assert rc == orc.E_RANGE
    assert np.all(np.isnan(pdf[1])) and tot[1] == 0
    assert np.all(np.isfinite(pdf[0])) and np.all(np.isfinite(pdf[2]))


def _tables(orc, s):
    rc, pdf, marg, cond, tot = orc.build_cdf(s)
    assert rc == 0
    return pdf, marg, cond


def test_one_hot_samples(orc):
    H, W = 16, 32
    s = np.zeros((1, H, W))
    s[0, 11, 5] = 1.0
    pdf, marg, cond = _tables(orc, s)
    rng = synth.rng_for(2)
    n = 5000
    u = np.stack([synth.uniforms(rng, n), synth.uniforms(rng, n)], 1)
    rc, d, p, b = orc.sample(pdf, marg, cond, np.zeros(n, np.uint32), u)
    assert rc == 0
    assert np.all(b == 11 * W + 5)
    assert np.all(p == np.float32(H * W / (4 * math.pi)))
    assert np.allclose(np.linalg.norm(d, axis=1), 1, atol=1e-12)
    rc, bins = orc.bin_dirs(d.astype(np.float32), H, W)
    assert np.mean(bins == 11 * W + 5) > 0.999


def test_chi_square_and_unbiasedness(orc):
    H, W = 32, 32
    s = synth.random_density(5, 1, H, W, zero_frac=0.2).astype(np.float64)
    pdf, marg, cond = _tables(orc, s)
    rng = synth.rng_for(6)
    n = 400_000
    u = np.stack([synth.uniforms(rng, n), synth.uniforms(rng, n)], 1)
    rc, d, p, b = orc.sample(pdf, marg, cond, np.zeros(n, np.uint32), u)
    assert rc == 0
    pk = (s[0] / s[0].sum()).ravel()
    assert np.all(pk[b] > 0)                       # zero bins never sampled
    obs = np.bincount(b, minlength=H * W)
    keep = pk * n >= 5
    e = pk[keep] * n
    o = obs[keep]
    assert stats.chisquare(o, e * o.sum() / e.sum()).pvalue > 1e-4
    # E[1/pdf] = solid angle of the support = 4 pi * (nonzero bins) / (H W)
    inv = 1.0 / p.astype(np.float64)
    se = inv.std() / math.sqrt(n)
    support = 4 * math.pi * np.count_nonzero(pk) / (H * W)
    assert abs(inv.mean() - support) < 5 * se
    # sampled directions evaluate to the pdf the sampler returned
    rc, pe = orc.eval_pdf(pdf, np.zeros(n, np.uint32), d.astype(np.float32))
    assert np.mean(pe != p) < 1e-4


def test_uniform_map_uniform_z_and_offsets(orc):
    H, W = 16, 16
    pdf, marg, cond = _tables(orc, np.ones((1, H, W)))
    rng = synth.rng_for(7)
    n = 100_000
    u = np.stack([synth.uniforms(rng, n), synth.uniforms(rng, n)], 1)
    rc, d, p, b = orc.sample(pdf, marg, cond, np.zeros(n, np.uint32), u)
    assert stats.kstest(d[:, 2], stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-4
    phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
    assert stats.kstest(phi, stats.uniform(scale=2 * np.pi).cdf).pvalue > 1e-4
    # in-bin offsets of a non-uniform map are uniform
    s = synth.random_density(8, 1, H, W).astype(np.float64)
    pdf, marg, cond = _tables(orc, s)
    rc, d, p, b = orc.sample(pdf, marg, cond, np.zeros(n, np.uint32), u)
    t1 = (d[:, 2] + 1) * H / 2 - b // W
    t2 = phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi) * W / (2 * np.pi) - b % W
    for t in (t1, t2):
        t = np.clip(t, 0, 1)
        assert stats.kstest(t, "uniform").pvalue > 1e-4


def test_hand_worked_4x4(orc):
    """Row masses 1/8, 3/8, 0, 1/2; row 1 split 1:2 over columns 0 and 3."""
    s = np.zeros((1, 4, 4))
    s[0, 0, :] = 1.0       # row 0: 4 units, uniform
    s[0, 1, 0] = 4.0       # row 1: 12 units, 1:2
    s[0, 1, 3] = 8.0
    s[0, 3, 2] = 16.0      # row 3: 16 units, one bin
    pdf, marg, cond = _tables(orc, s)
    assert list(marg[0]) == [0.0, 0.125, 0.5, 0.5, 1.0]
    assert np.allclose(cond[0, 1], [0, 1 / 3, 1 / 3, 1 / 3, 1])
    u = np.array([[0.0, 0.0],          # row 0 col 0, offsets 0 -> z = -1 (pole)
                  [0.125, 0.5],        # exactly M_1 -> row 1; u2 = 0.5 -> col 3
                  [0.4999999701976776, 0.2],   # just below M_2 -> row 1, col 0
                  [0.5, 0.0],          # M_2 = M_3 = 0.5 -> empty row 2 skipped -> row 3
                  [0.75, 0.999999940395355]], np.float32)
    rc, d, p, b = orc.sample(pdf, marg, cond, np.zeros(5, np.uint32), u)
    assert rc == 0
    assert list(b) == [0, 1 * 4 + 3, 1 * 4 + 0, 3 * 4 + 2, 3 * 4 + 2]
    assert np.allclose(d[0], [0, 0, -1])
    # query 1: t1 = 0 -> z = -1 + 2*1/4 = -0.5; t2 = (0.5 - 1/3)/(2/3) = 0.25 -> phi = 2pi*3.25/4
    z = -0.5
    phi = 2 * math.pi * 3.25 / 4
    r = math.sqrt(1 - z * z)
    assert np.allclose(d[1], [r * math.cos(phi), r * math.sin(phi), z], atol=1e-7)
    # query 3: row 3, t1 = 0, col 2 (C = [0,0,0,1,1]): t2 = 0 -> z = 0.5, phi = pi
    assert np.allclose(d[3], [-math.sqrt(0.75), 0, 0.5], atol=1e-7)
    assert np.allclose(p, pdf[0].ravel()[b])


def test_sample_and_eval_errors(orc):
    pdf, marg, cond = _tables(orc, np.ones((2, 4, 4)))
    leaf = np.array([0, 2, 1, 1], np.uint32)
    u = np.array([[0.5, 0.5], [0.5, 0.5], [1.0, 0.2], [-0.0, 0.2]], np.float32)
    rc, d, p, b = orc.sample(pdf, marg, cond, leaf, u)
    assert rc == orc.E_RANGE
    assert np.all(np.isfinite(d[0])) and np.all(np.isnan(d[1])) and np.all(np.isnan(d[2]))
    assert np.isfinite(p[3]) and b[1] == 0xFFFFFFFF and b[2] == 0xFFFFFFFF
    dirs = np.array([[0, 0, 1], [0, 0, 1], [np.nan, 0, 0]], np.float32)
    rc, pe = orc.eval_pdf(pdf, np.array([1, 5, 0], np.uint32), dirs)
    assert rc == orc.E_RANGE
    assert pe[0] == pdf[1, 3, 0] and pe[1] == 0 and pe[2] == 0


def test_fp32_tables_total_variation(orc):
    """The float32 tables select bins with probabilities (M_{i+1} - M_i) *
    (C_{i,j+1} - C_{i,j}); every stored prefix is within half an ulp (at most
    2^-25) of the float64 prefix, so the total-variation distance to p is at
    most (H + W) * 2^-24 / 2, even for spiky maps with zero rows."""
    for seed, (H, W), spike in ((21, (32, 32), False), (22, (64, 64), True), (23, (128, 16), True)):
        s = synth.random_density(seed, 6, H, W, zero_frac=0.3).astype(np.float64)
        if spike:
            s[1] *= 1e-12
            s[1, 3, 5] = 1.0                           # one dominant bin
            s[2, : H // 2] = 0.0                       # zero rows
        rc, pdf, marg, cond, tot = orc.build_cdf(s)
        assert rc == 0
        for l in range(s.shape[0]):
            p = s[l] / s[l].sum()
            m = np.diff(marg[l].astype(np.float64))
            c = np.diff(cond[l].astype(np.float64), axis=1)
            q = m[:, None] * c
            assert abs(q.sum() - 1.0) < 1e-12
            tv = 0.5 * np.abs(q - p).sum()
            assert tv <= (H + W) * 2.0 ** -25, (seed, l, tv)
