"""Pins of the oracle's one-sample MIS (Sec. 7.3, Eq. "mis_alpha" and
Eq. "mis_coef") with the cosine-lobe stand-in BSDF.

Checks: alpha on hand-computed cases (below 50 bounces per strategy, equal
averages, ratios that land inside and outside the clamp, averages over
different bounce counts, zero contributions, bad input); the Duff et al.
frame is orthonormal and right-handed; cosine samples lie in the hemisphere
with E[n.w] = 2/3 and E[(n.w)^2] = 1/2 (moments of the cosine lobe); the
cosine pdf and the mixture pdf integrate to 1 over the sphere (midpoint
quadrature); MIS samples pick the BSDF with frequency alpha, satisfy
E[1/pdf] = 4 pi (the mixture is positive everywhere), and their returned pdf
equals the mixture pdf evaluated at the returned direction.
"""
import math

import numpy as np

from paper_2010_01775_amd import synth


def test_alpha_hand_cases(orc):
    #            nu_B   nu_G   Q_B  Q_G   alpha
    cases = [(1.0, 1.0, 49, 500, 0.5),       # BSDF side below 50 bounces
             (1.0, 1.0, 500, 49, 0.5),       # guided side below 50
             (2.0, 2.0, 50, 50, 0.5),        # equal averages
             (3.0, 1.0, 50, 50, 0.75),       # 3/(3+1)
             (9.0, 1.0, 50, 50, 0.8),        # 0.9 clamped to 0.8
             (1.0, 9.0, 50, 50, 0.2),        # 0.1 clamped to 0.2
             (10.0, 30.0, 100, 50, 0.2),     # averages 0.1 and 0.6: 1/7 -> 0.2
             (30.0, 30.0, 100, 50, 1 / 3),   # averages 0.3 and 0.6
             (0.0, 0.0, 80, 80, 0.5),        # no contribution at all
             (0.0, 5.0, 80, 80, 0.2),        # guiding only -> lower clamp
             (7.0, 0.0, 80, 80, 0.8)]        # BSDF only -> upper clamp
    nb, ng, qb, qg, want = map(np.array, zip(*cases))
    rc, a = orc.mis_alpha(nb, ng, qb.astype(np.uint32), qg.astype(np.uint32))
    assert rc == 0
    assert np.array_equal(a, want.astype(np.float32))
    rc, a = orc.mis_alpha([np.nan, -1.0, 1.0], [1.0, 1.0, np.inf], [60] * 3, [60] * 3)
    assert rc == orc.E_RANGE and np.array_equal(a, np.float32([0.5, 0.5, 0.5]))


def _normals(n, seed=3):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    special = [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, -1e-9, -1]]   # poles, equator, near -z
    k = min(n, 4) if n >= 4 else 0
    v[:k] = special[:k]
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_frame_orthonormal(orc):
    n = _normals(2000)
    t, b = orc.onb(n)
    dot = lambda x, y: np.sum(x * y, axis=1)
    for v in (t, b):
        assert np.allclose(dot(v, v), 1.0, atol=1e-12)
        assert np.allclose(dot(v, n), 0.0, atol=1e-12)
    assert np.allclose(dot(t, b), 0.0, atol=1e-12)
    assert np.allclose(np.cross(t, b), n, atol=1e-12)


def test_cosine_sample_moments(orc):
    rng = np.random.default_rng(5)
    m = 400_000
    n = np.repeat(_normals(8, 9), m // 8, axis=0)
    w = orc.cosine_sample(n, rng.random(m), rng.random(m))
    c = np.sum(w * n, axis=1)
    assert np.allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-12)
    assert c.min() >= 0.0
    assert abs(c.mean() - 2 / 3) < 4 * math.sqrt(1 / 18 / m)          # var of cos = 1/2 - 4/9
    assert abs((c * c).mean() - 0.5) < 4 * math.sqrt((1 / 3 - 1 / 4) / m)


def _sphere_grid(k):
    z = -1 + (np.arange(k) + 0.5) * 2 / k
    phi = (np.arange(2 * k) + 0.5) * math.pi / k
    zz, pp = np.meshgrid(z, phi, indexing="ij")
    r = np.sqrt(1 - zz ** 2)
    d = np.stack([r * np.cos(pp), r * np.sin(pp), zz], -1).reshape(-1, 3)
    return d, 4 * math.pi / d.shape[0]        # equal-area cells


def test_pdfs_integrate_to_one(orc):
    d, dw = _sphere_grid(400)
    n = np.repeat(np.array([[0.3, -0.5, 0.8]]) / math.sqrt(0.98), d.shape[0], axis=0)
    assert abs(orc.cosine_pdf(n, d).sum() * dw - 1) < 1e-4
    rng = np.random.default_rng(7)
    s = rng.gamma(0.5, 1.0, (2, 16, 16))
    rc, pdf, marg, cond, tot = orc.build_cdf(s)
    for a in (0.2, 0.65):
        rc, p = orc.eval_pdf_mis(pdf, np.float32([a, a]), np.ones(d.shape[0], np.uint32), n,
                                 d.astype(np.float32))
        assert rc == 0
        assert abs(p.sum() * dw - 1) < 2e-3


def _tables(seed, L, H):
    rng = np.random.default_rng(seed)
    s = rng.gamma(0.7, 1.0, (L, H, H)) + 1e-3
    rc, pdf, marg, cond, tot = orc_build(s)
    return pdf, marg, cond


def orc_build(s):
    from oracle import oracle
    return oracle.build_cdf(s)


def test_mis_samples(orc):
    L, H, m = 3, 16, 300_000
    pdf, marg, cond = _tables(1, L, H)
    rng = synth.rng_for(17)
    alpha = np.float32([0.2, 0.5, 0.8])
    leaf = rng.integers(0, L, m).astype(np.uint32)
    normal = _normals(m, 19)
    u = synth.uniforms(rng, (m, 3))
    rc, d, p, strat = orc.sample_mis(pdf, marg, cond, alpha, leaf, normal, u)
    assert rc == 0
    for l in range(L):
        sel = leaf == l
        f = strat[sel].mean()
        assert abs(f - alpha[l]) < 5 * math.sqrt(alpha[l] * (1 - alpha[l]) / sel.sum()), (l, f)
        inv = 1.0 / p[sel]
        assert abs(inv.mean() - 4 * math.pi) < 5 * inv.std() / math.sqrt(sel.sum()), (l, inv.mean())
    rc, pe = orc.eval_pdf_mis(pdf, alpha, leaf, normal, d)
    g = strat == 0
    assert np.array_equal(p[~g], pe[~g])                 # BSDF samples: same bin rule
    mism = np.sum(np.abs(p[g] - pe[g]) > 1e-12 * pe[g])  # guided: sampled bin vs re-binned
    assert mism <= 3, mism


def test_mis_errors(orc):
    pdf, marg, cond = _tables(2, 2, 8)
    n = _normals(4, 23)
    n[3] = np.nan
    u = np.float32([[0.1, 0.2, 0.3], [0.5, 1.0, 0.1], [0.9, 0.1, 0.1], [0.5, 0.5, 0.5]])
    rc, d, p, s = orc.sample_mis(pdf, marg, cond, np.float32([0.5, 0.5]), np.uint32([0, 0, 5, 1]), n, u)
    assert rc == orc.E_RANGE
    assert np.all(np.isfinite(d[0])) and np.all(np.isnan(d[1:])) and np.all(np.isnan(p[1:]))
