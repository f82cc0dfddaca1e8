"""GPU tests of the one-sample MIS calls (npg_mis_alpha, npg_sample_mis,
npg_eval_pdf_mis) against the oracle on the same tables: alpha bit-exact,
the strategy choice bit-exact, directions within 2e-6, pdfs within FP32
rounding of the oracle's mixture; the returned pdf equals the evaluated
mixture at the returned direction; sample statistics (BSDF frequency alpha,
E[1/pdf] = 4 pi); error outputs."""
import math

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


def _normals(rng, n):
    v = rng.standard_normal((n, 3))
    v[:6] = [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0], [0, -1e-9, -1], [0.6, 0, 0.8]]
    return (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)


def _tables(orc, seed, L, H, W, zero_frac):
    s = synth.random_density(seed, L, H, W, zero_frac=zero_frac).astype(np.float64)
    rc, pdf, marg, cond, tot = orc.build_cdf(s)
    assert rc == 0
    return pdf, marg, cond


def test_alpha_bit_exact(ctx, npg, orc):
    rng = np.random.default_rng(3)
    L = 5000
    nb = (rng.lognormal(0, 2, L) * (rng.random(L) > 0.1)).astype(np.float32)
    ng = (rng.lognormal(0, 2, L) * (rng.random(L) > 0.1)).astype(np.float32)
    qb = rng.integers(0, 120, L).astype(np.uint32)
    qg = rng.integers(0, 120, L).astype(np.uint32)
    qb[:4], qg[:4] = [49, 50, 50, 51], [50, 49, 50, 50]
    rc, want = orc.mis_alpha(nb, ng, qb, qg)
    a = npg.mis_alpha(ctx, tf(nb), tf(ng), t32(qb), t32(qg)).cpu().numpy()
    assert rc == 0 and npg.sync_status(ctx) == 0
    assert np.array_equal(a, want)
    assert a.min() >= 0.2 and a.max() <= 0.8
    bad = npg.mis_alpha(ctx, tf([np.nan, 1.0]), tf([1.0, -2.0]), t32(np.uint32([60, 60])),
                        t32(np.uint32([60, 60]))).cpu().numpy()
    assert npg.sync_status(ctx) == npg.E_RANGE
    assert np.array_equal(bad, np.float32([0.5, 0.5]))


@pytest.mark.parametrize("L,H,W,n", [(5, 32, 32, 200000), (3, 128, 128, 100000), (2, 8, 64, 20000)])
def test_sample_mis_parity(ctx, npg, orc, L, H, W, n):
    pdf, marg, cond = _tables(orc, 40 + L, L, H, W, 0.2)
    rng = synth.rng_for(50 + L)
    alpha = rng.uniform(0.2, 0.8, L).astype(np.float32)
    leaf = rng.integers(0, L, n).astype(np.uint32)
    normal = _normals(rng, n)
    u = synth.uniforms(rng, (n, 3))
    rc, d_ref, p_ref, s_ref = orc.sample_mis(pdf, marg, cond, alpha, leaf, normal, u)
    assert rc == 0
    tabs = npg.CdfTables(tf(pdf), tf(marg), tf(cond), None)
    d, p, st = npg.sample_mis(ctx, tabs, tf(alpha), t32(leaf), tf(normal), tf(u))
    assert npg.sync_status(ctx) == 0
    d, p, st = d.cpu().numpy(), p.cpu().numpy().astype(np.float64), st.cpu().numpy()
    assert np.array_equal(st, s_ref)
    assert np.max(np.abs(d - d_ref)) < 2e-6
    # the mixture at the returned direction (exact bin rule on the float32
    # direction; the guided branch's sampled bin for guided samples)
    rc, p_at = orc.eval_pdf_mis(pdf, alpha, leaf, normal, d.astype(np.float64))
    rc, _, pg, _ = orc.sample(pdf, marg, cond, leaf, u[:, 1:3])     # guide term of the sampled bin
    a = alpha[leaf].astype(np.float64)
    p_g = a * orc.cosine_pdf(normal, d.astype(np.float64)) + (1 - a) * pg.astype(np.float64)
    g = st == 0
    bs = ~g
    assert np.all(np.abs(p[bs] - p_at[bs]) <= 2e-6 * p_at[bs] + 1e-7)
    assert np.all(np.abs(p[g] - p_g[g]) <= 2e-6 * p_g[g] + 1e-7)
    assert np.all(np.abs(p[g] - p_ref[g]) <= 1e-5 * p_ref[g] + 1e-6)
    # returned pdf = GPU mixture evaluated at the returned direction
    pe = npg.eval_pdf_mis(ctx, tabs, tf(alpha), t32(leaf), tf(normal), tf(d)).cpu().numpy()
    assert np.array_equal(pe[bs], p[bs].astype(np.float32))
    mism = np.count_nonzero(pe[g] != p[g].astype(np.float32))
    assert mism <= max(3, n // 20000), mism


def test_eval_mis_parity(ctx, npg, orc):
    L, H, W, n = 4, 64, 64, 100000
    pdf, marg, cond = _tables(orc, 61, L, H, W, 0.3)
    rng = np.random.default_rng(62)
    alpha = rng.uniform(0.2, 0.8, L).astype(np.float32)
    leaf = rng.integers(0, L, n).astype(np.uint32)
    normal = _normals(rng, n)
    dirs = synth.unit_vectors(rng, n).astype(np.float32)
    rc, want = orc.eval_pdf_mis(pdf, alpha, leaf, normal, dirs)
    tabs = npg.CdfTables(tf(pdf), tf(marg), tf(cond), None)
    got = npg.eval_pdf_mis(ctx, tabs, tf(alpha), t32(leaf), tf(normal), tf(dirs)).cpu().numpy()
    assert rc == 0 and npg.sync_status(ctx) == 0
    assert np.all(np.abs(got - want) <= 2e-6 * want + 1e-7)


def test_sample_mis_statistics(ctx, npg, orc):
    """BSDF fraction per leaf = alpha; E[1/pdf] = 4 pi (the mixture is
    positive everywhere when no guide bin is zero)."""
    L, H, W, per = 4, 32, 32, 400000
    pdf, marg, cond = _tables(orc, 71, L, H, W, 0.0)
    alpha = np.float32([0.2, 0.35, 0.6, 0.8])
    leaf = np.repeat(np.arange(L, dtype=np.uint32), per)
    rng = synth.rng_for(72)
    normal = _normals(rng, L * per)
    u = synth.uniforms(rng, (L * per, 3))
    tabs = npg.CdfTables(tf(pdf), tf(marg), tf(cond), None)
    d, p, st = npg.sample_mis(ctx, tabs, tf(alpha), t32(leaf), tf(normal), tf(u))
    assert npg.sync_status(ctx) == 0
    p = p.cpu().numpy().astype(np.float64).reshape(L, per)
    st = st.cpu().numpy().reshape(L, per)
    for l in range(L):
        f = st[l].mean()
        assert abs(f - alpha[l]) < 5 * math.sqrt(alpha[l] * (1 - alpha[l]) / per), (l, f)
        inv = 1.0 / p[l]
        assert abs(inv.mean() - 4 * math.pi) < 5 * inv.std() / math.sqrt(per), (l, inv.mean())


def test_mis_errors(ctx, npg, orc):
    pdf, marg, cond = _tables(orc, 81, 2, 8, 8, 0.0)
    tabs = npg.CdfTables(tf(pdf), tf(marg), tf(cond), None)
    normal = np.float32([[0, 0, 1], [0, 0, 1], [0, 0, 1], [np.nan, 0, 1]])
    u = np.float32([[0.1, 0.2, 0.3], [0.5, 1.0, 0.1], [0.9, 0.1, 0.1], [0.5, 0.5, 0.5]])
    leaf = np.uint32([0, 0, 5, 1])
    d, p, st = npg.sample_mis(ctx, tabs, tf([0.5, 0.5]), t32(leaf), tf(normal), tf(u))
    assert npg.sync_status(ctx) == npg.E_RANGE
    d, p = d.cpu().numpy(), p.cpu().numpy()
    assert np.all(np.isfinite(d[0])) and np.all(np.isnan(d[1:])) and np.all(np.isnan(p[1:]))
    pe = npg.eval_pdf_mis(ctx, tabs, tf([0.5, 0.5]), t32(leaf), tf(normal), tf([[0, 0, 1]] * 4)).cpu().numpy()
    assert npg.sync_status(ctx) == npg.E_RANGE
    assert pe[0] > 0 and pe[2] == 0 and pe[3] == 0
