"""Sanity pins of the seeded input generators (not the method)."""
import math

import numpy as np

from paper_2010_01775_amd import synth


def test_uniforms_exact_grid():
    u = synth.uniforms(synth.rng_for(1), 100000)
    assert u.dtype == np.float32 and u.min() >= 0 and u.max() < 1
    assert np.all((u * 2 ** 24) == np.floor(u * 2 ** 24))


def test_vmf_mean_resultant_length():
    """E[cos] of a vMF lobe = coth(k) - 1/k."""
    rng = synth.rng_for(2)
    n = 200000
    for k in (5.0, 20.0, 200.0):
        mu = synth.unit_vectors(rng, 1)[0]
        d = synth.vmf_directions(rng, np.tile(mu, (n, 1)), np.full(n, k))
        c = d @ mu
        want = 1 / math.tanh(k) - 1 / k
        assert abs(c.mean() - want) < 5 * c.std() / math.sqrt(n)
        assert np.allclose(np.linalg.norm(d, axis=1), 1, atol=1e-12)


def test_weights_quantised():
    w = synth.photon_weights(synth.rng_for(3), 100000)
    assert w.dtype == np.uint32
    # lognormal(0, 0.5) mean exp(1/8) in units of 2^-16
    assert abs(w.mean() / 65536 - math.exp(0.125)) < 0.01


def test_batches_deterministic():
    a = synth.uniform_batch(seed=9, L=4, per_leaf=64, n_queries=16)
    b = synth.uniform_batch(seed=9, L=4, per_leaf=64, n_queries=16)
    assert np.array_equal(a.dirs, b.dirs) and np.array_equal(a.w, b.w)
    assert a.model == b.model
    s = synth.single_leaf()
    assert s.dirs.shape == (4096, 3) and s.L == 1 and s.q_u.shape == (65536, 2)
