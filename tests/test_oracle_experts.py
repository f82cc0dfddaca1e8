"""Pins of the oracle's mixture of experts by photon count.

The paper trains five networks for the photon-count ranges [0,100),
[100,500), [500,1000), [1000,5000) and [5000,inf) (Sec. 8, Implementation,
training).  Checks: the counts at and around each range boundary land in the
paper's range (a literal table of the paper's numbers, so an off-by-one at a
boundary or a shifted range fails); five identical experts reproduce the
single network; two different experts give each leaf exactly its own
expert's map.
"""
import numpy as np

from paper_2010_01775_amd import synth

PAPER_BOUNDS = (100, 500, 1000, 5000)
# photon count -> index of the paper's range that contains it
PAPER_TABLE = {0: 0, 1: 0, 99: 0, 100: 1, 101: 1, 499: 1, 500: 2, 999: 2, 1000: 3, 4999: 3, 5000: 4,
               5001: 4, 78853: 4, 2**32 - 1: 4}


def test_expert_ranges_from_paper(orc):
    counts = np.array(list(PAPER_TABLE), dtype=np.int64)
    want = np.array([PAPER_TABLE[int(c)] for c in counts])
    assert np.array_equal(orc.expert_of(counts, PAPER_BOUNDS), want)


def test_single_expert_and_other_bounds(orc):
    assert np.array_equal(orc.expert_of([0, 7, 10**6], ()), [0, 0, 0])
    assert np.array_equal(orc.expert_of([0, 9, 10, 11], (10,)), [0, 0, 1, 1])


def _maps(seed, L, H):
    rng = np.random.default_rng(seed)
    x = rng.gamma(0.7, 1.0, (L, H, H))
    return x / x.reshape(L, -1).mean(1)[:, None, None]


def test_identical_experts_equal_one_network(orc):
    model = synth.cnn_model(5)
    x = _maps(1, 6, 8)
    photons = [0, 120, 700, 1500, 6000, 99]
    rc, one = orc.net_forward(model, x)
    rc2, mix = orc.experts_forward([model] * 5, photons, PAPER_BOUNDS, x)
    assert rc == 0 and rc2 == 0
    assert np.array_equal(one, mix)


def test_each_leaf_gets_its_own_expert(orc):
    a, b = synth.cnn_model(6), synth.cnn_model(7, random_bias=True)
    x = _maps(2, 5, 8)
    photons = [499, 500, 0, 501, 10]
    rc, mix = orc.experts_forward([a, b], photons, (500,), x)
    rc_a, ya = orc.net_forward(a, x)
    rc_b, yb = orc.net_forward(b, x)
    assert rc == rc_a == rc_b == 0
    for l, n in enumerate(photons):
        assert np.array_equal(mix[l], (ya if n < 500 else yb)[l]), l
    assert not np.array_equal(ya, yb)
