"""Pins for the oracle's weighted permutation (problem WRP, Sections 1 and 7).

WRP permutes the items by the sequential process of WRS-N run to k = n, so
the probability of an ordering is prod_j w_{s_j} / (W - sum_{l<j} w_{s_l}).
The checks: exact enumeration of those probabilities on tiny inputs against
frequencies over seeds, the first k entries form the oracle's own WRS-N
sample for every k, equal weights give uniform orderings, the output is a
permutation, and zero-weight items come last in index order.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chi2

import workloads


def order_probabilities(w):
    """P(ordering) of the positive-weight items, from the sequential definition."""
    pos = [i for i in range(len(w)) if w[i] > 0]
    W = sum(Fraction(int(w[i])) for i in pos)
    probs = {}
    for order in itertools.permutations(pos):
        p, rest = Fraction(1), W
        for i in order:
            p *= Fraction(int(w[i])) / rest
            rest -= Fraction(int(w[i]))
        probs[order] = p
    return probs


def chi2_orders(orc, w, trials):
    probs = order_probabilities(w)
    keys = sorted(probs)
    index = {o: j for j, o in enumerate(keys)}
    npos = len(keys[0])
    counts = np.zeros(len(keys))
    wf = np.array(w, np.float32)
    for seed in range(trials):
        out = orc.permutation(wf, seed, 0)
        counts[index[tuple(int(x) for x in out[:npos])]] += 1
    expect = np.array([float(probs[o]) for o in keys]) * trials
    stat = float(((counts - expect) ** 2 / expect).sum())
    return float(chi2.sf(stat, len(keys) - 1))


def test_perm_order_probabilities_tiny(orc):
    assert chi2_orders(orc, [1, 2, 3, 6], 24000) > 1e-4
    assert chi2_orders(orc, [5, 1, 0, 2, 3], 24000) > 1e-4


def test_perm_equal_weights_uniform(orc):
    w = np.full(4, 2.5, np.float32)
    counts = {}
    trials = 24000
    for seed in range(trials):
        o = tuple(int(x) for x in orc.permutation(w, 1000 + seed, 3))
        counts[o] = counts.get(o, 0) + 1
    assert len(counts) == 24
    c = np.array(list(counts.values()), float)
    stat = float(((c - trials / 24) ** 2 / (trials / 24)).sum())
    assert chi2.sf(stat, 23) > 1e-4


@pytest.mark.parametrize("kind", ["uniform", "power"])
def test_perm_prefix_is_the_wor_sample(orc, kind):
    n = 5000
    w = workloads.uniform(n, 8) if kind == "uniform" else workloads.power_law(n, 0.5, 8)
    out = orc.permutation(w, 77, 2)
    assert np.array_equal(np.sort(out), np.arange(n))
    for k in (1, 2, 17, 1000, 4999, 5000):
        s, _ = orc.sample_wor(w, k, 77, 2)
        assert np.array_equal(np.sort(out[:k]), s), k


def test_perm_zero_weights_last_in_index_order(orc):
    rng = np.random.default_rng(4)
    w = workloads.uniform(3000, 4)
    zero = rng.random(3000) < 0.3
    w[zero] = 0.0
    w[np.nonzero(zero)[0][::2]] = np.float32(-0.0)
    out = orc.permutation(w, 5, 0)
    npos = int((~zero).sum())
    assert np.array_equal(out[npos:], np.nonzero(zero)[0])
    assert not zero[out[:npos]].any()


def test_perm_keys_ascending_and_domain(orc):
    w = workloads.power_law(2000, 1.0, 6)
    out = orc.permutation(w, 9, 1)
    keys = orc.wor_keys(w, 9, 1)
    assert np.all(np.diff(keys[out]) >= 0)
    with pytest.raises(orc.OracleError):
        orc.permutation(np.array([1.0, -2.0], np.float32), 1, 0)
    with pytest.raises(orc.OracleError):
        orc.permutation(np.array([1.0, np.nan], np.float32), 1, 0)
