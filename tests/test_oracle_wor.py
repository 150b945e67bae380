"""Pins for the oracle's sampling without replacement (CPU only).

Problem WRS-N (Section 1) fixes the probability of every ordered sample:
P(s_1..s_k) = prod_j w_{s_j} / (W - sum_{l<j} w_{s_l}).  Section 2.3 reaches it
with exponential clocks.  The checks: exact enumeration of set probabilities on
tiny inputs against frequencies over seeds, k = 1 reduces to P(i) = w_i / W,
equal weights give uniform subsets, keys times weights are Exp(1), and the
selected set equals the k smallest keys found by brute force.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chi2, kstest

import workloads


def set_probabilities(w, k):
    """P(sample set = S) from the sequential-removal definition, exactly."""
    n = len(w)
    W = sum(Fraction(int(x)) for x in w)
    probs = {}
    for order in itertools.permutations([i for i in range(n) if w[i] > 0], k):
        p = Fraction(1)
        rest = W
        for i in order:
            p *= Fraction(int(w[i])) / rest
            rest -= Fraction(int(w[i]))
        key = tuple(sorted(order))
        probs[key] = probs.get(key, 0) + p
    return probs


def chi2_sets(orc, w, k, trials):
    probs = set_probabilities(w, k)
    keys = sorted(probs)
    index = {s: j for j, s in enumerate(keys)}
    counts = np.zeros(len(keys))
    wf = np.array(w, np.float32)
    for seed in range(trials):
        out, _ = orc.sample_wor(wf, k, seed, 0)
        counts[index[tuple(int(x) for x in out)]] += 1
    expect = np.array([float(probs[s]) for s in keys]) * trials
    stat = float(((counts - expect) ** 2 / expect).sum())
    return float(chi2.sf(stat, len(keys) - 1))


def test_wor_set_probabilities_tiny(orc):
    assert chi2_sets(orc, [1, 2, 3, 4, 6], 2, 20000) > 1e-4
    assert chi2_sets(orc, [5, 1, 1, 2, 0, 3], 3, 20000) > 1e-4


def test_wor_k1_is_weighted_choice(orc):
    w = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.float32)
    counts = np.zeros(w.size)
    trials = 40000
    for seed in range(trials):
        out, _ = orc.sample_wor(w, 1, seed, 7)
        counts[out[0]] += 1
    expect = trials * w / w.sum()
    stat = float(((counts - expect) ** 2 / expect).sum())
    assert chi2.sf(stat, w.size - 1) > 1e-4


def test_wor_equal_weights_uniform_subsets(orc):
    n, k, trials = 6, 2, 15000
    w = np.full(n, 2.5, np.float32)
    counts = {}
    for seed in range(trials):
        out, _ = orc.sample_wor(w, k, seed, 1)
        counts[tuple(out)] = counts.get(tuple(out), 0) + 1
    m = math.comb(n, k)
    assert len(counts) == m
    obs = np.array(list(counts.values()), np.float64)
    stat = float(((obs - trials / m) ** 2 / (trials / m)).sum())
    assert chi2.sf(stat, m - 1) > 1e-4


def test_wor_keys_are_exponential(orc):
    w = workloads.power_law(1 << 16, 0.5, 3)
    keys = orc.wor_keys(w, 3, 0)
    e = keys * w.astype(np.float64)          # -ln(u_i), must be Exp(1)
    assert kstest(e, "expon").pvalue > 1e-4
    assert np.all(e >= 0)


def test_wor_brute_force_selection(orc):
    rng = np.random.default_rng(8)
    for trial in range(40):
        n = int(rng.integers(1, 2000))
        w = rng.integers(0, 4, n).astype(np.float32)   # many equal keys' weights, zeros
        pos = int((w > 0).sum())
        if pos == 0:
            continue
        k = int(rng.integers(1, pos + 1))
        out, kth = orc.sample_wor(w, k, trial, 5)
        keys = orc.wor_keys(w, trial, 5)
        order = np.lexsort((np.arange(n), keys))     # by key, then by index
        want = np.sort(order[:k])
        assert np.array_equal(out, want)
        assert kth == keys[order[k - 1]]
        assert np.all(np.diff(out) > 0)


def test_wor_domain_errors(orc):
    w = np.array([1, 0, 2], np.float32)
    with pytest.raises(orc.OracleError) as e:
        orc.sample_wor(w, 3, 0, 0)                    # k > number of positive weights
    assert e.value.code == orc.EDOMAIN
    out, _ = orc.sample_wor(w, 2, 0, 0)
    assert list(out) == [0, 2]
    with pytest.raises(orc.OracleError):
        orc.sample_wor(np.array([1, -1], np.float32), 1, 0, 0)
