"""Pins of the oracle's output-sensitive sampling with replacement (Section 5).

What fixes it independently of the oracle's own code:
  - its logarithm, square root and log-factorial against the C library
    (math.log, math.sqrt, math.lgamma);
  - its binomial variates against the exact binomial law (scipy.stats.binom),
    by chi-square, in both generator regimes (mean below 10 and above), with
    the p > 1/2 reflection, and the degenerate cases;
  - the grouping by binary exponent against math.frexp on a hand-made input;
  - the sample: multiplicities add up to k over distinct positive items; the
    joint law of a k = 3 sample of five items spread over five groups against
    the exact multinomial probabilities; per-item frequencies of a large sample
    against w_i / W; the cases with one positive item, k = 0 and bad weights.
"""
import itertools
import math
from collections import Counter

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads


def test_elementary_functions_match_libm():
    xs = np.concatenate([np.geomspace(1e-300, 1e300, 2001), [0.5, 0.7071067811865476, 1.0, 1.0 + 2 ** -52,
                                                             2.0, 3.0, 10.0, 0.1]])
    for x in xs:
        ref = math.log(x)
        got = oracle.os_log(x)
        assert abs(got - ref) <= 4 * math.ulp(ref) + 1e-300, x
        assert abs(oracle.os_sqrt(x) - math.sqrt(x)) <= math.ulp(math.sqrt(x)), x
    assert oracle.os_log(0.0) == -math.inf
    for j in list(range(0, 40)) + [100, 12345, 10 ** 6, 2 ** 30, 2 ** 31 - 1]:
        ref = math.lgamma(j + 1)
        assert abs(oracle.os_lfact(j) - ref) <= 1e-10 * max(1.0, ref), j


def binomial_chi2(m, rho, draws, tag):
    x = np.array([oracle.os_binomial(m, rho, 11, h, tag) for h in range(draws)])
    assert x.min() >= 0 and x.max() <= m
    pmf = stats.binom.pmf(np.arange(m + 1), m, rho)
    exp = pmf * draws
    # bins with expected count >= 5; the tails are lumped
    lo = int(np.argmax(exp >= 5))
    hi = int(len(exp) - np.argmax(exp[::-1] >= 5))
    obs = np.bincount(x, minlength=m + 1).astype(float)
    o = np.concatenate([[obs[:lo].sum()], obs[lo:hi], [obs[hi:].sum()]])
    e = np.concatenate([[exp[:lo].sum()], exp[lo:hi], [exp[hi:].sum()]])
    keep = e > 0
    return stats.chisquare(o[keep], e[keep] * o[keep].sum() / e[keep].sum()).pvalue


@pytest.mark.parametrize("m,rho", [(1, 0.3), (7, 0.5), (40, 0.1), (30, 0.97), (100, 0.5), (1000, 0.23),
                                   (5000, 0.9), (200000, 0.001)])
def test_binomial_law(m, rho):
    assert binomial_chi2(m, rho, 20000, 3) > 1e-4


def test_binomial_large_m_moments_and_degenerate_cases():
    m = 2 ** 30
    for rho in (0.37, 1e-6, 0.999):
        x = np.array([oracle.os_binomial(m, rho, 5, h, 9) for h in range(4000)], dtype=float)
        mu, sd = m * rho, math.sqrt(m * rho * (1 - rho))
        assert abs(x.mean() - mu) < 5 * sd / math.sqrt(len(x))
        assert abs(x.std() / sd - 1) < 0.06
    assert oracle.os_binomial(0, 0.5, 1, 1, 0) == 0
    assert oracle.os_binomial(10, 0.0, 1, 1, 0) == 0
    assert oracle.os_binomial(10, 1.0, 1, 1, 0) == 10
    # a draw is a function of (seed, node, tag) only
    assert oracle.os_binomial(1000, 0.4, 3, 17, 2) == oracle.os_binomial(1000, 0.4, 3, 17, 2)


def test_groups_by_binary_exponent():
    w = np.array([3.0, 0.0, 1.5, 1e-40, 2.5, 0.75, 3.9, 1.4e-45, 0.0], np.float32)
    order, exps, starts, counts = oracle.os_groups(w)
    e = {i: math.frexp(float(w[i]))[1] - 1 for i in range(w.size) if w[i] > 0}
    want_exps = sorted(set(e.values()), reverse=True)
    assert list(exps) == want_exps
    want_order = [i for g in want_exps for i in sorted(i for i in e if e[i] == g)]
    assert list(order) == want_order
    assert list(counts) == [sum(1 for i in e if e[i] == g) for g in want_exps]
    assert list(starts) == list(np.concatenate([[0], np.cumsum(counts)[:-1]]))
    assert want_exps[-1] == -149 and -133 in want_exps


def check_sample(w, k, seed):
    items, counts = oracle.os_sample(w, k, seed)
    assert counts.sum() == k
    assert np.all(counts >= 1) and np.all(np.diff(items) > 0)
    assert np.all(w[items] > 0)
    return items, counts


@pytest.mark.parametrize("k", [1, 2, 17, 1000, 100000])
def test_sample_invariants(k):
    w = workloads.power_law(3000, 1.0, 4).copy()
    w[::7] = 0.0
    items, counts = check_sample(w, k, 8)
    assert len(items) <= min(k, int((w > 0).sum()))


def test_joint_law_of_a_small_sample():
    w = np.array([1.0, 0.3, 0.05, 2.5e-3, 7.0], np.float32)  # five groups
    p = w.astype(np.float64) / w.astype(np.float64).sum()
    k, R = 3, 30000
    seen = Counter()
    for seed in range(R):
        items, counts = check_sample(w, k, seed)
        seen[tuple(zip(items.tolist(), counts.tolist()))] += 1
    outcomes, probs = [], []
    for c in itertools.product(range(k + 1), repeat=len(w)):
        if sum(c) != k:
            continue
        key = tuple((i, ci) for i, ci in enumerate(c) if ci)
        outcomes.append(key)
        probs.append(stats.multinomial.pmf(c, k, p))
    exp = np.array(probs) * R
    obs = np.array([seen.get(o, 0) for o in outcomes], float)
    assert sum(seen.values()) == obs.sum()  # nothing outside the support
    big = exp >= 5
    o = np.concatenate([obs[big], [obs[~big].sum()]])
    e = np.concatenate([exp[big], [exp[~big].sum()]])
    assert stats.chisquare(o, e * o.sum() / e.sum()).pvalue > 1e-4


def test_item_frequencies_of_a_large_sample():
    w = workloads.power_law(2000, 1.0, 6)
    p = w.astype(np.float64) / w.astype(np.float64).sum()
    k = 1 << 30
    items, counts = check_sample(w, k, 21)
    full = np.zeros(w.size)
    full[items] = counts
    sd = np.sqrt(k * p * (1 - p))
    assert np.all(np.abs(full - k * p) <= 6 * sd + 1)
    k = 200000
    tot = np.zeros(w.size)
    for seed in range(5):
        items, counts = check_sample(w, k, 100 + seed)
        tot[items] += counts
    exp = p * 5 * k
    big = exp >= 5
    o, e = tot[big], exp[big]
    if (~big).any():
        o = np.concatenate([o, [tot[~big].sum()]])
        e = np.concatenate([e, [exp[~big].sum()]])
    assert stats.chisquare(o, e).pvalue > 1e-4


def test_special_cases():
    w = np.zeros(100, np.float32)
    w[37] = 0.25
    items, counts = oracle.os_sample(w, 12345, 1)
    assert list(items) == [37] and list(counts) == [12345]
    items, counts = oracle.os_sample(workloads.uniform(50, 1), 0, 1)
    assert items.size == 0
    for bad in (-1.0, float("nan"), float("inf")):
        x = workloads.uniform(10, 2).copy()
        x[3] = bad
        with pytest.raises(oracle.OracleError):
            oracle.os_sample(x, 10, 1)
    with pytest.raises(oracle.OracleError):
        oracle.os_sample(np.zeros(5, np.float32), 10, 1)


def test_distinct_count_matches_closed_form():
    """s, the number of distinct items in k draws, against
    E[X] = sum_i 1 - (1 - w_i/W)^k (the distinct-count closed form that the
    paper's query figure plots as output size / sample size)."""
    for s, n, k in ((1.0, 1 << 14, 1 << 16), (0.5, 1 << 12, 1 << 14), (2.0, 1 << 14, 1 << 20)):
        w = workloads.power_law(n, s, 22)
        items, counts = oracle.os_sample(w, k, 78)
        p = w.astype(np.float64) / w.astype(np.float64).sum()
        q = -np.expm1(k * np.log1p(-p))
        ex = float(q.sum())
        sd = math.sqrt(float((q * (1 - q)).sum()))  # indicators are negatively correlated
        assert abs(items.size - ex) <= 6 * sd + 1, (s, items.size, ex)


def test_single_group_is_uniform():
    """Equal weights form one group (the top tree is a single leaf): the
    sample is uniform over the items (chi-square over 20 seeds)."""
    n, k = 500, 20000
    w = np.full(n, 0.75, np.float32)
    order, exps, starts, cnts = oracle.os_groups(w)
    assert list(exps) == [-1] and list(cnts) == [n] and np.array_equal(order, np.arange(n))
    tot = np.zeros(n)
    for seed in range(20):
        items, counts = check_sample(w, k, 300 + seed)
        tot[items] += counts
    assert stats.chisquare(tot).pvalue > 1e-4
