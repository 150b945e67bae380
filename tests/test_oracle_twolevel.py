"""Pins for the oracle's 2-level alias table (Section 4.4, replicated top level).

The construction is tied to the plain sweep it must reduce to (one block
holding every item: a trivial top level over the sweep's table; blocks of one
item: a trivial block level under the sweep's table over the items), to the
alias-table definition applied twice (each item's probability, in exact
rationals, is w_i / W), and the two-step query to the distribution of its
draws (chi-square) and to its counter-addressed form.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chi2

import workloads
from test_oracle_tables import exact_masses


def _inputs():
    for trial in range(8):
        n = int(np.random.default_rng(70 + trial).integers(1, 2500))
        yield n, workloads.uniform(n, 70 + trial) if trial % 2 == 0 else workloads.power_law(n, 1.0, 70 + trial)


def test_one_block_is_the_sweep(orc):
    for n, w in _inputs():
        tt, at, t, a = orc.twolevel_build(w, n + 5)
        assert tt.tolist() == [1.0] and at.tolist() == [0]
        ts, as_ = orc.sweep_build(w)
        assert np.array_equal(t.view(np.uint32), ts.view(np.uint32)) and np.array_equal(a, as_), n


def test_blocks_of_one_item_are_the_sweep_over_items(orc):
    for n, w in _inputs():
        tt, at, t, a = orc.twolevel_build(w, 1)
        assert np.all(t == 1.0) and np.array_equal(a, np.arange(n))
        ts, as_ = orc.sweep_build(w)
        assert np.array_equal(tt.view(np.uint32), ts.view(np.uint32)) and np.array_equal(at, as_), n


@pytest.mark.parametrize("block", [2, 7, 64])
def test_item_probabilities_are_exact(orc, block):
    for n, w in list(_inputs())[:5]:
        w = w.copy()
        if n > 10:
            w[: min(block, n)] = 0.0  # a block of total weight zero
        if float(w.astype(np.float64).sum()) == 0.0:
            continue
        tt, at, t, a = orc.twolevel_build(w, block)
        G = tt.size
        W = sum(Fraction(float(x)) for x in w)
        pg = [m / G for m in exact_masses(np.zeros(G), tt, at)]  # P(block g)
        for g in range(G):
            b0, b1 = g * block, min(n, g * block + block)
            Wb = sum(Fraction(float(x)) for x in w[b0:b1])
            if Wb == 0:
                assert pg[g] == 0 and np.all(t[b0:b1] == 1.0) and np.array_equal(a[b0:b1], np.arange(b0, b1))
                continue
            m = b1 - b0
            local = exact_masses(np.zeros(m), t[b0:b1], a[b0:b1] - b0)
            for i in range(m):
                p = pg[g] * local[i] / m
                ref = Fraction(float(w[b0 + i])) / W
                # FP32 thresholds: a few half-ulp roundings per bucket at each level
                assert abs(p - ref) <= Fraction(8 * (G + m), 2 ** 24) * max(ref, Fraction(1, n * G)), (g, i)


def test_two_step_draws_follow_the_weights(orc):
    w = np.array([3, 1, 4, 1, 5, 9, 2, 6, 5, 3, 5, 0, 8], np.float32)
    tt, at, t, a = orc.twolevel_build(w, 4)
    k = 200000
    out = orc.twolevel_sample(tt, at, t, a, 4, 11, 2, 0, k)
    counts = np.bincount(out, minlength=w.size)
    assert counts[11] == 0
    pos = w > 0
    expect = w[pos] / w.sum() * k
    stat = float(((counts[pos] - expect) ** 2 / expect).sum())
    assert chi2.sf(stat, int(pos.sum()) - 1) > 1e-4
    idx = np.array([0, 5, 99, 123456, k - 1], np.uint64)
    assert np.array_equal(orc.twolevel_sample_at(tt, at, t, a, 4, 11, 2, idx), out[idx.astype(np.int64)])
