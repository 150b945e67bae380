"""Pins for the oracle's greedy-block construction (Section 4.2.1, PSA+).

The construction is tied to things other than itself: hand-worked tables,
the plain sweep it must reduce to (one block holding every item, or blocks of
one item, where nothing is packed greedily), blocks that each balance exactly
(then every block is an independent instance of the sweep), and the
alias-table definition (every item's mass, in exact rationals).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads
from test_oracle_tables import exact_masses

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _inputs():
    rng = np.random.default_rng(21)
    for trial in range(12):
        n = int(rng.integers(1, 3000))
        w = workloads.uniform(n, 100 + trial) if trial % 2 == 0 else workloads.power_law(n, 1.0, 100 + trial)
        yield n, w


def test_psaplus_hand_cases(orc):
    with open(os.path.join(GOLDEN, "psaplus_hand.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        w = np.array(c["w"], np.float32)
        t, a = orc.psaplus_build(w, c["block"])
        assert [Fraction(float(x)) for x in t] == [Fraction(x) for x in c["t"]], c["note"]
        assert a.tolist() == c["alias"], c["note"]
        assert orc.psaplus_leftovers(w, c["block"]) == c["left"], c["note"]


@pytest.mark.parametrize("mult", [1, 2, 7])
def test_one_block_is_the_plain_sweep(orc, mult):
    # a block holding every item: the greedy sweep is the whole sweep
    for n, w in _inputs():
        t, a = orc.psaplus_build(w, n * mult)
        ts, as_ = orc.sweep_build(w)
        assert np.array_equal(t.view(np.uint32), ts.view(np.uint32)), n
        assert np.array_equal(a, as_), n


def test_blocks_of_one_item_are_the_plain_sweep(orc):
    # a block of one item has no light or no heavy: every item is left with
    # its full size, and the second sweep is the plain sweep
    for n, w in _inputs():
        t, a = orc.psaplus_build(w, 1)
        ts, as_ = orc.sweep_build(w)
        assert np.array_equal(t.view(np.uint32), ts.view(np.uint32)), n
        assert np.array_equal(a, as_), n
        assert orc.psaplus_leftovers(w, 1) == n


@pytest.mark.parametrize("block", [4, 16, 61])
def test_balanced_blocks_are_independent_sweeps(orc, block):
    # every block is a permutation of one multiset, so each block's total is
    # exactly its share of W: the greedy sweep of a block is the sweep of the
    # block as an instance of its own (aliases shifted by the block start)
    rng = np.random.default_rng(block)
    base = workloads.uniform(block, block)
    nb = 9
    w = np.concatenate([base[rng.permutation(block)] for _ in range(nb)])
    t, a = orc.psaplus_build(w, block)
    for b in range(nb):
        ts, as_ = orc.sweep_build(w[b * block:(b + 1) * block])
        sl = slice(b * block, (b + 1) * block)
        assert np.array_equal(t[sl].view(np.uint32), ts.view(np.uint32)), b
        assert np.array_equal(a[sl], as_ + b * block), b


@pytest.mark.parametrize("block", [2, 3, 64, 2048])
def test_psaplus_masses_are_exact(orc, block):
    # alias-table definition: item i's mass is t_i plus (1 - t_r) over buckets
    # r aliased to i; it equals n w_i / W up to the FP32 rounding of each t
    for n, w in list(_inputs())[:6]:
        t, a = orc.psaplus_build(w, block)
        assert np.all((t >= 0) & (t <= 1)) and np.all((a >= 0) & (a < n))
        W = sum(Fraction(float(x)) for x in w)
        m = exact_masses(w, t, a)
        # each bucket contributes at most two roundings of half an FP32 ulp
        refs = [Fraction(n) * Fraction(float(x)) / W for x in w]
        deg = np.bincount(a, minlength=n) + 1
        for i in range(n):
            assert abs(m[i] - refs[i]) <= Fraction(int(deg[i]), 2 ** 24), (n, block, i)


def test_psaplus_mass_reconstruction_large(orc):
    # the same definition in double-double at a size with many blocks
    for kind in ("uniform", "power"):
        n = 1 << 17
        w = workloads.uniform(n, 7) if kind == "uniform" else workloads.power_law(n, 1.0, 7)
        t, a = orc.psaplus_build(w, 2048)
        _, err = orc.reconstruct(w, t, a)
        assert float(np.max(err)) <= 1e-6, kind


def test_psaplus_differs_from_the_sweep_and_leaves_few_items(orc):
    # a real greedy stage: on uniform weights most items are packed inside
    # their block, so the table is not the plain sweep's
    n = 1 << 15
    w = workloads.uniform(n, 3)
    t, a = orc.psaplus_build(w, 2048)
    ts, as_ = orc.sweep_build(w)
    assert not np.array_equal(a, as_)
    assert orc.psaplus_leftovers(w, 2048) < n // 10


def test_psaplus_rejects_bad_inputs(orc):
    with pytest.raises(orc.OracleError):
        orc.psaplus_build(np.array([1.0, -1.0], np.float32), 4)
    with pytest.raises(orc.OracleError):
        orc.psaplus_build(np.array([0.0, 0.0], np.float32), 4)
    with pytest.raises(orc.OracleError):
        orc.psaplus_build(np.array([1.0], np.float32), 0)
