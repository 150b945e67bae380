"""Property-based pins for the oracle (hypothesis, CPU only).

Random instances with n in [1, 2^12] and weights drawn from mixtures that
include zeros, duplicates, one dominant item, all-equal runs, subnormals and
huge ratios.  For each: the sweep and the greedy-block constructions give
tables whose every item mass, in exact rationals, is n w_i / W up to the FP32
rounding of the thresholds (the alias-table definition, Section 2.2); Vose's
table reconstructs within its FP64 drift; invalid inputs give the exact error
codes; the permutation is a permutation whose prefixes are the WRS-N samples;
output-sensitive samples are distinct positive items whose multiplicities sum
to k, grouped by binary exponent.
"""
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from test_oracle_tables import exact_masses

SUBNORMAL = np.float32(1e-40)


@st.composite
def weights(draw, max_n=1 << 12):
    n = draw(st.integers(1, max_n))
    seed = draw(st.integers(0, 2 ** 32 - 1))
    kind = draw(st.sampled_from(["mixed", "dupes", "dominant", "equal", "subnormal", "ratios", "ints"]))
    rng = np.random.default_rng(seed)
    if kind == "mixed":
        w = rng.random(n).astype(np.float32)
        w[rng.random(n) < 0.2] = 0.0
    elif kind == "dupes":
        w = rng.choice(np.array([0.5, 1.0, 3.0, 0.0], np.float32), n)
    elif kind == "dominant":
        w = rng.random(n).astype(np.float32)
        w[rng.integers(0, n)] = np.float32(1e6)
    elif kind == "equal":
        w = np.full(n, np.float32(rng.random() + 0.1), np.float32)
    elif kind == "subnormal":
        w = rng.random(n).astype(np.float32)
        w[rng.random(n) < 0.3] = SUBNORMAL
    elif kind == "ratios":
        w = (10.0 ** rng.uniform(-20, 20, n)).astype(np.float32)
    else:
        w = rng.integers(0, 1025, n).astype(np.float32)
    if float(w.astype(np.float64).sum()) == 0.0:
        w[0] = 1.0
    return w


def assert_exact_masses(w, t, a):
    n = w.size
    assert np.all((t >= 0) & (t <= 1)) and np.all((a >= 0) & (a < n))
    W = sum(Fraction(float(x)) for x in w)
    m = exact_masses(w, t, a)
    deg = np.bincount(a, minlength=n) + 1
    for i in range(n):
        ref = Fraction(n) * Fraction(float(w[i])) / W
        assert abs(m[i] - ref) <= Fraction(int(deg[i]), 2 ** 24), i


FAST = settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@FAST
@given(weights(max_n=600))
def test_sweep_masses_exact(orc, w):
    t, a = orc.sweep_build(w)
    assert_exact_masses(w, t, a)


@FAST
@given(weights(max_n=600), st.sampled_from([1, 2, 5, 64, 2048]))
def test_psaplus_masses_exact(orc, w, block):
    t, a = orc.psaplus_build(w, block)
    assert_exact_masses(w, t, a)


@FAST
@given(weights())
def test_vose_and_sweep_reconstruct(orc, w):
    # the 1e-6 bar holds where n w_i / W is a normal FP32 number; a subnormal
    # threshold has fewer mantissa bits (the absolute error stays below the
    # FP32 subnormal spacing, which the exact-mass properties above check)
    wd = w.astype(np.float64)
    ref = wd * w.size / wd.sum()
    normal = (w > 0) & (ref >= 2.0 ** -125)
    for build in (orc.sweep_build, orc.vose_build):
        t, a = build(w)
        _, err = orc.reconstruct(w, t, a)
        if normal.any():
            assert err[normal].max() <= (1e-6 if build is orc.sweep_build else 1e-4)


@FAST
@given(weights(max_n=2000), st.integers(0, 2 ** 63), st.integers(0, 7))
def test_permutation_prefixes(orc, w, seed, sid):
    out = orc.permutation(w, seed, sid)
    assert np.array_equal(np.sort(out), np.arange(w.size))
    npos = int((w > 0).sum())
    for k in sorted({1, npos // 2, npos} - {0}):
        s, _ = orc.sample_wor(w, k, seed, sid)
        assert np.array_equal(np.sort(out[:k]), s)


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 50), st.sampled_from(["neg", "nan", "inf", "zero"]), st.integers(0, 10 ** 6))
def test_invalid_inputs_error_codes(orc, n, bad, seed):
    rng = np.random.default_rng(seed)
    w = rng.random(n).astype(np.float32) + np.float32(0.1)
    if bad == "zero":
        w[:] = 0.0
    else:
        w[rng.integers(0, n)] = {"neg": -1.0, "nan": np.nan, "inf": np.inf}[bad]
    for fn in (lambda: orc.sweep_build(w), lambda: orc.vose_build(w), lambda: orc.psaplus_build(w, 4),
               lambda: orc.total_weight(w)):
        with pytest.raises(orc.OracleError) as e:
            fn()
        assert e.value.code == orc.EDOMAIN


@FAST
@given(weights(max_n=2000), st.integers(0, 2 ** 31 - 1), st.integers(0, 2 ** 63))
def test_output_sensitive_invariants(orc, w, k, seed):
    """Section 5's sample: distinct positive items, ascending, multiplicities
    summing to k, a pure function of (weights, k, seed); groups by binary
    exponent, heaviest first, items of a group by index (against frexp)."""
    items, counts = orc.os_sample(w, k, seed)
    assert int(counts.sum()) == k and np.all(counts >= 1)
    assert np.all(np.diff(items) > 0) and np.all(w[items] > 0)
    assert items.size <= min(k, int((w > 0).sum()))
    i2, c2 = orc.os_sample(w, k, seed)
    assert np.array_equal(items, i2) and np.array_equal(counts, c2)
    order, exps, starts, cnts = orc.os_groups(w)
    pos = np.nonzero(w > 0)[0]
    e = np.frexp(w[pos])[1] - 1
    assert np.array_equal(order, pos[np.lexsort((pos, -e))])
    assert list(exps) == sorted(set(e.tolist()), reverse=True)
    assert int(cnts.sum()) == pos.size
