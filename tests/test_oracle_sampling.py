"""Pins for the oracle's random bits and its sampling with replacement (CPU only).

* Philox-4x32-10 is checked against PyTorch's independent Philox engine (ATen
  header, compiled here with g++); the paper itself uses Mersenne Twisters, so
  nothing in the paper fixes these bits.
* The alias query (Section 2.2) is checked by the exact output distribution
  implied by the bit mapping, by chi-square tests of actual draws against
  w_i / W (problem WRS-R, Section 1), and by the expected number of distinct
  items, E[X] = sum_i 1 - (1 - w_i/W)^k (Section 6), which itself is pinned to
  the distinct fractions printed in the paper's query figure.
"""
import json
import math
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- Philox against PyTorch's engine ----------------------------------------

TORCH_PHILOX_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  // args: seed subsequence offset  ->  four 32-bit outputs of one block
  unsigned long long seed = strtoull(argv[1], 0, 10), sub = strtoull(argv[2], 0, 10),
                     off = strtoull(argv[3], 0, 10);
  at::philox_engine e(seed, sub, off);
  for (int i = 0; i < 4; ++i) printf("%u\n", e());
  return 0;
}
"""


@pytest.fixture(scope="module")
def torch_philox_exe():
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    d = tempfile.mkdtemp(prefix="wrs_philox_")
    src = os.path.join(d, "p.cpp")
    exe = os.path.join(d, "p")
    with open(src, "w") as f:
        f.write(TORCH_PHILOX_SRC)
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, src, "-o", exe], check=True)
    return exe


def test_philox_matches_pytorch_engine(orc, torch_philox_exe):
    rng = np.random.default_rng(123)
    cases = [(0, 0, 0), (1, 0, 0), (2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1)]
    cases += [tuple(int(x) for x in rng.integers(0, 2 ** 63, 3, dtype=np.int64)) for _ in range(40)]
    for seed, sub, off in cases:
        out = subprocess.run([torch_philox_exe, str(seed), str(sub), str(off)], check=True,
                             capture_output=True, text=True).stdout.split()
        want = [int(x) for x in out]
        ctr = [off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        got = [int(x) for x in orc.philox4x32_10(ctr, key)]
        assert got == want, (seed, sub, off)


# --- exact output distribution of the alias query ----------------------------

def bucket_probability(r, n):
    """P(floor(X n / 2^64) = r) for X uniform on 64-bit integers."""
    lo = -(-(r * 2 ** 64) // n)
    hi = -(-((r + 1) * 2 ** 64) // n)
    return Fraction(hi - lo, 2 ** 64)


def heads_probability(t):
    """P(v 2^-24 < t) for v uniform on 24-bit integers, t in [0, 1]."""
    x = Fraction(float(t)) * 2 ** 24
    return Fraction(min(2 ** 24, math.ceil(x)), 2 ** 24)


def test_query_distribution_is_exactly_the_weights(orc):
    """Enumerate the query's bit mapping exactly: the output distribution must
    match w_i / W up to the FP32 rounding of t (2^-25 relative), the 2^-24 coin
    grid and the 2^-64 bucket grid, per contributing bucket."""
    rng = np.random.default_rng(7)
    for trial in range(60):
        n = int(rng.integers(1, 12))
        w = rng.integers(0, 9, n).astype(np.float32)
        if w.sum() == 0:
            w[0] = 1
        for build in (orc.sweep_build, orc.vose_build):
            t, a = build(w)
            p = [Fraction(0)] * n
            contrib = [0] * n
            for r in range(n):
                pr = bucket_probability(r, n)
                ph = heads_probability(t[r])
                p[r] += pr * ph
                p[int(a[r])] += pr * (1 - ph)
                contrib[r] += 1
                contrib[int(a[r])] += 1
            W = sum(Fraction(int(x)) for x in w)
            for i in range(n):
                bound = contrib[i] * (Fraction(1, n) * Fraction(3, 2 ** 25) + Fraction(1, 2 ** 63))
                assert abs(p[i] - Fraction(int(w[i])) / W) <= bound, (w, t, a, i)


def chi2_pvalue(observed, expected):
    from scipy.stats import chi2
    observed = np.asarray(observed, np.float64)
    expected = np.asarray(expected, np.float64)
    stat = float(((observed - expected) ** 2 / expected).sum())
    return float(chi2.sf(stat, len(observed) - 1))


def test_query_chi_square_small(orc):
    w = np.array([1, 2, 3, 4, 10, 0.5, 7], np.float32)
    k = 1 << 20
    for build in (orc.sweep_build, orc.vose_build):
        t, a = build(w)
        out = orc.alias_sample(t, a, seed=99, stream_id=3, first_counter=0, k=k)
        counts = np.bincount(out, minlength=w.size)
        assert chi2_pvalue(counts, k * w / w.sum()) > 1e-4


def test_query_chi_square_first_config(orc):
    """n = 2^16 uniform weights (seed 1), k = 2^20 draws (key 1, counter = draw
    index); expected counts pooled into 256 bins of 256 consecutive items."""
    w = workloads.uniform(1 << 16, 1)
    t, a = orc.sweep_build(w)
    k = 1 << 20
    out = orc.alias_sample(t, a, seed=1, stream_id=0, first_counter=0, k=k)
    counts = np.bincount(out, minlength=w.size).reshape(256, 256).sum(1)
    expect = (k * w.astype(np.float64) / w.astype(np.float64).sum()).reshape(256, 256).sum(1)
    assert chi2_pvalue(counts, expect) > 1e-4


def test_query_counter_offsets(orc):
    w = workloads.power_law(1000, 1.0, 9)
    t, a = orc.sweep_build(w)
    full = orc.alias_sample(t, a, 5, 2, 0, 5000)
    part = orc.alias_sample(t, a, 5, 2, 1234, 100)
    assert np.array_equal(part, full[1234:1334])
    at = orc.alias_sample_at(t, a, 5, 2, np.array([7, 4999, 0], np.uint64))
    assert list(at) == [full[7], full[4999], full[0]]


def test_query_special_tables(orc):
    """t = 1 everywhere returns the bucket (uniform over buckets); t = 0 always
    returns the alias."""
    n = 97
    k = 200000
    out = orc.alias_sample(np.ones(n, np.float32), np.zeros(n, np.int32), 4, 0, 0, k)
    assert chi2_pvalue(np.bincount(out, minlength=n), np.full(n, k / n)) > 1e-4
    alias = np.full(n, 13, np.int32)
    out = orc.alias_sample(np.zeros(n, np.float32), alias, 4, 0, 0, 1000)
    assert np.all(out == 13)


# --- expected number of distinct items ---------------------------------------

def expected_distinct_power(n, s, k, explicit=10 ** 6):
    """E[X] = sum_i 1 - (1 - p_i)^k for p_i = i^-s / W_s, i = 1..n.  The first
    `explicit` terms are summed directly, the rest by the midpoint rule as an
    integral over x (the summand varies slowly there)."""
    from scipy.integrate import quad
    m = min(n, explicit)
    i = np.arange(1, m + 1, dtype=np.float64)
    head_w = float(np.sum(i ** -s))
    a, b = m + 0.5, n + 0.5
    if s == 1.0:
        tail_w = math.log(b / a)
    else:
        tail_w = (b ** (1 - s) - a ** (1 - s)) / (1 - s)
    W = head_w + (tail_w if n > m else 0.0)
    head = float(np.sum(-np.expm1(k * np.log1p(-(i ** -s) / W))))
    if n <= m:
        return head
    f = lambda y: math.exp(y) * -math.expm1(k * math.log1p(-math.exp(-s * y) / W))
    tail, _ = quad(f, math.log(a), math.log(b), limit=400, epsabs=1e-6, epsrel=1e-12)
    return head + tail


def expected_distinct_uniform(n, k):
    """For w_i uniform on (0,1] and W ~ n/2: E[X] = n (1 - E[exp(-2 k w / n)])
    = n (1 - (n / 2k) (1 - exp(-2k/n)))."""
    x = 2.0 * k / n
    return n * (1.0 - (1.0 - math.exp(-x)) / x)


def test_distinct_fraction_matches_paper():
    with open(os.path.join(GOLDEN, "paper_distinct_fraction.json")) as f:
        g = json.load(f)
    n = g["n"]
    for c in g["cases"]:
        if c["family"] == "uniform":
            ex = expected_distinct_uniform(n, c["k"])
        else:
            ex = expected_distinct_power(n, c["s"], c["k"])
        frac = ex / c["k"]
        assert abs(frac - c["printed"]) <= c["rtol"] * c["printed"], (c, frac)


def test_oracle_distinct_count_matches_closed_form(orc):
    for s, n, k in ((1.0, 1 << 14, 1 << 16), (0.5, 1 << 12, 1 << 14), (2.0, 1 << 14, 1 << 16)):
        w = workloads.power_law(n, s, 21)
        t, a = orc.sweep_build(w)
        out = orc.alias_sample(t, a, 77, 0, 0, k)
        x = np.unique(out).size
        p = w.astype(np.float64) / w.astype(np.float64).sum()
        ex = float(np.sum(-np.expm1(k * np.log1p(-p))))
        assert abs(x - ex) <= 5 * math.sqrt(ex) + 1, (s, x, ex)
