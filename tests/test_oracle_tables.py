"""Pins for the oracle's table construction (CPU only).

Each check ties the oracle to something other than itself: hand-worked tables,
exact rational arithmetic, Python's correctly rounded sum, the alias-table
definition (Section 2.2) and the merge characterisation of the sweep.
"""
import json
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def exact_masses(w, t, a):
    """Item masses in buckets implied by a table, in exact rationals (Section 2.2)."""
    n = len(w)
    m = [Fraction(0)] * n
    for r in range(n):
        tr = Fraction(float(t[r]))
        m[r] += tr
        m[int(a[r])] += 1 - tr
    return m


def is_nearest_f32(f: np.float32, x: Fraction) -> bool:
    f = np.float32(f)
    fx = Fraction(float(f))
    up = np.nextafter(f, np.float32(np.inf))
    dn = np.nextafter(f, np.float32(-np.inf))
    d = abs(fx - x)
    du = abs(Fraction(float(up)) - x)
    dd = abs(Fraction(float(dn)) - x)
    if d < du and d < dd:
        return True
    if d == du or d == dd:  # tie: the even mantissa wins
        return int(np.array(f, np.float32).view(np.uint32)) % 2 == 0
    return False


# --- total weight -----------------------------------------------------------

def test_total_weight_matches_fsum_and_exact(orc):
    rng = np.random.default_rng(11)
    for trial in range(20):
        n = int(rng.integers(1, 3000))
        w = (rng.random(n) ** 8 * 10.0 ** rng.integers(-20, 20, n)).astype(np.float32)
        hi, lo = orc.total_weight(w)
        assert hi == math.fsum(w.astype(np.float64))  # correctly rounded sum
        exact = sum(Fraction(float(x)) for x in w)
        assert Fraction(hi) + Fraction(lo) - exact == 0 or abs(Fraction(hi) + Fraction(lo) - exact) <= abs(exact) * Fraction(1, 2 ** 104)


def test_total_weight_rejects_bad_inputs(orc):
    for bad in ([1.0, -1.0], [1.0, float("nan")], [float("inf")], [0.0, 0.0]):
        with pytest.raises(orc.OracleError) as e:
            orc.total_weight(np.array(bad, np.float32))
        assert e.value.code == orc.EDOMAIN


# --- correctly rounded ratio helper ------------------------------------------

def test_ratio_rounding_is_nearest_even(orc):
    rng = random.Random(5)
    for _ in range(3000):
        wa = np.float32(rng.uniform(0, 1) * 2.0 ** rng.randint(-140, 20))
        wb = np.float32(rng.uniform(0.5, 1) * 2.0 ** rng.randint(-20, 20))
        ma, mb = rng.randint(1, 2 ** 31 - 1), rng.randint(1, 2 ** 31 - 1)
        if wb == 0:
            continue
        x = Fraction(float(wa)) * ma / (Fraction(float(wb)) * mb)
        f = orc.ratio_f32(wa, ma, wb, mb)
        if x > Fraction(float(np.finfo(np.float32).max)):
            continue
        assert is_nearest_f32(f, x), (wa, ma, wb, mb, f, float(x))


def test_ratio_rounding_exact_ties(orc):
    # 1 + 2^-24 lies exactly between two FP32 values: ties go to the even one (1.0);
    # 1 + 3*2^-24 goes up to 1 + 2^-22.
    assert orc.ratio_f32(np.float32(2 ** 24 + 1), 1, np.float32(2 ** 24), 1) == np.float32(1.0)
    assert orc.ratio_f32(np.float32(2 ** 24 + 3), 1, np.float32(2 ** 24), 1) == np.float32(1 + 2 ** -22)
    # subnormal results
    f = orc.ratio_f32(np.float32(2.0 ** -140), 1, np.float32(2.0 ** 9), 1)
    assert f == np.float32(2.0 ** -149)


# --- sweeping construction (Algorithm 2, Section 4.1) ------------------------

def test_sweep_hand_worked_cases(orc):
    with open(os.path.join(GOLDEN, "sweep_hand.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        t, a = orc.sweep_build(np.array(c["w"], np.float32))
        want_t = [np.float32(float(Fraction(s))) for s in c["t"]]
        assert list(a) == c["alias"], c
        assert [np.float32(x) for x in t] == want_t, c


def _random_small_instance(rng, n):
    kind = rng.integers(0, 5)
    if kind == 0:
        return rng.integers(0, 21, n).astype(np.float32)          # small integers, zeros, ties
    if kind == 1:
        return rng.integers(1, 1025, n).astype(np.float32)
    if kind == 2:
        return workloads.uniform(n, int(rng.integers(1 << 30)))
    if kind == 3:
        return workloads.power_law(n, float(rng.choice([0.5, 1.0, 2.0])), int(rng.integers(1 << 30)))
    w = rng.random(n).astype(np.float32)
    w[rng.integers(0, n)] = np.float32(1e6)                       # one dominant item
    return w


def test_sweep_is_an_exact_alias_table(orc):
    """Reconstruction (Section 2.2) with every t exactly representable: integer
    weights with W = 16 n and n a power of two make n w_i / W and every residual
    dyadic, so the masses must equal n w_i / W exactly."""
    rng = np.random.default_rng(2)
    for trial in range(200):
        n = int(2 ** rng.integers(0, 7))
        w = rng.integers(0, 33, n).astype(np.int64)
        diff = 16 * n - int(w.sum())
        while diff != 0:                 # adjust so that the total is exactly 16 n
            i = int(rng.integers(0, n))
            step = min(diff, 8) if diff > 0 else -min(-diff, int(w[i]))
            w[i] += step
            diff -= step
        wf = w.astype(np.float32)
        if wf.sum() == 0:
            continue
        t, a = orc.sweep_build(wf)
        masses = exact_masses(wf, t, a)
        W = sum(Fraction(int(x)) for x in w)
        for i in range(n):
            assert masses[i] == n * Fraction(int(w[i])) / W, (w, t, a)


def merge_closed_form(w):
    """Tables from the merge characterisation of the sweep, in exact rationals.

    With c = W/n, light items (w <= c) and heavy items in index order,
    D(i) = sum_{x<=i} (c - w_light[x]) and E(j) = sum_{x<=j} (w_heavy[x] - c),
    the sweep emits light i when D(i-1) < E(J+1) and heavy J+1 otherwise; light i
    takes alias h[J+1] (J heavies emitted before it), heavy j keeps
    t = 1 + (E(j) - D(I)) / c where I lights were emitted before it."""
    n = len(w)
    W = sum(Fraction(float(x)) for x in w)
    c = W / n
    L = [i for i in range(n) if Fraction(float(w[i])) <= c]
    H = [i for i in range(n) if Fraction(float(w[i])) > c]
    D = [Fraction(0)]
    for i in L:
        D.append(D[-1] + c - Fraction(float(w[i])))
    E = [Fraction(0)]
    for j in H:
        E.append(E[-1] + Fraction(float(w[j])) - c)
    t = [None] * n
    a = [None] * n
    I = J = 0
    while I < len(L) or J < len(H):
        heavy_next = J < len(H) and (I >= len(L) or E[J + 1] <= D[I])
        if heavy_next:
            j = H[J]
            t[j] = min(Fraction(1), 1 + (E[J + 1] - D[I]) / c)
            a[j] = H[J + 1] if J + 1 < len(H) else j
            J += 1
        else:
            i = L[I]
            t[i] = Fraction(float(w[i])) / c
            a[i] = H[J] if J < len(H) else i
            if J >= len(H):
                t[i] = min(t[i], Fraction(1))
            I += 1
    return t, a


def test_sweep_equals_merge_characterisation(orc):
    rng = np.random.default_rng(3)
    for trial in range(400):
        n = int(rng.integers(1, 40))
        w = _random_small_instance(rng, n)
        if w.astype(np.float64).sum() == 0:
            continue
        t, a = orc.sweep_build(w)
        tf, af = merge_closed_form(w)
        assert list(a) == af, (w, list(a), af)
        for i in range(n):
            assert is_nearest_f32(t[i], tf[i]), (w, i, t[i], float(tf[i]))


def test_sweep_structure(orc):
    """Sweep invariants: heavy buckets chain to the next heavy item in index
    order (the last to itself); light aliases never decrease along the light
    order; every alias target is a heavy item or the bucket's own item."""
    rng = np.random.default_rng(4)
    for trial in range(50):
        n = int(rng.integers(2, 3000))
        w = _random_small_instance(rng, n)
        if w.astype(np.float64).sum() == 0:
            continue
        t, a = orc.sweep_build(w)
        W = sum(Fraction(float(x)) for x in w)
        heavy = [Fraction(float(x)) * n > W for x in w]
        H = [i for i in range(n) if heavy[i]]
        for k, j in enumerate(H):
            assert a[j] == (H[k + 1] if k + 1 < len(H) else j)
        rank = {j: k for k, j in enumerate(H)}
        last = -1
        for i in range(n):
            if heavy[i]:
                continue
            if a[i] == i:
                last = len(H)
                continue
            assert heavy[a[i]]
            assert rank[a[i]] >= last
            last = rank[a[i]]


def test_sweep_reconstruction_large(orc):
    """n = 2^16 from the first configuration's input family: exact table masses
    within FP32 rounding of every t (at most 2^-24 per contributing bucket)."""
    w = workloads.uniform(1 << 16, 1)
    t, a = orc.sweep_build(w)
    mass, err = orc.reconstruct(w, t, a)
    assert err.max() < 1e-6


def test_sweep_rejects_bad_inputs(orc):
    for bad in ([1.0, -1.0], [1.0, float("nan")], [float("inf"), 1.0], [0.0]):
        with pytest.raises(orc.OracleError) as e:
            orc.sweep_build(np.array(bad, np.float32))
        assert e.value.code == orc.EDOMAIN


# --- Vose (Algorithm 1, Section 2.2) in FP64 ---------------------------------

def test_vose_special_cases(orc):
    t, a = orc.vose_build(np.full(7, 3.5, np.float32))     # all equal
    assert np.all(t == 1.0) and list(a) == list(range(7))
    t, a = orc.vose_build(np.array([2.0], np.float32))      # n = 1
    assert t[0] == 1.0 and a[0] == 0
    t, a = orc.vose_build(np.array([0, 0, 5, 0], np.float32))  # one non-zero weight
    assert list(a) == [2, 2, 2, 2] and t[2] == 1.0 and np.all(t[[0, 1, 3]] == 0)
    t, a = orc.vose_build(np.array([1, 3], np.float32))      # two items
    m = exact_masses([1, 3], t, a)
    assert m == [Fraction(1, 2), Fraction(3, 2)]


def test_vose_reconstruction(orc):
    rng = np.random.default_rng(6)
    for trial in range(30):
        n = int(rng.integers(1, 5000))
        w = _random_small_instance(rng, n)
        if w.astype(np.float64).sum() == 0:
            continue
        t, a = orc.vose_build(w)
        mass, err = orc.reconstruct(w, t, a)
        pos = w > 0
        assert err[pos].max() < 1e-5
        assert np.all(mass[~pos] == 0)


# --- reconstruction checker itself --------------------------------------------

def test_reconstruct_detects_errors(orc):
    w = np.array([1, 5, 1, 5], np.float32)
    t = np.array([1 / 3, 1, 1 / 3, 1], np.float32)
    a = np.array([1, 3, 3, 3], np.int32)
    mass, err = orc.reconstruct(w, t, a)
    assert err.max() < 1e-7
    a_bad = a.copy()
    a_bad[2] = 1                                   # moves 2/3 bucket from item 3 to 1
    mass, err = orc.reconstruct(w, t, a_bad)
    assert abs(mass[1] - (5 / 3 + 2 / 3)) < 1e-7 and err[1] > 0.3
    with pytest.raises(orc.OracleError):
        orc.reconstruct(w, np.array([1.5, 1, 1, 1], np.float32), a)
    with pytest.raises(orc.OracleError):
        orc.reconstruct(w, t, np.array([4, 3, 3, 3], np.int32))
