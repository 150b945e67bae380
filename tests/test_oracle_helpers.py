"""Pins of the oracle's per-item checker helpers against the full oracle.

The GPU tests at full size cannot afford the whole oracle and call two
per-item helpers instead: ``light_t_at`` (is item i light, and its correctly
rounded t = n w_i / W) and ``wor_keys_at`` (the exponential-clock key of item
i).  Here each helper is tied to the oracle function it stands in for:

* ``light_t_at`` against the exact sweep (Algorithm 2).  In the sweep's table
  a light bucket keeps its own item's whole size, so its t is n w_i / W, and a
  heavy item is exactly an item that some other bucket names as its alias
  (heavy j >= 2 is the alias of heavy j - 1, heavy 1 the alias of the first
  light; a light is never anyone's alias).  So the helper's classification must
  equal "aliased by another bucket" and its t must equal the sweep's t on every
  light, bit for bit.
* ``wor_keys_at`` against ``wor_keys`` (Section 2.3) bit for bit, and with the
  same rejection of negative, NaN and infinite weights.

Instances: random n up to 2^16 with zero weights and ties at the mean
(w_i = W / n exactly, which the sweep classifies as light).
"""
import numpy as np
import pytest

import oracle


def _instance(rng, n, kind):
    if kind == "uniform":
        return (1.0 - rng.random(n, dtype=np.float32)).astype(np.float32)
    if kind == "zeros":
        w = (1.0 - rng.random(n, dtype=np.float32)).astype(np.float32)
        w[rng.random(n) < 0.3] = 0.0
        if not (w > 0).any():
            w[0] = 1.0
        return w
    if kind == "ties":
        # integer weights whose mean is an integer: items equal to the mean are
        # ties (n w = W) and must count as light
        w = rng.integers(0, 7, n).astype(np.float32)
        w[0] = 0.0
        s = float(w.sum())
        mean = int(np.ceil(s / n)) if s > 0 else 1
        w[0] = np.float32(mean * n - s + w[0]) if mean * n - s >= 0 else 0.0
        w[1:][rng.random(n - 1) < 0.2] = np.float32(mean)
        # re-balance so that the total is mean * n again
        diff = mean * n - float(w.sum())
        w[0] = np.float32(max(0.0, float(w[0]) + diff))
        return w
    if kind == "power":
        base = (np.arange(1, n + 1, dtype=np.float64) ** -1.0).astype(np.float32)
        return base[rng.permutation(n)]
    if kind == "equal":
        return np.full(n, 0.375, np.float32)
    raise ValueError(kind)


CASES = [(n, kind, seed) for seed, n in enumerate([1, 2, 3, 17, 1000, 4097, 30011, 65536])
         for kind in ("uniform", "zeros", "ties", "power", "equal")]


@pytest.mark.parametrize("n,kind,seed", CASES)
def test_light_t_at_matches_sweep(n, kind, seed):
    rng = np.random.default_rng(100 + seed)
    w = _instance(rng, n, kind)
    t_sw, a_sw = oracle.sweep_build(w)
    aliased = np.zeros(n, bool)
    other = a_sw != np.arange(n)
    aliased[a_sw[other]] = True
    idx = np.arange(n) if n <= 4096 else np.unique(rng.integers(0, n, 4096))
    light, t = oracle.light_t_at(w, idx)
    assert np.array_equal(light, ~aliased[idx]), "classification differs from the sweep's heavy set"
    lt = light.nonzero()[0]
    assert np.array_equal(t[lt].view(np.int32), t_sw[idx[lt]].view(np.int32)), "light t differs from the sweep"


def test_light_t_at_ties_are_light():
    # every weight equal: each item is exactly W / n, a tie, light with t = 1
    w = np.full(12, 2.5, np.float32)
    light, t = oracle.light_t_at(w, np.arange(12))
    assert light.all() and (t == 1.0).all()
    t_sw, a_sw = oracle.sweep_build(w)
    assert (a_sw == np.arange(12)).all() and (t_sw == 1.0).all()


def test_light_t_at_ties_instance_has_ties():
    rng = np.random.default_rng(7)
    w = _instance(rng, 1000, "ties")
    s = float(np.sum(w.astype(np.float64)))
    assert s == round(s) and int(s) % 1000 == 0
    mean = s / 1000
    assert (w == mean).sum() > 50
    light, _ = oracle.light_t_at(w, np.nonzero(w == mean)[0])
    assert light.all()


@pytest.mark.parametrize("n,kind,seed", CASES)
def test_wor_keys_at_matches_wor_keys(n, kind, seed):
    rng = np.random.default_rng(200 + seed)
    w = _instance(rng, n, kind)
    full = oracle.wor_keys(w, 3 + seed, seed)
    idx = np.arange(n) if n <= 4096 else rng.integers(0, n, 4096)
    at = oracle.wor_keys_at(w, 3 + seed, seed, idx)
    assert np.array_equal(at.view(np.int64), full[idx].view(np.int64))


@pytest.mark.parametrize("bad", [np.float32(-1.0), np.float32(np.nan), np.float32(np.inf)])
def test_wor_keys_at_rejects_bad_weights_like_wor_keys(bad):
    w = np.ones(50, np.float32)
    w[37] = bad
    with pytest.raises(oracle.OracleError) as e1:
        oracle.wor_keys(w, 1, 0)
    # the bad weight is not among the requested items: still rejected
    with pytest.raises(oracle.OracleError) as e2:
        oracle.wor_keys_at(w, 1, 0, np.array([0, 1, 2]))
    assert e1.value.code == e2.value.code == oracle.EDOMAIN


def test_light_t_at_rejects_bad_weights():
    w = np.ones(10, np.float32)
    w[3] = -2.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.light_t_at(w, np.array([0]))
    assert e.value.code == oracle.EDOMAIN
    with pytest.raises(oracle.OracleError) as e:
        oracle.light_t_at(np.zeros(4, np.float32), np.array([0]))
    assert e.value.code == oracle.EDOMAIN
