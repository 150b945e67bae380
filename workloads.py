"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws inputs; it holds none of the sampling method's arithmetic.
The input families are the paper's (Section 10, "Input Data"): weights uniform
in (0,1], and random permutations of the power-law weights {1^-s, ..., n^-s}.

Recipes (numpy ``default_rng(seed)``, i.e. PCG64):
  uniform(n, seed)       1 - rng.random(n, float32): FP32 values on the 2^-24
                         grid in (0, 1].
  power_law(n, s, seed)  i^-s for i = 1..n computed in FP64, rounded once to
                         FP32, then permuted by rng.permutation(n).
  batch_jobs(seed)       4096 tables, n_i = floor(2^(6 + 14 U)) clamped to
                         [2^6, 2^20]; per table a fair coin picks uniform or
                         power law (s = 1); k_i = 4 n_i; stream id = table id.
  serve_trace(seed, ...) Poisson arrivals; half build requests with
                         n = floor(2^U), U ~ U[10, 24]; half sample requests with
                         k = floor(2^U), U ~ U[10, 22] against a resident table.
"""
from __future__ import annotations

import numpy as np


def uniform(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (np.float32(1.0) - rng.random(n, dtype=np.float32)).astype(np.float32)


def power_law(n: int, s: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    base = (np.arange(1, n + 1, dtype=np.float64) ** (-float(s))).astype(np.float32)
    perm = rng.permutation(n)
    return base[perm]


def batch_jobs(seed: int = 4, count: int = 4096, lo_log2: int = 6, hi_log2: int = 20):
    """List of dicts {n, kind, seed_w, k, stream_id} for the batched workload."""
    rng = np.random.default_rng(seed)
    u = rng.random(count)
    n = np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
    n = np.clip(n, 2 ** lo_log2, 2 ** hi_log2)
    kind = rng.integers(0, 2, size=count)
    wseed = rng.integers(0, 2 ** 31, size=count)
    return [dict(n=int(n[i]), kind="uniform" if kind[i] == 0 else "power", seed_w=int(wseed[i]),
                 k=int(4 * n[i]), stream_id=i) for i in range(count)]


def job_weights(job) -> np.ndarray:
    if job["kind"] == "uniform":
        return uniform(job["n"], job["seed_w"])
    return power_law(job["n"], 1.0, job["seed_w"])


def serve_trace(seed: int = 5, count: int = 2000, rate_hz: float = 1000.0,
                n_log2=(10, 24), k_log2=(10, 22)):
    """Request list: dicts {t_arrive (s), op ('build'|'sample'), n or k, kind, seed_w,
    table_pick (uniform in [0,1), selects among resident tables), seed}."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps)
    ops = rng.integers(0, 2, size=count)
    ub = rng.random(count)
    us = rng.random(count)
    kinds = rng.integers(0, 2, size=count)
    picks = rng.random(count)
    wseeds = rng.integers(0, 2 ** 31, size=count)
    reqs = []
    for i in range(count):
        if ops[i] == 0:
            n = int(np.floor(2.0 ** (n_log2[0] + (n_log2[1] - n_log2[0]) * ub[i])))
            reqs.append(dict(t_arrive=float(t[i]), op="build", n=n,
                             kind="uniform" if kinds[i] == 0 else "power", seed_w=int(wseeds[i])))
        else:
            k = int(np.floor(2.0 ** (k_log2[0] + (k_log2[1] - k_log2[0]) * us[i])))
            reqs.append(dict(t_arrive=float(t[i]), op="sample", k=k, table_pick=float(picks[i]),
                             seed=int(wseeds[i])))
    return reqs
