"""GPU parity of sampling with replacement (C ABI wrs_alias_sample).

Bar: every drawn index bit-identical to the oracle querying the same (GPU-built)
table with the same Philox counters.
"""
import math

import numpy as np
import pytest

import workloads
from gpu_common import family, gpu_build, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


def gpu_sample(wrs, table, n, seed, sid, first, k):
    import torch
    out = torch.empty(max(k, 1), dtype=torch.int32, device=table.device)
    wrs.alias_sample(table, n, seed, sid, first, k, out)
    torch.cuda.synchronize()
    return out[:k].cpu().numpy()


def test_sample_first_config(wrs, orc):
    """n = 2^16 uniform (seed 1), k = 2^20 draws, Philox key 1, counter = draw index."""
    w = workloads.uniform(1 << 16, 1)
    say("sample config n=2^16 k=2^20")
    t, a, st, table, *_ = gpu_build(wrs, w)
    got = gpu_sample(wrs, table, w.size, 1, 0, 0, 1 << 20)
    want = orc.alias_sample(t, a, 1, 0, 0, 1 << 20)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,k,seed,sid,first", [
    (1, 100, 3, 0, 0), (2, 5000, 4, 1, 7), (1000, 1, 5, 2, 0), (1000, 2047, 6, 0, 2 ** 32 - 5),
    (4097, 2049, 7, 9, 123456789012), (65536 + 3, 300001, 2 ** 63 + 5, 2 ** 32 - 1, 2 ** 40), (300, 0, 1, 0, 0)])
def test_sample_edges(wrs, orc, n, k, seed, sid, first):
    w = family("power1", n, n)
    say("sample", n, k, seed, sid, first)
    t, a, st, table, *_ = gpu_build(wrs, w)
    got = gpu_sample(wrs, table, n, seed, sid, first, k)
    want = orc.alias_sample(t, a, seed, sid, first, k)
    assert np.array_equal(got, want)


def test_sample_from_oracle_table(wrs, orc):
    """The sampler on a table it did not build (the oracle's Vose table)."""
    import torch
    w = workloads.power_law(5000, 0.5, 1)
    t, a = orc.vose_build(w)
    tab = np.stack([t.view(np.int32), a], axis=1)
    table = torch.from_numpy(tab).to("cuda:0")
    say("sample vose table")
    got = gpu_sample(wrs, table, w.size, 42, 0, 0, 100000)
    assert np.array_equal(got, orc.alias_sample(t, a, 42, 0, 0, 100000))


def test_sample_distinct_count(wrs, orc):
    """Distinct items among k draws against E[X] = sum_i 1 - (1 - w_i/W)^k."""
    w = workloads.power_law(1 << 20, 1.0, 3)
    say("distinct count")
    t, a, st, table, *_ = gpu_build(wrs, w)
    k = 1 << 22
    got = gpu_sample(wrs, table, w.size, 8, 0, 0, k)
    x = np.unique(got).size
    p = w.astype(np.float64) / w.astype(np.float64).sum()
    ex = float(np.sum(-np.expm1(k * np.log1p(-p))))
    assert abs(x - ex) <= 5 * math.sqrt(ex)


@pytest.mark.parametrize("fam", ["uniform", "power1"])
def test_sample_full_size(wrs, orc, fam):
    """n = 2^28 table from the GPU build, k = 2^30 draws (key 2): the first and
    last 2^20 draws and every 1021st draw equal the oracle's queries."""
    import torch
    n, k = 1 << 28, 1 << 30
    w = workloads.uniform(n, 2) if fam == "uniform" else workloads.power_law(n, 1.0, 2)
    say("sample full size", fam)
    t, a, st, table, wt, ws = gpu_build(wrs, w)
    del wt, ws
    out = torch.empty(k, dtype=torch.int32, device="cuda:0")
    wrs.alias_sample(table, n, 2, 0, 0, k, out)
    torch.cuda.synchronize()
    cnt = np.concatenate([np.arange(0, 1 << 20), np.arange(k - (1 << 20), k), np.arange(0, k, 1021)])
    got = out[torch.from_numpy(cnt).to("cuda:0")].cpu().numpy()
    want = orc.alias_sample_at(t, a, 2, 0, cnt.astype(np.uint64))
    assert np.array_equal(got, want)
