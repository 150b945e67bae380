"""GPU parity of sampling without replacement (C ABI wrs_sample_wor).

Bar: the GPU's index set equals the oracle's (exponential-clock keys in FP64,
k smallest by (key, index)), except for items whose key lies within 1e-6
relative of the oracle's k-th key (both sides compute -ln(u) to about one FP64
ulp, so only such near-ties may swap).
"""
import numpy as np
import pytest

import workloads
from gpu_common import family, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


def gpu_wor(wrs, w_np, k, seed, sid):
    import torch
    n = w_np.size
    w = torch.from_numpy(np.ascontiguousarray(w_np, np.float32)).to("cuda:0")
    out = torch.empty(max(k, 1), dtype=torch.int32, device="cuda:0")
    ws = wrs.new_workspace(wrs.OP_WOR, n, k, "cuda:0")
    wrs.sample_wor(w, n, k, seed, sid, out, ws)
    st = wrs.status(ws)
    return out[:k].cpu().numpy(), st


def compare_sets(orc, w, k, seed, sid, got):
    want, kth = orc.sample_wor(w, k, seed, sid)
    assert np.all(np.diff(got) > 0), "output must be strictly ascending"
    diff = np.setxor1d(got, want)
    if diff.size:
        keys = orc.wor_keys_at(w, seed, sid, diff)
        assert np.all(np.abs(keys - kth) <= 1e-6 * kth), f"{diff.size} differing items away from the boundary"


@pytest.mark.parametrize("fam", ["uniform", "power0.5", "power1", "ints", "equal", "dominant", "wide"])
def test_wor_small(wrs, orc, fam):
    for n, k in [(1, 1), (10, 3), (1000, 1), (1000, 999), (5000, 100), (70000, 4096), (70000, 60000)]:
        w = family(fam, n, n + 3)
        k = min(k, int((w > 0).sum()))
        if k < 1:
            continue
        say("wor", fam, n, k)
        got, st = gpu_wor(wrs, w, k, 17, 2)
        assert st == wrs.OK
        compare_sets(orc, w, k, 17, 2, got)


def test_wor_zero_weights_and_full(wrs, orc):
    w = np.array([0, 3, 0, 1, 2, 0, 5], np.float32)
    say("wor k = #positive")
    got, st = gpu_wor(wrs, w, 4, 1, 0)
    assert st == wrs.OK and list(got) == [1, 3, 4, 6]
    say("wor k > #positive")
    got, st = gpu_wor(wrs, w, 5, 1, 0)
    assert st == wrs.EDOMAIN


def test_wor_bad_weights(wrs):
    for bad in ([1.0, -1.0, 2.0], [1.0, float("nan"), 1.0]):
        say("wor domain", bad)
        _, st = gpu_wor(wrs, np.array(bad, np.float32), 1, 0, 0)
        assert st == wrs.EDOMAIN


@pytest.mark.parametrize("k", [1 << 10, 1 << 16, 1 << 20])
def test_wor_config(wrs, orc, k):
    """n = 2^26 power law s = 0.5 permuted (seed 3), Philox key 3."""
    w = workloads.power_law(1 << 26, 0.5, 3)
    say("wor config", k)
    got, st = gpu_wor(wrs, w, k, 3, 0)
    assert st == wrs.OK
    compare_sets(orc, w, k, 3, 0, got)


def gpu_wor_counts(wrs, w_np, k, seed, sid):
    """As gpu_wor, also returning the candidate counts of the threshold pass and
    of the fallback pass with an infinite threshold (the third and fourth words
    of the workspace's scalars)."""
    import torch
    n = w_np.size
    w = torch.from_numpy(np.ascontiguousarray(w_np, np.float32)).to("cuda:0")
    out = torch.empty(max(k, 1), dtype=torch.int32, device="cuda:0")
    ws = wrs.new_workspace(wrs.OP_WOR, n, k, "cuda:0")
    wrs.sample_wor(w, n, k, seed, sid, out, ws)
    st = wrs.status(ws)
    words = ws[:16].cpu().numpy().view(np.uint32)
    return out[:k].cpu().numpy(), st, int(words[2]), int(words[3])


@pytest.mark.parametrize("n,k", [(50000, 64), (50000, 1000), (50000, 20000), (3 * (1 << 20) + 5, 1 << 16)])
def test_wor_fallback_pass(wrs, orc, n, k):
    """The threshold is estimated from the 4096 weights at positions
    floor(s n / 4096).  Dominant weights on exactly those positions make the
    estimate count each of them n / 4096 times, so the threshold pass finds
    about 4096 / n of its targeted count of candidates, fewer than k (for k of
    at least 64 here), and the fallback
    pass (threshold +infinity, every item a candidate) must produce the sample."""
    rng = np.random.default_rng(n + k)
    w = (1.0 - rng.random(n, dtype=np.float32)).astype(np.float32)
    sub = np.minimum((np.arange(4096, dtype=np.float64) * (n / 4096.0)).astype(np.int64), n - 1)
    w[sub] = np.float32(1e30)
    say("wor fallback", n, k)
    got, st, c1, c2 = gpu_wor_counts(wrs, w, k, 41, 3)
    assert st == wrs.OK
    assert c1 < k and c2 > 0, (c1, c2)
    compare_sets(orc, w, k, 41, 3, got)
