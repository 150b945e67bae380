"""GPU parity of output-sensitive sampling with replacement (Section 5).

The device draws its binomial variates and bucket rejections from the same
Philox counter blocks as the oracle, by the same definitions in IEEE basic
operations, so the sample -- the set of (item, multiplicity) pairs -- must be
identical: bit-exact integers, compared after sorting by item (the device
emits pairs in no particular order).  Cases span many weight groups (uniform
weights cover exponents down to 2^-24, power laws, subnormals, zeros), the
degenerate inputs, ragged sizes, multiplicities large enough for the
transformed-rejection generator, and the maximum-size run's invariants.  At
the paper's n = 10^9 the number of distinct items drawn is checked against
the closed form and against the output size / sample size the paper prints.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_common import family, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


def gpu_os(wrs, w_np, ks, seed, dev="cuda:0"):
    """Build once, sample each k; returns [(items, counts)] sorted by item."""
    import torch
    n = w_np.size
    w = torch.from_numpy(np.ascontiguousarray(w_np, np.float32)).to(dev)
    st = wrs.new_os(n, dev)
    ws = wrs.new_workspace(wrs.OP_OS, n, max(ks), dev)
    wrs.os_build(w, n, st, ws)
    assert wrs.status(st) == wrs.OK
    res = []
    for k in ks:
        cap = max(1, min(k, n))
        items = torch.full((cap,), -1, dtype=torch.int32, device=dev)
        counts = torch.zeros(cap, dtype=torch.int32, device=dev)
        s = torch.full((1,), -1, dtype=torch.int64, device=dev)
        wrs.os_sample(st, n, k, seed, items, counts, s, ws)
        assert wrs.status(ws) == wrs.OK
        s = int(s.item())
        it = items[:s].cpu().numpy()
        ct = counts[:s].cpu().numpy().astype(np.int64)
        o = np.argsort(it, kind="stable")
        res.append((it[o], ct[o]))
    return res


def mixed_groups(n, seed):
    """Weights over the whole FP32 range: subnormals, zeros, large values."""
    rng = np.random.default_rng(seed)
    w = (rng.random(n) * np.exp2(rng.integers(-149, 120, n))).astype(np.float32)
    w[rng.random(n) < 0.05] = 0.0
    w[rng.integers(0, n, 5)] = np.float32(2.0 ** 100)
    return w


CASES = [
    ("uniform", lambda: workloads.uniform(5000, 31), [1, 2, 100, 10000, 1 << 20]),
    ("power1", lambda: workloads.power_law(20000, 1.0, 32), [1, 7, 5000, 1 << 20]),
    ("power2", lambda: family("power2", 3001, 33), [3, 1000, 1 << 22]),
    ("mixed", lambda: mixed_groups(7777, 34), [1, 50, 4096, 1 << 21]),
    ("equal", lambda: family("equal", 4099, 35), [10, 4099, 100000]),
    ("one", lambda: family("one", 1000, 36), [1, 12345]),
    ("n1", lambda: np.array([0.3], np.float32), [1, 5]),
    ("heavy k", lambda: workloads.power_law(300, 1.0, 37), [(1 << 31) - 1]),
]


@pytest.mark.parametrize("name,make,ks", CASES, ids=[c[0] for c in CASES])
def test_os_matches_oracle(wrs, name, make, ks):
    w = make()
    for seed in (1, 2):
        say("os", name, "seed", seed, "k", ks)
        got = gpu_os(wrs, w, ks, seed)
        for k, (it, ct) in zip(ks, got):
            ref_it, ref_ct = oracle.os_sample(w, k, seed)
            assert np.array_equal(it, ref_it), (name, k, seed)
            assert np.array_equal(ct, ref_ct), (name, k, seed)
            assert ct.sum() == k


def test_os_zero_draws_and_errors(wrs):
    import torch
    say("os: k = 0 and bad weights")
    (it, ct), = gpu_os(wrs, workloads.uniform(100, 3), [0], 1)
    assert it.size == 0
    for bad in (-1.0, float("nan"), float("inf")):
        w = torch.from_numpy(workloads.uniform(1000, 4)).cuda()
        w[500] = bad
        st = wrs.new_os(1000)
        ws = wrs.new_workspace(wrs.OP_OS, 1000, 10)
        wrs.os_build(w, 1000, st, ws)
        assert wrs.status(st) == wrs.EDOMAIN
        items = torch.empty(10, dtype=torch.int32, device="cuda")
        counts = torch.empty(10, dtype=torch.int32, device="cuda")
        s = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        wrs.os_sample(st, 1000, 10, 1, items, counts, s, ws)
        assert wrs.status(ws) == wrs.EDOMAIN and int(s.item()) == 0
    w = torch.zeros(64, dtype=torch.float32, device="cuda")
    st = wrs.new_os(64)
    ws = wrs.new_workspace(wrs.OP_OS, 64, 1)
    wrs.os_build(w, 64, st, ws)
    assert wrs.status(st) == wrs.EDOMAIN
    # a structure queried with another n than it was built for is refused
    w = torch.from_numpy(workloads.uniform(5000, 5)).cuda()
    st = wrs.new_os(5000)
    ws = wrs.new_workspace(wrs.OP_OS, 5000, 100)
    wrs.os_build(w, 5000, st, ws)
    assert wrs.status(st) == wrs.OK
    items = torch.empty(100, dtype=torch.int32, device="cuda")
    counts = torch.empty(100, dtype=torch.int32, device="cuda")
    s = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    wrs.os_sample(st, 4000, 100, 1, items, counts, s, ws)
    assert wrs.status(ws) == wrs.EINVAL and int(s.item()) == 0


def test_os_ragged_mid_size(wrs):
    n = (1 << 20) + 123
    w = workloads.power_law(n, 1.0, 38)
    w[::97] = 0.0
    ks = [1 << 10, 1 << 22]
    say("os: n = 2^20 + 123, power law with zeros")
    for k, (it, ct) in zip(ks, gpu_os(wrs, w, ks, 9)):
        ref_it, ref_ct = oracle.os_sample(w, k, 9)
        assert np.array_equal(it, ref_it) and np.array_equal(ct, ref_ct), k


def test_os_full_size_invariants(wrs):
    """n = 2^28 (power law s = 1), k = 2^30, where the oracle is too slow:
    multiplicities sum to k over distinct positive items, and the 64 heaviest
    items' multiplicities are within 6 sigma of k w_i / W."""
    import torch
    n, k = 1 << 28, 1 << 30
    say("os: n = 2^28, k = 2^30")
    w_np = workloads.power_law(n, 1.0, 2)
    w = torch.from_numpy(w_np).cuda()
    st = wrs.new_os(n)
    ws = wrs.new_workspace(wrs.OP_OS, n, k)
    wrs.os_build(w, n, st, ws)
    assert wrs.status(st) == wrs.OK
    del w
    cap = min(k, n)
    items = torch.empty(cap, dtype=torch.int32, device="cuda")
    counts = torch.empty(cap, dtype=torch.int32, device="cuda")
    s = torch.zeros(1, dtype=torch.int64, device="cuda")
    wrs.os_sample(st, n, k, 2, items, counts, s, ws)
    assert wrs.status(ws) == wrs.OK
    s = int(s.item())
    it = items[:s]
    ct = counts[:s]
    assert int(ct.to(torch.int64).sum()) == k and int(ct.min()) >= 1
    srt = torch.sort(it).values
    assert int(srt[0]) >= 0 and int(srt[-1]) < n and bool((srt[1:] > srt[:-1]).all())
    it_np, ct_np = it.cpu().numpy(), ct.cpu().numpy()
    assert np.all(w_np[it_np] > 0)
    W = w_np.astype(np.float64).sum()
    top = np.argsort(w_np)[-64:]
    got = np.zeros(n, np.int64)
    got[it_np] = ct_np
    p = w_np[top].astype(np.float64) / W
    assert np.all(np.abs(got[top] - k * p) <= 6 * np.sqrt(k * p * (1 - p)) + 1)


def test_os_distinct_fraction_at_paper_size(wrs):
    """n = 10^9, as in the paper's query figure: s / k of an output-sensitive
    sample against the printed output size / sample size (golden fixture, within
    its rtol) and against the closed form sum_i 1 - (1 - w_i/W)^k for these very
    weights (within 6 sigma; the indicators are negatively correlated)."""
    import json
    import math
    import os
    import torch
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "golden", "paper_distinct_fraction.json")) as f:
        g = json.load(f)
    n = g["n"]
    dev = torch.device("cuda:0")
    kmax = max(c["k"] for c in g["cases"])
    st = wrs.new_os(n, dev)
    ws = wrs.new_workspace(wrs.OP_OS, n, kmax, dev)
    cap = min(kmax, n)
    items = torch.empty(cap, dtype=torch.int32, device=dev)
    counts = torch.empty(cap, dtype=torch.int32, device=dev)
    s = torch.zeros(1, dtype=torch.int64, device=dev)
    gen = torch.Generator(device=dev)
    for c in g["cases"]:
        say("os at n = 10^9:", c["family"], c["s"], "k", c["k"])
        if c["family"] == "uniform":
            gen.manual_seed(41)
            w = 1.0 - torch.rand(n, generator=gen, device=dev, dtype=torch.float32)
        else:
            w = torch.arange(1, n + 1, device=dev, dtype=torch.float64).pow(-c["s"]).to(torch.float32)
        wrs.os_build(w, n, st, ws)
        assert wrs.status(st) == wrs.OK
        k = c["k"]
        wrs.os_sample(st, n, k, 3, items, counts, s, ws)
        assert wrs.status(ws) == wrs.OK
        sv = int(s.item())
        assert int(counts[:sv].to(torch.int64).sum()) == k
        W = float(w.double().sum())
        ex, var = 0.0, 0.0
        for a in range(0, n, 1 << 27):
            p = w[a:a + (1 << 27)].double() / W
            q = -torch.expm1(k * torch.log1p(-p))
            ex += float(q.sum())
            var += float((q * (1 - q)).sum())
        del w
        say("  s/k", sv / k, "closed form", ex / k, "printed", c["printed"])
        assert abs(sv - ex) <= 6 * math.sqrt(var) + 1, (c, sv, ex)
        assert abs(sv / k - c["printed"]) <= c["rtol"] * c["printed"], (c, sv / k)
