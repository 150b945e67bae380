"""The greedy-block build, the 2-level table and the weighted permutation at
the largest size the C ABI accepts: n = 2^31 - 1 FP32 weights (uniform, seed 6;
ragged last tile and block).  Int32 item indices, 2^20 greedy blocks and
meta-items, 2^19 radix blocks and 64-bit offsets are at their limits here.

Checks (test infrastructure only: torch on the device for per-item sums, the
oracle for exact values):
  - greedy-block build: t in [0, 1], alias in [0, n), every item's mass within
    1e-6 relative of n w_i / W (W the oracle's exact total);
  - 2-level table: every item's probability P(block) P(item | block) within
    1e-6 relative of w_i / W, and 2^20 draws equal the oracle's two-step query
    of the same tables;
  - permutation: every item exactly once, and at 2^16 sampled positions the
    oracle keys of neighbouring items ascend (up to 1e-12 relative);
  - sampling without replacement (k = 2^16): ascending distinct indices, 2^20
    random unselected items all have oracle keys at or above the largest
    selected key, and the selection is the permutation's first k items;
  - output-sensitive sampling (k = 2^20): distinct items in range with
    positive weights, multiplicities summing to k, and the draws of each
    weight group (binary exponent) within 6 sigma of k times its share of W.
"""
import numpy as np
import pytest

import workloads
from gpu_common import say

pytestmark = pytest.mark.gpu

N = (1 << 31) - 1
CHUNK = 1 << 28


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


@pytest.fixture(scope="module")
def weights(orc):
    say("max size (next): generating", N, "weights")
    w_np = workloads.uniform(N, 6)
    hi, lo = orc.total_weight(w_np)
    return w_np, hi + lo


def item_mass(torch, t, a, n):
    """t_i plus the sum of (1 - t_r) over buckets r != i aliasing to i (FP64)."""
    dev = t.device
    mass = t.double()
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        own = torch.arange(s, e, device=dev, dtype=torch.int64)
        al = a[s:e].long()
        m = al != own
        mass.index_add_(0, al[m], (1.0 - t[s:e].double())[m])
        del own, al, m
    return mass


def test_max_size_build_plus(wrs, orc, weights):
    import torch
    w_np, W = weights
    dev = torch.device("cuda:0")
    w = torch.from_numpy(w_np).to(dev)
    table = wrs.new_table(N, dev)
    ws = wrs.new_workspace(wrs.OP_BUILD_PLUS, N, 0, dev)
    say("max size: build plus")
    wrs.alias_build_plus(w, N, table, ws)
    assert wrs.status(ws) == wrs.OK
    left = wrs.plus_leftovers(ws)
    assert 0 < left < N // 10
    del ws
    torch.cuda.empty_cache()
    t = table[:, 0].view(torch.float32)
    a = table[:, 1]
    assert bool(((t >= 0) & (t <= 1)).all()) and bool(((a >= 0) & (a < N)).all())
    say("max size: plus per-item mass")
    mass = item_mass(torch, t, a, N)
    worst = 0.0
    for s in range(0, N, CHUNK):
        e = min(N, s + CHUNK)
        want = w[s:e].double() * (float(N) / W)
        worst = max(worst, ((mass[s:e] - want).abs() / want).max().item())
    assert worst <= 1e-6, worst
    del mass, table, w
    torch.cuda.empty_cache()


def test_max_size_twolevel(wrs, orc, weights):
    import torch
    w_np, W = weights
    dev = torch.device("cuda:0")
    B = wrs.TWOLEVEL_BLOCK
    G = -(-N // B)
    w = torch.from_numpy(w_np).to(dev)
    table = wrs.new_table(N, dev)
    top = wrs.new_table(G, dev)
    ws = wrs.new_workspace(wrs.OP_TWOLEVEL, N, 0, dev)
    say("max size: two-level build")
    wrs.twolevel_build(w, N, table, top, ws)
    assert wrs.status(ws) == wrs.OK
    t = table[:, 0].view(torch.float32)
    a = table[:, 1]
    tt = top[:, 0].view(torch.float32)
    at = top[:, 1]
    assert bool(((tt >= 0) & (tt <= 1)).all()) and bool(((at >= 0) & (at < G)).all())
    say("max size: two-level probabilities")
    mt = tt.double().clone()
    mt.index_add_(0, at.long(), 1.0 - tt.double())
    pg = mt / G
    mass = item_mass(torch, t, a, N)
    worst = 0.0
    for s in range(0, N, CHUNK):
        e = min(N, s + CHUNK)
        idx = torch.arange(s, e, device=dev, dtype=torch.int64)
        g = idx // B
        m = torch.clamp(N - g * B, max=B).double()
        p = pg[g] * mass[s:e] / m
        want = w[s:e].double() / W
        worst = max(worst, ((p - want).abs() / want).max().item())
        del idx, g, m, p, want
    assert worst <= 1e-6, worst
    del mass
    say("max size: two-level draws")
    k = 1 << 20
    out = torch.empty(k, dtype=torch.int32, device=dev)
    wrs.twolevel_sample(top, table, N, 6, 1, 0, k, out)
    got = out.cpu().numpy()
    ref = orc.twolevel_sample(tt.contiguous().cpu().numpy(), at.contiguous().cpu().numpy(),
                              t.contiguous().cpu().numpy(), a.contiguous().cpu().numpy(), B, 6, 1, 0, k)
    assert np.array_equal(got, ref)
    del table, top, ws, w, out
    torch.cuda.empty_cache()


def test_max_size_permutation(wrs, orc, weights):
    import torch
    w_np, _ = weights
    dev = torch.device("cuda:0")
    w = torch.from_numpy(w_np).to(dev)
    out = torch.empty(N, dtype=torch.int32, device=dev)
    ws = wrs.new_workspace(wrs.OP_PERM, N, 0, dev)
    say("max size: permutation")
    wrs.permutation(w, N, 6, 0, out, ws)
    assert wrs.status(ws) == wrs.OK
    del ws, w
    torch.cuda.empty_cache()
    say("max size: permutation is one")
    seen = torch.zeros(N, dtype=torch.bool, device=dev)
    seen[out.long()] = True
    assert bool(seen.all())
    del seen
    say("max size: sampled neighbours ascend")
    pos = np.random.default_rng(9).integers(0, N - 1, 1 << 16)
    o = out.cpu().numpy()
    ka = orc.wor_keys_at(w_np, 6, 0, o[pos].astype(np.int64))
    kb = orc.wor_keys_at(w_np, 6, 0, o[pos + 1].astype(np.int64))
    assert np.all(kb >= ka * (1 - 1e-12))


def test_max_size_wor(wrs, orc, weights):
    import torch
    w_np, _ = weights
    dev = torch.device("cuda:0")
    k = 1 << 16
    w = torch.from_numpy(w_np).to(dev)
    sel = torch.empty(k, dtype=torch.int32, device=dev)
    ws = wrs.new_workspace(wrs.OP_WOR, N, k, dev)
    say("max size: without replacement")
    wrs.sample_wor(w, N, k, 6, 0, sel, ws)
    assert wrs.status(ws) == wrs.OK
    del ws
    torch.cuda.empty_cache()
    s = sel.cpu().numpy()
    assert np.all(np.diff(s) > 0) and s[0] >= 0 and s[-1] < N
    kappa = orc.wor_keys_at(w_np, 6, 0, s.astype(np.int64)).max()
    rng = np.random.default_rng(12)
    others = np.setdiff1d(rng.integers(0, N, 1 << 20), s)
    assert np.all(orc.wor_keys_at(w_np, 6, 0, others.astype(np.int64)) >= kappa * (1 - 1e-6))
    say("max size: without replacement against the permutation's prefix")
    out = torch.empty(N, dtype=torch.int32, device=dev)
    pws = wrs.new_workspace(wrs.OP_PERM, N, 0, dev)
    wrs.permutation(w, N, 6, 0, out, pws)
    assert wrs.status(pws) == wrs.OK
    assert np.array_equal(np.sort(out[:k].cpu().numpy()), s)


def test_max_size_output_sensitive(wrs, weights):
    import torch
    w_np, W = weights
    dev = torch.device("cuda:0")
    k = 1 << 20
    w = torch.from_numpy(w_np).to(dev)
    st = wrs.new_os(N, dev)
    ws = wrs.new_workspace(wrs.OP_OS, N, k, dev)
    say("max size: output-sensitive build and sample")
    wrs.os_build(w, N, st, ws)
    assert wrs.status(st) == wrs.OK
    items = torch.empty(k, dtype=torch.int32, device=dev)
    counts = torch.empty(k, dtype=torch.int32, device=dev)
    s = torch.zeros(1, dtype=torch.int64, device=dev)
    wrs.os_sample(st, N, k, 4, items, counts, s, ws)
    assert wrs.status(ws) == wrs.OK
    del st, ws
    s = int(s.item())
    it, ct = items[:s], counts[:s].to(torch.int64)
    assert int(ct.sum()) == k and int(ct.min()) >= 1 and s > k - 4096
    srt = torch.sort(it).values
    assert int(srt[0]) >= 0 and int(srt[-1]) < N and bool((srt[1:] > srt[:-1]).all())
    assert bool((w[it.long()] > 0).all())
    del w
    # per-group masses on the host, in chunks (few groups: device atomics on
    # a handful of bins would serialize)
    mass = np.zeros(400)
    for s0 in range(0, N, CHUNK):
        c = w_np[s0:s0 + CHUNK]
        _, e = np.frexp(c)
        mass += np.bincount(e + 200, weights=c.astype(np.float64), minlength=400)
        say("max size: group masses through item", s0 + c.size)
    it_np, ct_np = it.cpu().numpy(), ct.cpu().numpy()
    _, e_it = np.frexp(w_np[it_np])
    g = np.bincount(e_it + 200, weights=ct_np.astype(np.float64), minlength=400)
    p = mass / W
    assert np.all(np.abs(g - k * p) <= 6 * np.sqrt(k * p * (1 - p)) + 1)

