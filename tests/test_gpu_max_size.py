"""The largest table the C ABI accepts: n = 2^31 - 1 FP32 weights (uniform,
seed 6; a ragged last tile).  Int32 item indices, tile counts and 64-bit
offsets are all at their limits here.

Checks (test infrastructure only: torch on the device for the per-item sums,
the oracle for exact values):
  - every bucket has t in [0, 1] and alias in [0, n);
  - every item's reconstructed mass t_i + sum of (1 - t_r) over buckets r != i
    aliasing to i is within 1e-6 relative of n w_i / W, with W the oracle's
    exact total (FP64 sums in chunks of 2^28 buckets);
  - 2^16 sampled light buckets hold the correctly rounded n w_i / W (1 ulp);
  - 2^20 draws from the table (and every 4099th of 2^26) equal the oracle's
    queries of the same table with the same counters.
"""
import numpy as np
import pytest

import workloads
from gpu_common import say, ulp_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


def test_max_size_build_and_sample(wrs, orc):
    import torch
    dev = torch.device("cuda:0")
    n = (1 << 31) - 1
    say("max size: generating", n, "weights")
    w_np = workloads.uniform(n, 6)
    W_hi, W_lo = orc.total_weight(w_np)
    w = torch.from_numpy(w_np).to(dev)
    table = wrs.new_table(n, dev)
    ws = wrs.new_workspace(wrs.OP_BUILD, n, 0, dev)
    say("max size: build")
    wrs.alias_build(w, n, table, ws)
    assert wrs.status(ws) == wrs.OK
    del ws
    torch.cuda.empty_cache()
    t = table[:, 0].view(torch.float32)
    a = table[:, 1]
    assert bool(((t >= 0) & (t <= 1)).all()) and bool(((a >= 0) & (a < n)).all())

    say("max size: per-item mass")
    mass = t.double()
    chunk = 1 << 28
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        own = torch.arange(s, e, device=dev, dtype=torch.int64)
        al = a[s:e].long()
        m = al != own
        mass.index_add_(0, al[m], (1.0 - t[s:e].double())[m])
        del own, al, m
    W = W_hi + W_lo
    worst = 0.0
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        want = w[s:e].double() * (float(n) / W)
        err = ((mass[s:e] - want).abs() / want).max().item()
        worst = max(worst, err)
    del mass
    assert worst <= 1e-6, worst

    say("max size: sampled light buckets")
    t_host = table[:, 0].contiguous().view(torch.float32).cpu().numpy()
    a_host = table[:, 1].contiguous().cpu().numpy()
    idx = np.random.default_rng(7).integers(0, n, 1 << 16)
    light, tl = orc.light_t_at(w_np, idx)
    assert light.mean() > 0.4
    assert np.all(ulp_diff(t_host[idx[light]], tl[light]) <= 1)

    say("max size: draws")
    k = 1 << 26
    out = torch.empty(k, dtype=torch.int32, device=dev)
    wrs.alias_sample(table, n, 6, 0, 0, k, out)
    torch.cuda.synchronize()
    cnt = np.concatenate([np.arange(0, 1 << 20), np.arange(0, k, 4099)]).astype(np.uint64)
    got = out[torch.from_numpy(cnt.astype(np.int64)).to(dev)].cpu().numpy()
    want = orc.alias_sample_at(t_host, a_host, 6, 0, cnt)
    assert np.array_equal(got, want)
