"""Property-based GPU parity (hypothesis, a bounded number of examples): random
instances with n in [1, 2^12] from weight mixtures with zeros, duplicates,
one dominant item, all-equal runs, subnormals, huge ratios and integers, built
by wrs_alias_build, wrs_alias_build_plus and wrs_twolevel_build and sampled by
wrs_alias_sample, each against the oracle with the bars of the dedicated
parity tests (aliases bit for bit, thresholds within their error bounds,
draws bit-exact on the GPU's own table); output-sensitive samples of random
size k < 2^31 bit for bit."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from gpu_common import gpu_build, say
from test_oracle_properties import weights

pytestmark = pytest.mark.gpu

SETTINGS = settings(max_examples=25, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


def t_tol(n, t_ref, units):
    unit = 2.0 ** (int(n).bit_length() - 1 - 60)
    return np.spacing(np.abs(t_ref).astype(np.float32)).astype(np.float64) + units * unit


@SETTINGS
@given(weights())
def test_random_builds_match_oracle(wrs, orc, w):
    n = w.size
    say("property build", n)
    t, a, st_, table, *_ = gpu_build(wrs, w)
    assert st_ == wrs.OK
    t_ref, a_ref = orc.sweep_build(w)
    assert np.array_equal(a, a_ref)
    assert np.all(np.abs(t.astype(np.float64) - t_ref) <= t_tol(n, t_ref, 513))
    import torch
    k = 4 * n + 17
    out = torch.empty(k, dtype=torch.int32, device=table.device)
    wrs.alias_sample(table, n, 5, 1, 3, k, out)
    assert np.array_equal(out.cpu().numpy(), orc.alias_sample(t, a, 5, 1, 3, k))
    tp, ap, st_p, *_ = gpu_build(wrs, w, plus=True)
    assert st_p == wrs.OK
    tr, ar = orc.psaplus_build(w, 2048)
    assert np.array_equal(ap, ar)
    assert np.all(np.abs(tp.astype(np.float64) - tr) <= t_tol(n, tr, 1025))


@SETTINGS
@given(weights())
def test_random_twolevel_match_oracle(wrs, orc, w):
    import torch
    n = w.size
    G = -(-n // 2048)
    say("property twolevel", n)
    dev = torch.device("cuda:0")
    wt = torch.from_numpy(w).to(dev)
    table, top = wrs.new_table(n, dev), wrs.new_table(G, dev)
    ws = wrs.new_workspace(wrs.OP_TWOLEVEL, n, 0, dev)
    wrs.twolevel_build(wt, n, table, top, ws)
    assert wrs.status(ws) == wrs.OK
    tb, tp = table.cpu().numpy(), top.cpu().numpy()
    rtt, rat, rt, ra = orc.twolevel_build(w, 2048)
    assert np.array_equal(tp[:, 1], rat) and np.array_equal(tb[:, 1], ra)
    tt, t = tp[:, 0].copy().view(np.float32), tb[:, 0].copy().view(np.float32)
    assert np.all(np.abs(t.astype(np.float64) - rt) <= t_tol(1, rt, 1025))
    assert np.all(np.abs(tt.astype(np.float64) - rtt) <= t_tol(G, rtt, 513))
    k = 2 * n + 5
    out = torch.empty(k, dtype=torch.int32, device=dev)
    wrs.twolevel_sample(top, table, n, 8, 2, 1, k, out)
    assert np.array_equal(out.cpu().numpy(), orc.twolevel_sample(tt, tp[:, 1], t, tb[:, 1], 2048, 8, 2, 1, k))


@SETTINGS
@given(weights(), st.integers(0, 2 ** 31 - 1), st.integers(0, 2 ** 63))
def test_random_output_sensitive_match_oracle(wrs, orc, w, k, seed):
    """wrs_os_build + wrs_os_sample against the oracle: the same (item,
    multiplicity) pairs, bit for bit (compared sorted by item)."""
    import torch
    n = w.size
    say("property output-sensitive", n, k)
    dev = torch.device("cuda:0")
    wt = torch.from_numpy(np.ascontiguousarray(w)).to(dev)
    st_ = wrs.new_os(n, dev)
    ws = wrs.new_workspace(wrs.OP_OS, n, k, dev)
    wrs.os_build(wt, n, st_, ws)
    assert wrs.status(st_) == wrs.OK
    cap = max(1, min(k, n))
    items = torch.empty(cap, dtype=torch.int32, device=dev)
    counts = torch.empty(cap, dtype=torch.int32, device=dev)
    s = torch.zeros(1, dtype=torch.int64, device=dev)
    wrs.os_sample(st_, n, k, seed, items, counts, s, ws)
    assert wrs.status(ws) == wrs.OK
    s = int(s.item())
    it, ct = items[:s].cpu().numpy(), counts[:s].cpu().numpy().astype(np.int64)
    o = np.argsort(it)
    ref_it, ref_ct = orc.os_sample(w, k, seed)
    assert np.array_equal(it[o], ref_it) and np.array_equal(ct[o], ref_ct)
