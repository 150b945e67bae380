"""GPU parity of 2-level alias tables (C ABI wrs_twolevel_build /
wrs_twolevel_sample, Section 4.4 replicated top level) against the oracle.

Bar: block tables and top table have the oracle's aliases bit for bit.  Light
thresholds are within 1 ulp.  Heavy thresholds come from 64-bit keys: inside a
block the key unit is below 2^-48 of a bucket (<= 1025 units of error); the
top table is the splitting construction over G meta-items (513 units of
2^(floor(log2 G) - 60)).  Every item's probability P(block) P(item | block) is
within 1e-6 relative of w_i / W.  Draws are bit-identical to the oracle's
two-step query on the GPU's own tables.
"""
import numpy as np
import pytest

from gpu_common import family, say, ulp_diff

pytestmark = pytest.mark.gpu

BLOCK = 2048


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    assert w.TWOLEVEL_BLOCK == BLOCK
    return w


def gpu_twolevel(wrs, w_np):
    import torch
    dev = torch.device("cuda:0")
    n = w_np.size
    G = -(-n // BLOCK)
    w = torch.from_numpy(np.ascontiguousarray(w_np, np.float32)).to(dev)
    table = wrs.new_table(n, dev)
    top = wrs.new_table(G, dev)
    ws = wrs.new_workspace(wrs.OP_TWOLEVEL, n, 0, dev)
    wrs.twolevel_build(w, n, table, top, ws)
    st = wrs.status(ws)
    tb, tp = table.cpu().numpy(), top.cpu().numpy()
    return (tp[:, 0].copy().view(np.float32), tp[:, 1].copy(), tb[:, 0].copy().view(np.float32), tb[:, 1].copy(),
            st, table, top)


def probabilities(n, tt, at, t, a):
    """P(item) = P(block) P(item | block) implied by the tables (FP64)."""
    G = tt.size
    mt = tt.astype(np.float64) + np.bincount(at, weights=1.0 - tt.astype(np.float64), minlength=G)
    mi = t.astype(np.float64) + np.bincount(a, weights=1.0 - t.astype(np.float64), minlength=n)
    g = np.arange(n) // BLOCK
    m = np.minimum(BLOCK, n - g * BLOCK)
    return (mt / G)[g] * mi / m


def check(orc, w, tt, at, t, a):
    n = w.size
    rtt, rat, rt, ra = orc.twolevel_build(w, BLOCK)
    for name, x, y in (("top", at, rat), ("block", a, ra)):
        bad = np.nonzero(x != y)[0]
        assert bad.size == 0, f"{name}: {bad.size} alias mismatches, first at {bad[:5]}: gpu {x[bad[:5]]} ref {y[bad[:5]]}"
    G = tt.size
    for x, y, unit in ((tt, rtt, 513 * 2.0 ** (int(G).bit_length() - 1 - 60)), (t, rt, 1025 * 2.0 ** -48)):
        tol = np.spacing(np.abs(y)).astype(np.float64) + unit
        assert np.all(np.abs(x.astype(np.float64) - y) <= tol)
    wd = np.abs(w.astype(np.float64))
    light = wd * np.minimum(BLOCK, n) <= wd.sum() * (1 - 1e-12)
    p = probabilities(n, tt, at, t, a)
    ref = wd / wd.sum()
    pos = wd > 0
    assert np.max(np.abs(p[pos] - ref[pos]) / ref[pos]) <= 1e-6
    assert np.all(p[~pos] == 0)
    del light


SIZES = [1, 2, 2047, 2048, 2049, 5000, 3 * 2048 + 17, 40000, 200001, (1 << 20) + 5]
FAMILIES = ["uniform", "power0.5", "power1", "power2", "ints", "equal", "one", "dominant", "sorted_power1",
            "tiny_heavies", "negzero", "wide", "ties"]


@pytest.mark.parametrize("fam", FAMILIES)
def test_twolevel_matches_oracle(wrs, orc, fam):
    for n in SIZES:
        w = family(fam, n, 900 + n)
        if np.abs(w.astype(np.float64)).sum() == 0:
            continue
        say("twolevel", fam, n)
        tt, at, t, a, st, *_ = gpu_twolevel(wrs, w)
        assert st == wrs.OK
        check(orc, w, tt, at, t, a)


def test_twolevel_zero_block_and_draws(wrs, orc):
    import torch
    n = 5 * BLOCK + 100
    w = family("uniform", n, 3)
    w[BLOCK:2 * BLOCK] = 0.0  # a block of weight zero
    say("twolevel zero block")
    tt, at, t, a, st, table, top = gpu_twolevel(wrs, w)
    assert st == wrs.OK
    check(orc, w, tt, at, t, a)
    assert np.all(t[BLOCK:2 * BLOCK] == 1.0) and np.array_equal(a[BLOCK:2 * BLOCK], np.arange(BLOCK, 2 * BLOCK))
    k = 1 << 20
    out = torch.empty(k, dtype=torch.int32, device=table.device)
    wrs.twolevel_sample(top, table, n, 21, 4, 7, k, out)
    got = out.cpu().numpy()
    ref = orc.twolevel_sample(tt, at, t, a, BLOCK, 21, 4, 7, k)
    assert np.array_equal(got, ref)
    assert not np.any((got >= BLOCK) & (got < 2 * BLOCK))


@pytest.mark.parametrize("fam", ["uniform", "power1"])
def test_twolevel_full_size(wrs, orc, fam):
    """n = 2^28 (seed 2): 256 sampled blocks against the oracle's sweep of the
    block, every item's probability within 1e-6 of w_i / W, and 2^30 draws
    sampled at the first and last 2^16 counters and every 4099th."""
    import torch
    import workloads
    n = 1 << 28
    w = workloads.uniform(n, 2) if fam == "uniform" else workloads.power_law(n, 1.0, 2)
    say("twolevel full size", fam)
    tt, at, t, a, st, table, top = gpu_twolevel(wrs, w)
    assert st == wrs.OK
    G = tt.size
    assert np.all((tt >= 0) & (tt <= 1)) and np.all((at >= 0) & (at < G))
    for g in np.random.default_rng(6).choice(G, 256, replace=False):
        b0 = int(g) * BLOCK
        rt, ra = orc.sweep_build(w[b0:b0 + BLOCK])
        assert np.array_equal(a[b0:b0 + BLOCK], ra + b0), g
        tol = np.spacing(np.abs(rt)).astype(np.float64) + 1025 * 2.0 ** -48
        assert np.all(np.abs(t[b0:b0 + BLOCK].astype(np.float64) - rt) <= tol), g
    p = probabilities(n, tt, at, t, a)
    wd = w.astype(np.float64)
    ref = wd / wd.sum()
    assert np.max(np.abs(p - ref) / ref) <= 1e-6
    del p, ref, wd
    k = 1 << 30
    out = torch.empty(k, dtype=torch.int32, device=table.device)
    wrs.twolevel_sample(top, table, n, 2, 0, 0, k, out)
    idx = np.unique(np.concatenate([np.arange(1 << 16), np.arange(k - (1 << 16), k), np.arange(0, k, 4099)]))
    got = out.cpu().numpy()[idx]
    assert np.array_equal(got, orc.twolevel_sample_at(tt, at, t, a, BLOCK, 2, 0, idx.astype(np.uint64)))


def test_twolevel_domain_errors(wrs):
    for bad in ([1.0, -1.0, 2.0], [1.0, float("nan")], [float("inf"), 1.0], [0.0, 0.0]):
        say("twolevel domain", bad)
        *_, st, _, _ = gpu_twolevel(wrs, np.array(bad, np.float32))
        assert st == wrs.EDOMAIN
