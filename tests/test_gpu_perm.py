"""GPU parity of the weighted permutation (C ABI wrs_permutation, problem WRP,
Sections 1 and 7) against the oracle.

Bar: the output is a permutation of 0..n-1 in ascending order of the oracle's
FP64 keys -ln(u_i)/w_i, ties by index, where two keys within 1e-12 relative may
appear in either order.  Both sides compute -ln u in FP64 to about an ulp (the
GPU through log1p for u >= 1/2, the oracle through log), so only such near-ties
can swap; everything else equals the oracle's permutation.  Independently of
the oracle, the first k items form exactly the GPU's own sample without
replacement of size k (the same keys), for several k.
"""
import numpy as np
import pytest

from gpu_common import family, say

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


def gpu_perm(wrs, w_np, seed, sid):
    import torch
    dev = torch.device("cuda:0")
    n = w_np.size
    w = torch.from_numpy(np.ascontiguousarray(w_np, np.float32)).to(dev)
    out = torch.full((n,), -1, dtype=torch.int32, device=dev)
    ws = wrs.new_workspace(wrs.OP_PERM, n, 0, dev)
    wrs.permutation(w, n, seed, sid, out, ws)
    st = wrs.status(ws)
    return out.cpu().numpy(), st, w, ws


def check_against_oracle(orc, w, seed, sid, p):
    n = w.size
    assert np.array_equal(np.sort(p), np.arange(n)), "not a permutation"
    ref = orc.permutation(w, seed, sid)
    keys = orc.wor_keys(w, seed, sid)
    kp = keys[p]
    fin = np.isfinite(kp)
    # ascending up to near-ties; the +inf (zero-weight) items last
    assert np.all(fin[:-1] >= fin[1:]), "an infinite key before a finite one"
    a, b = kp[:-1], kp[1:]
    both = fin[:-1] & fin[1:]
    assert np.all(b[both] >= a[both] * (1 - REL)), "keys out of order"
    # exact ties (equal oracle keys) in index order
    tie = (a == b) | (~fin[:-1] & ~fin[1:])
    assert np.all(p[1:][tie] > p[:-1][tie]), "tie not broken by index"
    diff = np.nonzero(p != ref)[0]
    if diff.size:
        # each differing position holds a key within REL of the oracle's key there
        kr = keys[ref[diff]]
        assert np.all(np.abs(kp[diff] - kr) <= REL * np.abs(kr)), f"{diff.size} positions differ beyond near-ties"


SIZES = [1, 2, 63, 4095, 4096, 4097, 10000, 100003, (1 << 20) + 17]
FAMILIES = ["uniform", "power0.5", "power1", "ints", "equal", "one", "negzero", "sorted_power1", "tiny_heavies",
            "wide", "ties"]


@pytest.mark.parametrize("fam", FAMILIES)
def test_perm_matches_oracle(wrs, orc, fam):
    for n in SIZES:
        w = family(fam, n, 500 + n)
        say("perm", fam, n)
        p, st, *_ = gpu_perm(wrs, w, 7 + n, 3)
        assert st == wrs.OK
        check_against_oracle(orc, w, 7 + n, 3, p)


def test_perm_prefix_is_the_gpu_wor_sample(wrs):
    import torch
    import workloads
    dev = torch.device("cuda:0")
    n = 300000
    w_np = workloads.power_law(n, 0.5, 12)
    say("perm prefix vs wor", n)
    p, st, w, _ = gpu_perm(wrs, w_np, 12, 5)
    assert st == wrs.OK
    for k in (1, 1000, 65536, 299999):
        out = torch.empty(k, dtype=torch.int32, device=dev)
        ws = wrs.new_workspace(wrs.OP_WOR, n, k, dev)
        wrs.sample_wor(w, n, k, 12, 5, out, ws)
        assert wrs.status(ws) == wrs.OK
        assert np.array_equal(np.sort(p[:k]), out.cpu().numpy()), k


def test_perm_deterministic_and_streams_differ(wrs):
    w = family("uniform", 50000, 3)
    say("perm determinism")
    a, *_ = gpu_perm(wrs, w, 1, 0)
    b, *_ = gpu_perm(wrs, w, 1, 0)
    c, *_ = gpu_perm(wrs, w, 1, 1)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_perm_domain_errors(wrs):
    for bad in ([1.0, -1.0, 2.0], [1.0, float("nan")], [float("inf"), 1.0]):
        say("perm domain", bad)
        _, st, *_ = gpu_perm(wrs, np.array(bad, np.float32), 1, 0)
        assert st == wrs.EDOMAIN


def test_perm_large(wrs, orc):
    """n = 2^26, the sampling-without-replacement input (power law s = 0.5,
    seed 3, Philox key 3), checked against the oracle in full."""
    import workloads
    n = 1 << 26
    w = workloads.power_law(n, 0.5, 3)
    say("perm 2^26")
    p, st, *_ = gpu_perm(wrs, w, 3, 0)
    assert st == wrs.OK
    check_against_oracle(orc, w, 3, 0, p)
