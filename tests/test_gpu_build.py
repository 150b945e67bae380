"""GPU parity of alias-table construction (C ABI wrs_alias_build) against the oracle.

Bar: aliases bit-identical to the exact sequential sweep (Algorithm 2,
Section 4.1); every item's mass within 1e-6 relative of n w_i / W; thresholds
within the error the kernel's arithmetic allows:
  * a light bucket's t = n w / W goes through two FP64 products before the FP32
    rounding, so it is within 1 ulp of the correctly rounded value;
  * a heavy bucket's t = 1 + (E - D) / W uses 64-bit merge keys: exact tile
    prefix sums plus item sizes rounded to the key unit u <= 2^(floor(log2 n) - 60)
    bucket, so E - D is off by at most (TILE/2 + 1) u, TILE = 1024, plus 1 ulp.
"""
import numpy as np
import pytest

from gpu_common import check_against_sweep, family, gpu_build, say, t_tolerance, ulp_diff  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


SIZES = [1, 2, 3, 5, 63, 1000, 1023, 1024, 1025, 2047, 4096, 5000, 3 * 1024 + 17, 40000, 65536, 65536 + 37]
FAMILIES = ["uniform", "power0.5", "power1", "power2", "ints", "equal", "one", "dominant", "sorted_power1",
            "tiny_heavies", "negzero", "wide", "ties"]


@pytest.mark.parametrize("fam", FAMILIES)
def test_build_matches_sweep(wrs, orc, fam):
    for n in SIZES:
        w = family(fam, n, 100 + n)
        if w.astype(np.float64).sum() == 0:
            continue
        say("build", fam, n)
        t, a, st, *_ = gpu_build(wrs, w)
        assert st == wrs.OK
        check_against_sweep(orc, w, t, a)


def test_build_first_config(wrs, orc):
    """n = 2^16 uniform weights, seed 1."""
    import workloads
    w = workloads.uniform(1 << 16, 1)
    say("build config n=2^16 uniform seed 1")
    t, a, st, *_ = gpu_build(wrs, w)
    assert st == wrs.OK
    check_against_sweep(orc, w, t, a)


@pytest.mark.parametrize("fam", ["uniform", "power1", "wide", "ties"])
def test_build_2pow21(wrs, orc, fam):
    """Many tiles and pack blocks (2^21 items: 2048 tiles, 256 pack blocks)."""
    w = family(fam, 1 << 21, 9)
    say("build", fam, 1 << 21)
    t, a, st, *_ = gpu_build(wrs, w)
    assert st == wrs.OK
    check_against_sweep(orc, w, t, a)


def test_total_weight_matches_exact(wrs, orc):
    import workloads
    w = workloads.power_law(300000, 1.0, 4)
    say("total weight")
    *_, ws = gpu_build(wrs, w)
    hi, lo = wrs.total_weight(ws)
    ohi, olo = orc.total_weight(w)
    assert hi == ohi and abs(lo - olo) <= abs(ohi) * 2.0 ** -100


def test_build_domain_errors(wrs):
    for bad in ([1.0, -1.0, 2.0], [1.0, float("nan")], [float("inf"), 1.0], [0.0, 0.0, 0.0]):
        say("domain", bad)
        *_, st, _, _, _ = gpu_build(wrs, np.array(bad, np.float32))
        assert st == wrs.EDOMAIN


def test_build_host_errors(wrs):
    import torch
    dev = torch.device("cuda:0")
    w = torch.ones(10, device=dev)
    table = wrs.new_table(10, dev)
    ws = wrs.new_workspace(wrs.OP_BUILD, 10, 0, dev)
    with pytest.raises(wrs.WrsError) as e:
        wrs.alias_build(w, 0, table, ws)
    assert e.value.code == wrs.EINVAL
    small = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(wrs.WrsError) as e:
        wrs.alias_build(w, 10, table, small)
    assert e.value.code == wrs.EINVAL


@pytest.mark.parametrize("fam", ["uniform", "power1"])
def test_build_full_size(wrs, orc, fam):
    """n = 2^28 (the large configuration, seed 2): every item's mass within 1e-6,
    and 2^16 sampled light buckets equal to n w_i / W correctly rounded."""
    import workloads
    n = 1 << 28
    w = workloads.uniform(n, 2) if fam == "uniform" else workloads.power_law(n, 1.0, 2)
    say("build full size", fam)
    t, a, st, table, wt, ws = gpu_build(wrs, w)
    del table, wt, ws
    assert st == wrs.OK
    assert np.all((t >= 0) & (t <= 1)) and np.all((a >= 0) & (a < n))
    mass, err = orc.reconstruct(w, t, a)
    del mass
    assert err.max() <= 1e-6, f"max relative mass error {err.max()} at {np.argmax(err)}"
    idx = np.random.default_rng(5).integers(0, n, 1 << 16)
    light, tl = orc.light_t_at(w, idx)
    il = idx[light]
    assert np.all(ulp_diff(t[il], tl[light]) <= 1)


def test_build_exact_instances_bit_identical(wrs, orc):
    """Integer weights in [0, 2^10] with n up to 2^16 (exact-arithmetic
    instances): every prefix sum is exact and every item size is an exact
    multiple of the key unit, so the merge is the exact sweep's.  On these
    fixed instances the whole table, thresholds included, is bit-identical to
    the oracle's (the general bar for thresholds is 1 ulp: a light's t passes
    through FP64 before its one FP32 rounding)."""
    rng = np.random.default_rng(31)
    for n in (1, 7, 1000, 1024, 1025, 4097, 65536):
        w = rng.integers(0, 1025, n).astype(np.float32)
        if w.sum() == 0:
            w[0] = 1.0
        say("exact instance", n)
        t, a, st, *_ = gpu_build(wrs, w)
        assert st == wrs.OK
        t_ref, a_ref = orc.sweep_build(w)
        assert np.array_equal(a, a_ref), n
        assert np.array_equal(t.view(np.uint32), t_ref.view(np.uint32)), n
