"""wrs_alias_build_noalloc (the build with the library's fixed scratch array as
workspace) against wrs_alias_build, through the C ABI: two calls in a row, the
second with a smaller input, each giving wrs_alias_build's table bit for bit
and its status, and that table equal to the exact sweep (Algorithm 2) within
the bars of the build tests; an out-of-domain weight reported as WRS_EDOMAIN
through the status output, after which the array serves a good build again."""
import ctypes

import numpy as np
import pytest

from gpu_common import check_against_sweep, cur_stream, family, say, split_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


def build_both(wrs, w_np):
    """(no-alloc table, its status, wrs_alias_build's table, its status)."""
    import torch
    dev = torch.device("cuda:0")
    n = w_np.size
    w = torch.from_numpy(w_np).to(dev)
    got = torch.full((n, 2), -7, dtype=torch.int32, device=dev)
    status = torch.full((1,), 12345, dtype=torch.int32, device=dev)
    L = wrs.lib()
    assert L.wrs_alias_build_noalloc(ctypes.c_void_p(w.data_ptr()), n, ctypes.c_void_p(got.data_ptr()),
                                     ctypes.c_void_p(status.data_ptr()), ctypes.c_void_p(cur_stream())) == wrs.OK
    ref = wrs.new_table(n, dev)
    ws = wrs.new_workspace(wrs.OP_BUILD, n, 0, dev)
    assert L.wrs_alias_build(ctypes.c_void_p(w.data_ptr()), n, ctypes.c_void_p(ref.data_ptr()),
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(cur_stream())) == wrs.OK
    torch.cuda.synchronize()
    return got.cpu().numpy(), int(status.item()), ref.cpu().numpy(), wrs.status(ws)


def test_noalloc_two_calls_match_build(wrs, orc):
    for n, fam in (((5 << 20) + 77, "power1"), (70001, "uniform")):
        say("no-alloc build", fam, n)
        w_np = family(fam, n, 11 + n)
        got, st, ref, st_ref = build_both(wrs, w_np)
        assert st == st_ref == wrs.OK
        assert np.array_equal(got, ref)
        t, a = split_table(got)
        check_against_sweep(orc, w_np, t, a)


def test_noalloc_status_out(wrs):
    n = 5000
    w_np = family("uniform", n, 3)
    w_np[17] = np.float32("nan")
    say("no-alloc build with a NaN weight", n)
    _, st, _, st_ref = build_both(wrs, w_np)
    assert st == st_ref == wrs.EDOMAIN
    w_np = family("dominant", 3001, 4)
    say("no-alloc build after it", w_np.size)
    got, st, ref, st_ref = build_both(wrs, w_np)
    assert st == st_ref == wrs.OK and np.array_equal(got, ref)


def test_noalloc_limits(wrs):
    import torch
    dev = torch.device("cuda:0")
    L = wrs.lib()
    w = torch.ones(16, device=dev)
    table = wrs.new_table(16, dev)
    n = 1 << 25  # workspace above the scratch array: refused before any launch
    assert L.wrs_workspace_bytes(wrs.OP_BUILD, n, 0) > wrs.NOALLOC_SCRATCH_BYTES
    assert L.wrs_alias_build_noalloc(ctypes.c_void_p(w.data_ptr()), n, ctypes.c_void_p(table.data_ptr()), None,
                                     ctypes.c_void_p(cur_stream())) == wrs.EINVAL
    assert "scratch" in wrs.last_error()
