"""CPU-only checks of the C ABI library: it loads, exports every function that
include/wrs.h declares, and rejects bad arguments on the host before any GPU work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "wrs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wrs_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    if not os.path.exists(w.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    w.lib()
    return w


def test_every_declared_symbol_is_exported(wrs):
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(wrs.lib(), name), name
        assert name in wrs.EXPORTS, f"binding lacks {name}"


def test_host_validation_without_gpu_work(wrs):
    L = wrs.lib()
    assert L.wrs_workspace_bytes(wrs.OP_BUILD, 0, 0) == 0
    assert L.wrs_workspace_bytes(wrs.OP_BUILD, 2 ** 31, 0) == 0
    assert L.wrs_workspace_bytes(wrs.OP_BUILD, 1 << 28, 0) > (1 << 28) // 1024 * 40
    assert L.wrs_workspace_bytes(7, 100, 0) == 0
    assert L.wrs_alias_build(None, 10, None, None, 0, None) == wrs.EINVAL
    assert "null" in wrs.last_error()
    assert L.wrs_alias_sample(None, 10, 0, 0, 0, 10, None, None) == wrs.EINVAL
    assert L.wrs_sample_wor(None, 10, 1, 0, 0, None, None, 0, None) == wrs.EINVAL
    # server configurations out of range are rejected before touching the device:
    # a budget below 1 MiB, batches or concurrent batches outside their limits
    srv = ctypes.c_void_p()
    for cfg in (wrs.ServeConfig(1024, 8, 0, 1), wrs.ServeConfig(1 << 30, 0, 0, 1),
                wrs.ServeConfig(1 << 30, wrs.SERVE_MAX_BATCH + 1, 0, 1), wrs.ServeConfig(1 << 30, 8, 0, 0),
                wrs.ServeConfig(1 << 30, 8, 0, wrs.SERVE_MAX_INFLIGHT + 1)):
        assert L.wrs_serve_create(ctypes.byref(cfg), ctypes.byref(srv)) == wrs.EINVAL


def test_workspace_depends_on_n_only(wrs):
    L = wrs.lib()
    a = L.wrs_workspace_bytes(wrs.OP_WOR, 1 << 20, 1)
    b = L.wrs_workspace_bytes(wrs.OP_WOR, 1 << 20, 1 << 19)
    assert a == b
    jobs = (wrs.Job * 3)()
    for i, n in enumerate((10, 5000, 1 << 20)):
        jobs[i] = wrs.Job(None, n, None, 4 * n, 0, i, None)
    total = L.wrs_batch_workspace_bytes(jobs, 3)
    assert total >= sum(L.wrs_workspace_bytes(wrs.OP_BUILD, n, 0) for n in (10, 5000, 1 << 20))


def test_build_plus_host_validation(wrs):
    L = wrs.lib()
    n = 10000
    plain = L.wrs_workspace_bytes(wrs.OP_BUILD, n, 0)
    plus = L.wrs_workspace_bytes(wrs.OP_BUILD_PLUS, n, 0)
    # the greedy stage's arrays come after the build workspace: staging and
    # list (index + weight each), partitioned indices, per-block counts
    assert plus >= plain + 5 * 4 * n
    assert L.wrs_workspace_bytes(wrs.OP_BUILD_PLUS, 0, 0) == 0
    assert L.wrs_workspace_bytes(wrs.OP_BUILD_PLUS, 2 ** 31, 0) == 0
    assert L.wrs_alias_build_plus(None, n, None, None, 0, None) == wrs.EINVAL
    assert "null" in wrs.last_error()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every check below fails on the host
    assert L.wrs_alias_build_plus(fake, 0, fake, fake, plus, None) == wrs.EINVAL
    assert L.wrs_alias_build_plus(fake, n, fake, fake, plus - 1, None) == wrs.EINVAL
    assert "workspace" in wrs.last_error()
    assert L.wrs_alias_build_plus(fake, n, fake, ctypes.c_void_p((1 << 20) + 8), plus, None) == wrs.EINVAL
    assert "aligned" in wrs.last_error()
    assert L.wrs_alias_build_plus(fake, n, ctypes.c_void_p((1 << 20) + 4), fake, plus, None) == wrs.EINVAL
    assert wrs.PSAPLUS_BLOCK == 2048


def test_permutation_host_validation(wrs):
    L = wrs.lib()
    n = 100000
    nb = L.wrs_workspace_bytes(wrs.OP_PERM, n, 0)
    assert nb >= 24 * n  # two key and two index buffers
    assert L.wrs_workspace_bytes(wrs.OP_PERM, 0, 0) == 0
    assert L.wrs_permutation(None, n, 0, 0, None, None, 0, None) == wrs.EINVAL
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every check below fails on the host
    assert L.wrs_permutation(fake, 0, 0, 0, fake, fake, nb, None) == wrs.EINVAL
    assert L.wrs_permutation(fake, n, 0, 0, fake, fake, nb - 1, None) == wrs.EINVAL
    assert "workspace" in wrs.last_error()
    assert L.wrs_permutation(fake, n, 0, 0, fake, ctypes.c_void_p((1 << 20) + 16), nb, None) == wrs.EINVAL
    assert L.wrs_permutation(fake, n, 0, 0, ctypes.c_void_p((1 << 20) + 2), fake, nb, None) == wrs.EINVAL


def test_twolevel_host_validation(wrs):
    L = wrs.lib()
    n = 1 << 20
    nb = L.wrs_workspace_bytes(wrs.OP_TWOLEVEL, n, 0)
    assert 0 < nb < n // 4 + (1 << 20)  # small: reduction partials, the top job, the meta-items
    assert L.wrs_twolevel_build(None, n, None, None, None, 0, None) == wrs.EINVAL
    fake = ctypes.c_void_p(1 << 20)
    assert L.wrs_twolevel_build(fake, n, fake, fake, fake, nb - 1, None) == wrs.EINVAL
    assert "workspace" in wrs.last_error()
    assert L.wrs_twolevel_build(fake, n, fake, ctypes.c_void_p((1 << 20) + 4), fake, nb, None) == wrs.EINVAL
    assert L.wrs_twolevel_sample(None, fake, n, 0, 0, 0, 10, fake, None) == wrs.EINVAL
    assert L.wrs_twolevel_sample(fake, fake, 0, 0, 0, 0, 10, fake, None) == wrs.EINVAL
    assert L.wrs_twolevel_sample(fake, fake, n, 0, 0, 0, -1, fake, None) == wrs.EINVAL
    assert wrs.TWOLEVEL_BLOCK == 2048


def test_output_sensitive_host_validation(wrs):
    L = wrs.lib()
    n, k = 100000, 1 << 20
    sb = L.wrs_os_bytes(n)
    assert 12 * n <= sb < 12 * n + (1 << 16)  # item order + prefix sums, small header and top tree
    assert L.wrs_os_bytes(0) == 0 and L.wrs_os_bytes(1 << 31) == 0
    wb0 = L.wrs_workspace_bytes(wrs.OP_OS, n, 0)
    wbk = L.wrs_workspace_bytes(wrs.OP_OS, n, k)
    assert wbk >= wb0 > 0 and wbk >= 2 * 24 * n  # two frontiers of min(k, n) nodes
    assert L.wrs_workspace_bytes(wrs.OP_OS, n, 1 << 31) == 0
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every check below fails on the host
    odd = ctypes.c_void_p((1 << 20) + 4)
    assert L.wrs_os_build(None, n, fake, sb, fake, wb0, None) == wrs.EINVAL
    assert L.wrs_os_build(fake, 0, fake, sb, fake, wb0, None) == wrs.EINVAL
    assert L.wrs_os_build(fake, n, fake, sb - 1, fake, wb0, None) == wrs.EINVAL
    assert "structure" in wrs.last_error()
    assert L.wrs_os_build(fake, n, fake, sb, fake, wb0 - 1, None) == wrs.EINVAL
    assert "workspace" in wrs.last_error()
    assert L.wrs_os_build(fake, n, odd, sb, fake, wb0, None) == wrs.EINVAL
    s = ctypes.c_void_p((1 << 20) + 8)
    assert L.wrs_os_sample(None, n, k, 1, fake, fake, s, fake, wbk, None) == wrs.EINVAL
    assert L.wrs_os_sample(fake, n, k, 1, None, fake, s, fake, wbk, None) == wrs.EINVAL
    assert L.wrs_os_sample(fake, n, -1, 1, fake, fake, s, fake, wbk, None) == wrs.EINVAL
    assert L.wrs_os_sample(fake, n, 1 << 31, 1, fake, fake, s, fake, wbk, None) == wrs.EINVAL
    assert L.wrs_os_sample(fake, n, k, 1, fake, fake, s, fake, wbk - 1, None) == wrs.EINVAL
    assert L.wrs_os_sample(fake, n, k, 1, fake, fake, odd, fake, wbk, None) == wrs.EINVAL
    assert L.wrs_os_sample(fake, n, k, 1, fake, fake, s, odd, wbk, None) == wrs.EINVAL


def test_noalloc_host_validation(wrs):
    L = wrs.lib()
    hdr = open(os.path.join(ROOT, "include", "wrs.h")).read()
    m = re.search(r"#define WRS_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", hdr)
    assert m and wrs.NOALLOC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every check below fails on the host
    n = 1 << 20
    assert L.wrs_alias_build_noalloc(None, n, fake, None, None) == wrs.EINVAL
    assert L.wrs_alias_build_noalloc(fake, n, None, None, None) == wrs.EINVAL
    assert L.wrs_alias_build_noalloc(fake, 0, fake, None, None) == wrs.EINVAL
    assert L.wrs_alias_build_noalloc(fake, n, ctypes.c_void_p((1 << 20) + 4), None, None) == wrs.EINVAL
    assert L.wrs_alias_build_noalloc(fake, n, fake, ctypes.c_void_p((1 << 20) + 2), None) == wrs.EINVAL
    # the largest n whose workspace fits the scratch array, and the next one
    lo, hi = 1, (1 << 31) - 1
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if L.wrs_workspace_bytes(wrs.OP_BUILD, mid, 0) <= wrs.NOALLOC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid - 1
    assert lo > 1 << 24
    assert L.wrs_alias_build_noalloc(fake, lo + 1, fake, None, None) == wrs.EINVAL
    assert "scratch" in wrs.last_error()
    assert L.wrs_alias_build_noalloc(fake, 1 << 30, fake, None, None) == wrs.EINVAL


def test_batch_fuse_small_host_validation(wrs):
    L = wrs.lib()
    hdr = open(os.path.join(ROOT, "include", "wrs.h")).read()
    m = re.search(r"#define WRS_FUSE_MAX_N (\d+)", hdr)
    assert m and wrs.FUSE_MAX_N == int(m.group(1))
    assert L.wrs_batch_fuse_small(-1) == wrs.EINVAL
    assert L.wrs_batch_fuse_small(wrs.FUSE_MAX_N + 1) == wrs.EINVAL
    assert "max_n" in wrs.last_error()
    assert L.wrs_batch_fuse_small(wrs.FUSE_MAX_N) == wrs.OK
    assert L.wrs_batch_fuse_small(0) == wrs.OK
