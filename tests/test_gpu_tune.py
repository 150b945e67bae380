"""Launch-parameter tuning on the GPU: every value of the two tunable launch
parameters (tile events per merge block, draws per sampler thread) gives
bit-identical tables and samples, and wrs_autotune picks one of the candidates
and round-trips through the JSON cache."""
import json

import numpy as np
import pytest

from gpu_common import family, gpu_build, say

pytestmark = pytest.mark.gpu

BUILD_VALUES = [4, 8, 16, 32]
SAMPLE_VALUES = [1, 2, 4, 8]


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


@pytest.mark.parametrize("fam,n", [("uniform", 5000), ("power1", 1 << 21), ("sorted_power1", 300000),
                                   ("tiny_heavies", 70000)])
def test_pack_steps_do_not_change_the_table(wrs, orc, fam, n):
    w = family(fam, n, 31 + n)
    ref = None
    try:
        for ps in BUILD_VALUES:
            wrs.tune_set(wrs.TUNE_BUILD, n, ps)
            assert wrs.tune_get(wrs.TUNE_BUILD, n) == ps
            say("build", fam, n, "events per block", ps)
            t, a, st, *_ = gpu_build(wrs, w)
            assert st == wrs.OK
            if ref is None:
                ref = (t.copy(), a.copy())
                mass, err = orc.reconstruct(w, t, a)
                assert err[w > 0].max() <= 1e-6
            else:
                assert np.array_equal(t.view(np.int32), ref[0].view(np.int32)), ps
                assert np.array_equal(a, ref[1]), ps
    finally:
        wrs.tune_set(wrs.TUNE_BUILD, n, 0)


@pytest.mark.parametrize("n,k", [(1000, 100003), (65536, 1 << 20)])
def test_sample_unroll_does_not_change_draws(wrs, orc, n, k):
    import torch
    w = family("power1", n, 5)
    t, a, st, table, *_ = gpu_build(wrs, w)
    want = orc.alias_sample(t, a, 77, 3, 1 << 33, k)
    out = torch.empty(k, dtype=torch.int32, device=table.device)
    try:
        for u in SAMPLE_VALUES:
            wrs.tune_set(wrs.TUNE_SAMPLE, k, u)
            say("sample", n, k, "draws per thread", u)
            out.fill_(-1)
            wrs.alias_sample(table, n, 77, 3, 1 << 33, k, out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), want), u
    finally:
        wrs.tune_set(wrs.TUNE_SAMPLE, k, 0)


def test_bad_values_rejected(wrs):
    with pytest.raises(wrs.WrsError) as e:
        wrs.tune_set(wrs.TUNE_BUILD, 1000, 12)
    assert e.value.code == wrs.EINVAL
    with pytest.raises(wrs.WrsError) as e:
        wrs.tune_set(wrs.TUNE_SAMPLE, 1000, 16)
    assert e.value.code == wrs.EINVAL


def test_autotune_and_cache_roundtrip(wrs, tmp_path):
    n, k = 1 << 20, 1 << 22
    try:
        say("autotune build", n)
        b = wrs.autotune(wrs.TUNE_BUILD, n)
        say("autotune sample", n, k)
        s = wrs.autotune(wrs.TUNE_SAMPLE, n, k)
        assert b in BUILD_VALUES and s in SAMPLE_VALUES
        assert wrs.tune_get(wrs.TUNE_BUILD, n) == b
        assert wrs.tune_get(wrs.TUNE_SAMPLE, k) == s
        path = str(tmp_path / "tune.json")
        wrs.tune_save(path)
        doc = json.load(open(path))
        ops = {(e["op"], e["log2"]): e for e in doc["entries"]}
        assert ops[("build", 20)]["value"] == b and ops[("build", 20)]["us"] > 0
        assert ops[("sample", 22)]["value"] == s
        assert ops[("build", 20)]["arch"].startswith("gfx")
        other = [v for v in BUILD_VALUES if v != b][0]
        wrs.tune_set(wrs.TUNE_BUILD, n, other)
        assert wrs.tune_get(wrs.TUNE_BUILD, n) == other
        wrs.tune_load(path)
        assert wrs.tune_get(wrs.TUNE_BUILD, n) == b
    finally:
        wrs.tune_set(wrs.TUNE_BUILD, n, 0)
        wrs.tune_set(wrs.TUNE_SAMPLE, k, 0)


def test_batch_results_independent_of_tuning(wrs, orc):
    """The same batch under other launch parameters (a new recorded graph) draws the same samples."""
    import torch
    dev = torch.device("cuda:0")
    ns = [300, 5000, 70000]
    ws_ = [torch.from_numpy(family("uniform", n, n)).to(dev) for n in ns]
    tables = [wrs.new_table(n, dev) for n in ns]
    outs = [torch.empty(4 * n, dtype=torch.int32, device=dev) for n in ns]
    jobs = wrs.make_jobs([dict(w=w, n=n, table=tb, k=4 * n, seed=9, stream_id=j, out=o)
                          for j, (w, n, tb, o) in enumerate(zip(ws_, ns, tables, outs))])
    bws = torch.empty(wrs.batch_workspace_bytes(jobs), dtype=torch.uint8, device=dev)
    try:
        res = []
        for ps in (4, 32):
            for n in ns:
                wrs.tune_set(wrs.TUNE_BUILD, n, ps)
            for o in outs:
                o.fill_(-1)
            say("batch with events per block", ps)
            wrs.batch_build_sample(jobs, bws)
            assert wrs.batch_status(bws, len(ns)) == [wrs.OK] * len(ns)
            res.append([o.cpu().numpy().copy() for o in outs])
        for a_, b_ in zip(*res):
            assert np.array_equal(a_, b_)
    finally:
        for n in ns:
            wrs.tune_set(wrs.TUNE_BUILD, n, 0)
