"""Batched and served operation: every job's or request's results must be
bit-identical to the single-call results for the same weights, seed and stream."""
import numpy as np
import pytest

import workloads
from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    w.lib()
    return w


def single(wrs, w, n, k, seed, sid):
    import torch
    table = wrs.new_table(n, w.device)
    ws = wrs.new_workspace(wrs.OP_BUILD, n, 0, w.device)
    wrs.alias_build(w, n, table, ws)
    assert wrs.status(ws) == wrs.OK
    out = torch.empty(max(k, 1), dtype=torch.int32, device=w.device)
    if k:
        wrs.alias_sample(table, n, seed, sid, 0, k, out)
    torch.cuda.synchronize()
    return table.cpu().numpy(), out[:k].cpu().numpy()


def make_batch(wrs, jobs):
    import torch
    specs = []
    for j in jobs:
        w = torch.from_numpy(workloads.job_weights(j)).to("cuda:0")
        specs.append(dict(w=w, n=j["n"], table=wrs.new_table(j["n"], "cuda:0"), k=j["k"], seed=4,
                          stream_id=j["stream_id"], out=torch.empty(max(j["k"], 1), dtype=torch.int32, device="cuda:0")))
    return specs


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_single_calls(wrs, graph):
    import torch
    jobs = workloads.batch_jobs(seed=4, count=300, lo_log2=0, hi_log2=17)
    specs = make_batch(wrs, jobs)
    arr = wrs.make_jobs(specs)
    ws = torch.empty(wrs.batch_workspace_bytes(arr), dtype=torch.uint8, device="cuda:0")
    wrs.batch_graph_mode(graph)
    say("batch", len(jobs), "graph" if graph else "stream")
    for rep in range(4):  # later calls replay the recorded graph, with eager work in between
        for s in specs:
            s["table"].fill_(-1)
            s["out"].fill_(-1)
        wrs.batch_build_sample(arr, ws)
        torch.cuda.synchronize()
        assert all(st == wrs.OK for st in wrs.batch_status(ws, len(jobs)))
        for i in range(0, len(jobs), 7):
            s = specs[i]
            tab, smp = single(wrs, s["w"], s["n"], s["k"], 4, s["stream_id"])
            assert np.array_equal(s["table"].cpu().numpy(), tab), (rep, i)
            assert np.array_equal(s["out"][:s["k"]].cpu().numpy(), smp), (rep, i)
    wrs.batch_graph_mode(True)


def test_batch_graphs_share_a_workspace(wrs):
    """Two different batches alternate on one workspace: replaying the first
    batch's recorded graph must use its own descriptors again."""
    import torch
    ja = workloads.batch_jobs(seed=11, count=40, lo_log2=4, hi_log2=15)
    jb = workloads.batch_jobs(seed=12, count=7, lo_log2=10, hi_log2=16)
    sa, sb = make_batch(wrs, ja), make_batch(wrs, jb)
    aa, ab = wrs.make_jobs(sa), wrs.make_jobs(sb)
    nb = max(wrs.batch_workspace_bytes(aa), wrs.batch_workspace_bytes(ab))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    wrs.batch_graph_mode(True)
    for step, (arr, specs) in enumerate([(aa, sa), (ab, sb), (aa, sa), (ab, sb), (aa, sa)]):
        say("shared workspace, call", step)
        for s in specs:
            s["table"].fill_(-1)
            s["out"].fill_(-1)
        wrs.batch_build_sample(arr, ws)
        torch.cuda.synchronize()
        assert all(st == wrs.OK for st in wrs.batch_status(ws, len(specs)))
        for i in range(0, len(specs), 3):
            s = specs[i]
            tab, smp = single(wrs, s["w"], s["n"], s["k"], 4, s["stream_id"])
            assert np.array_equal(s["table"].cpu().numpy(), tab), (step, i)
            assert np.array_equal(s["out"][:s["k"]].cpu().numpy(), smp), (step, i)


def test_batch_reports_bad_job(wrs):
    import torch
    jobs = workloads.batch_jobs(seed=6, count=5, lo_log2=3, hi_log2=10)
    specs = make_batch(wrs, jobs)
    specs[2]["w"][1] = float("nan")
    arr = wrs.make_jobs(specs)
    ws = torch.empty(wrs.batch_workspace_bytes(arr), dtype=torch.uint8, device="cuda:0")
    say("batch with a bad job")
    wrs.batch_build_sample(arr, ws)
    st = wrs.batch_status(ws, len(jobs))
    assert st[2] == wrs.EDOMAIN and all(st[i] == wrs.OK for i in (0, 1, 3, 4))


def run_server(wrs, reqs, weights, one_at_a_time, budget=8 << 30):
    """Submit (op, ...) requests, wait for all; return tables and outputs."""
    import ctypes
    import torch
    cfg = wrs.ServeConfig(budget, 64, 1 if one_at_a_time else 0, 2)
    srv = ctypes.c_void_p()
    assert wrs.lib().wrs_serve_create(ctypes.byref(cfg), ctypes.byref(srv)) == wrs.OK
    tid, rid = ctypes.c_uint64(), ctypes.c_uint64()
    table_ids, req_ids, outs = [], [], []
    for r in reqs:
        if r[0] == "build":
            w = weights[r[1]]
            assert wrs.lib().wrs_serve_submit_build(srv, w.data_ptr(), w.numel(), ctypes.byref(tid),
                                                    ctypes.byref(rid)) == wrs.OK
            table_ids.append(tid.value)
        else:
            _, ti, k, seed = r
            out = torch.full((k,), -1, dtype=torch.int32, device="cuda:0")
            assert wrs.lib().wrs_serve_submit_sample(srv, table_ids[ti], k, seed, out.data_ptr(),
                                                     ctypes.byref(rid)) == wrs.OK
            outs.append(out)
        req_ids.append(rid.value)
    st = ctypes.c_int()
    for q in req_ids:
        assert wrs.lib().wrs_serve_wait(srv, q, ctypes.byref(st)) == wrs.OK
        assert st.value == wrs.OK
    tables = []
    for i, tid_ in enumerate(table_ids):
        n = weights[i].numel()
        h = np.empty((n, 2), np.int32)
        assert wrs.lib().wrs_serve_read_table(srv, tid_, h.ctypes.data, n) == wrs.OK
        tables.append(h)
    stats = wrs.ServeStats()
    wrs.lib().wrs_serve_stats(srv, ctypes.byref(stats))
    wrs.lib().wrs_serve_destroy(srv)
    torch.cuda.synchronize()
    return tables, [o.cpu().numpy() for o in outs], stats


def test_serve_alone_vs_mix(wrs):
    """Each request's result is the same alone (single calls) and in the mix."""
    import torch
    rng = np.random.default_rng(5)
    sizes = [int(2 ** rng.uniform(10, 18)) for _ in range(12)]
    weights = [torch.from_numpy(workloads.uniform(n, 50 + i) if i % 2 else workloads.power_law(n, 1.0, 50 + i)).to("cuda:0")
               for i, n in enumerate(sizes)]
    reqs = []
    for i in range(len(sizes)):
        reqs.append(("build", i))
        for _ in range(3):
            reqs.append(("sample", int(rng.integers(0, i + 1)), int(2 ** rng.uniform(10, 16)), int(rng.integers(1 << 40))))
    say("serve mix")
    tabs_mix, outs_mix, stats = run_server(wrs, reqs, weights, one_at_a_time=False)
    tabs_one, outs_one, _ = run_server(wrs, reqs, weights, one_at_a_time=True)
    si = 0
    for r in reqs:
        if r[0] == "build":
            tab, _ = single(wrs, weights[r[1]], weights[r[1]].numel(), 0, 0, 0)
            assert np.array_equal(tabs_mix[r[1]], tab) and np.array_equal(tabs_one[r[1]], tab)
        else:
            _, ti, k, seed = r
            w = weights[ti]
            _, smp = single(wrs, w, w.numel(), k, seed, 0)
            assert np.array_equal(outs_mix[si], smp) and np.array_equal(outs_one[si], smp)
            si += 1
    assert stats.completed == len(reqs) and stats.failed == 0
    assert stats.bytes_peak <= 8 << 30
