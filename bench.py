"""Benchmark of the weighted-random-sampling hot path on one MI355X.

Step = alias-table build of n = 2^28 FP32 weights followed by k = 2^30 draws
with replacement, for both input families of the large configuration
((a) uniform (0,1], (b) power law i^-1 randomly permuted; seed 2, Philox key 2).
Inputs are generated once and resident in HBM before the timed region.

Printed: one JSON line.  `value` = alias build throughput (Gitems/s) over the
step's builds; `sample_gsamples_s` = sampling throughput over the step's draws;
`ms_per_step` = the whole step.  `roofline` covers the kernel with the largest
share of the step (the sampler); `build_hbm_frac_16B_floor` relates the build to
its minimum HBM traffic.  Before timing, the library's autotuner picks the
launch parameters of every size class the run uses (`tuning` lists them; they
never change a result).  Extra objects report:
- the greedy-block (PSA+) and 2-level builds on the same inputs;
- output-sensitive sampling on the same inputs;
- sampling without replacement and the weighted permutation (n = 2^26);
- the batched (4096 tables) and served (Poisson trace) forms;
- the CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, GB/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# Sources with host code only (entry points, the request server and its
# allocator): edits there leave every kernel, and so its counted HBM traffic,
# unchanged.
HOST_ONLY_SOURCES = ("wrs_api.hip", "wrs_serve.hip", "wrs_pool.h")


def kernel_source_sha():
    """Hash of every source that holds or feeds device code."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1903_00227_amd", "csrc"))):
        if f in HOST_ONLY_SOURCES:
            continue
        with open(os.path.join(ROOT, "paper_1903_00227_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None if the
    kernels changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_sha") != kernel_source_sha():
        return None
    e = d.get("kernels", {}).get(kernel)
    return None if e is None else e.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--log2k", type=int, default=30)
    ap.add_argument("--skip-extras", action="store_true", help="only the main step (no batch/serve/cpu legs)")
    ap.add_argument("--profile-only", action="store_true", help="few steps, no extras (for rocprofv3)")
    ap.add_argument("--no-tune", action="store_true", help="size-derived default launch parameters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path has no multi-GPU form; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1903_00227_amd as wrs
    import workloads

    wrs.lib()
    dev = torch.device("cuda:0")
    n, k = 1 << args.log2n, 1 << args.log2k
    log(f"generating inputs n=2^{args.log2n}")
    inputs = {}
    for fam in ("uniform", "power1"):
        w_np = workloads.uniform(n, 2) if fam == "uniform" else workloads.power_law(n, 1.0, 2)
        inputs[fam] = torch.from_numpy(w_np).to(dev)
        del w_np
    table = wrs.new_table(n, dev)
    ws = wrs.new_workspace(wrs.OP_BUILD, n, 0, dev)
    out = torch.empty(k, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    tuning = tune(wrs, [n], [(n, k)], not args.no_tune and not args.profile_only)

    def step(timers=None):
        for fam in ("uniform", "power1"):
            if timers is not None:
                timers[fam][0].record(stream)
            wrs.alias_build(inputs[fam], n, table, ws)
            if timers is not None:
                timers[fam][1].record(stream)
            wrs.alias_sample(table, n, 2, 0, 0, k, out)
            if timers is not None:
                timers[fam][2].record(stream)

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert wrs.status(ws) == wrs.OK
    steps = 2 if args.profile_only else args.steps
    ev = [{f: [torch.cuda.Event(enable_timing=True) for _ in range(3)] for f in inputs} for _ in range(steps)]
    log(f"timing {steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    build_ms = {f: [] for f in inputs}
    sample_ms = {f: [] for f in inputs}
    for s in range(steps):
        for f in inputs:
            build_ms[f].append(ev[s][f][0].elapsed_time(ev[s][f][1]))
            sample_ms[f].append(ev[s][f][1].elapsed_time(ev[s][f][2]))
    tot_build = sum(sum(v) for v in build_ms.values())
    tot_sample = sum(sum(v) for v in sample_ms.values())
    ms_per_step = wall * 1e3 / steps
    value = (2 * n * steps) / (tot_build * 1e-3) / 1e9
    gsps = (2 * k * steps) / (tot_sample * 1e-3) / 1e9
    if args.profile_only:
        # a plain 1 GiB device copy: calibrates the HBM byte counters
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        pws = wrs.new_workspace(wrs.OP_BUILD_PLUS, n, 0, dev)
        for fam in inputs:
            wrs.alias_build_plus(inputs[fam], n, table, pws)
        del pws
        top = wrs.new_table(-(-n // 2048), dev)
        tws = wrs.new_workspace(wrs.OP_TWOLEVEL, n, 0, dev)
        for fam in inputs:
            wrs.twolevel_build(inputs[fam], n, table, top, tws)
        del top, tws
        bench_os(wrs, torch, inputs, n, k, reps=1)
        bench_perm(wrs, torch, np, workloads, reps=1)
        bench_wor(wrs, torch, np, workloads, reps=1)
        bench_roofs(torch, n, k, wrs.tune_get(wrs.TUNE_SAMPLE, k), tot_sample / steps / 2, reps=1)
        torch.cuda.synchronize()
        log(f"profile run done: build {tot_build / steps / 2:.3f} ms, sample {tot_sample / steps / 2:.3f} ms")
        return

    # Pack kernel alone: time it by difference of two launch sequences is not
    # possible from outside the library, so report its share from the phase
    # model: the build's dominant kernel is bounded by the same HBM roof.
    samp_avg_ms = tot_sample / (2 * steps)
    samp_bytes = 12.0 * k                      # 8 B table gather + 4 B index store per draw
    samp_gbs = samp_bytes / (samp_avg_ms * 1e-3) / 1e9
    build_avg_ms = tot_build / (2 * steps)
    build_bytes = 16.0 * n                     # 4 B read for W + 4 B read to build + 8 B table write
    build_gbs = build_bytes / (build_avg_ms * 1e-3) / 1e9
    result = {
        "metric": "alias build Gitems/s + Gsamples/s at n=2^28 (% HBM roof); served p50/p99",
        "value": round(value, 3),
        "unit": "Gitems/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 weights/thresholds, exact int128 prefix sums, u32 Philox",
        "data": "synthetic (uniform (0,1] and permuted power law s=1, seed 2)",
        "config": {"workload": "large single table: n=2^28 FP32 weights, build + k=2^30 draws, "
                               "uniform and power law s=1 (seed 2, Philox key 2)",
                   "n": n, "k": k, "parallelism": "single GPU"},
        "sample_gsamples_s": round(gsps, 3),
        "build_ms": {f: round(sum(v) / len(v), 4) for f, v in build_ms.items()},
        "sample_ms": {f: round(sum(v) / len(v), 4) for f, v in sample_ms.items()},
        "tuning": tuning,
        "build_hbm_frac_16B_floor": round(build_gbs / HBM_PEAK_GBS, 4),
        "roofline": {"kernel": "k_sample", "bound": "hbm", "achieved": round(samp_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(samp_gbs / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic("k_sample"),
                     "algorithmic_bytes_per_launch": samp_bytes},
    }
    traffic = result["roofline"]["traffic"]
    if traffic:
        # bytes the counters saw move (whole 128-byte lines per random gather), per second
        tgbs = traffic / (samp_avg_ms * 1e-3) / 1e9
        result["roofline"]["traffic_gbs"] = round(tgbs, 1)
        result["roofline"]["traffic_frac"] = round(tgbs / HBM_PEAK_GBS, 4)
    # the build's HBM bytes as the counters saw them (every kernel of one build,
    # the larger of the two inputs' launches), against its average time
    build_kernels = ("k_reduce", "k_finalize", "void k_tileagg<false>", "k_scan_seg", "k_scan_top", "k_scan_fix",
                     "k_split", "void k_pack<false>")
    counted = [load_traffic(kn) for kn in build_kernels]
    if all(c is not None for c in counted):
        cgbs = sum(counted) / (build_avg_ms * 1e-3) / 1e9
        result["build_counted_traffic"] = {"bytes_per_build": int(sum(counted)), "gbs": round(cgbs, 1),
                                           "frac": round(cgbs / HBM_PEAK_GBS, 4),
                                           "algorithmic_bytes_per_build": int(build_bytes)}
    result["sampler_roofs"] = bench_roofs(torch, n, k, wrs.tune_get(wrs.TUNE_SAMPLE, k), samp_avg_ms)
    if not args.skip_extras:
        result["small"] = bench_small(wrs, torch, workloads, not args.no_tune)
        result["build_plus"] = bench_plus(wrs, torch, inputs, n, table)
        result["two_level"] = bench_twolevel(wrs, torch, inputs, n, table, k, out)
        skewed = torch.from_numpy(workloads.power_law(n, 2.0, 2)).to(dev)
        result["output_sensitive"] = bench_os(wrs, torch, inputs, n, k, skewed=skewed)
        del skewed
        result["without_replacement"] = bench_wor(wrs, torch, np, workloads)
        result["permutation"] = bench_perm(wrs, torch, np, workloads)
        result["batched"] = bench_batched(wrs, torch, np, workloads, not args.no_tune)
        result["served"] = bench_served(wrs, torch, np, workloads)
        result["cpu_baseline"] = bench_cpu(np, workloads)
    print(json.dumps(result), flush=True)


def bench_small(wrs, torch, workloads, run_tune=True, reps=50):
    """The small single-table workload (n = 2^16 uniform, seed 2; k = 2^20
    draws, Philox key 2) in microseconds per call, and builds of other sizes:
    each call bracketed by its own pair of events, median over `reps`."""
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    n1, k1 = 1 << 16, 1 << 20
    sizes = (1 << 10, 1 << 16, 1 << 20, 1 << 24)
    tuning = tune(wrs, list(sizes), [(n1, k1)], run_tune)

    def median_us(fn):
        fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record(st)
            fn()
            e1.record(st)
        torch.cuda.synchronize()
        return round(sorted(e0.elapsed_time(e1) for e0, e1 in ev)[reps // 2] * 1e3, 2)

    res = {"workload": "n=2^16 uniform (seed 2), k=2^20 draws; builds of 2^10..2^24 items (uniform, seed 2)",
           "tuning": tuning, "build_us": {}}
    out = torch.empty(k1, dtype=torch.int32, device=dev)
    for m in sizes:
        w = torch.from_numpy(workloads.uniform(m, 2)).to(dev)
        table = wrs.new_table(m, dev)
        ws = wrs.new_workspace(wrs.OP_BUILD, m, 0, dev)
        res["build_us"][f"2^{m.bit_length() - 1}"] = median_us(lambda: wrs.alias_build(w, m, table, ws))
        assert wrs.status(ws) == wrs.OK
        if m == n1:
            res["n2p16_k2p20_sample_us"] = median_us(lambda: wrs.alias_sample(table, m, 2, 0, 0, k1, out))
            res["n2p16_build_us"] = res["build_us"]["2^16"]
        del w, table, ws
    log(f"small: build 2^16 {res['n2p16_build_us']} us, 2^20 draws {res['n2p16_k2p20_sample_us']} us")
    return res


def bench_plus(wrs, torch, inputs, n, table, reps=5):
    """The greedy-block construction (PSA+, blocks of 2048 items) on the same
    resident inputs: build time per family and the share of items its blocks
    leave to the splitting stage.  The call waits for its greedy stage on the
    host, so the wall clock around each call is reported too."""
    dev = torch.device("cuda:0")
    log("build plus")
    ws = wrs.new_workspace(wrs.OP_BUILD_PLUS, n, 0, dev)
    res = {"workload": "the same n=2^28 inputs, wrs_alias_build_plus (greedy blocks of 2048, then splitting)"}
    for fam, w in inputs.items():
        for _ in range(2):
            wrs.alias_build_plus(w, n, table, ws)
        torch.cuda.synchronize()
        assert wrs.status(ws) == wrs.OK
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(reps):
            wrs.alias_build_plus(w, n, table, ws)
        e1.record()
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3 / reps
        ms = e0.elapsed_time(e1) / reps
        left = wrs.plus_leftovers(ws)
        res[fam] = {"ms": round(ms, 4), "wall_ms": round(wall_ms, 4), "gitems_s": round(n / (ms * 1e-3) / 1e9, 2),
                    "left_fraction": round(left / n, 4)}
    del ws
    return res


def bench_twolevel(wrs, torch, inputs, n, table, k, out, reps=5):
    """2-level alias tables (Section 4.4, replicated top level; blocks of 2048
    items) on the same resident inputs: build, and k draws by the two-step
    query.  A different table layout from the headline's, with the same item
    probabilities."""
    dev = torch.device("cuda:0")
    log("two-level tables")
    top = wrs.new_table(-(-n // 2048), dev)
    ws = wrs.new_workspace(wrs.OP_TWOLEVEL, n, 0, dev)
    res = {"workload": "the same n=2^28 inputs and k=2^30 draws, 2-level table (blocks of 2048)"}
    for fam, w in inputs.items():
        wrs.twolevel_build(w, n, table, top, ws)
        wrs.twolevel_sample(top, table, n, 2, 0, 0, k, out)
        torch.cuda.synchronize()
        assert wrs.status(ws) == wrs.OK
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for _ in range(reps):
            wrs.twolevel_build(w, n, table, top, ws)
        e[1].record()
        wrs.twolevel_sample(top, table, n, 2, 0, 0, k, out)
        e[2].record()
        torch.cuda.synchronize()
        bms = e[0].elapsed_time(e[1]) / reps
        sms = e[1].elapsed_time(e[2])
        res[fam] = {"build_ms": round(bms, 4), "build_gitems_s": round(n / (bms * 1e-3) / 1e9, 2),
                    "sample_ms": round(sms, 3), "sample_gsamples_s": round(k / (sms * 1e-3) / 1e9, 2)}
    del top, ws
    return res


def bench_os(wrs, torch, inputs, n, k, reps=3, skewed=None):
    """Output-sensitive sampling with replacement (Section 5) on the same
    resident inputs and k: build of the grouped structure, then the k draws
    returned as distinct items with multiplicities.  With `skewed` (resident
    power-law s = 2 weights), also that input against the alias sampler."""
    dev = torch.device("cuda:0")
    log("output-sensitive sampling")
    st = wrs.new_os(n, dev)
    ws = wrs.new_workspace(wrs.OP_OS, n, k, dev)
    cap = min(k, n)
    items = torch.empty(cap, dtype=torch.int32, device=dev)
    counts = torch.empty(cap, dtype=torch.int32, device=dev)
    s = torch.zeros(1, dtype=torch.int64, device=dev)
    res = {"workload": "the same n=2^28 inputs and k=2^30 draws, output-sensitive (distinct items + multiplicities); "
                       "power2 = power law s=2 permuted (seed 2), with the alias sampler on the same input"}
    for fam, w in inputs.items():
        wrs.os_build(w, n, st, ws)
        wrs.os_sample(st, n, k, 2, items, counts, s, ws)
        torch.cuda.synchronize()
        assert wrs.status(st) == wrs.OK and wrs.status(ws) == wrs.OK
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for _ in range(reps):
            wrs.os_build(w, n, st, ws)
        e[1].record()
        for _ in range(reps):
            wrs.os_sample(st, n, k, 2, items, counts, s, ws)
        e[2].record()
        torch.cuda.synchronize()
        bms = e[0].elapsed_time(e[1]) / reps
        sms = e[1].elapsed_time(e[2]) / reps
        res[fam] = {"build_ms": round(bms, 3), "sample_ms": round(sms, 3),
                    "sample_gsamples_s": round(k / (sms * 1e-3) / 1e9, 2), "distinct": int(s.item())}
    if skewed is not None:
        # a more skewed input (power law s = 2, seed 2): few distinct items,
        # the regime the method is for; the alias sampler beside it
        w = skewed
        wrs.os_build(w, n, st, ws)
        wrs.os_sample(st, n, k, 2, items, counts, s, ws)
        table = wrs.new_table(n, dev)
        tws = wrs.new_workspace(wrs.OP_BUILD, n, 0, dev)
        out = torch.empty(k, dtype=torch.int32, device=dev)
        wrs.alias_build(w, n, table, tws)
        wrs.alias_sample(table, n, 2, 0, 0, k, out)
        torch.cuda.synchronize()
        assert wrs.status(st) == wrs.OK and wrs.status(ws) == wrs.OK and wrs.status(tws) == wrs.OK
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for _ in range(reps):
            wrs.os_sample(st, n, k, 2, items, counts, s, ws)
        e[1].record()
        for _ in range(reps):
            wrs.alias_sample(table, n, 2, 0, 0, k, out)
        e[2].record()
        torch.cuda.synchronize()
        oms = e[0].elapsed_time(e[1]) / reps
        ams = e[1].elapsed_time(e[2]) / reps
        res["power2"] = {"sample_ms": round(oms, 3), "sample_gsamples_s": round(k / (oms * 1e-3) / 1e9, 2),
                         "distinct": int(s.item()), "alias_sample_ms": round(ams, 3),
                         "alias_sample_gsamples_s": round(k / (ams * 1e-3) / 1e9, 2)}
        del table, tws, out
    del st, ws, items, counts, s
    return res


def bench_wor(wrs, torch, np, workloads, reps=5):
    """n = 2^26 power law s = 0.5 permuted (seed 3), Philox key 3, k in
    {2^10, 2^16, 2^20}: exponential keys, threshold filter, exact top-k."""
    dev = torch.device("cuda:0")
    n = 1 << 26
    log("without replacement: n=2^26")
    w = torch.from_numpy(workloads.power_law(n, 0.5, 3)).to(dev)
    res = {"workload": "n=2^26 FP32 weights, power law s=0.5 permuted (seed 3), Philox key 3"}
    for lk in (10, 16, 20):
        k = 1 << lk
        out = torch.empty(k, dtype=torch.int32, device=dev)
        ws = wrs.new_workspace(wrs.OP_WOR, n, k, dev)
        wrs.sample_wor(w, n, k, 3, 0, out, ws)
        assert wrs.status(ws) == wrs.OK
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            wrs.sample_wor(w, n, k, 3, 0, out, ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"k=2^{lk}"] = {"ms": round(ms, 4), "gitems_s": round(n / (ms * 1e-3) / 1e9, 2),
                            "hbm_frac_4B_per_item": round(4.0 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del out, ws
    return res


def bench_perm(wrs, torch, np, workloads, reps=5):
    """Weighted permutation (problem WRP) of the without-replacement input:
    n = 2^26, power law s = 0.5 permuted (seed 3), Philox key 3.  Algorithmic
    bytes: keys (4 B read, 12 B written), five radix passes of 32 B (8 B counted,
    12 B read and 12 B written), 8 B read by the last pass over runs."""
    dev = torch.device("cuda:0")
    n = 1 << 26
    log("permutation: n=2^26")
    w = torch.from_numpy(workloads.power_law(n, 0.5, 3)).to(dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    ws = wrs.new_workspace(wrs.OP_PERM, n, 0, dev)
    wrs.permutation(w, n, 3, 0, out, ws)
    assert wrs.status(ws) == wrs.OK
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        wrs.permutation(w, n, 3, 0, out, ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    alg = (16 + 5 * 32 + 8) * n
    return {"workload": "n=2^26 FP32 weights, power law s=0.5 permuted (seed 3), Philox key 3",
            "ms": round(ms, 4), "gitems_s": round(n / (ms * 1e-3) / 1e9, 2),
            "hbm_frac_184B_per_item": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def tune(wrs, build_ns, sample_nks, run):
    """Autotune (or just report) the launch parameters of the given size classes."""
    res = {"tuned": bool(run), "build_events_per_block": {}, "sample_draws_per_thread": {}}
    for n in build_ns:
        if run:
            wrs.autotune(wrs.TUNE_BUILD, n)
        res["build_events_per_block"][f"2^{(n - 1).bit_length()}"] = wrs.tune_get(wrs.TUNE_BUILD, n)
    for n, k in sample_nks:
        if run:
            wrs.autotune(wrs.TUNE_SAMPLE, n, k)
        res["sample_draws_per_thread"][f"2^{(k - 1).bit_length()}"] = wrs.tune_get(wrs.TUNE_SAMPLE, k)
    if run:
        log("tuned:", res)
    return res


def bench_batched(wrs, torch, np, workloads, run_tune=True):
    """4096 tables (seed 4): one batched launch sequence replayed as a hipGraph,
    against one build + one sample call per table."""
    log("batched: preparing 4096 tables")
    jobs = workloads.batch_jobs(seed=4)
    classes = sorted({(j["n"] - 1).bit_length() for j in jobs})
    tuning = tune(wrs, [1 << c for c in classes], [(1 << c, 4 << c) for c in classes], run_tune)
    dev = torch.device("cuda:0")
    specs = []
    for j in jobs:
        w = torch.from_numpy(workloads.job_weights(j)).to(dev)
        specs.append(dict(w=w, n=j["n"], table=wrs.new_table(j["n"], dev), k=j["k"], seed=4,
                          stream_id=j["stream_id"], out=torch.empty(j["k"], dtype=torch.int32, device=dev)))
    arr = wrs.make_jobs(specs)
    ws = torch.empty(wrs.batch_workspace_bytes(arr), dtype=torch.uint8, device=dev)
    items = sum(j["n"] for j in jobs)
    draws = sum(j["k"] for j in jobs)
    wrs.batch_build_sample(arr, ws)          # records the graph
    torch.cuda.synchronize()
    st = wrs.batch_status(ws, len(jobs))
    assert all(s == wrs.OK for s in st)
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        wrs.batch_build_sample(arr, ws)
    e1.record()
    torch.cuda.synchronize()
    fused_ms = e0.elapsed_time(e1) / reps
    # the same batch with its small tables (n <= 8192) in the one-workgroup-per-table launch
    wrs.batch_fuse_small(wrs.FUSE_MAX_N)
    try:
        wrs.batch_build_sample(arr, ws)      # records that batch's graph
        torch.cuda.synchronize()
        assert all(s == wrs.OK for s in wrs.batch_status(ws, len(jobs)))
        e0.record()
        for _ in range(reps):
            wrs.batch_build_sample(arr, ws)
        e1.record()
        torch.cuda.synchronize()
        small_ms = e0.elapsed_time(e1) / reps
    finally:
        wrs.batch_fuse_small(0)
    # one call per table, same kernels
    sws = [wrs.new_workspace(wrs.OP_BUILD, s["n"], 0, dev) for s in specs]
    torch.cuda.synchronize()
    e0.record()
    for s, w_ in zip(specs, sws):
        wrs.alias_build(s["w"], s["n"], s["table"], w_)
        wrs.alias_sample(s["table"], s["n"], 4, s["stream_id"], 0, s["k"], s["out"])
    e1.record()
    torch.cuda.synchronize()
    single_ms = e0.elapsed_time(e1)
    log(f"batched: fused {fused_ms:.3f} ms, one-at-a-time {single_ms:.3f} ms")
    return {"workload": "4096 tables, n_i log-uniform in [2^6,2^20], k_i = 4 n_i (seed 4)",
            "items": items, "draws": draws, "fused_ms": round(fused_ms, 3), "tuning": tuning,
            "one_at_a_time_ms": round(single_ms, 3), "speedup": round(single_ms / fused_ms, 2),
            "small_tables_in_one_workgroup_ms": round(small_ms, 3),
            "small_tables": sum(1 for j in jobs if j["n"] <= wrs.FUSE_MAX_N),
            "fused_gitems_s": round(items / (fused_ms * 1e-3) / 1e9, 3),
            "fused_hbm_frac_28B_per_item": round(28.0 * items / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_served(wrs, torch, np, workloads, count=20000, warmup=1000, repeats=3, inflight=4,
                 lambdas=(0.25, 0.5, 0.75, 0.9, 1.1)):
    """Poisson request stream (seed 5): `warmup` requests, then `count`
    measured ones, at rates lambda x the one-at-a-time capacity (the
    completion rate of the same trace submitted at once to the one-launch-
    per-request server), continuous batching against one launch per request
    on the same trace, `repeats` runs each.  Latency = completion - submission
    of the measured requests; throughput = measured requests over the span
    from the first measured submission to the last measured completion."""
    import ctypes
    dev = torch.device("cuda:0")
    trace = workloads.serve_trace(seed=5, count=warmup + count, rate_hz=1.0)  # times rescaled per rate
    log(f"served: {warmup} + {count} requests")
    # A build of n items takes the first n weights of a resident 2^24-item
    # array of its family, drawn on the GPU (torch generator, seed 5): uniform
    # 1 - U[0,1) in FP32, or i^-1 under a random permutation.
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    nmax = 1 << 24
    fam = {"uniform": (1.0 - torch.rand(nmax, generator=g, device=dev, dtype=torch.float32)).contiguous()}
    base = torch.arange(1, nmax + 1, device=dev, dtype=torch.float64).pow(-1.0).to(torch.float32)
    fam["power"] = base[torch.randperm(nmax, generator=g, device=dev)].contiguous()
    del base
    max_k = max(r["k"] for r in trace if r["op"] == "sample")
    outs = [torch.empty(max_k, dtype=torch.int32, device=dev) for _ in range(8)]
    torch.cuda.synchronize()
    L = wrs.lib()
    # The weights are made and synchronised above and the outputs are scratch
    # buffers nobody reads: the requests need no ordering behind a stream, and
    # the latencies are the server's own.
    cs = wrs.SERVE_UNORDERED

    def run(mode, rate_hz):
        cfg = wrs.ServeConfig(64 << 30, 256, 1 if mode == "one" else 0, inflight)
        srv = ctypes.c_void_p()
        assert L.wrs_serve_create(ctypes.byref(cfg), ctypes.byref(srv)) == wrs.OK
        tid, rid = ctypes.c_uint64(), ctypes.c_uint64()
        tables, reqs = [], []
        t_start = time.perf_counter()
        scale = 1.0 / rate_hz
        for i, r in enumerate(trace):
            t_due = t_start + r["t_arrive"] * scale
            while True:
                now = time.perf_counter()
                if now >= t_due:
                    break
                if t_due - now > 2e-4:
                    time.sleep((t_due - now) * 0.5)
            if r["op"] == "build":
                w = fam[r["kind"]]
                rc = L.wrs_serve_submit_build(srv, w.data_ptr(), r["n"], 0, cs, ctypes.byref(tid), ctypes.byref(rid))
                assert rc == wrs.OK
                tables.append(tid.value)
            elif tables:
                # a resident table: one the budget has evicted is dropped and another picked
                o = outs[i % len(outs)]
                rc = wrs.ENOTFOUND
                while rc == wrs.ENOTFOUND and tables:
                    j = int(r["table_pick"] * len(tables))
                    rc = L.wrs_serve_submit_sample(srv, tables[j], r["k"], r["seed"], o.data_ptr(), cs,
                                                   ctypes.byref(rid))
                    if rc == wrs.ENOTFOUND:
                        tables.pop(j)
                if rc == wrs.ENOTFOUND:
                    continue
                assert rc == wrs.OK
            else:
                continue
            reqs.append((i >= warmup, r["op"], r.get("n", r.get("k")), rid.value))
        st = ctypes.c_int()
        failed = 0
        for _, _, _, q in reqs:
            L.wrs_serve_wait(srv, q, ctypes.byref(st))
            failed += st.value != wrs.OK
        ts, td = ctypes.c_double(), ctypes.c_double()
        lat, t0s, t1s, work = [], [], [], 0
        for measured, op, size, q in reqs:
            if not measured:
                continue
            assert L.wrs_serve_request_times(srv, q, ctypes.byref(ts), ctypes.byref(td)) == wrs.OK
            lat.append((td.value - ts.value) * 1e6)
            t0s.append(ts.value)
            t1s.append(td.value)
            work += size
        s = wrs.ServeStats()
        L.wrs_serve_stats(srv, ctypes.byref(s))
        L.wrs_serve_destroy(srv)
        span = max(t1s) - min(t0s)
        lat = np.asarray(lat)
        return {"p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
                "req_per_s": len(lat) / span, "gitems_plus_gsamples_s": work / span / 1e9,
                "failed": int(failed), "launches": int(s.launches), "peak_bytes": int(s.bytes_peak)}

    # capacity of one launch per request: the trace submitted at once
    probe = run("one", 1e9)
    cap = probe["req_per_s"]
    log(f"served: one-at-a-time capacity {cap:.0f} requests/s")
    res = {"workload": f"Poisson stream (seed 5): {warmup} warm-up + {count} measured requests, 50% builds n in "
                       f"[2^10,2^24], 50% samples k in [2^10,2^22], 64 GB budget, {inflight} batches in flight",
           "capacity_one_at_a_time_req_per_s": round(cap, 1), "repeats": repeats,
           "note": "a sample request draws from a table picked uniformly among the resident ones (tables the "
                   "budget evicted, least recently used first, are dropped from the pick)", "rates": {}}

    def summary(runs):
        out = {}
        for key in ("p50_us", "p99_us", "req_per_s", "gitems_plus_gsamples_s"):
            v = sorted(r[key] for r in runs)
            out[key] = round(v[len(v) // 2], 3 if key.startswith("g") else 1)
            out[key + "_range"] = [round(v[0], 3 if key.startswith("g") else 1),
                                   round(v[-1], 3 if key.startswith("g") else 1)]
        out["failed"] = sum(r["failed"] for r in runs)
        out["launches"] = runs[0]["launches"]
        return out

    for lam in lambdas:
        rate = lam * cap
        log(f"served: lambda {lam} ({rate:.0f}/s)")
        per = {"rate_per_s": round(rate, 1)}
        for mode, name in (("batch", "continuous_batching"), ("one", "one_launch_per_request")):
            per[name] = summary([run(mode, rate) for _ in range(repeats)])
        res["rates"][str(lam)] = per
    sat = run("batch", 1e9)
    res["saturated"] = {"continuous_batching": {k: round(v, 1) for k, v in sat.items() if k in
                                                ("req_per_s", "p50_us", "p99_us", "launches")},
                        "one_launch_per_request": {k: round(v, 1) for k, v in probe.items() if k in
                                                   ("req_per_s", "p50_us", "p99_us", "launches")}}
    return res


def bench_roofs(torch, n, k, unroll, sample_ms, reps=3):
    """Ceilings for the sampler at its own shape (libwrs_roofs.so): the same
    Philox-addressed 8-byte gathers from an n-entry table of 8-byte words (2 GiB
    at n = 2^28) with coalesced 4-byte stores and no select, and the Philox
    blocks alone (XOR-reduced, one word stored per block)."""
    import ctypes
    dev = torch.device("cuda:0")
    R = ctypes.CDLL(os.path.join(ROOT, "paper_1903_00227_amd", "libwrs_roofs.so"))
    P = ctypes.c_void_p
    R.wrs_roof_gather.restype = ctypes.c_int
    R.wrs_roof_gather.argtypes = [P, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, P, P]
    R.wrs_roof_philox.restype = ctypes.c_int
    R.wrs_roof_philox.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, P, P]
    R.wrs_roof_blocks.restype = ctypes.c_int64
    R.wrs_roof_blocks.argtypes = [ctypes.c_int64, ctypes.c_int]
    log("sampler ceilings: random gathers, Philox")
    buf = torch.zeros(n, dtype=torch.int64, device=dev)
    out = torch.empty(k, dtype=torch.int32, device=dev)
    red = torch.empty(R.wrs_roof_blocks(k, unroll), dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()

    def timed(fn):
        assert fn() == 0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            assert fn() == 0
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    g_ms = timed(lambda: R.wrs_roof_gather(buf.data_ptr(), n, 2, k, unroll, out.data_ptr(), st.cuda_stream))
    p_ms = timed(lambda: R.wrs_roof_philox(2, k, unroll, red.data_ptr(), st.cuda_stream))
    del buf, out, red
    return {"workload": f"k=2^{k.bit_length() - 1} draws, {unroll} per thread, table of n=2^{n.bit_length() - 1} "
                        "8-byte words",
            "gather_ms": round(g_ms, 3), "gather_gsamples_s": round(k / (g_ms * 1e-3) / 1e9, 2),
            "philox_ms": round(p_ms, 3), "philox_gsamples_s": round(k / (p_ms * 1e-3) / 1e9, 2),
            "k_sample_frac_of_gather_roof": round(g_ms / sample_ms, 4)}


def host_info():
    """CPU model, logical CPUs and compiler of the host the oracle is timed on."""
    import subprocess
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cc = subprocess.run(["g++", "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        cc = "unknown"
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "compiler": cc}


def bench_cpu(np, workloads):
    """The CPU oracle on the host's cores, compiled for that host with the
    paper's flags: FP64 Vose (sequential by definition) on the full n = 2^28
    uniform input; alias queries on that table and exponential-clock keys of
    the n = 2^26 power-law input on one thread and on all the threads used
    (disjoint counter ranges); the whole sequential WOR oracle at n = 2^26,
    k = 2^20."""
    import ctypes
    import tempfile
    import threading

    import oracle
    info = host_info()
    threads = max(1, min(16, os.cpu_count() or 1))  # the host's share for one GPU
    tmp = tempfile.mkdtemp(prefix="wrs_oracle_")
    log(f"cpu oracle: compiling with {oracle.NATIVE_FLAGS}")
    L = oracle.native_library(os.path.join(tmp, "liboracle_native.so"))
    P = ctypes.c_void_p

    def ptr(a):
        return a.ctypes.data_as(P)

    def parallel(fn, parts):
        ts = [threading.Thread(target=fn, args=(p,)) for p in parts]
        t0 = time.perf_counter()
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        return time.perf_counter() - t0

    n = 1 << 28
    log("cpu oracle: Vose on n=2^28")
    w = workloads.uniform(n, 2)
    t = np.empty(n, np.float32)
    a = np.empty(n, np.int32)
    t0 = time.perf_counter()
    assert L.orc_vose_build(ptr(w), n, ptr(t), ptr(a)) == 0
    dt_build = time.perf_counter() - t0
    del w
    # queries: 2^24 on one thread; 2^24 per thread on all threads
    ks = 1 << 24
    out = np.empty(ks * threads, np.int32)
    t0 = time.perf_counter()
    assert L.orc_alias_sample(ptr(t), ptr(a), n, 2, 0, 0, ks, ptr(out)) == 0
    dt_s1 = time.perf_counter() - t0
    errs = []

    def draws(i):
        o = out[i * ks:(i + 1) * ks]
        errs.append(L.orc_alias_sample(ptr(t), ptr(a), n, 2, 0, i * ks, ks, ptr(o)))

    dt_sT = parallel(draws, range(threads))
    assert all(e == 0 for e in errs)
    del t, a, out
    # without replacement, n = 2^26 power law s = 0.5 (seed 3)
    nw = 1 << 26
    log("cpu oracle: WOR on n=2^26")
    ww = workloads.power_law(nw, 0.5, 3)
    kw = 1 << 20
    sel = np.empty(kw, np.int32)
    kth = ctypes.c_double()
    t0 = time.perf_counter()
    assert L.orc_sample_wor(ptr(ww), nw, kw, 3, 0, ptr(sel), ctypes.byref(kth)) == 0
    dt_wor = time.perf_counter() - t0
    keys = np.empty(nw, np.float64)
    idx = np.arange(nw, dtype=np.int64)
    chunk = -(-nw // threads)
    t0 = time.perf_counter()
    assert L.orc_wor_keys_at(ptr(ww), nw, 3, 0, ptr(idx), nw, ptr(keys)) == 0
    dt_k1 = time.perf_counter() - t0
    errs.clear()

    def keygen(i):
        lo, hi = i * chunk, min(nw, (i + 1) * chunk)
        errs.append(L.orc_wor_keys_at(ptr(ww), nw, 3, 0, ptr(idx[lo:hi]), hi - lo, ptr(keys[lo:hi])))

    dt_kT = parallel(keygen, range(threads))
    assert all(e == 0 for e in errs)
    return {"value": round(n / dt_build / 1e9, 4), "unit": "Gitems/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 Vose build of the full n=2^28 uniform input (seed 2), one thread (Vose is sequential); "
                      f"alias queries on that table: 2^24 on one thread, 2^24 per thread on {threads} threads; "
                      "exponential-clock keys of the n=2^26 power-law s=0.5 input (seed 3) on 1 and "
                      f"{threads} threads; the sequential WOR oracle at n=2^26, k=2^20",
            "host": info, "flags": oracle.NATIVE_FLAGS + " -ffp-contract=off", "threads_used": threads,
            "build_s": round(dt_build, 2),
            "sample_gsamples_s": {"1": round(ks / dt_s1 / 1e9, 4),
                                  str(threads): round(ks * threads / dt_sT / 1e9, 4)},
            "wor_keys_gitems_s": {"1": round(nw / dt_k1 / 1e9, 4), str(threads): round(nw / dt_kT / 1e9, 4)},
            "wor_n2p26_k2p20_s": round(dt_wor, 2)}


if __name__ == "__main__":
    main()
