"""Helpers shared by the GPU parity tests (test infrastructure)."""
import sys

import numpy as np

import workloads


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    return torch.device("cuda:0")


def gpu_build(wrs, w_np, dev=None, plus=False):
    """Build on the GPU through the C ABI (plus: the greedy-block construction);
    returns (t, alias, status, table tensor, w tensor, workspace)."""
    import torch
    dev = dev or torch_dev()
    n = w_np.size
    w = torch.from_numpy(np.ascontiguousarray(w_np, np.float32)).to(dev)
    table = wrs.new_table(n, dev)
    ws = wrs.new_workspace(wrs.OP_BUILD_PLUS if plus else wrs.OP_BUILD, n, 0, dev)
    (wrs.alias_build_plus if plus else wrs.alias_build)(w, n, table, ws)
    st = wrs.status(ws)
    tab = table.cpu().numpy()
    t = tab[:, 0].copy().view(np.float32)
    a = tab[:, 1].copy()
    return t, a, st, table, w, ws


def ulp_diff(a, b):
    a = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b)


def family(name, n, seed):
    rng = np.random.default_rng(seed)
    if name == "uniform":
        return workloads.uniform(n, seed)
    if name == "power0.5":
        return workloads.power_law(n, 0.5, seed)
    if name == "power1":
        return workloads.power_law(n, 1.0, seed)
    if name == "power2":
        return workloads.power_law(n, 2.0, seed)
    if name == "ints":
        return rng.integers(0, 21, n).astype(np.float32)
    if name == "equal":
        return np.full(n, 0.75, np.float32)
    if name == "one":
        w = np.zeros(n, np.float32)
        w[rng.integers(0, n)] = 3.0
        return w
    if name == "dominant":
        w = rng.random(n).astype(np.float32)
        w[rng.integers(0, n)] = np.float32(1e7)
        return w
    if name == "sorted_power1":
        return (np.arange(1, n + 1, dtype=np.float64) ** -1.0).astype(np.float32)
    if name == "negzero":
        # zero weights written as -0.0 (accepted: -0 >= 0), the rest uniform
        w = workloads.uniform(n, seed)
        w[rng.random(n) < 0.1] = np.float32(-0.0)
        return w
    if name == "tiny_heavies":
        # many heavy items barely above the mean, a few very light items
        w = np.full(n, 1.0, np.float32)
        w[rng.integers(0, n, max(1, n // 50))] = np.float32(1e-3)
        return w
    raise ValueError(name)
