"""Helpers shared by the GPU parity tests (test infrastructure)."""
import sys

import numpy as np

import workloads


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def cur_stream():
    """Handle of torch's current HIP stream (the stream the serve submits order against)."""
    import torch
    return torch.cuda.current_stream().cuda_stream


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
    if name == "ties":
        # weights 1, 2 and 3 with as many 1s as 3s: the mean is exactly 2, every
        # 2 sits on the light/heavy boundary, and the deficit and excess sums
        # are integers that tie over and over in the merge
        k = n // 3
        w = np.full(n, 2.0, np.float32)
        pos = rng.permutation(n)
        w[pos[:k]] = 1.0
        w[pos[k:2 * k]] = 3.0
        return w
    if name == "wide":
        # binary exponents uniform in [-60, 60] (ratios up to 2^121: sizes below
        # the quantization grid, wide tile sums), 5 % zeros
        w = np.ldexp(1.0 + rng.random(n), rng.integers(-60, 61, n)).astype(np.float32)
        w[rng.random(n) < 0.05] = 0.0
        return w
    if name == "tiny_heavies":
        # many heavy items barely above the mean, a few very light items
        w = np.full(n, 1.0, np.float32)
        w[rng.integers(0, n, max(1, n // 50))] = np.float32(1e-3)
        return w
    raise ValueError(name)


def t_tolerance(n, t_ref):
    """Threshold bar against the exact sweep: 1 ulp, plus for a heavy bucket
    (TILE/2 + 1) merge-key units of at most 2^(floor(log2 n) - 60) bucket each."""
    unit = 2.0 ** (int(n).bit_length() - 1 - 60)
    ulp = np.spacing(np.abs(t_ref).astype(np.float32)).astype(np.float64)
    return ulp + 513 * unit


def check_against_sweep(orc, w, t, a):
    """Aliases equal to the exact sequential sweep (Algorithm 2), thresholds
    within t_tolerance (lights within 1 ulp), every positive item's mass within
    1e-6 relative of n w_i / W, zero-weight items with mass 0."""
    t_ref, a_ref = orc.sweep_build(w)
    bad = np.nonzero(a != a_ref)[0]
    assert bad.size == 0, f"{bad.size} alias mismatches, first at {bad[:5]}: gpu {a[bad[:5]]} ref {a_ref[bad[:5]]}"
    dt = np.abs(t.astype(np.float64) - t_ref.astype(np.float64))
    tol = t_tolerance(w.size, t_ref)
    assert np.all(dt <= tol), f"threshold off by {dt.max()} at {np.argmax(dt - tol)}"
    light = w.astype(np.float64) * w.size <= w.astype(np.float64).sum() * (1 - 1e-12)
    assert ulp_diff(t[light], t_ref[light]).max(initial=0) <= 1
    check_masses(orc, w, t, a)


def check_masses(orc, w, t, a):
    """Every positive item's reconstructed mass within 1e-6 relative of
    n w_i / W, zero-weight items with mass 0, t in [0, 1], aliases in [0, n)."""
    assert np.all((t >= 0) & (t <= 1)) and np.all((a >= 0) & (a < w.size))
    mass, err = orc.reconstruct(w, t, a)
    pos = w > 0
    if pos.any():
        assert err[pos].max() <= 1e-6
    assert np.all(mass[~pos] == 0)


def split_table(tab):
    """(t, alias) arrays of a table read back as an (n, 2) int32 array."""
    tab = np.asarray(tab)
    return tab[:, 0].copy().view(np.float32), tab[:, 1].copy()
