"""CPU oracle for weighted random sampling -- TEST INFRASTRUCTURE ONLY.

A plain sequential reference (FP64 Vose, exact sweeping construction, alias
queries, exponential-clock sampling without replacement) for the method of
Huebschle-Schneider & Sanders, "Parallel Weighted Random Sampling".  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import this
module.  It shares no code with the HIP library and never imports it.

The arithmetic lives in ``wrs_oracle.cpp`` (built by ``build.sh`` into
``liboracle.so``); this file only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, EDOMAIN, ENOMEM = 0, -1, -2, -3


class OracleError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} returned {code}")
        self.code = code


def build() -> None:
    """Compile the oracle library (g++)."""
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)


NATIVE_FLAGS = "-O3 -march=native"


def native_library(path):
    """Compile a copy of the oracle for the host it runs on (g++ with
    NATIVE_FLAGS, as the paper's experiments compile) into `path`, and load it
    with the same signatures.  For timing the oracle on the CPU."""
    subprocess.run(["sh", os.path.join(_HERE, "build.sh"), os.path.abspath(path), *NATIVE_FLAGS.split()],
                   check=True)
    return _bind(ctypes.CDLL(os.path.abspath(path)))


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _bind(lib):
    P = ctypes.c_void_p
    i64, u64, u32, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
    sig = {
        "orc_philox4x32_10": (None, [P, P, P]),
        "orc_total_weight": (ctypes.c_int, [P, i64, P, P]),
        "orc_vose_build": (ctypes.c_int, [P, i64, P, P]),
        "orc_sweep_build": (ctypes.c_int, [P, i64, P, P]),
        "orc_psaplus_build": (ctypes.c_int, [P, i64, i64, P, P]),
        "orc_psaplus_leftovers": (ctypes.c_int64, [P, i64, i64]),
        "orc_ratio_f32": (ctypes.c_float, [ctypes.c_float, u32, ctypes.c_float, u32]),
        "orc_light_t_at": (ctypes.c_int, [P, i64, P, i64, P, P]),
        "orc_alias_sample": (ctypes.c_int, [P, P, i64, u64, u32, u64, i64, P]),
        "orc_alias_sample_at": (ctypes.c_int, [P, P, i64, u64, u32, P, i64, P]),
        "orc_reconstruct": (ctypes.c_int, [P, P, P, i64, P, P]),
        "orc_wor_keys": (ctypes.c_int, [P, i64, u64, u32, P]),
        "orc_wor_keys_at": (ctypes.c_int, [P, i64, u64, u32, P, i64, P]),
        "orc_sample_wor": (ctypes.c_int, [P, i64, i64, u64, u32, P, P]),
        "orc_permutation": (ctypes.c_int, [P, i64, u64, u32, P]),
        "orc_twolevel_build": (ctypes.c_int, [P, i64, i64, P, P, P, P]),
        "orc_twolevel_sample": (ctypes.c_int, [P, P, P, P, i64, i64, u64, u32, u64, i64, P]),
        "orc_twolevel_sample_at": (ctypes.c_int, [P, P, P, P, i64, i64, u64, u32, P, i64, P]),
        "orc_os_log": (ctypes.c_double, [ctypes.c_double]),
        "orc_os_sqrt": (ctypes.c_double, [ctypes.c_double]),
        "orc_os_lfact": (ctypes.c_double, [ctypes.c_double]),
        "orc_os_binomial": (ctypes.c_int, [i64, ctypes.c_double, u64, u64, u32, P]),
        "orc_os_groups": (ctypes.c_int, [P, i64, P, P, P, P, P, P]),
        "orc_os_sample": (ctypes.c_int, [P, i64, i64, u64, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(w) -> np.ndarray:
    return np.ascontiguousarray(w, dtype=np.float32)


def _check(fn, rc):
    if rc != OK:
        raise OracleError(fn, rc)


def philox4x32_10(counter, key) -> np.ndarray:
    """One Philox-4x32-10 block: counter = 4 words, key = 2 words -> 4 words."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def total_weight(w):
    """Exact W as (hi, lo): hi = W rounded to FP64, lo = (W - hi) rounded."""
    w = _f32(w)
    hi, lo = ctypes.c_double(), ctypes.c_double()
    _check("orc_total_weight", _load().orc_total_weight(_ptr(w), w.size, ctypes.byref(hi), ctypes.byref(lo)))
    return hi.value, lo.value


def vose_build(w):
    """Algorithm 1 (Vose) in FP64 -> (t float32[n], alias int32[n])."""
    w = _f32(w)
    t = np.empty(w.size, np.float32)
    a = np.empty(w.size, np.int32)
    _check("orc_vose_build", _load().orc_vose_build(_ptr(w), w.size, _ptr(t), _ptr(a)))
    return t, a


def sweep_build(w):
    """Algorithm 2 (sweep) in exact arithmetic -> (t float32[n], alias int32[n])."""
    w = _f32(w)
    t = np.empty(w.size, np.float32)
    a = np.empty(w.size, np.int32)
    _check("orc_sweep_build", _load().orc_sweep_build(_ptr(w), w.size, _ptr(t), _ptr(a)))
    return t, a


def psaplus_build(w, block):
    """Section 4.2.1 (PSA+): the sweep inside consecutive blocks of `block`
    items until a block runs out of lights or heavies, then the sweep over all
    items left, in exact arithmetic -> (t float32[n], alias int32[n])."""
    w = _f32(w)
    t = np.empty(w.size, np.float32)
    a = np.empty(w.size, np.int32)
    _check("orc_psaplus_build", _load().orc_psaplus_build(_ptr(w), w.size, int(block), _ptr(t), _ptr(a)))
    return t, a


def psaplus_leftovers(w, block) -> int:
    """How many items the greedy blocks of psaplus_build leave over."""
    w = _f32(w)
    r = int(_load().orc_psaplus_leftovers(_ptr(w), w.size, int(block)))
    if r < 0:
        raise OracleError("orc_psaplus_leftovers", r)
    return r


def ratio_f32(wa, ma, wb, mb) -> np.float32:
    """Correctly rounded FP32 value of (ma*wa)/(mb*wb) for FP32 wa, wb."""
    return np.float32(_load().orc_ratio_f32(float(np.float32(wa)), int(ma), float(np.float32(wb)), int(mb)))


def light_t_at(w, idx):
    """For each index: (is the item light, correctly rounded t = n w_i / W)."""
    w = _f32(w)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    t = np.empty(idx.size, np.float32)
    light = np.empty(idx.size, np.int32)
    _check("orc_light_t_at", _load().orc_light_t_at(_ptr(w), w.size, _ptr(idx), idx.size, _ptr(t), _ptr(light)))
    return light.astype(bool), t


def alias_sample(t, alias, seed, stream_id, first_counter, k):
    t = _f32(t)
    a = np.ascontiguousarray(alias, dtype=np.int32)
    out = np.empty(k, np.int32)
    _check("orc_alias_sample", _load().orc_alias_sample(_ptr(t), _ptr(a), t.size, seed, stream_id,
                                                        first_counter, k, _ptr(out)))
    return out


def alias_sample_at(t, alias, seed, stream_id, counters):
    t = _f32(t)
    a = np.ascontiguousarray(alias, dtype=np.int32)
    c = np.ascontiguousarray(counters, dtype=np.uint64)
    out = np.empty(c.size, np.int32)
    _check("orc_alias_sample_at", _load().orc_alias_sample_at(_ptr(t), _ptr(a), t.size, seed, stream_id,
                                                              _ptr(c), c.size, _ptr(out)))
    return out


def reconstruct(w, t, alias):
    """Per-item mass (in buckets) implied by a table, and its relative error
    against n*w_i/W (for w_i == 0 the error entry is the mass itself)."""
    w = _f32(w)
    t = _f32(t)
    a = np.ascontiguousarray(alias, dtype=np.int32)
    mass = np.empty(w.size, np.float64)
    err = np.empty(w.size, np.float64)
    _check("orc_reconstruct", _load().orc_reconstruct(_ptr(w), _ptr(t), _ptr(a), w.size, _ptr(mass), _ptr(err)))
    return mass, err


def wor_keys(w, seed, stream_id):
    w = _f32(w)
    keys = np.empty(w.size, np.float64)
    _check("orc_wor_keys", _load().orc_wor_keys(_ptr(w), w.size, seed, stream_id, _ptr(keys)))
    return keys


def wor_keys_at(w, seed, stream_id, idx):
    w = _f32(w)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    keys = np.empty(idx.size, np.float64)
    _check("orc_wor_keys_at", _load().orc_wor_keys_at(_ptr(w), w.size, seed, stream_id, _ptr(idx),
                                                      idx.size, _ptr(keys)))
    return keys


def sample_wor(w, k, seed, stream_id):
    """Exponential-clock sample without replacement: (ascending indices, k-th key)."""
    w = _f32(w)
    out = np.empty(k, np.int32)
    kth = ctypes.c_double()
    _check("orc_sample_wor", _load().orc_sample_wor(_ptr(w), w.size, k, seed, stream_id, _ptr(out),
                                                    ctypes.byref(kth)))
    return out, kth.value


def permutation(w, seed, stream_id):
    """Problem WRP: every item, in ascending order of its exponential-clock key
    (ties by index; zero weights last, in index order)."""
    w = _f32(w)
    out = np.empty(w.size, np.int32)
    _check("orc_permutation", _load().orc_permutation(_ptr(w), w.size, seed, stream_id, _ptr(out)))
    return out


def twolevel_build(w, block):
    """Section 4.4, replicated top level: per-block alias tables (the sweep on
    each block of `block` items, global alias indices) and a top-level table
    over the block sums -> (t_top, a_top, t, alias)."""
    w = _f32(w)
    G = (w.size + block - 1) // block
    tt = np.empty(G, np.float32)
    at = np.empty(G, np.int32)
    t = np.empty(w.size, np.float32)
    a = np.empty(w.size, np.int32)
    _check("orc_twolevel_build", _load().orc_twolevel_build(_ptr(w), w.size, int(block), _ptr(tt), _ptr(at),
                                                            _ptr(t), _ptr(a)))
    return tt, at, t, a


def twolevel_sample(t_top, a_top, t, alias, block, seed, stream_id, first_counter, k):
    args = [np.ascontiguousarray(x, d) for x, d in ((t_top, np.float32), (a_top, np.int32), (t, np.float32),
                                                    (alias, np.int32))]
    out = np.empty(k, np.int32)
    _check("orc_twolevel_sample", _load().orc_twolevel_sample(*[_ptr(x) for x in args], args[2].size, int(block),
                                                              seed, stream_id, first_counter, k, _ptr(out)))
    return out


def twolevel_sample_at(t_top, a_top, t, alias, block, seed, stream_id, counters):
    args = [np.ascontiguousarray(x, d) for x, d in ((t_top, np.float32), (a_top, np.int32), (t, np.float32),
                                                    (alias, np.int32))]
    c = np.ascontiguousarray(counters, dtype=np.uint64)
    out = np.empty(c.size, np.int32)
    _check("orc_twolevel_sample_at", _load().orc_twolevel_sample_at(*[_ptr(x) for x in args], args[2].size,
                                                                    int(block), seed, stream_id, _ptr(c), c.size,
                                                                    _ptr(out)))
    return out


# --- output-sensitive sampling with replacement (Section 5) -------------------

def os_log(x):
    """ln x from IEEE basic operations (the binomial generator's logarithm)."""
    return _load().orc_os_log(float(x))


def os_sqrt(x):
    return _load().orc_os_sqrt(float(x))


def os_lfact(j):
    """ln(j!) (sum of logarithms below 10, Stirling's series above)."""
    return _load().orc_os_lfact(float(j))


def os_binomial(m, rho, seed, heap, tag):
    """Binomial(m, rho) drawn with the counter blocks (heap, tag, attempt)."""
    out = ctypes.c_int64()
    _check("orc_os_binomial", _load().orc_os_binomial(int(m), float(rho), seed, heap, tag, ctypes.byref(out)))
    return out.value


def os_groups(w):
    """Groups of the output-sensitive structure -> (order, exps, starts, counts):
    order[j] = item at position j (groups heaviest first, items by index)."""
    w = _f32(w)
    order = np.empty(w.size, np.int32)
    ge = np.empty(300, np.int32)
    gs = np.empty(300, np.int64)
    gc = np.empty(300, np.int64)
    u, npos = ctypes.c_int64(), ctypes.c_int64()
    _check("orc_os_groups", _load().orc_os_groups(_ptr(w), w.size, _ptr(order), _ptr(ge), _ptr(gs), _ptr(gc),
                                                  ctypes.byref(u), ctypes.byref(npos)))
    return order[: npos.value], ge[: u.value], gs[: u.value], gc[: u.value]


def os_sample(w, k, seed):
    """k draws with replacement, output-sensitively (Section 5) -> (items,
    counts): the distinct items drawn, ascending, and their multiplicities."""
    w = _f32(w)
    cap = max(1, min(int(k), w.size))
    items = np.empty(cap, np.int32)
    counts = np.empty(cap, np.int64)
    s = ctypes.c_int64()
    _check("orc_os_sample", _load().orc_os_sample(_ptr(w), w.size, int(k), seed, _ptr(items), _ptr(counts),
                                                  ctypes.byref(s)))
    return items[: s.value], counts[: s.value]
