"""Python binding of libwrs.so, the gfx950 weighted-random-sampling library.

Argument marshalling only: every step runs in the HIP kernels behind the C ABI
declared in include/wrs.h.  Device buffers are torch tensors (used for memory
and streams only); their data pointers and the current HIP stream are passed
through ctypes.  If the library is not built, every call raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwrs.so")

OK, EINVAL, EDOMAIN, ENOMEM, EDEVICE, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
OP_BUILD, OP_WOR, OP_BUILD_PLUS, OP_PERM, OP_TWOLEVEL, OP_OS = 1, 2, 3, 4, 5, 6
TWOLEVEL_BLOCK = 2048  # items per block (meta-item) of the 2-level tables
PSAPLUS_BLOCK = 2048  # items per greedy block of alias_build_plus
NOALLOC_SCRATCH_BYTES = 128 << 20  # the fixed workspace of alias_build_noalloc
FUSE_MAX_N = 8192  # largest batched table the fused small-table launch takes
SERVE_UNORDERED = (1 << 64) - 1  # serve submits: no ordering behind a caller's stream
SERVE_MAX_BATCH = 4096  # limits of ServeConfig.max_batch and ServeConfig.inflight
SERVE_MAX_INFLIGHT = 16
TUNE_BUILD, TUNE_SAMPLE = 1, 2

_lib = None


class WrsError(RuntimeError):
    def __init__(self, fn, code, msg=""):
        super().__init__(f"{fn} failed with {code}: {msg}")
        self.code = code


class Job(ctypes.Structure):
    _fields_ = [("d_w", ctypes.c_void_p), ("n", ctypes.c_int64), ("d_table", ctypes.c_void_p),
                ("k", ctypes.c_int64), ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32),
                ("d_out", ctypes.c_void_p)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_batch", ctypes.c_int32),
                ("one_at_a_time", ctypes.c_int32), ("inflight", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("host_stage_bytes", ctypes.c_size_t)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("builds", ctypes.c_uint64), ("samples", ctypes.c_uint64),
                ("items_built", ctypes.c_uint64), ("samples_drawn", ctypes.c_uint64),
                ("launches", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("bytes_in_use", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t),
                ("tables_resident", ctypes.c_uint64)]


EXPORTS = {
    "wrs_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64]),
    "wrs_alias_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p]),
    "wrs_alias_build_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "wrs_alias_build_plus": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_size_t, ctypes.c_void_p]),
    "wrs_permutation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "wrs_os_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "wrs_os_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "wrs_os_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_void_p]),
    "wrs_twolevel_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "wrs_twolevel_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                           ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "wrs_plus_leftovers": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "wrs_alias_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "wrs_sample_wor": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                      ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p]),
    "wrs_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    "wrs_total_weight": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "wrs_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Job), ctypes.c_int32]),
    "wrs_batch_build_sample": (ctypes.c_int, [ctypes.POINTER(Job), ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_size_t, ctypes.c_void_p]),
    "wrs_batch_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_int)]),
    "wrs_batch_graph_mode": (ctypes.c_int, [ctypes.c_int]),
    "wrs_batch_fuse_small": (ctypes.c_int, [ctypes.c_int32]),
    "wrs_tune_get": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]),
    "wrs_tune_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int32]),
    "wrs_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_int32)]),
    "wrs_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "wrs_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "wrs_serve_create": (ctypes.c_int, [ctypes.POINTER(ServeConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "wrs_serve_submit_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                              ctypes.POINTER(ctypes.c_uint64)]),
    "wrs_serve_submit_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                                               ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.POINTER(ctypes.c_uint64)]),
    "wrs_serve_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]),
    "wrs_serve_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]),
    "wrs_serve_request_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double)]),
    "wrs_serve_release_table": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "wrs_serve_read_table": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int64]),
    "wrs_serve_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServeStats)]),
    "wrs_serve_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "wrs_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libwrs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_1903_00227_amd/build.py (or __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    # Loading torch first makes the dynamic loader bind libwrs.so to that one
    # runtime; two HIP runtimes in one process do not share the device.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().wrs_last_error().decode()


def _check(fn, rc):
    if rc != OK:
        raise WrsError(fn, rc, last_error())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- allocation helpers (torch memory; the library never allocates for these) ----

def new_workspace(op: int, n: int, k: int = 0, device="cuda"):
    import torch
    nb = workspace_bytes(op, n, k)
    return torch.empty(max(nb, 256), dtype=torch.uint8, device=device)


def new_table(n: int, device="cuda"):
    """An (n, 2) int32 tensor holding n wrs_entry {float t; int32 alias}."""
    import torch
    return torch.empty((n, 2), dtype=torch.int32, device=device)


def table_t(table):
    return table[:, 0].view(table.dtype).contiguous().view(__import__("torch").float32)


# ---- the C ABI, same names ----

def workspace_bytes(op: int, n: int, k: int = 0) -> int:
    return int(lib().wrs_workspace_bytes(op, n, k))


def alias_build(w, n, table, ws, stream=None):
    _check("wrs_alias_build", lib().wrs_alias_build(_ptr(w), n, _ptr(table), _ptr(ws), ws.numel() if hasattr(ws, "numel") else ws_bytes_of(ws), _stream(stream)))


def alias_build_noalloc(w, n, table, status_out=None, stream=None):
    """Build with the library's fixed scratch array as workspace (allocates nothing)."""
    _check("wrs_alias_build_noalloc", lib().wrs_alias_build_noalloc(_ptr(w), n, _ptr(table), _ptr(status_out),
                                                                  _stream(stream)))


def alias_build_plus(w, n, table, ws, stream=None):
    """Greedy blocks, then the splitting construction on the items left
    (blocks the calling thread until the greedy stage has run)."""
    _check("wrs_alias_build_plus", lib().wrs_alias_build_plus(_ptr(w), n, _ptr(table), _ptr(ws), ws.numel() if hasattr(ws, "numel") else ws_bytes_of(ws), _stream(stream)))


def permutation(w, n, seed, stream_id, out, ws, stream=None):
    """Weighted random permutation of the n items into out (int32)."""
    _check("wrs_permutation", lib().wrs_permutation(_ptr(w), n, seed, stream_id, _ptr(out), _ptr(ws), ws.numel() if hasattr(ws, "numel") else ws_bytes_of(ws), _stream(stream)))


def new_os(n: int, device="cuda"):
    """Device memory for an output-sensitive sampling structure of n items."""
    import torch
    return torch.empty(max(lib().wrs_os_bytes(n), 256), dtype=torch.uint8, device=device)


def os_build(w, n, os_, ws, stream=None):
    """Output-sensitive sampling structure (Section 5) for the n weights."""
    _check("wrs_os_build", lib().wrs_os_build(_ptr(w), n, _ptr(os_), os_.numel(), _ptr(ws), ws.numel(),
                                              _stream(stream)))


def os_sample(os_, n, k, seed, items, counts, s, ws, stream=None):
    """k draws with replacement: distinct items into items, multiplicities into
    counts (min(k, n) int32 each, unordered), their number into s (int64[1])."""
    _check("wrs_os_sample", lib().wrs_os_sample(_ptr(os_), n, k, seed, _ptr(items), _ptr(counts), _ptr(s),
                                                _ptr(ws), ws.numel(), _stream(stream)))


def twolevel_build(w, n, table, top, ws, stream=None):
    """2-level alias table: block tables into table (n entries), top table over
    the blocks into top (ceil(n / 2048) entries)."""
    _check("wrs_twolevel_build", lib().wrs_twolevel_build(_ptr(w), n, _ptr(table), _ptr(top), _ptr(ws), ws.numel() if hasattr(ws, "numel") else ws_bytes_of(ws), _stream(stream)))


def twolevel_sample(top, table, n, seed, stream_id, first_counter, k, out, stream=None):
    _check("wrs_twolevel_sample", lib().wrs_twolevel_sample(_ptr(top), _ptr(table), n, seed, stream_id, first_counter, k, _ptr(out), _stream(stream)))


def plus_leftovers(ws, stream=None) -> int:
    """Items the greedy blocks of the last alias_build_plus on ws left over."""
    v = ctypes.c_int64()
    _check("wrs_plus_leftovers", lib().wrs_plus_leftovers(_ptr(ws), _stream(stream), ctypes.byref(v)))
    return v.value


def ws_bytes_of(ws):
    raise TypeError("pass the workspace as a torch tensor")


def alias_sample(table, n, seed, stream_id, first_counter, k, out, stream=None):
    _check("wrs_alias_sample", lib().wrs_alias_sample(_ptr(table), n, seed, stream_id, first_counter, k,
                                                      _ptr(out), _stream(stream)))


def sample_wor(w, n, k, seed, stream_id, out, ws, stream=None):
    _check("wrs_sample_wor", lib().wrs_sample_wor(_ptr(w), n, k, seed, stream_id, _ptr(out), _ptr(ws),
                                                  ws.numel(), _stream(stream)))


def status(ws, stream=None) -> int:
    s = ctypes.c_int()
    _check("wrs_status", lib().wrs_status(_ptr(ws), _stream(stream), ctypes.byref(s)))
    return s.value


def total_weight(ws, stream=None):
    hi, lo = ctypes.c_double(), ctypes.c_double()
    _check("wrs_total_weight", lib().wrs_total_weight(_ptr(ws), _stream(stream), ctypes.byref(hi), ctypes.byref(lo)))
    return hi.value, lo.value


def make_jobs(specs):
    """specs: iterable of dicts with tensors w, table, out (or None) and ints n, k, seed, stream_id."""
    specs = list(specs)
    arr = (Job * len(specs))()
    for i, s in enumerate(specs):
        arr[i] = Job(_ptr(s["w"]), s["n"], _ptr(s["table"]), s.get("k", 0), s.get("seed", 0),
                     s.get("stream_id", 0), _ptr(s.get("out")))
    return arr


def batch_workspace_bytes(jobs) -> int:
    return int(lib().wrs_batch_workspace_bytes(jobs, len(jobs)))


def batch_build_sample(jobs, ws, stream=None):
    _check("wrs_batch_build_sample", lib().wrs_batch_build_sample(jobs, len(jobs), _ptr(ws), ws.numel(),
                                                                  _stream(stream)))


def batch_status(ws, njobs, stream=None):
    arr = (ctypes.c_int * njobs)()
    _check("wrs_batch_status", lib().wrs_batch_status(_ptr(ws), njobs, _stream(stream), arr))
    return list(arr)


def batch_graph_mode(enable: bool):
    lib().wrs_batch_graph_mode(1 if enable else 0)


def batch_fuse_small(max_n: int):
    """Batched jobs with n <= max_n (0: none) go to the fused small-table launch."""
    _check("wrs_batch_fuse_small", lib().wrs_batch_fuse_small(max_n))


# ---- launch-parameter tuning (result-neutral) ----

def tune_get(op: int, size: int) -> int:
    v = ctypes.c_int32()
    _check("wrs_tune_get", lib().wrs_tune_get(op, size, ctypes.byref(v)))
    return v.value


def tune_set(op: int, size: int, value: int):
    _check("wrs_tune_set", lib().wrs_tune_set(op, size, value))


def autotune(op: int, n: int, k: int = 0, stream=None) -> int:
    v = ctypes.c_int32()
    _check("wrs_autotune", lib().wrs_autotune(op, n, k, _stream(stream), ctypes.byref(v)))
    return v.value


def tune_save(path: str):
    _check("wrs_tune_save", lib().wrs_tune_save(path.encode()))


def tune_load(path: str):
    _check("wrs_tune_load", lib().wrs_tune_load(path.encode()))
