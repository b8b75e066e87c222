"""Python binding of libmps, the gfx950 multiway-Powersort library.

Argument marshalling only: every step of the sort runs in the HIP kernels of
``_lib/libmps.so`` behind the C ABI declared in ``include/mps.h``.  PyTorch
supplies device memory (the workspace is a torch tensor) and the stream.
There is no CPU fallback: if the library is not built, or no GPU is present,
the calls raise.

    import torch, paper_2209_06909_amd as mps
    keys = torch.tensor([...], dtype=torch.int64, device="cuda")
    idx = torch.arange(keys.numel(), dtype=torch.int32, device="cuda")
    mps.sort(keys, idx)                 # stable, in place; idx becomes the permutation
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmps.so")

MPS_OK, MPS_PENDING = 0, 1
_STATUS = {-1: "MPS_E_INVALID", -2: "MPS_E_NOMEM", -3: "MPS_E_HIP", -4: "MPS_E_UNSUPPORTED",
           -5: "MPS_E_NOTFOUND", -6: "MPS_E_DEVICE"}
KEY_I32, KEY_I64, KEY_F32 = 0, 1, 2

EXPORTED = ["mps_workspace_bytes", "mps_sort", "mps_sort_i32", "mps_sort_i64", "mps_sort_f32",
            "mps_sort_ex", "mps_sort_noalloc", "mps_noalloc_scratch_bytes", "mps_sort_kv64",
            "mps_sort_batched", "mps_autotune", "mps_sort_status",
            "mps_free_workspaces", "mps_trace_fetch",
            "mps_last_level_stats", "mps_stream_copy", "mps_serve_create", "mps_serve_submit", "mps_serve_poll",
            "mps_serve_release", "mps_serve_stats", "mps_serve_destroy", "mps_serve_selftest",
            "mps_last_error"]


class MpsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


OPT_TIME_LEVELS = 1
OPT_GRAPH = 2
OPT_MERGE_DOWN = 4
OPT_TEST_DEVICE_ERROR = 8
# merge tile configurations: (outputs per tile, outputs per thread per LDS stage)
TILE_CONFIGS = [(1024, 4), (2048, 8), (2048, 4), (4096, 8), (4096, 4)]


class _Opts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("tile", ctypes.c_uint32), ("lane_slice", ctypes.c_uint32),
                ("min_run", ctypes.c_uint32), ("error_out", ctypes.c_void_p)]


def _opts(k, ws, *, time_levels=False, graph=False, tile=None, lane_slice=None,
          min_run=1, merge_down=False, error_out=None, test_device_error=False) -> _Opts:
    flags = ((OPT_TIME_LEVELS if time_levels else 0) | (OPT_GRAPH if graph else 0)
             | (OPT_MERGE_DOWN if merge_down else 0)
             | (OPT_TEST_DEVICE_ERROR if test_device_error else 0))
    return _Opts(k=k, flags=flags, workspace=ws.data_ptr(), workspace_bytes=ws.numel(),
                 tile=int(tile or 0), lane_slice=int(lane_slice or 0),
                 min_run=int(min_run or 1),
                 error_out=error_out.data_ptr() if error_out is not None else None)


class _Trace(ctypes.Structure):
    _fields_ = [("r", ctypes.c_uint64), ("n_nodes", ctypes.c_uint64),
                ("merge_cost", ctypes.c_uint64), ("n_levels", ctypes.c_uint32),
                ("k", ctypes.c_uint32), ("r_cap", ctypes.c_uint64),
                ("run_start", ctypes.c_void_p), ("run_desc", ctypes.c_void_p),
                ("power", ctypes.c_void_p), ("leaf_depth", ctypes.c_void_p),
                ("node_begin", ctypes.c_void_p), ("node_end", ctypes.c_void_p),
                ("node_first", ctypes.c_void_p), ("node_arity", ctypes.c_void_p),
                ("node_power", ctypes.c_void_p), ("node_depth", ctypes.c_void_p)]


class _ServeCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("n_streams", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("k", ctypes.c_uint32), ("tile", ctypes.c_uint32),
                ("lane_slice", ctypes.c_uint32), ("poll_us", ctypes.c_uint32),
                ("fail_every", ctypes.c_uint32)]


class _Request(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("payload", ctypes.c_void_p),
                ("keys_out", ctypes.c_void_p), ("payload_out", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("kt", ctypes.c_int), ("ready_event", ctypes.c_void_p)]


class _ReqInfo(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("batch", ctypes.c_uint64),
                ("batch_requests", ctypes.c_uint32), ("status", ctypes.c_int)]


class _ServeStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_uint64), ("arena_used", ctypes.c_uint64),
                ("busy_streams", ctypes.c_uint32)]


_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """Load libmps.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing; build it with "
                                  "`python -m paper_2209_06909_amd.build`")
            # torch ships its own HIP runtime; load it first so that libmps binds to
            # that same runtime (its libamdhip64 soname) instead of bringing in a second one.
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            l = ctypes.CDLL(LIB_PATH)
            P, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
            l.mps_workspace_bytes.argtypes = [u64, u64, i32, i32, u32]
            l.mps_workspace_bytes.restype = u64
            l.mps_sort.argtypes = [P, i32, P, u64, P]
            l.mps_sort.restype = i32
            for name in ("mps_sort_i32", "mps_sort_i64", "mps_sort_f32"):
                getattr(l, name).argtypes = [P, P, u64, P]
                getattr(l, name).restype = i32
            l.mps_sort_ex.argtypes = [P, i32, P, u64, ctypes.POINTER(_Opts), ctypes.POINTER(_Trace), P]
            l.mps_sort_ex.restype = i32
            l.mps_sort_noalloc.argtypes = [P, i32, P, u64, ctypes.POINTER(_Opts), P]
            l.mps_sort_noalloc.restype = i32
            l.mps_noalloc_scratch_bytes.argtypes = []
            l.mps_noalloc_scratch_bytes.restype = u64
            l.mps_sort_kv64.argtypes = [P, i32, P, u64, ctypes.POINTER(_Opts), ctypes.POINTER(_Trace), P]
            l.mps_sort_kv64.restype = i32
            l.mps_sort_batched.argtypes = [P, i32, P, P, P, u64, u64, ctypes.POINTER(_Opts),
                                           ctypes.POINTER(_Trace), P]
            l.mps_sort_batched.restype = i32
            l.mps_autotune.argtypes = [P, i32, P, P, u64, u64, u32, ctypes.POINTER(_Opts), P, P]
            l.mps_autotune.restype = i32
            l.mps_sort_status.argtypes = [P, P]
            l.mps_sort_status.restype = i32
            l.mps_free_workspaces.argtypes = []
            l.mps_free_workspaces.restype = i32
            l.mps_trace_fetch.argtypes = [P, ctypes.POINTER(_Trace)]
            l.mps_trace_fetch.restype = i32
            l.mps_last_level_stats.argtypes = [u32, P, P, P, P]
            l.mps_last_level_stats.restype = i32
            l.mps_stream_copy.argtypes = [P, P, u64, P]
            l.mps_stream_copy.restype = i32
            l.mps_serve_create.argtypes = [ctypes.POINTER(_ServeCfg), ctypes.POINTER(P)]
            l.mps_serve_create.restype = i32
            l.mps_serve_submit.argtypes = [P, ctypes.POINTER(_Request), ctypes.POINTER(u64)]
            l.mps_serve_submit.restype = i32
            l.mps_serve_poll.argtypes = [P, u64, ctypes.POINTER(_ReqInfo)]
            l.mps_serve_poll.restype = i32
            l.mps_serve_release.argtypes = [P, u64]
            l.mps_serve_release.restype = i32
            l.mps_serve_stats.argtypes = [P, ctypes.POINTER(_ServeStats)]
            l.mps_serve_stats.restype = i32
            l.mps_serve_destroy.argtypes = [P]
            l.mps_serve_destroy.restype = i32
            l.mps_serve_selftest.argtypes = []
            l.mps_serve_selftest.restype = i32
            l.mps_last_error.argtypes = []
            l.mps_last_error.restype = ctypes.c_char_p
            _lib = l
        return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise MpsError(rc, lib().mps_last_error().decode())
    return rc


def _torch():
    import torch
    return torch


def key_type_of(t) -> int:
    torch = _torch()
    kt = {torch.int32: KEY_I32, torch.int64: KEY_I64, torch.float32: KEY_F32}.get(t.dtype)
    if kt is None:
        raise TypeError(f"unsupported key dtype {t.dtype} (int32, int64, float32)")
    return kt


def workspace_bytes(n: int, m: int = 1, key_type: int = KEY_I32, has_payload: int = 1,
                    k: int = 4) -> int:
    return int(lib().mps_workspace_bytes(n, m, key_type, int(has_payload), k))


_ws = {}
_ws_lock = threading.Lock()


def _workspace(device, stream, nbytes: int):
    """A cached torch uint8 workspace of at least nbytes for sorts on `stream`.

    One buffer per (device, stream): sorts on one stream run one after another, so
    they may share it, while sorts on two streams never do.  The buffer is allocated
    with `stream` current, so torch's caching allocator ties it to that stream: when
    a larger one replaces it, its memory is handed out again only in that stream's
    order, after the sorts already enqueued there."""
    torch = _torch()
    key = (device.type, device.index, stream.cuda_stream)
    with _ws_lock:
        buf = _ws.get(key)
        if buf is None or buf.numel() < nbytes:
            # drop every reference to the old buffer first, so that its memory can be
            # reused for the larger one
            buf = None
            _ws.pop(key, None)
            with torch.cuda.stream(stream):
                buf = torch.empty(int(nbytes * 1.05) + 4096, dtype=torch.uint8, device=device)
            _ws[key] = buf
        return buf


def release_workspaces():
    """Drop the cached torch workspaces (they are reallocated on the next call) and
    free the library-managed ones (mps_free_workspaces)."""
    with _ws_lock:
        _ws.clear()
    if os.path.exists(LIB_PATH) and _lib is not None:
        _check(lib().mps_free_workspaces())


def _check_tensors(keys, payload, wide_ok=False):
    """wide_ok: an int64 payload (8-byte records) is accepted, for sort() only."""
    torch = _torch()
    if not keys.is_cuda:
        raise ValueError("keys must be a GPU tensor")
    if not keys.is_contiguous():
        raise ValueError("keys must be contiguous")
    if payload is not None:
        if payload.dtype == torch.int64 and not wide_ok:
            raise TypeError("an 8-byte payload is supported by sort() only")
        if payload.dtype not in (torch.int32, torch.uint32, torch.int64):
            raise TypeError("payload must be int32/uint32 (4 bytes per key) or int64 (8 bytes)")
        if payload.device != keys.device or not payload.is_contiguous():
            raise ValueError("payload must be contiguous and on the keys' device")
        if payload.numel() != keys.numel():
            raise ValueError("payload and keys differ in length")


@dataclass
class Trace:
    """Runs, powers and merge-tree nodes of one sort (host numpy arrays)."""
    r: int
    n_nodes: int
    merge_cost: int
    n_levels: int
    k: int
    run_start: np.ndarray | None = None    # uint64[r+1]
    run_desc: np.ndarray | None = None     # uint8[r]
    power: np.ndarray | None = None        # uint8[r-1]
    leaf_depth: np.ndarray | None = None   # uint8[r]
    node_begin: np.ndarray | None = None   # uint64[n_nodes], ordered by first boundary
    node_end: np.ndarray | None = None
    node_first: np.ndarray | None = None   # uint32
    node_arity: np.ndarray | None = None   # uint8
    node_power: np.ndarray | None = None   # uint8
    node_depth: np.ndarray | None = None   # uint8


def _fetch_trace(ws_ptr, t: _Trace, arrays: bool) -> Trace:
    tr = Trace(r=int(t.r), n_nodes=int(t.n_nodes), merge_cost=int(t.merge_cost),
               n_levels=int(t.n_levels), k=int(t.k))
    if not arrays:
        return tr
    r, nn = tr.r, tr.n_nodes
    cap = max(r + 1, nn, 1)
    bufs = dict(run_start=np.zeros(cap, np.uint64), run_desc=np.zeros(cap, np.uint8),
                power=np.zeros(cap, np.uint8), leaf_depth=np.zeros(cap, np.uint8),
                node_begin=np.zeros(cap, np.uint64), node_end=np.zeros(cap, np.uint64),
                node_first=np.zeros(cap, np.uint32), node_arity=np.zeros(cap, np.uint8),
                node_power=np.zeros(cap, np.uint8), node_depth=np.zeros(cap, np.uint8))
    t2 = _Trace()
    t2.r_cap = cap
    for name, a in bufs.items():
        setattr(t2, name, a.ctypes.data)
    _check(lib().mps_trace_fetch(ws_ptr, ctypes.byref(t2)))
    tr.run_start = bufs["run_start"][: r + 1]
    tr.run_desc = bufs["run_desc"][:r]
    tr.power = bufs["power"][: max(r - 1, 0)]
    tr.leaf_depth = bufs["leaf_depth"][:r]
    for name in ("node_begin", "node_end", "node_first", "node_arity", "node_power", "node_depth"):
        setattr(tr, name, bufs[name][:nn])
    return tr


def _stream_of(device, stream):
    torch = _torch()
    return stream if stream is not None else torch.cuda.current_stream(device)


def _stream_ptr(device, stream):
    return ctypes.c_void_p(_stream_of(device, stream).cuda_stream)


def status(ws_ptr, stream_ptr):
    """mps_sort_status: synchronise the stream and raise MpsError(MPS_E_DEVICE) if the
    last sort that used the workspace failed a device-side check."""
    _check(lib().mps_sort_status(ws_ptr, stream_ptr))


def check_last(device=None, stream=None):
    """After sorts run with check=False: synchronise `stream` (default: the current
    stream of `device`) and raise MpsError if the last sort() / sort_batched() on it
    failed a device-side check."""
    torch = _torch()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    st = _stream_of(dev, stream)
    with _ws_lock:
        buf = _ws.get((dev.type, dev.index, st.cuda_stream))
    if buf is None:
        raise MpsError(-5, "no sort has run on this stream")
    status(ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(st.cuda_stream))


def last_trace(device=None, stream=None, arrays: bool = True) -> Trace:
    """mps_trace_fetch: the trace of the last sort() / sort_batched() on `stream`
    (default: the current stream of `device`), also when it ran without trace=True;
    synchronises the device."""
    torch = _torch()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    st = _stream_of(dev, stream)
    with _ws_lock:
        buf = _ws.get((dev.type, dev.index, st.cuda_stream))
    if buf is None:
        raise MpsError(-5, "no sort has run on this stream")
    t = _Trace()
    _check(lib().mps_trace_fetch(ctypes.c_void_p(buf.data_ptr()), ctypes.byref(t)))
    return _fetch_trace(ctypes.c_void_p(buf.data_ptr()), t, arrays)


def sort(keys, payload=None, *, k: int = 4, trace: bool = False, trace_arrays: bool = True,
         stream=None, time_levels: bool = False, graph: bool = False, tile: int | None = None,
         lane_slice: int | None = None, min_run: int = 1, merge_down: bool = False,
         check: bool = True, error_out=None, test_device_error: bool = False):
    """Stable multiway Powersort of a 1-D GPU tensor, in place.

    keys: int32 / int64 / float32 (float32 by the IEEE-754 total order).
    payload: optional int32/uint32 tensor of the same length, permuted with the keys; an
        int64 payload (8-byte records such as pointers) goes through mps_sort_kv64.
    trace: if True, synchronise and return a Trace (runs, powers, nodes, merge cost).
    graph: capture the launch sequence in a HIP graph (replayed on identical calls).
    tile, lane_slice: merge tile configuration, one of TILE_CONFIGS (default 2048, 4).
    min_run: minimal run length (Appendix A.3; 1 = natural runs, at most 32).
    merge_down: Appendix A.3's final phase (every merge after the first on the right
        spine is k-way) instead of Algorithm 2's equal-power groups.
    check: synchronise the stream after the sort and raise MpsError (MPS_E_DEVICE) if
        a device-side check failed.  check=False keeps the call asynchronous; the
        device error word then reaches the caller through `error_out` (a GPU int32
        tensor of one element that the sort ORs its error bits into) or status().
    test_device_error: testing only -- the sort runs normally but reports a failed check.
    """
    _check_tensors(keys, payload, wide_ok=True)
    kt = key_type_of(keys)
    n = keys.numel()
    dev = keys.device
    wide = payload is not None and payload.element_size() == 8
    need = workspace_bytes(max(n, 2), 1, kt, 2 if wide else int(payload is not None), k)
    if need == 0:
        raise MpsError(-4, f"unsupported arity k={k}")
    st = _stream_of(dev, stream)
    ws = _workspace(dev, st, need)
    opts = _opts(k, ws, time_levels=time_levels, graph=graph, tile=tile, lane_slice=lane_slice,
                 min_run=min_run, merge_down=merge_down, error_out=error_out,
                 test_device_error=test_device_error)
    t = _Trace() if trace else None
    entry = lib().mps_sort_kv64 if wide else lib().mps_sort_ex
    sp = ctypes.c_void_p(st.cuda_stream)
    _check(entry(ctypes.c_void_p(keys.data_ptr()), kt,
                             ctypes.c_void_p(payload.data_ptr()) if payload is not None else None,
                             n, ctypes.byref(opts), ctypes.byref(t) if t is not None else None,
                             sp))
    if t is None:
        if check and n > 1:
            status(ctypes.c_void_p(ws.data_ptr()), sp)
        return None
    if n <= 1:
        tr = Trace(r=n, n_nodes=0, merge_cost=0, n_levels=0, k=k)
        if trace_arrays:
            tr.run_start = np.array([0, 1] if n else [0], np.uint64)
            tr.run_desc = np.zeros(n, np.uint8)
            tr.power = np.zeros(0, np.uint8)
            tr.leaf_depth = np.zeros(n, np.uint8)
            for name in ("node_begin", "node_end"):
                setattr(tr, name, np.zeros(0, np.uint64))
            tr.node_first = np.zeros(0, np.uint32)
            for name in ("node_arity", "node_power", "node_depth"):
                setattr(tr, name, np.zeros(0, np.uint8))
        return tr
    return _fetch_trace(ctypes.c_void_p(ws.data_ptr()), t, trace_arrays)


def noalloc_scratch_bytes() -> int:
    """Size of the fixed device scratch behind sort_noalloc (mps_noalloc_scratch_bytes)."""
    return int(lib().mps_noalloc_scratch_bytes())


def sort_noalloc(keys, payload=None, *, k: int = 4, stream=None, tile: int | None = None,
                 lane_slice: int | None = None, min_run: int = 1, merge_down: bool = False,
                 error_out=None):
    """sort() through mps_sort_noalloc: the workspace is the library's fixed device
    scratch, so the call allocates nothing (neither here nor in the library).  Only
    for arrays whose workspace fits that scratch (MpsError MPS_E_NOMEM otherwise).
    Asynchronous on `stream`; device-side check results go to `error_out` (a GPU
    int32 tensor of one element) if given.  Calls that can overlap on one device
    share the scratch and must not be issued concurrently."""
    _check_tensors(keys, payload)
    kt = key_type_of(keys)
    st = _stream_of(keys.device, stream)
    opts = _Opts(k=k, flags=(OPT_MERGE_DOWN if merge_down else 0), workspace=None,
                 workspace_bytes=0, tile=int(tile or 0), lane_slice=int(lane_slice or 0),
                 min_run=int(min_run or 1),
                 error_out=error_out.data_ptr() if error_out is not None else None)
    _check(lib().mps_sort_noalloc(ctypes.c_void_p(keys.data_ptr()), kt,
                                  ctypes.c_void_p(payload.data_ptr()) if payload is not None else None,
                                  keys.numel(), ctypes.byref(opts), ctypes.c_void_p(st.cuda_stream)))


def sort_batched(keys, payload, offsets, *, k: int = 4, trace: bool = False,
                 trace_arrays: bool = True, stream=None, host_offsets=None,
                 time_levels: bool = False, graph: bool = False, tile: int | None = None,
                 lane_slice: int | None = None, check: bool = True, error_out=None,
                 test_device_error: bool = False):
    """Sort m independent arrays packed back to back in `keys` (and `payload`).

    offsets: GPU int64/uint64 tensor of m+1 entries (offsets[0] = 0, offsets[m] = len(keys)).
    Every array is sorted exactly as sort() would sort it alone.  graph / tile /
    lane_slice / check / error_out as for sort().
    """
    torch = _torch()
    _check_tensors(keys, payload)
    if offsets.dtype not in (torch.int64, torch.uint64) or not offsets.is_contiguous():
        raise TypeError("offsets must be a contiguous int64/uint64 tensor")
    if offsets.device != keys.device:
        raise ValueError("offsets must be on the keys' device")
    kt = key_type_of(keys)
    m = offsets.numel() - 1
    n = keys.numel()
    dev = keys.device
    hoff = None
    if host_offsets is not None:
        hoff = np.ascontiguousarray(host_offsets, dtype=np.uint64)
    need = workspace_bytes(max(n, 2), max(m, 1), kt, payload is not None, k)
    if need == 0:
        raise MpsError(-4, f"unsupported arity k={k}")
    st = _stream_of(dev, stream)
    ws = _workspace(dev, st, need)
    opts = _opts(k, ws, time_levels=time_levels, graph=graph, tile=tile, lane_slice=lane_slice,
                 error_out=error_out, test_device_error=test_device_error)
    t = _Trace() if trace else None
    sp = ctypes.c_void_p(st.cuda_stream)
    _check(lib().mps_sort_batched(
        ctypes.c_void_p(keys.data_ptr()), kt,
        ctypes.c_void_p(payload.data_ptr()) if payload is not None else None,
        ctypes.c_void_p(offsets.data_ptr()),
        hoff.ctypes.data_as(ctypes.c_void_p) if hoff is not None else None,
        max(m, 0), n, ctypes.byref(opts), ctypes.byref(t) if t is not None else None,
        sp))
    if t is None:
        if check and m > 0 and n > 0:
            status(ctypes.c_void_p(ws.data_ptr()), sp)
        return None
    return _fetch_trace(ctypes.c_void_p(ws.data_ptr()), t, trace_arrays)


# candidate order of mps_autotune: arity outer, tile configuration inner
TUNE_CANDIDATES = [(k, t, e) for k in (4, 2, 8)
                   for (t, e) in ((2048, 8), (1024, 4), (2048, 4), (4096, 8), (4096, 4))]


def autotune(keys, payload, host_offsets, *, sample_keys: int = 1 << 27, graph: bool = True,
             stream=None, with_times: bool = False):
    """Pick arity and merge tile configuration for batched sorts of this shape by
    timing every candidate on a sample of the batch (see mps_autotune).  Returns
    dict(k=, tile=, lane_slice=) and, with with_times, the per-candidate times."""
    _check_tensors(keys, payload)
    kt = key_type_of(keys)
    hoff = np.ascontiguousarray(host_offsets, dtype=np.uint64)
    m = hoff.size - 1
    best = _Opts()
    times = np.zeros(len(TUNE_CANDIDATES), np.float32) if with_times else None
    _check(lib().mps_autotune(
        ctypes.c_void_p(keys.data_ptr()), kt,
        ctypes.c_void_p(payload.data_ptr()) if payload is not None else None,
        hoff.ctypes.data_as(ctypes.c_void_p), m, int(sample_keys), OPT_GRAPH if graph else 0,
        ctypes.byref(best), times.ctypes.data_as(ctypes.c_void_p) if times is not None else None,
        _stream_ptr(keys.device, stream)))
    out = dict(k=int(best.k), tile=int(best.tile), lane_slice=int(best.lane_slice))
    if with_times:
        out["candidates"] = [dict(k=k, tile=t, lane_slice=e, ms=float(x))
                             for (k, t, e), x in zip(TUNE_CANDIDATES, times)]
    return out


def stream_copy(dst, src, stream=None):
    """mps_stream_copy: copy the bytes of tensor src into tensor dst (same size, both
    16-byte aligned) with the library's streaming copy kernel, on `stream`."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise MpsError(-1, "size mismatch")
    st = _stream_of(src.device, stream)
    _check(lib().mps_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                 nbytes, ctypes.c_void_p(st.cuda_stream)))


def level_stats(cap: int = 64):
    """Per-level (merged elements, co-rank ms, merge ms) of the last sort run with
    time_levels=True on the current device; waits for it to finish."""
    nl = ctypes.c_uint32(0)
    elems = np.zeros(cap, np.uint64)
    cms = np.zeros(cap, np.float32)
    mms = np.zeros(cap, np.float32)
    _check(lib().mps_last_level_stats(cap, ctypes.byref(nl), elems.ctypes.data, cms.ctypes.data,
                                      mms.ctypes.data))
    n = min(int(nl.value), cap)
    return elems[:n].copy(), cms[:n].copy(), mms[:n].copy()


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching sort server (mps_serve_*): submit device tensors at any
    time, poll for completion.  Each result equals sort() of that request alone.

        with mps.Server(hbm_budget_bytes=8 << 30) as srv:
            rid = srv.submit(keys, payload, keys_out, payload_out)
            srv.wait(rid)
    """

    def __init__(self, hbm_budget_bytes: int, *, n_streams: int = 2, max_batch: int = 256,
                 k: int = 4, tile: int = 0, lane_slice: int = 0, poll_us: int = 0,
                 fail_every: int = 0):
        cfg = _ServeCfg(hbm_budget_bytes=int(hbm_budget_bytes), n_streams=n_streams,
                        max_batch=max_batch, k=k, tile=tile, lane_slice=lane_slice,
                        poll_us=poll_us, fail_every=fail_every)
        h = ctypes.c_void_p()
        _check(lib().mps_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._live = {}

    def submit(self, keys, payload=None, keys_out=None, payload_out=None) -> int:
        """Queue a sort of `keys` (and `payload`) into keys_out / payload_out (default:
        in place).  The tensors are kept alive until release(); the request waits for
        the work queued so far on the current stream."""
        torch = _torch()
        _check_tensors(keys, payload)
        keys_out = keys if keys_out is None else keys_out
        if payload is not None and payload_out is None:
            payload_out = payload
        if keys_out.dtype != keys.dtype or keys_out.numel() != keys.numel() or not keys_out.is_contiguous():
            raise ValueError("keys_out must match keys")
        if payload_out is not None and (payload is None or payload_out.numel() != keys.numel()):
            raise ValueError("payload_out needs a payload of the same length")
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(keys.device))
        req = _Request(keys=keys.data_ptr(), payload=payload.data_ptr() if payload is not None else None,
                       keys_out=keys_out.data_ptr(),
                       payload_out=payload_out.data_ptr() if payload_out is not None else None,
                       n=keys.numel(), kt=key_type_of(keys), ready_event=ev.cuda_event)
        rid = ctypes.c_uint64(0)
        _check(lib().mps_serve_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        self._live[rid.value] = (keys, payload, keys_out, payload_out, ev)
        return rid.value

    def poll(self, rid: int):
        """(status, info): status is MPS_PENDING (1), MPS_OK (0) or raises MpsError."""
        info = _ReqInfo()
        rc = lib().mps_serve_poll(self._h, rid, ctypes.byref(info))
        if rc < 0:
            raise MpsError(rc, lib().mps_last_error().decode())
        return rc, dict(t_submit_ns=info.t_submit_ns, t_admit_ns=info.t_admit_ns,
                        t_done_ns=info.t_done_ns, batch=info.batch,
                        batch_requests=info.batch_requests)

    def wait(self, rid: int, timeout: float | None = None, sleep: float = 50e-6):
        import time
        t0 = time.perf_counter()
        while True:
            rc, info = self.poll(rid)
            if rc == MPS_OK:
                return info
            if timeout is not None and time.perf_counter() - t0 > timeout:
                raise TimeoutError(f"request {rid} still pending after {timeout} s")
            time.sleep(sleep)

    def release(self, rid: int):
        _check(lib().mps_serve_release(self._h, rid))
        self._live.pop(rid, None)

    def stats(self) -> dict:
        st = _ServeStats()
        _check(lib().mps_serve_stats(self._h, ctypes.byref(st)))
        return dict(queued=st.queued, batches=st.batches, arena_bytes=st.arena_bytes,
                    arena_used=st.arena_used, busy_streams=st.busy_streams)

    def close(self):
        if self._h is not None:
            _check(lib().mps_serve_destroy(self._h))
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def serve_selftest() -> int:
    """Host-only self-test of the server's allocator and batching policy (no GPU)."""
    return int(lib().mps_serve_selftest())
