"""The C-ABI library (no GPU needed): it loads, exports every function that
include/mps.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_2209_06909_amd as mps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mps_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = mps.lib()
    names = declared_functions()
    assert "mps_sort" in names and "mps_sort_batched" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(mps.EXPORTED)


def test_workspace_bytes_host_logic():
    lib = mps.lib()
    n = 1 << 20
    a = lib.mps_workspace_bytes(n, 1, mps.KEY_I32, 1, 4)
    b = lib.mps_workspace_bytes(n, 1, mps.KEY_I64, 1, 4)
    c = lib.mps_workspace_bytes(n, 1, mps.KEY_I32, 0, 4)
    d = lib.mps_workspace_bytes(n, 1, mps.KEY_I64, 2, 4)
    assert lib.mps_workspace_bytes(n, 1, mps.KEY_I32, 1, 3) == 0   # k must be 2, 4 or 8
    assert lib.mps_workspace_bytes(n, 1, 7, 1, 4) == 0             # unknown key type
    assert lib.mps_workspace_bytes(n, 2, mps.KEY_I64, 2, 4) == 0   # 8-byte payloads: single arrays
    # the ping-pong buffer alone is n*(key+payload) bytes
    assert a >= n * 8 and b >= n * 12 and c >= n * 4 and d >= n * 16
    # the tree's scratch shares the ping-pong buffer where it fits: an int64 key
    # with a u32 payload needs at most 32 bytes per key
    assert lib.mps_workspace_bytes(1 << 24, 1, mps.KEY_I64, 1, 4) <= 32 * (1 << 24)


def test_argument_errors_need_no_gpu():
    lib = mps.lib()
    assert lib.mps_sort(None, mps.KEY_I32, None, 10, None) == -1           # keys NULL, n > 0
    assert b"NULL" in lib.mps_last_error()
    assert lib.mps_sort(None, 9, None, 10, None) == -1                     # bad key type
    fake = ctypes.c_void_p(1 << 40)                                        # never dereferenced
    assert lib.mps_sort(fake, mps.KEY_I32, None, (1 << 31) + 1, None) == -4
    opts = mps._Opts(k=3)
    assert lib.mps_sort_ex(fake, mps.KEY_I32, None, 100, ctypes.byref(opts), None, None) == -4
    assert lib.mps_sort(fake, mps.KEY_I32, None, 1, None) == 0            # n <= 1 is a no-op
    assert lib.mps_sort(fake, mps.KEY_I32, None, 0, None) == 0
    # batched: bad host offsets are rejected before any launch
    off = (ctypes.c_uint64 * 3)(0, 5, 4)
    assert lib.mps_sort_batched(fake, mps.KEY_I32, None, fake, off, 2, 4, None, None, None) == -1
    off = (ctypes.c_uint64 * 3)(0, 3, 7)
    assert lib.mps_sort_batched(fake, mps.KEY_I32, None, fake, off, 2, 8, None, None, None) == -1
    off = (ctypes.c_uint64 * 2)(0, (1 << 31) + 5)
    assert lib.mps_sort_batched(fake, mps.KEY_I32, None, fake, off, 1, (1 << 31) + 5, None, None,
                                None) == -4


def test_stream_copy_argument_errors_need_no_gpu():
    lib = mps.lib()
    fake = ctypes.c_void_p(1 << 40)                                        # never dereferenced
    assert lib.mps_stream_copy(None, fake, 64, None) == -1
    assert lib.mps_stream_copy(ctypes.c_void_p((1 << 40) + 8), fake, 64, None) == -1   # misaligned
    assert b"aligned" in lib.mps_last_error()
    assert lib.mps_stream_copy(fake, fake, 0, None) == 0                   # nothing to copy


def test_min_run_argument_errors_need_no_gpu():
    """min_run above 32, or with several arrays, is rejected before the
    workspace or the GPU is touched; 0 and 1 both mean natural runs."""
    lib = mps.lib()
    fake = ctypes.c_void_p(1 << 40)                                        # never dereferenced
    opts = mps._Opts(k=4, min_run=33)
    assert lib.mps_sort_ex(fake, mps.KEY_I64, None, 1000, ctypes.byref(opts), None, None) == -4
    assert b"min_run" in lib.mps_last_error()
    opts = mps._Opts(k=4, min_run=24)
    off = (ctypes.c_uint64 * 3)(0, 500, 1000)
    assert lib.mps_sort_batched(fake, mps.KEY_I32, None, fake, off, 2, 1000, ctypes.byref(opts),
                                None, None) == -4
    assert b"single-array" in lib.mps_last_error()
    opts = mps._Opts(k=4, flags=mps.OPT_MERGE_DOWN)                        # merge-down: single arrays
    assert lib.mps_sort_batched(fake, mps.KEY_I32, None, fake, off, 2, 1000, ctypes.byref(opts),
                                None, None) == -4
    assert b"MERGE_DOWN" in lib.mps_last_error()
    opts = mps._Opts(k=4, min_run=24)                                      # n <= 1: a no-op
    assert lib.mps_sort_ex(fake, mps.KEY_I64, None, 1, ctypes.byref(opts), None, None) == 0
    # a single-array workspace has room for the natural runs and chunk maps: apart
    # when they do not fit in the ping-pong buffer (4-byte keys, no payload) ...
    assert (lib.mps_workspace_bytes(1 << 20, 1, mps.KEY_I32, 0, 4)
            > lib.mps_workspace_bytes(1 << 20, 2, mps.KEY_I32, 0, 4) + 8 * (1 << 19))
    # ... and inside it when they do (int64 keys with a payload)
    assert (lib.mps_workspace_bytes(1 << 20, 1, mps.KEY_I64, 1, 4)
            < lib.mps_workspace_bytes(1 << 20, 2, mps.KEY_I64, 1, 4) + 8 * (1 << 19))


def test_serve_host_selftest():
    """The request server's arena allocator and batch-formation policy (host code,
    no GPU): first-fit allocation, coalescing, accounting under random churn, and
    arrival-order batches split by key type, count and memory."""
    assert mps.serve_selftest() == 0


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asked for more it exits with a message before
    touching a device."""
    import subprocess
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_noalloc_argument_errors_need_no_gpu():
    """mps_sort_noalloc checks its arguments and the fixed scratch's limit on the
    host, before it looks up the scratch or enqueues anything."""
    lib = mps.lib()
    fake = ctypes.c_void_p(1 << 40)                                        # never dereferenced
    scratch = lib.mps_noalloc_scratch_bytes()
    assert scratch == 64 << 20
    assert lib.mps_sort_noalloc(None, mps.KEY_I32, None, 10, None, None) == -1
    assert lib.mps_sort_noalloc(fake, 9, None, 10, None, None) == -1
    assert lib.mps_sort_noalloc(fake, mps.KEY_I32, None, 1, None, None) == 0   # no-op
    assert lib.mps_sort_noalloc(fake, mps.KEY_I32, None, (1 << 31) + 1, None, None) == -4
    o = mps._Opts(k=4, workspace=1 << 40, workspace_bytes=1 << 30)
    assert lib.mps_sort_noalloc(fake, mps.KEY_I32, fake, 1000, ctypes.byref(o), None) == -1
    for flag in (mps.OPT_GRAPH, mps.OPT_TIME_LEVELS):
        o = mps._Opts(k=4, flags=flag)
        assert lib.mps_sort_noalloc(fake, mps.KEY_I32, fake, 1000, ctypes.byref(o), None) == -4
    o = mps._Opts(k=3)
    assert lib.mps_sort_noalloc(fake, mps.KEY_I32, fake, 1000, ctypes.byref(o), None) == -4
    # the largest fitting size and one past it, by the workspace formula
    n = 1
    while lib.mps_workspace_bytes(2 * n, 1, mps.KEY_I64, 1, 4) <= scratch:
        n *= 2
    assert lib.mps_sort_noalloc(fake, mps.KEY_I64, fake, 2 * n, None, None) == -2
    assert b"fixed scratch" in lib.mps_last_error()
