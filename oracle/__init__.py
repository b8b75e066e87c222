"""Reference CPU implementation of k-way Powersort (TEST INFRASTRUCTURE ONLY).

This package is the checker the GPU library is compared against.  Only the
test suite, the package smoke check at the repository root and the CPU-baseline leg of
``bench.py`` may import it; the product path never does, and it shares no
code with the GPU library.  The arithmetic lives in ``oracle.c`` (plain C,
single-threaded); this module only marshals numpy arrays through ctypes.

Each function follows the paper (arXiv 2209.06909):
  runs()            Section 2, run definition (greedy left-to-right scan);
                    with min_run > 1, Appendix A.3's extension of short runs
  power()/powers()  Definition 3.1, run-boundary power (exact integers)
  sort()            Algorithm 2 (KwayPowerSort_k) with stable k-way merges;
                    merge_down: the final phase of Appendix A.3
  kway_tree()       Algorithm 1 (KwayTree_k), independent cross-check
  tree_from_runs()  Algorithm 2's tree without moving elements
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_REF_PATH = os.path.join(_HERE, "libstableref.so")
_REF_SRC = os.path.join(_HERE, "stable_ref.cpp")

KEY_TYPES = {np.dtype(np.int32): 0, np.dtype(np.int64): 1, np.dtype(np.float32): 2}

NODE_DTYPE = np.dtype({
    "names": ["begin", "end", "first_boundary", "arity", "power", "depth", "parent"],
    "formats": ["<u8", "<u8", "<u8", "<u4", "<u4", "<u4", "<i8"],
    "offsets": [0, 8, 16, 24, 28, 32, 40],
    "itemsize": 48,
})


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no tuning), and beside it the
    std::stable_sort reference (libstableref.so, g++ -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-o", tmp, _SRC], cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    if force or not os.path.exists(_REF_PATH):
        tmp = _REF_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                               "-o", tmp, _REF_SRC], cwd=_HERE)
        os.replace(tmp, _REF_PATH)
    return _LIB_PATH


_ref = None


def stable_sort_ref(keys: np.ndarray, payload: np.ndarray | None = None):
    """std::stable_sort of (key, payload) records on one thread (the library
    reference); returns (keys, payload) sorted.  Float32 keys follow the
    IEEE-754 total order, like the oracle."""
    global _ref
    if _ref is None:
        build()
        _ref = ctypes.CDLL(_REF_PATH)
        _ref.ref_stable_sort.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        _ref.ref_stable_sort.restype = ctypes.c_int
    keys = np.ascontiguousarray(keys)
    kt = KEY_TYPES[keys.dtype]
    ko = np.empty_like(keys)
    po = np.empty(keys.size, np.uint32)
    pin = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32)
    rc = _ref.ref_stable_sort(keys.ctypes.data, None if pin is None else pin.ctypes.data,
                              keys.size, kt, ko.ctypes.data, po.ctypes.data)
    if rc != 0:
        raise ValueError("unsupported key type")
    return ko, po


class _Node(ctypes.Structure):
    _fields_ = [("begin", ctypes.c_uint64), ("end", ctypes.c_uint64),
                ("first_boundary", ctypes.c_uint64), ("arity", ctypes.c_uint32),
                ("power", ctypes.c_uint32), ("depth", ctypes.c_uint32),
                ("parent", ctypes.c_int64)]


class _Trace(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("r", ctypes.c_uint64), ("k", ctypes.c_uint32),
                ("run_start", ctypes.POINTER(ctypes.c_uint64)),
                ("run_desc", ctypes.POINTER(ctypes.c_uint8)),
                ("power", ctypes.POINTER(ctypes.c_uint8)),
                ("n_nodes", ctypes.c_uint64),
                ("nodes", ctypes.POINTER(_Node)),
                ("boundary_node", ctypes.POINTER(ctypes.c_uint64)),
                ("leaf_depth", ctypes.POINTER(ctypes.c_uint32)),
                ("merge_cost", ctypes.c_uint64),
                ("max_stack", ctypes.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        assert ctypes.sizeof(_Node) == NODE_DTYPE.itemsize
        l = ctypes.CDLL(build())
        P = ctypes.c_void_p
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        l.oracle_runs.argtypes = [P, i32, u64, P, P]
        l.oracle_runs.restype = u64
        l.oracle_power.argtypes = [u64, u64, u64, u64, u32]
        l.oracle_power.restype = i32
        l.oracle_powers.argtypes = [P, u64, u32, P]
        l.oracle_powers.restype = i32
        l.oracle_sort.argtypes = [P, i32, P, u64, u32, ctypes.POINTER(_Trace)]
        l.oracle_sort.restype = i32
        l.oracle_sort_ex.argtypes = [P, i32, P, u64, u32, u32, i32, ctypes.POINTER(_Trace)]
        l.oracle_sort_ex.restype = i32
        l.oracle_runs_min.argtypes = [P, i32, P, u64, u32, P, P]
        l.oracle_runs_min.restype = u64
        l.oracle_trace_free.argtypes = [ctypes.POINTER(_Trace)]
        l.oracle_trace_free.restype = None
        l.oracle_kway_tree.argtypes = [P, u64, P, P]
        l.oracle_kway_tree.restype = ctypes.c_int64
        l.oracle_tree_from_runs.argtypes = [P, u64, u32, ctypes.POINTER(_Trace)]
        l.oracle_tree_from_runs.restype = i32
        l.oracle_tree_from_runs_ex.argtypes = [P, u64, u32, i32, ctypes.POINTER(_Trace)]
        l.oracle_tree_from_runs_ex.restype = i32
        l.oracle_sort_many.argtypes = [P, i32, P, P, u64, u32, P]
        l.oracle_sort_many.restype = i32
        l.oracle_key_cmp.argtypes = [P, i32, u64, u64]
        l.oracle_key_cmp.restype = i32
        _lib = l
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _kt(keys: np.ndarray) -> int:
    try:
        return KEY_TYPES[keys.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {keys.dtype}") from None


@dataclass
class Trace:
    """What Algorithm 2 did: runs, powers, merge-tree nodes and merge cost."""
    n: int
    r: int
    k: int
    run_start: np.ndarray       # uint64[r+1]
    run_desc: np.ndarray        # uint8[r]
    power: np.ndarray           # uint8[r-1], power[i-1] = P_i
    nodes: np.ndarray           # NODE_DTYPE[n_nodes], in merge order
    boundary_node: np.ndarray   # uint64[r-1], node owning boundary i
    leaf_depth: np.ndarray      # uint32[r]
    merge_cost: int
    max_stack: int


def _take_trace(t: _Trace) -> Trace:
    r, nn = int(t.r), int(t.n_nodes)

    def arr(p, count, dt):
        if count == 0:
            return np.zeros(0, dtype=dt)
        return np.ctypeslib.as_array(p, shape=(count,)).copy().view(dt)

    nodes = np.zeros(nn, dtype=NODE_DTYPE)
    if nn:
        # a byte view (ctypes.string_at takes a C int size, too small past 2 GiB)
        raw = np.ctypeslib.as_array(ctypes.cast(t.nodes, ctypes.POINTER(ctypes.c_uint8)),
                                    shape=(nn * NODE_DTYPE.itemsize,))
        nodes = raw.copy().view(NODE_DTYPE)
    tr = Trace(n=int(t.n), r=r, k=int(t.k),
               run_start=arr(t.run_start, r + 1, np.uint64),
               run_desc=arr(t.run_desc, r, np.uint8),
               power=arr(t.power, max(r - 1, 0), np.uint8),
               nodes=nodes,
               boundary_node=arr(t.boundary_node, max(r - 1, 0), np.uint64),
               leaf_depth=arr(t.leaf_depth, r, np.uint32),
               merge_cost=int(t.merge_cost), max_stack=int(t.max_stack))
    lib().oracle_trace_free(ctypes.byref(t))
    return tr


def key_cmp(keys: np.ndarray, i: int, j: int) -> int:
    keys = np.ascontiguousarray(keys)
    return int(lib().oracle_key_cmp(_ptr(keys), _kt(keys), i, j))


def runs(keys: np.ndarray, min_run: int = 1):
    """Greedy run partition (Section 2) -> (run_start uint64[r+1], run_desc uint8[r]).

    min_run > 1: runs shorter than min_run are extended (Appendix A.3); the
    partition depends only on the input, which is not modified."""
    keys = np.ascontiguousarray(keys)
    n = keys.size
    rs = np.empty(n + 1, dtype=np.uint64)
    rd = np.empty(max(n, 1), dtype=np.uint8)
    if min_run <= 1:
        r = int(lib().oracle_runs(_ptr(keys), _kt(keys), n, _ptr(rs), _ptr(rd)))
    else:
        work = keys.copy()
        r = int(lib().oracle_runs_min(_ptr(work), _kt(work), None, n, min_run,
                                      _ptr(rs), _ptr(rd)))
    return rs[: r + 1].copy(), rd[:r].copy()


def power(n: int, s_prev: int, s_cur: int, s_next: int, k: int) -> int:
    """Definition 3.1 for one boundary."""
    return int(lib().oracle_power(n, s_prev, s_cur, s_next, k))


def powers(run_start: np.ndarray, k: int) -> np.ndarray:
    """All boundary powers; run_start may describe a segment (normalised by its own length)."""
    rs = np.ascontiguousarray(run_start, dtype=np.uint64)
    r = rs.size - 1
    out = np.zeros(max(r - 1, 0), dtype=np.uint8)
    if r >= 2:
        rc = lib().oracle_powers(_ptr(rs), r, k, _ptr(out))
        if rc:
            raise ValueError("invalid run partition")
    return out


def sort(keys: np.ndarray, payload: np.ndarray | None = None, k: int = 4, min_run: int = 1,
         merge_down: bool = False):
    """Stable k-way Powersort (Algorithm 2).  Returns (keys, payload, Trace); inputs are copied.

    min_run > 1 extends short runs first (Appendix A.3); merge_down uses the
    final phase of Appendix A.3 (s mod (k-1) entries first, then k-way)."""
    keys = np.array(keys, copy=True, order="C")
    pl = None if payload is None else np.array(payload, dtype=np.uint32, copy=True, order="C")
    if pl is not None and pl.size != keys.size:
        raise ValueError("payload size mismatch")
    t = _Trace()
    rc = lib().oracle_sort_ex(_ptr(keys), _kt(keys), None if pl is None else _ptr(pl),
                              keys.size, k, max(int(min_run), 1), int(bool(merge_down)),
                              ctypes.byref(t))
    if rc:
        raise RuntimeError(f"oracle_sort failed ({rc})")
    return keys, pl, _take_trace(t)


def tree_from_runs(run_start: np.ndarray, k: int, merge_down: bool = False) -> Trace:
    """Algorithm 2's merge tree for a given run partition (no element movement)."""
    rs = np.ascontiguousarray(run_start, dtype=np.uint64)
    t = _Trace()
    rc = lib().oracle_tree_from_runs_ex(_ptr(rs), rs.size - 1, k, int(bool(merge_down)),
                                        ctypes.byref(t))
    if rc:
        raise RuntimeError(f"oracle_tree_from_runs failed ({rc})")
    return _take_trace(t)


def kway_tree(run_start: np.ndarray, power_arr: np.ndarray) -> np.ndarray:
    """Algorithm 1 (KwayTree) -> nodes in post-order."""
    rs = np.ascontiguousarray(run_start, dtype=np.uint64)
    pw = np.ascontiguousarray(power_arr, dtype=np.uint8)
    r = rs.size - 1
    nodes = np.zeros(max(r - 1, 1), dtype=NODE_DTYPE)
    cnt = int(lib().oracle_kway_tree(_ptr(rs), r, _ptr(pw), _ptr(nodes)))
    if cnt < 0:
        raise RuntimeError("oracle_kway_tree failed")
    return nodes[:cnt].copy()


def sort_many(keys: np.ndarray, payload: np.ndarray | None, offsets: np.ndarray, k: int = 4):
    """Sort every segment [offsets[i], offsets[i+1]) on its own.

    Returns (keys, payload, merge_cost uint64[m]); inputs are copied."""
    keys = np.array(keys, copy=True, order="C")
    pl = None if payload is None else np.array(payload, dtype=np.uint32, copy=True, order="C")
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    m = off.size - 1
    mc = np.zeros(max(m, 1), dtype=np.uint64)
    rc = lib().oracle_sort_many(_ptr(keys), _kt(keys), None if pl is None else _ptr(pl),
                                _ptr(off), m, k, _ptr(mc))
    if rc:
        raise RuntimeError(f"oracle_sort_many failed ({rc})")
    return keys, pl, mc[:m]
