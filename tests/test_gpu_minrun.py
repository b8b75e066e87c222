"""GPU parity for the minimal run length (Appendix A.3) against the CPU oracle.

With min_run = m > 1, natural runs shorter than m are extended to m elements
(sorted stably) and the next run starts where the extended one ends; the
powers and the merge tree are those of the extended runs.  The bar is the
same as for natural runs: output keys and payload, run starts and flags,
every power, the merge tree and the merge cost, all bit-exact.

Inputs are chosen to exercise the chunked resolution of the run chain
(chunks of 4096 positions): runs with lengths around m, long runs that cross
several chunk edges (the chain then enters a chunk past its first m
positions), alternating and constant inputs, arrays shorter than m and
arrays that end exactly on or just past a chunk edge.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2209_06909_amd as mps  # noqa: E402

from test_gpu_parity import (bits, check_stable_sort_properties, check_trace, pay_dev,  # noqa: E402
                             to_dev)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_sort(keys, pay, k, m, trace=True, graph=False):
    kd = to_dev(keys)
    pd = pay_dev(pay) if pay is not None else None
    tr = mps.sort(kd, pd, k=k, trace=trace, min_run=m, graph=graph)
    torch.cuda.synchronize()
    gk = kd.cpu().numpy()
    gp = pd.cpu().numpy().view(np.uint32) if pd is not None else None
    return gk, gp, tr


def check_vs_oracle(keys, pay, k, m):
    """With a trace requested (whole tree built while sorting) and without (the
    tree inside small subtrees is built only when the trace is fetched)."""
    ok, op, ot = oracle.sort(keys, pay, k=k, min_run=m)
    gk, gp, gt = gpu_sort(keys, pay, k, m)
    assert np.array_equal(bits(gk), bits(ok))
    if pay is not None:
        assert np.array_equal(gp, op)
    check_trace(gt, ot)
    lk, lp, _ = gpu_sort(keys, pay, k, m, trace=False)
    assert np.array_equal(bits(lk), bits(ok))
    if pay is not None:
        assert np.array_equal(lp, op)
    check_trace(mps.last_trace("cuda:0"), ot)
    return gt


def near_m(n, m, seed, long_every=0):
    """Runs of m-3 .. m+3 elements in random directions; every long_every-th
    run is 5000-20000 long instead (crossing chunk edges)."""
    rng = np.random.default_rng(seed)
    parts, total, j = [], 0, 0
    while total < n:
        if long_every and j % long_every == long_every - 1:
            L = int(rng.integers(5000, 20000))
        else:
            L = int(rng.integers(max(m - 3, 1), m + 4))
        v = np.sort(rng.integers(-1000, 1000, size=L))
        parts.append(v if rng.random() < 0.5 else v[::-1].copy())
        total += L
        j += 1
    return np.concatenate(parts)[:n].astype(np.int32)


def crossing(n, seed):
    """Long ascending and strictly descending stretches (9000 keys) between
    alternating stretches, so that long runs span chunk edges."""
    rng = np.random.default_rng(seed)
    parts, total, j = [], 0, 0
    while total < n:
        if j % 2 == 0:
            L = 9000
            v = np.arange(L) * 3 + int(rng.integers(0, 100))
            parts.append(v if j % 4 == 0 else v[::-1].copy())
        else:
            L = int(rng.integers(1, 300))
            parts.append(np.tile(np.array([5, -5]), L)[:L] + int(rng.integers(0, 3)))
        total += L
        j += 1
    return np.concatenate(parts)[:n].astype(np.int64)


def named(name, n, m):
    if name == "near_m":
        return near_m(n, m, 31)
    if name == "near_m_long":
        return near_m(n, m, 32, long_every=7)
    if name == "crossing":
        return crossing(n, 33)
    if name == "f32_near_m":    # float keys: ties, and -0 / +0 (ordered -0 < +0)
        keys = near_m(n, m, 34, long_every=11).astype(np.float32) * np.float32(-0.25)
        rng = np.random.default_rng(35)
        z = rng.integers(0, n, size=n // 50)
        keys[z] = np.where(rng.random(z.size) < 0.5, np.float32(-0.0), np.float32(0.0))
        return keys
    keys, _ = workloads.WORKLOADS[name](n=n)
    return keys


CASES = [("perm_i64", (1 << 16) + 77), ("runs_i32", (1 << 17) + 5), ("ties_i32", (1 << 17) + 3),
         ("f32_near_m", (1 << 16) + 9), ("near_m", 150001), ("near_m_long", 200003),
         ("crossing", 100000)]


@pytest.mark.parametrize("m", [24, 2, 3, 32])
@pytest.mark.parametrize("name,n", CASES)
def test_min_run_vs_oracle(name, n, m):
    keys = named(name, n, m)
    say(f"[gpu] min_run {name} n={n} m={m}")
    pay = np.arange(n, dtype=np.uint32)
    check_vs_oracle(keys, pay, 4, m)


@pytest.mark.parametrize("k", [2, 8])
def test_min_run_other_arities(k):
    keys = near_m(120007, 24, 41, long_every=5)
    say(f"[gpu] min_run near_m_long k={k}")
    check_vs_oracle(keys, np.arange(keys.size, dtype=np.uint32), k, 24)


EDGE_N = [2, 3, 5, 23, 24, 25, 31, 33, 4095, 4096, 4097, 4096 * 3 + 1, 8192]


@pytest.mark.parametrize("n", EDGE_N)
def test_min_run_small_sizes(n):
    rng = np.random.default_rng(n)
    for m in (2, 24, 32):
        keys = rng.integers(0, 4, size=n).astype(np.int32)
        say(f"[gpu] min_run small n={n} m={m}")
        check_vs_oracle(keys, np.arange(n, dtype=np.uint32), 4, m)


EDGE = {
    "ascending": np.arange(10003, dtype=np.int32),
    "strict_desc": np.arange(10003, 0, -1).astype(np.int32),
    "all_equal": np.full(10003, 7, np.int32),
    "zigzag": np.tile(np.array([1, 0], np.int32), 5001),
    "zigzag_odd": np.concatenate([np.tile(np.array([1, 0], np.int32), 5001), [1]]).astype(np.int32),
    "pairs_down": np.repeat(np.arange(6000, 0, -1), 2).astype(np.int32),
}


@pytest.mark.parametrize("m", [2, 24])
@pytest.mark.parametrize("name", sorted(EDGE))
def test_min_run_edge_inputs(name, m):
    keys = EDGE[name]
    say(f"[gpu] min_run edge {name} m={m}")
    gt = check_vs_oracle(keys, np.arange(keys.size, dtype=np.uint32), 4, m)
    if name in ("ascending", "strict_desc", "all_equal"):
        assert gt.r == 1


def test_min_run_keys_only():
    keys = near_m(70001, 24, 51, long_every=9)
    ok, _, ot = oracle.sort(keys, None, k=4, min_run=24)
    gk, _, gt = gpu_sort(keys, None, 4, 24)
    assert np.array_equal(gk, ok)
    check_trace(gt, ot)


def test_min_run_graph_replay():
    """Graph capture of a min-run sort, replayed on new contents."""
    n = 90001
    kd = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    pd = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    for seed in (61, 62, 63):
        keys = near_m(n, 24, seed, long_every=6)
        pay = np.arange(n, dtype=np.uint32)
        kd.copy_(torch.from_numpy(keys))
        pd.copy_(torch.from_numpy(pay.view(np.int32)))
        say(f"[gpu] min_run graph seed={seed}")
        mps.sort(kd, pd, k=4, min_run=24, graph=True)
        torch.cuda.synchronize()
        ok, op, _ = oracle.sort(keys, pay, k=4, min_run=24)
        assert np.array_equal(kd.cpu().numpy(), ok)
        assert np.array_equal(pd.cpu().numpy().view(np.uint32), op)


def test_min_run_rejected_values():
    kd = torch.arange(1000, dtype=torch.int32, device="cuda:0")
    with pytest.raises(mps.MpsError):
        mps.sort(kd, None, min_run=33)


def test_min_run_one_is_natural():
    keys, pay = workloads.WORKLOADS["runs_i32"](n=50000)
    a = gpu_sort(keys, pay, 4, 1)
    b = gpu_sort(keys, pay, 4, 0)
    ok, op, ot = oracle.sort(keys, pay, k=4)
    for gk, gp, gt in (a, b):
        assert np.array_equal(gk, ok) and np.array_equal(gp, op)
        check_trace(gt, ot)


def test_min_run_full_size_permutation():
    """2^28 int64 keys, a random permutation, m = 24 (the paper's setting):
    stable-sort properties of the output; runs, flags, powers and the merge
    tree against the oracle's."""
    n = 1 << 28
    say("[gpu] min_run full perm_i64: generating")
    keys, pay = workloads.WORKLOADS["perm_i64"](n=n)
    say("[gpu] min_run full perm_i64: sorting")
    gk, gp, gt = gpu_sort(keys, pay, 4, 24)
    say(f"[gpu] min_run full perm_i64: checking r={gt.r}")
    check_stable_sort_properties(keys, gk, gp)
    rs, rd = oracle.runs(keys, min_run=24)
    assert np.array_equal(gt.run_start, rs) and np.array_equal(gt.run_desc, rd)
    ot = oracle.tree_from_runs(rs, 4)
    assert np.array_equal(gt.power, ot.power)
    assert gt.merge_cost == ot.merge_cost
    nodes = np.sort(ot.nodes, order="first_boundary")
    assert np.array_equal(gt.node_first.astype(np.int64), nodes["first_boundary"].astype(np.int64))
    assert np.array_equal(gt.node_depth.astype(np.int64), nodes["depth"].astype(np.int64))
