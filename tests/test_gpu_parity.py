"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Everything here is integer/comparison work, so the bar is bit-exact: output
keys and payload permutation, run boundaries and directions, every node
power, the merge tree (span, first boundary, arity, power, depth of every
node), leaf depths and the merge cost.

Sizes: the oracle cases span many 2048-key tiles and end in a ragged tail.
The full-size cases (the benchmark workloads) check the output by properties
that single out the stable sort at any size -- the payload is a permutation,
every key is the input key its payload points to, keys are non-decreasing,
and equal keys keep increasing payloads -- and compare runs, powers and the
merge tree with the oracle's (which is fast for those).
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2209_06909_amd as mps  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def pay_dev(p):
    return torch.from_numpy(np.ascontiguousarray(p).view(np.int32)).to(DEV)


def gpu_sort(keys, pay, k, trace=True):
    kd = to_dev(keys)
    pd = pay_dev(pay) if pay is not None else None
    tr = mps.sort(kd, pd, k=k, trace=trace)
    torch.cuda.synchronize()
    gk = kd.cpu().numpy()
    gp = pd.cpu().numpy().view(np.uint32) if pd is not None else None
    return gk, gp, tr


def bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


def check_trace(gt, ot):
    assert gt.r == ot.r
    assert np.array_equal(gt.run_start, ot.run_start)
    assert np.array_equal(gt.run_desc, ot.run_desc)
    assert np.array_equal(gt.power, ot.power)
    assert np.array_equal(gt.leaf_depth.astype(np.int64), ot.leaf_depth.astype(np.int64))
    assert gt.merge_cost == ot.merge_cost
    nodes = np.sort(ot.nodes, order="first_boundary")
    assert gt.n_nodes == len(nodes)
    assert np.array_equal(gt.node_first.astype(np.int64), nodes["first_boundary"].astype(np.int64))
    assert np.array_equal(gt.node_begin, nodes["begin"])
    assert np.array_equal(gt.node_end, nodes["end"])
    assert np.array_equal(gt.node_arity.astype(np.int64), nodes["arity"].astype(np.int64))
    assert np.array_equal(gt.node_power.astype(np.int64), nodes["power"].astype(np.int64))
    assert np.array_equal(gt.node_depth.astype(np.int64), nodes["depth"].astype(np.int64))


def check_vs_oracle(keys, pay, k):
    """Both ways of running the sort against the oracle: with a trace requested
    (the whole tree is built while sorting) and without (only the tree above the
    small subtrees is built; fetching the trace afterwards builds the rest)."""
    ok, op, ot = oracle.sort(keys, pay, k=k)
    gk, gp, gt = gpu_sort(keys, pay, k)
    assert np.array_equal(bits(gk), bits(ok))
    if pay is not None:
        assert np.array_equal(gp, op)
    check_trace(gt, ot)
    lk, lp, _ = gpu_sort(keys, pay, k, trace=False)
    assert np.array_equal(bits(lk), bits(ok))
    if pay is not None:
        assert np.array_equal(lp, op)
    check_trace(mps.last_trace(DEV), ot)
    return gt


# ---------------------------------------------------------------- workloads vs oracle

CASES = [("runs_i32", (1 << 18) + 777), ("runs_i64", (1 << 18) + 777),
         ("perm_i64", (1 << 17) + 333), ("ties_i32", (1 << 18) + 999)]


@pytest.mark.parametrize("k", [4, 2, 8])
@pytest.mark.parametrize("name,n", CASES)
def test_workload_vs_oracle(name, n, k):
    say(f"[gpu] {name} n={n} k={k}")
    keys, pay = workloads.WORKLOADS[name](n=n, seed=1000 + n % 97)
    check_vs_oracle(keys, pay, k)


def test_runs_i32_full_size_vs_oracle():
    """The n = 2^20 run-structured int32 workload, full size, full oracle parity."""
    say("[gpu] runs_i32 full 2^20")
    keys, pay = workloads.runs_i32()
    check_vs_oracle(keys, pay, 4)


@pytest.mark.parametrize("k", [2, 4])
def test_keys_only(k):
    keys, _ = workloads.ties_i32(n=50000, seed=3)
    ok, _, ot = oracle.sort(keys, None, k=k)
    gk, _, gt = gpu_sort(keys, None, k)
    assert np.array_equal(gk, ok)
    check_trace(gt, ot)


# ---------------------------------------------------------------- edge cases

I32 = np.iinfo(np.int32)
I64 = np.iinfo(np.int64)
EDGE = {
    "empty": np.zeros(0, np.int32),
    "one": np.array([5], np.int32),
    "two_up": np.array([1, 2], np.int32),
    "two_down": np.array([2, 1], np.int32),
    "two_eq": np.array([3, 3], np.int32),
    "three": np.array([3, 1, 2], np.int32),
    "all_equal": np.full(5000, 7, np.int32),
    "ascending": np.arange(5000, dtype=np.int32),
    "strict_desc": np.arange(5000, 0, -1, dtype=np.int32),
    "zigzag": np.tile(np.array([1, 0], np.int32), 2500),
    "zigzag_odd": np.concatenate([np.tile(np.array([1, 0], np.int32), 2500), [1]]).astype(np.int32),
    "zigzag_long": np.tile(np.array([5, 3], np.int32), 70000),     # carry chain across blocks
    "updown": np.tile(np.array([0, 1, 2, 1], np.int32), 30000),
    "extremes": np.array([I32.max, I32.min, I32.max, I32.min, 0, I32.min, I32.max] * 1000, np.int32),
    "i64_range": np.array([I64.max, I64.min, -1, 0, I64.max, I64.min, 1] * 999, np.int64),
    "two_runs": np.concatenate([np.arange(3000), np.arange(3000)]).astype(np.int32),
    "one_big_one_small": np.concatenate([np.arange(100000), [5, 4]]).astype(np.int32),
    "tile_edge": np.concatenate([np.arange(2048), np.arange(2048), np.arange(1)]).astype(np.int32),
    # runs of 8, shifted so a 2048-position block overlaps 257 of them: the
    # placement's staged run table (256 entries) just overflows
    "runs8_up": np.concatenate([np.arange(4), np.tile(np.arange(8), 1000)]).astype(np.int32),
    "runs8_down": np.concatenate([np.arange(4)[::-1], np.tile(np.arange(8)[::-1], 1000)]).astype(np.int32),
}


@pytest.mark.parametrize("k", [2, 4, 8])
@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_case(name, k):
    say(f"[gpu] edge {name} k={k}")
    keys = EDGE[name]
    pay = np.arange(keys.size, dtype=np.uint32)
    if keys.size <= 1:
        gk, gp, gt = gpu_sort(keys, pay, k)
        assert np.array_equal(gk, keys) and np.array_equal(gp, pay)
        assert gt.r == keys.size and gt.merge_cost == 0
        return
    check_vs_oracle(keys, pay, k)


def test_many_small_random_arrays():
    rng = np.random.default_rng(77)
    for it in range(120):
        n = int(rng.integers(2, 600))
        hi = int(rng.choice([2, 3, 10, 1000, 2 ** 31 - 1]))
        keys = rng.integers(-hi, hi, size=n).astype(np.int32)
        if it % 3 == 0:  # add runs
            cut = np.sort(rng.choice(n, size=min(n - 1, 5), replace=False))
            for a, b in zip(cut[:-1], cut[1:]):
                keys[a:b] = np.sort(keys[a:b])[:: (1 if rng.random() < 0.5 else -1)]
        k = int(rng.choice([2, 4, 8]))
        check_vs_oracle(keys, np.arange(n, dtype=np.uint32), k)


def test_float_keys_total_order():
    rng = np.random.default_rng(5)
    specials = np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45, 3.4e38, -3.4e38, 1.0, -1.0],
                        dtype=np.float32)
    keys = np.concatenate([rng.standard_normal(20000).astype(np.float32), np.repeat(specials, 300)])
    rng.shuffle(keys)
    for L in (1, 7, 100):  # some runs
        keys[: L * 50] = np.sort(keys[: L * 50])
    check_vs_oracle(keys, np.arange(keys.size, dtype=np.uint32), 4)


# ---------------------------------------------------------------- batched

def test_batched_vs_oracle_and_single():
    say("[gpu] batched small")
    keys, pay, off = workloads.batch_i32(m=300, seed=21, lo_exp=0, hi_exp=15)
    # a few empty arrays in the middle
    sizes = np.diff(off.astype(np.int64))
    sizes[[5, 6, 100]] = 0
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys, pay = keys[: int(off[-1])], pay[: int(off[-1])]
    ok, op, omc = oracle.sort_many(keys, pay, off, k=4)
    kd, pd = to_dev(keys), pay_dev(pay)
    od = torch.from_numpy(off.view(np.int64)).to(DEV)
    gt = mps.sort_batched(kd, pd, od, k=4, trace=True, host_offsets=off)
    gk, gp = kd.cpu().numpy(), pd.cpu().numpy().view(np.uint32)
    assert np.array_equal(gk, ok)
    assert np.array_equal(gp, op)
    assert gt.merge_cost == int(omc.sum())
    # runs and powers: per-array oracle results, concatenated; array edges carry power 0
    rs_all, pw_all = [], []
    for i in range(len(off) - 1):
        s, e = int(off[i]), int(off[i + 1])
        if e == s:
            continue
        rs, _ = oracle.runs(keys[s:e])
        if rs_all:
            pw_all.append(np.zeros(1, np.uint8))
        pw_all.append(oracle.powers(rs, 4))
        rs_all.append(rs[:-1] + s)
    rs_all.append(np.array([off[-1]], np.uint64))
    assert np.array_equal(gt.run_start, np.concatenate(rs_all))
    assert np.array_equal(gt.power, np.concatenate(pw_all))
    # each array alone through the single-array entry gives the same bits
    for i in range(0, len(off) - 1, 17):
        s, e = int(off[i]), int(off[i + 1])
        sk, sp, _ = gpu_sort(keys[s:e], pay[s:e], 4, trace=False)
        assert np.array_equal(sk, gk[s:e]) and np.array_equal(sp, gp[s:e])


# ---------------------------------------------------------------- full-size workloads

def order_key(a):
    if a.dtype == np.float32:
        u = a.view(np.uint32).astype(np.uint64)
        return np.where(u >> 31, (~u) & 0xFFFFFFFF, u | 0x80000000)
    if a.dtype == np.int64:
        return a.view(np.uint64) ^ np.uint64(1 << 63)
    return (a.view(np.uint32) ^ np.uint32(1 << 31)).astype(np.uint64)


def check_stable_sort_properties(keys_in, keys_out, pay_out):
    n = keys_in.size
    assert pay_out.max(initial=0) < n
    seen = np.zeros(n, dtype=bool)
    seen[pay_out] = True
    assert seen.all()                                        # payload is a permutation
    assert np.array_equal(bits(keys_out), bits(keys_in[pay_out]))   # keys travel with payload
    ko = order_key(keys_out)
    assert not np.any(ko[1:] < ko[:-1])                      # sorted
    eq = ko[1:] == ko[:-1]
    assert np.all(pay_out[1:][eq] > pay_out[:-1][eq])        # stable


FULL = [("ties_i32", 1 << 27), ("runs_i64", 1 << 28), ("perm_i64", 1 << 28)]


@pytest.mark.parametrize("name,n", FULL)
def test_full_size(name, n):
    say(f"[gpu] full {name} n={n}: generating")
    keys, pay = workloads.WORKLOADS[name](n=n)
    say(f"[gpu] full {name}: sorting")
    gk, gp, _ = gpu_sort(keys, pay, 4, trace=False)     # as the benchmark runs it
    gt = mps.last_trace(DEV)
    say(f"[gpu] full {name}: checking r={gt.r} nodes={gt.n_nodes}")
    check_stable_sort_properties(keys, gk, gp)
    tk, tp, tt = gpu_sort(keys, pay, 4, trace=True)     # the whole tree built while sorting
    assert np.array_equal(bits(tk), bits(gk)) and np.array_equal(tp, gp)
    for f in ("r", "n_nodes", "merge_cost", "n_levels"):
        assert getattr(tt, f) == getattr(gt, f), f
    for f in ("run_start", "power", "leaf_depth", "node_first", "node_arity", "node_depth"):
        assert np.array_equal(getattr(tt, f), getattr(gt, f)), f
    rs, rd = oracle.runs(keys)
    assert np.array_equal(gt.run_start, rs) and np.array_equal(gt.run_desc, rd)
    ot = oracle.tree_from_runs(rs, 4)
    assert np.array_equal(gt.power, ot.power)
    assert gt.merge_cost == ot.merge_cost
    nodes = np.sort(ot.nodes, order="first_boundary")
    assert np.array_equal(gt.node_first.astype(np.int64), nodes["first_boundary"].astype(np.int64))
    assert np.array_equal(gt.node_depth.astype(np.int64), nodes["depth"].astype(np.int64))
    assert np.array_equal(gt.node_arity.astype(np.int64), nodes["arity"].astype(np.int64))


ZIGZAG_BIG = [
    # strictly alternating: every pair type changes, so the odd-streak rule's carry runs
    # through the whole array and across every iteration of the run-detection block scan
    ("zigzag_i32", np.tile(np.array([5, 3], np.int32), (1 << 24) + 1)),
    ("zigzag_i32_odd", np.concatenate([np.tile(np.array([5, 3], np.int32), 1 << 24),
                                       np.array([9, 1, 2], np.int32)])),
    ("zigzag_i64_shifted", np.concatenate([np.array([7], np.int64),
                                           np.tile(np.array([2, 8], np.int64), (1 << 24) + 7)])),
]


@pytest.mark.parametrize("name,keys", ZIGZAG_BIG, ids=[z[0] for z in ZIGZAG_BIG])
def test_zigzag_crosses_detect_blocks(name, keys):
    """Zig-zag inputs of more than 2^25 keys (Section 2's runs: every run is a
    strictly descending pair, or the pair it starts is ascending): runs,
    directions, powers, tree and output equal the oracle's."""
    say(f"[gpu] zigzag {name} n={keys.size}")
    assert keys.size > 1 << 25
    pay = np.arange(keys.size, dtype=np.uint32)
    check_vs_oracle(keys, pay, 4)
