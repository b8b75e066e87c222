"""Pins for the CPU oracle (no GPU).

The oracle is only trusted because these tests tie it to things other than
itself: the worked examples printed in the paper (Figures 1 and 3), library
stable sorts, brute force over every tie pattern of tiny inputs, an
independent formulation of the node power (the "tick" form used in the proof
of Theorem 3.3), and the invariants of Section 3 (Fact 3.2, the leaf-depth
identity, Theorem 3.3, Proposition 3.5).  A plausible slip anywhere in the
oracle (wrong tie rule, off-by-one power, wrong final merge phase, dropped
reversal) breaks at least one of them.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.filterwarnings("ignore")


# ---------------------------------------------------------------- helpers

def starts_from_lengths(lengths):
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint64)


def ceil_log_plus1(k, x_num, x_den=1):
    """Least integer c with k**(c-1) >= x_num/x_den, i.e. ceil(log_k(x) + 1)."""
    c = 0
    while Fraction(k) ** (c - 1) < Fraction(x_num, x_den):
        c += 1
    return c


def tick_power(n, s_prev, s_cur, s_next, k):
    """Power via the tick form from the proof of Theorem 3.3: the least p such
    that some multiple c*k^-p lies in the half-open midpoint interval (a, b]."""
    a = Fraction(s_prev + s_cur, 2 * n)
    b = Fraction(s_cur + s_next, 2 * n)
    p = 0
    while True:
        step = Fraction(1, k ** p)
        c = (b // step)             # largest tick <= b
        if c * step > a:
            return p
        p += 1


def stable_order(keys):
    return np.argsort(keys, kind="stable")


def canonical_nodes(nodes):
    rows = [(int(v["begin"]), int(v["end"]), int(v["first_boundary"]), int(v["arity"]),
             int(v["power"]), int(v["depth"])) for v in nodes]
    return sorted(rows)


def check_tree_invariants(tr, k):
    """Section 3 invariants on one oracle trace."""
    r, n = tr.r, tr.n
    rs = tr.run_start.astype(np.int64)
    L = np.diff(rs)
    nodes = tr.nodes
    assert len(nodes) == (r - 1 if r >= 1 else 0) or k > 2
    # Algorithm 1 builds the same tree (stated right after Algorithm 1).
    alg1 = oracle.kway_tree(tr.run_start, tr.power)
    assert canonical_nodes(alg1) == canonical_nodes(nodes)
    if r <= 1:
        assert tr.merge_cost == 0
        return
    depth = nodes["depth"].astype(np.int64)
    bnode = tr.boundary_node.astype(np.int64)
    P = tr.power.astype(np.int64)
    # every node merges 2..k runs; all its boundaries carry its power
    assert np.all(nodes["arity"] >= 2) and np.all(nodes["arity"] <= k)
    assert np.all(nodes["power"][bnode] == P)
    counts = np.bincount(bnode, minlength=len(nodes))
    assert np.all(counts == nodes["arity"] - 1)
    # Fact 3.2: depth(m(B_j)) <= P_j - 1
    assert np.all(depth[bnode] <= P - 1)
    # leaf depth d_i = 1 + max(depth m(B_i), depth m(B_{i+1})), outer terms -1
    bd = np.concatenate([[-1], depth[bnode], [-1]])
    assert np.array_equal(tr.leaf_depth.astype(np.int64), 1 + np.maximum(bd[:-1], bd[1:]))
    # merge cost: sum over nodes of merged lengths = sum_i d_i L_i
    spans = (nodes["end"] - nodes["begin"]).astype(np.int64)
    assert tr.merge_cost == int(spans.sum()) == int((tr.leaf_depth.astype(np.int64) * L).sum())
    # powers: 1 <= P_i and P_i, P_{i+1} <= ceil(log_k(1/l_i) + 1) (proof of Thm 3.3)
    assert np.all(P >= 1)
    for i in range(r):
        bound = ceil_log_plus1(k, n, int(L[i]))
        if i >= 1:
            assert P[i - 1] <= bound
        if i + 1 <= r - 1:
            assert P[i] <= bound
    # Theorem 3.3 (sharper form from its proof): M/n <= sum l_i ceil(log_k(1/l_i) + 1)
    rhs = sum(int(Li) * ceil_log_plus1(k, n, int(Li)) for Li in L)
    assert tr.merge_cost <= rhs
    H = float(sum((Li / n) * math.log2(n / Li) for Li in L))
    assert tr.merge_cost <= H * n / math.log2(k) + 2 * n + 1e-6
    # Proposition 3.5: stack height <= (k-1) * ceil(log_k n + 1)
    assert tr.max_stack <= (k - 1) * ceil_log_plus1(k, n)


def lt(a, b):
    """Elementwise a < b in the key order (float32: numeric, with -0 < +0)."""
    if a.dtype == np.float32:
        return (a < b) | ((a == b) & np.signbit(a) & ~np.signbit(b))
    return a < b


def check_runs(keys, rs, rd):
    n = keys.size
    rs = rs.astype(np.int64)
    assert rs[0] == 0 and rs[-1] == n
    r = rs.size - 1
    for i in range(r):
        s, e = rs[i], rs[i + 1]
        assert e > s
        seg = keys[s:e]
        if e - s >= 2:
            if rd[i]:
                assert np.all(lt(seg[1:], seg[:-1]))
            else:
                assert not np.any(lt(seg[1:], seg[:-1]))
        else:
            assert i == r - 1 and rd[i] == 0     # only the last run can be a single element
        if e < n:                                # maximal: the next element breaks the run
            if rd[i]:
                assert not lt(keys[e:e + 1], keys[e - 1:e])[0]
            else:
                assert lt(keys[e:e + 1], keys[e - 1:e])[0]


def weak_orderings(n):
    """Every sequence of length n over {0..m-1} that uses all m values: one
    representative of every possible pattern of ties and order."""
    if n == 0:
        return np.zeros((1, 0), dtype=np.int32)
    grid = np.array(list(itertools.product(range(n), repeat=n)), dtype=np.int8)
    srt = np.sort(grid, axis=1)
    ok = (srt[:, 0] == 0) & np.all(np.diff(srt, axis=1) <= 1, axis=1)
    return grid[ok].astype(np.int32)


FUBINI = [1, 1, 3, 13, 75, 541, 4683, 47293]


# ---------------------------------------------------------------- paper pins

def test_fig1_powers(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "fig1.json")))
    rs = starts_from_lengths(g["run_lengths"])
    assert int(rs[-1]) == g["n"]
    assert oracle.powers(rs, 2).tolist() == g["power_k2"]
    assert oracle.powers(rs, 4).tolist() == g["power_k4"]


@pytest.mark.parametrize("k", [2, 4])
def test_fig1_trees(golden_dir, k):
    g = json.load(open(os.path.join(golden_dir, "fig1.json")))
    rs = starts_from_lengths(g["run_lengths"])
    tr = oracle.tree_from_runs(rs, k)
    spans = sorted((int(v["begin"]), int(v["end"])) for v in tr.nodes)
    want = sorted(tuple(s) for s in g[f"tree_k{k}_spans"])
    assert spans == want
    # merge cost is the total length of all merge results (Section 2.3)
    assert tr.merge_cost == sum(e - b for b, e in want)
    check_tree_invariants(tr, k)


def test_fig3_power(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "fig3.json")))
    # runs [8,10) and [10,28) of an array of length 40 have midpoints 9/40 and 19/40
    n, s = 40, (8, 10, 28)
    assert Fraction(s[0] + s[1], 2 * n) == Fraction(g["a"])
    assert Fraction(s[1] + s[2], 2 * n) == Fraction(g["b"])
    assert oracle.power(n, *s, g["k"]) == g["power"]


def test_half_open_interval():
    # a tick exactly at b counts: (1/8, 1/2] contains 1/2 -> P = 1 for k = 2 and 4
    assert oracle.power(8, 0, 2, 6, 2) == 1
    assert oracle.power(8, 0, 2, 6, 4) == 1
    # a tick exactly at a does not: (1/2, 3/4] needs p = 2 for k = 2 (tick 3/4)
    assert oracle.power(16, 6, 10, 14, 2) == 2
    # invalid partitions are rejected
    assert oracle.power(16, 6, 6, 14, 2) == -1
    assert oracle.power(16, 6, 10, 17, 2) == -1


@pytest.mark.parametrize("k", [2, 3, 4, 5, 8, 16])
def test_power_matches_tick_form(k):
    rng = np.random.default_rng(100 + k)
    for _ in range(300):
        n = int(rng.integers(3, 10 ** int(rng.integers(1, 7))))
        cuts = np.sort(rng.choice(np.arange(1, n), size=2, replace=False))
        s_prev = int(rng.integers(0, cuts[0]))
        s = (s_prev, int(cuts[0]), int(cuts[1]))
        assert oracle.power(n, *s, k) == tick_power(n, *s, k)


def test_power_extremes():
    n = 2 ** 31
    for s in [(0, 1, 2), (n - 3, n - 2, n - 1), (n - 2, n - 1, n), (0, n // 2, n), (0, 1, n)]:
        for k in (2, 4, 8):
            assert oracle.power(n, *s, k) == tick_power(n, *s, k)


def test_squish_identity():
    """Section 3.1: P^(4) = floor((P^(2)-1)/2) + 1; generalised to k = 2^q."""
    rng = np.random.default_rng(7)
    for _ in range(40):
        n = int(rng.integers(2, 200000))
        lengths = workloads._run_lengths(rng, n, lambda g, c: g.integers(1, 1 + int(rng.integers(1, 5000)), size=c))
        rs = starts_from_lengths(lengths)
        p2 = oracle.powers(rs, 2).astype(np.int64)
        for q, k in [(2, 4), (3, 8), (4, 16)]:
            assert np.array_equal(oracle.powers(rs, k).astype(np.int64), (p2 - 1) // q + 1)


def test_merge_cost_ratio_table1(golden_dir):
    """Hypothesis 3 / Table 1: 4-way merge cost is about 52% of 2-way on random runs.
    Different random inputs and no minimal run length here, so only a loose band."""
    g = json.load(open(os.path.join(golden_dir, "table1.json")))
    paper_ratio = g["merge_cost_k4"] / g["merge_cost_k2"]
    assert 0.51 < paper_ratio < 0.53
    keys, _ = workloads.runs_i64(n=1 << 20, seed=11)
    rs, _ = oracle.runs(keys)
    m2 = oracle.tree_from_runs(rs, 2).merge_cost
    m4 = oracle.tree_from_runs(rs, 4).merge_cost
    assert abs(m4 / m2 - paper_ratio) < 0.08


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("n", range(0, 9))
def test_bruteforce_sort_all_tie_patterns(n):
    """Every tie/order pattern of length n (Fubini many): the output is the
    unique stable sort (library stable argsort), for several k."""
    rows = weak_orderings(n)
    if n <= 7:
        assert rows.shape[0] == FUBINI[n]
    m = rows.shape[0]
    flat = rows.reshape(-1)
    offsets = (np.arange(m + 1, dtype=np.uint64) * n)
    local = np.tile(np.arange(n, dtype=np.uint32), m)
    want_perm = np.argsort(rows, axis=1, kind="stable").astype(np.uint32)
    want_keys = np.take_along_axis(rows, want_perm.astype(np.int64), axis=1)
    for k in (2, 3, 4):
        sk, sp, _ = oracle.sort_many(flat, local, offsets, k=k)
        assert np.array_equal(sk.reshape(m, n), want_keys)
        assert np.array_equal(sp.reshape(m, n), want_perm)
    # the same patterns as int64 and float32 keys (spread over negative values)
    for dt, scale in ((np.int64, -(2 ** 40)), (np.float32, -1.5)):
        vals = (rows.astype(np.float64) * scale).astype(dt)
        sk, sp, _ = oracle.sort_many(vals.reshape(-1), local, offsets, k=4)
        wp = np.argsort(vals, axis=1, kind="stable").astype(np.uint32)
        assert np.array_equal(sp.reshape(m, n), wp)


@pytest.mark.parametrize("n", range(0, 8))
def test_bruteforce_runs_all_tie_patterns(n):
    for row in weak_orderings(n):
        rs, rd = oracle.runs(row)
        check_runs(row, rs, rd)


@pytest.mark.parametrize("n", range(1, 7))
@pytest.mark.parametrize("k", [2, 3, 4])
def test_bruteforce_tree_all_tie_patterns(n, k):
    for row in weak_orderings(n):
        sk, sp, tr = oracle.sort(row, np.arange(n, dtype=np.uint32), k=k)
        assert np.array_equal(sp, stable_order(row))
        check_runs(row, tr.run_start, tr.run_desc)
        check_tree_invariants(tr, k)


def test_all_run_length_compositions():
    """Every composition of n <= 12 into run lengths: Algorithm 1 = Algorithm 2
    and all Section 3 invariants, for k = 2..5 and 8."""
    for n in range(1, 13):
        for mask in range(1 << (n - 1)):
            cuts = [i + 1 for i in range(n - 1) if mask >> i & 1]
            rs = np.array([0] + cuts + [n], dtype=np.uint64)
            for k in (2, 3, 4, 5, 8):
                check_tree_invariants(oracle.tree_from_runs(rs, k), k)


# ---------------------------------------------------------------- at scale

@pytest.mark.parametrize("name,n", [("runs_i32", 1 << 18), ("runs_i64", 1 << 18),
                                    ("perm_i64", 1 << 16), ("ties_i32", 1 << 18)])
@pytest.mark.parametrize("k", [2, 4, 8])
def test_matches_library_stable_sort(name, n, k):
    keys, pay = workloads.WORKLOADS[name](n=n)
    sk, sp, tr = oracle.sort(keys, pay, k=k)
    order = stable_order(keys)
    assert np.array_equal(sp, pay[order])
    assert np.array_equal(sk, keys[order])
    if k == 4:
        check_runs(keys, tr.run_start, tr.run_desc)
        check_tree_invariants(tr, k)


@pytest.mark.parametrize("name,n", [("runs_i32", 1 << 17), ("runs_i64", 1 << 17),
                                    ("ties_i32", 1 << 17)])
def test_matches_std_stable_sort(name, n):
    """The oracle against C++ std::stable_sort of (key, payload) records."""
    keys, pay = workloads.WORKLOADS[name](n=n)
    rk, rp = oracle.stable_sort_ref(keys, pay)
    for k in (2, 4):
        sk, sp, _ = oracle.sort(keys, pay, k=k)
        assert np.array_equal(sk, rk) and np.array_equal(sp, rp)


def test_float_total_order_matches_std_stable_sort():
    """Signed zeros and both signs under the total order, against std::stable_sort."""
    rng = np.random.default_rng(12)
    f = rng.standard_normal(50000).astype(np.float32)
    f[::7] = -0.0
    f[::11] = 0.0
    f[::13] = np.float32(1e-42)        # subnormal
    pay = np.arange(f.size, dtype=np.uint32)
    rk, rp = oracle.stable_sort_ref(f, pay)
    sk, sp, _ = oracle.sort(f, pay, k=4)
    assert np.array_equal(sk.view(np.uint32), rk.view(np.uint32)) and np.array_equal(sp, rp)


def test_permutation_exact():
    keys, pay = workloads.perm_i64(n=1 << 17, seed=5)
    sk, sp, _ = oracle.sort(keys, pay, k=4)
    assert np.array_equal(sk, np.arange(keys.size, dtype=np.int64))
    inv = np.empty_like(pay)
    inv[keys] = pay
    assert np.array_equal(sp, inv)


def test_float_total_order():
    rng = np.random.default_rng(3)
    specials = np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45, 3.4e38, -3.4e38,
                         1.0, -1.0], dtype=np.float32)
    vals = np.concatenate([specials, rng.standard_normal(3000).astype(np.float32),
                           rng.choice(specials, 500)])
    rng.shuffle(vals)
    pay = np.arange(vals.size, dtype=np.uint32)
    sk, sp, _ = oracle.sort(vals, pay, k=4)
    # numeric order; among equal numbers (only +-0 differ in bits) -0 first; then index
    neg_bit = np.signbit(vals)
    want = np.lexsort((pay, ~neg_bit, vals.astype(np.float64)))
    assert np.array_equal(sp, pay[want])
    assert np.array_equal(sk.view(np.uint32), vals[want].view(np.uint32))


def test_segments_sort_independently():
    keys, pay, off = workloads.batch_i32(m=40, seed=9, lo_exp=1, hi_exp=12)
    sk, sp, mc = oracle.sort_many(keys, pay, off, k=4)
    for i in range(40):
        s, e = int(off[i]), int(off[i + 1])
        k1, p1, t1 = oracle.sort(keys[s:e], pay[s:e], k=4)
        assert np.array_equal(sk[s:e], k1) and np.array_equal(sp[s:e], p1)
        assert mc[i] == t1.merge_cost


# ---------------------------------------------------------------- edge cases

I32 = np.iinfo(np.int32)
I64 = np.iinfo(np.int64)

EDGE = {
    "empty": np.zeros(0, np.int32),
    "one": np.array([5], np.int32),
    "two_up": np.array([1, 2], np.int32),
    "two_down": np.array([2, 1], np.int32),
    "two_eq": np.array([3, 3], np.int32),
    "all_equal": np.full(1000, 7, np.int32),
    "ascending": np.arange(1000, dtype=np.int32),
    "strict_desc": np.arange(1000, 0, -1, dtype=np.int32),
    "zigzag": np.tile(np.array([1, 0], np.int32), 500),
    "zigzag_odd": np.concatenate([np.tile(np.array([1, 0], np.int32), 500), [1]]).astype(np.int32),
    "extremes": np.array([I32.max, I32.min, I32.max, I32.min, 0, I32.min, I32.max], np.int32),
    "i64_range": np.array([I64.max, I64.min, -1, 0, I64.max, I64.min, 1], np.int64),
}


@pytest.mark.parametrize("name", sorted(EDGE))
@pytest.mark.parametrize("k", [2, 4])
def test_edge_cases(name, k):
    keys = EDGE[name]
    pay = np.arange(keys.size, dtype=np.uint32)
    sk, sp, tr = oracle.sort(keys, pay, k=k)
    assert np.array_equal(sp, stable_order(keys))
    check_runs(keys, tr.run_start, tr.run_desc)
    check_tree_invariants(tr, k)
    if name == "strict_desc":
        assert tr.r == 1 and tr.run_desc[0] == 1
    if name == "zigzag":
        assert tr.r == keys.size // 2 and np.all(tr.run_desc == 1)
    if name in ("all_equal", "ascending"):
        assert tr.r == 1 and tr.merge_cost == 0


# ---------------------------------------------------------------- minimal run length

def check_min_runs(keys, rs, rd, m):
    """The partition Appendix A.3's scan must produce, stated as properties of
    the input: runs longer than m are maximal natural runs from their start;
    runs of exactly m (or the shorter last one) are not: the natural run from
    their start ends inside them, or exactly at their end; desc flags mark the
    runs that are strictly decreasing as they stand in the input."""
    n = keys.size
    rs = rs.astype(np.int64)
    assert rs[0] == 0 and rs[-1] == n
    r = rs.size - 1
    for i in range(r):
        s, e = int(rs[i]), int(rs[i + 1])
        L = e - s
        assert L >= 1
        if L < m:
            assert e == n                          # only the tail may stay short
        seg = keys[s:e]
        down = L >= 2 and bool(np.all(lt(seg[1:], seg[:-1])))
        up = not np.any(lt(seg[1:], seg[:-1]))
        assert rd[i] == (1 if down else 0)
        if L > m:                                  # a natural run, maximal
            assert up or down
            if e < n:
                if down:
                    assert not lt(keys[e:e + 1], keys[e - 1:e])[0]
                else:
                    assert lt(keys[e:e + 1], keys[e - 1:e])[0]
        elif e < n and (up or down) and L >= 2:    # natural over [s, e): must stop at e
            if down:
                assert not lt(keys[e:e + 1], keys[e - 1:e])[0]
            else:
                assert lt(keys[e:e + 1], keys[e - 1:e])[0]


def test_min_run_worked_example():
    """Worked by hand, minimal run length 4 (Appendix A.3's scan):
    5 3 | 8 9 ...: the natural run from 0 is (5, 3), decreasing, length 2 < 4,
    so the run is [0, 4), sorted to 3 5 8 9.  From 4: 2 2 7 is weakly
    increasing (1 breaks it), length 3 < 4: run [4, 8) = 1 2 2 7.  From 8:
    0 4 6 6 (5 breaks it), length 4: a natural run [8, 12), not extended.
    From 12: the single 5, which cannot be extended past the end."""
    keys = np.array([5, 3, 8, 9, 2, 2, 7, 1, 0, 4, 6, 6, 5], np.int32)
    rs, rd = oracle.runs(keys, min_run=4)
    assert rs.tolist() == [0, 4, 8, 12, 13]
    assert rd.tolist() == [0, 0, 0, 0]
    pay = np.arange(keys.size, dtype=np.uint32)
    sk, sp, tr = oracle.sort(keys, pay, k=4, min_run=4)
    assert sp.tolist() == stable_order(keys).tolist()
    assert tr.run_start.tolist() == [0, 4, 8, 12, 13]
    # natural runs of the same input, for contrast: (5 3)(8 9)(2 2 7)(1 0)(4 6 6)(5)
    assert oracle.runs(keys)[0].tolist() == [0, 2, 4, 7, 9, 12, 13]


@pytest.mark.parametrize("n", range(1, 7))
def test_min_run_bruteforce_all_tie_patterns(n):
    """Every tie pattern of length n, minimal run lengths 2..4 and 8: the
    partition has the properties of Appendix A.3's scan, the output is the
    unique stable sort and the tree over the partition keeps every Section 3
    invariant."""
    rows = weak_orderings(n)
    for m in (2, 3, 4, 8):
        for row in rows:
            rs, rd = oracle.runs(row, min_run=m)
            check_min_runs(row, rs, rd, m)
            sk, sp, tr = oracle.sort(row, np.arange(n, dtype=np.uint32), k=4, min_run=m)
            assert np.array_equal(sp, stable_order(row))
            assert np.array_equal(tr.run_start, rs) and np.array_equal(tr.run_desc, rd)
            check_tree_invariants(tr, 4)


def test_min_run_random_small_alphabets():
    """Longer inputs over 2-4 values (many ties, many short runs): the same
    properties for minimal run lengths 2..6."""
    rng = np.random.default_rng(14)
    for _ in range(300):
        n = int(rng.integers(20, 80))
        row = rng.integers(0, int(rng.integers(2, 5)), size=n).astype(np.int32)
        m = int(rng.integers(2, 7))
        rs, rd = oracle.runs(row, min_run=m)
        check_min_runs(row, rs, rd, m)
        sk, sp, tr = oracle.sort(row, np.arange(n, dtype=np.uint32), k=4, min_run=m)
        assert np.array_equal(sp, stable_order(row))
        check_tree_invariants(tr, 4)


def test_min_run_one_is_natural():
    rng = np.random.default_rng(11)
    for _ in range(20):
        keys = rng.integers(0, 6, size=int(rng.integers(1, 300))).astype(np.int32)
        rs0, rd0 = oracle.runs(keys)
        rs1, rd1 = oracle.runs(keys, min_run=1)
        assert np.array_equal(rs0, rs1) and np.array_equal(rd0, rd1)
        a = oracle.sort(keys, None, k=4)
        b = oracle.sort(keys, None, k=4, min_run=1)
        assert np.array_equal(a[0], b[0]) and a[2].merge_cost == b[2].merge_cost


@pytest.mark.parametrize("m", [3, 5, 24])
def test_min_run_zigzag_closed_form(m):
    """Every natural run of an alternating input has length 2, so every run
    from any start is shorter than m >= 3: the runs start at 0, m, 2m, ..."""
    keys = np.tile(np.array([1, 0], np.int32), 500)
    rs, rd = oracle.runs(keys, min_run=m)
    want = list(range(0, keys.size, m)) + [keys.size]
    assert rs.tolist() == want and not rd.any()
    rs2, rd2 = oracle.runs(keys, min_run=2)        # length-2 runs are not extended
    assert rs2.tolist() == list(range(0, keys.size + 1, 2)) and rd2.all()


def test_min_run_covering_everything_is_insertion_sort():
    rng = np.random.default_rng(12)
    for n in (1, 5, 17, 40):
        keys = rng.integers(-3, 3, size=n).astype(np.int64)
        pay = np.arange(n, dtype=np.uint32)
        sk, sp, tr = oracle.sort(keys, pay, k=4, min_run=n + 3)
        assert tr.r == 1 and tr.merge_cost == 0
        assert np.array_equal(sp, stable_order(keys))


def test_min_run_long_natural_runs_unchanged():
    """Natural runs of length >= m are never extended: the partition is the
    natural one."""
    rng = np.random.default_rng(13)
    m = 24
    for _ in range(10):
        lens = rng.integers(m, 4 * m, size=40)
        # increasing segments in a high band, decreasing ones in a low band:
        # every segment edge breaks the run before it, so each segment is
        # exactly one natural run
        parts = [10 ** 6 + np.arange(L) if j % 2 == 0 else np.arange(L, 0, -1)
                 for j, L in enumerate(lens)]
        keys = np.concatenate(parts).astype(np.int64)
        nat = oracle.runs(keys)[0]
        assert np.array_equal(nat, starts_from_lengths(lens))
        assert np.array_equal(oracle.runs(keys, min_run=m)[0], nat)


@pytest.mark.parametrize("name,n", [("perm_i64", 1 << 16), ("runs_i32", 1 << 17),
                                    ("ties_i32", 1 << 17)])
def test_min_run_matches_library_stable_sort(name, n):
    keys, _ = getattr(workloads, name)(n=n)
    pay = np.arange(n, dtype=np.uint32)
    sk, sp, tr = oracle.sort(keys, pay, k=4, min_run=24)
    assert np.array_equal(sp, stable_order(keys))
    assert np.array_equal(sk, keys[stable_order(keys)])
    check_tree_invariants(tr, 4)
    if name == "perm_i64":          # natural runs have mean length ~2.5: nearly every run is 24
        lens = np.diff(tr.run_start.astype(np.int64))
        assert np.mean(lens[:-1] == 24) > 0.99


# ---------------------------------------------------------------- merge-down final phase

def spine_boundaries(power):
    """Boundaries i (1-based) whose power is <= every power to their right."""
    out, m = [], 10 ** 9
    for i in range(len(power), 0, -1):
        if power[i - 1] <= m:
            out.append(i)
            m = power[i - 1]
    return out[::-1]


def node_rows(nodes):
    return sorted((int(v["begin"]), int(v["end"]), int(v["first_boundary"]), int(v["arity"]))
                  for v in nodes)


@pytest.mark.parametrize("k", [3, 4, 5, 8])
def test_merge_down_properties(k):
    """Appendix A.3's final phase on random run partitions: the merge cost is
    never above the pure tree's (the appendix states it can only go down);
    nodes that do not end at n are the pure tree's; the nodes that end at n
    split the array exactly at the weak suffix minima of the powers (the
    boundaries left on the stack), every one of them k-way except the
    smallest, which takes the remaining s mod (k-1) entries."""
    rng = np.random.default_rng(100 + k)
    lower = 0
    for _ in range(400):
        r = int(rng.integers(2, 120))
        lens = rng.integers(1, int(rng.choice([3, 50, 5000])), size=r)
        rs = starts_from_lengths(lens)
        n = int(rs[-1])
        pure = oracle.tree_from_runs(rs, k)
        md = oracle.tree_from_runs(rs, k, merge_down=True)
        assert md.merge_cost <= pure.merge_cost
        lower += md.merge_cost < pure.merge_cost
        off_p = [x for x in node_rows(pure.nodes) if x[1] != n]
        off_m = [x for x in node_rows(md.nodes) if x[1] != n]
        assert off_p == off_m
        spine = [x for x in node_rows(md.nodes) if x[1] == n]
        sp = spine_boundaries(pure.power.tolist())
        s = len(sp)
        spine_ids = {i for i, v in enumerate(md.nodes) if int(v["end"]) == n}
        owned = [b for b in range(1, r) if int(md.boundary_node[b - 1]) in spine_ids]
        assert owned == sp
        arities = sorted((x[1] - x[0], x[3]) for x in spine)      # smallest span first
        e = s % (k - 1)
        want = ([e + 1] if e else []) + [k] * ((s - e) // (k - 1))
        assert [a for _, a in arities] == want
    assert lower > 0          # the variant does change some trees


def test_merge_down_binary_is_pure():
    """With k = 2 every merge is 2-way in both final phases: the same tree."""
    rng = np.random.default_rng(120)
    for _ in range(200):
        rs = starts_from_lengths(rng.integers(1, 40, size=int(rng.integers(2, 80))))
        a, b = oracle.tree_from_runs(rs, 2), oracle.tree_from_runs(rs, 2, merge_down=True)
        assert node_rows(a.nodes) == node_rows(b.nodes) and a.merge_cost == b.merge_cost


@pytest.mark.parametrize("name,n", [("runs_i32", 1 << 16), ("perm_i64", 1 << 14),
                                    ("ties_i32", 1 << 16)])
def test_merge_down_sort_is_stable_sort(name, n):
    keys, _ = getattr(workloads, name)(n=n)
    pay = np.arange(n, dtype=np.uint32)
    for k in (2, 4, 8):
        sk, sp, tr = oracle.sort(keys, pay, k=k, merge_down=True)
        assert np.array_equal(sp, stable_order(keys))
        pure = oracle.sort(keys, pay, k=k)[2]
        assert tr.merge_cost <= pure.merge_cost


@pytest.mark.parametrize("k", [3, 4, 8])
def test_merge_down_is_kway_tree_of_regrouped_powers(k):
    """An independent construction of the merge-down tree: Algorithm 1 over
    the powers in which every group of spine boundaries (taken from the right,
    s mod (k-1) first, then k-1 at a time) carries the power of its leftmost
    boundary.  Spine powers rise weakly to the right with at most k-1 equal in
    a row (Fact 3.2), so these groups are exactly Algorithm 1's equal-power
    groups; it must give the stack's merge-down tree node for node."""
    rng = np.random.default_rng(130 + k)
    for _ in range(300):
        r = int(rng.integers(2, 150))
        lens = rng.integers(1, int(rng.choice([3, 40, 4000])), size=r)
        rs = starts_from_lengths(lens)
        pw = oracle.tree_from_runs(rs, k).power.tolist()
        sp = spine_boundaries(pw)[::-1]                 # rightmost first
        v = list(pw)
        at, length = 0, len(sp) % (k - 1)
        while at < len(sp):
            if length:
                lead = pw[sp[at + length - 1] - 1]
                for b in sp[at:at + length]:
                    v[b - 1] = lead
                at += length
            length = k - 1
        alg1 = oracle.kway_tree(rs, np.array(v, dtype=np.uint8))
        md = oracle.tree_from_runs(rs, k, merge_down=True)
        rows = lambda nodes: sorted((int(x["begin"]), int(x["end"]), int(x["first_boundary"]),
                                     int(x["arity"]), int(x["power"]), int(x["depth"]))
                                    for x in nodes)
        assert rows(alg1) == rows(md.nodes)
