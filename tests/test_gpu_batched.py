"""GPU parity of the batching layer: merge tile configurations, the work-queue
merge kernels, HIP-graph replay and batched sorts of many uneven arrays, all
against the CPU oracle (bit-exact keys, payload permutation, runs, powers and
merge cost) or against the eager single-array path.
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


def bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


def batch_truth(keys, pay, off, k):
    """Oracle outputs and the per-array runs / powers concatenated as the batched trace
    reports them (array edges carry power 0)."""
    ok, op, omc = oracle.sort_many(keys, pay, off, k=k)
    rs_all, pw_all = [], []
    for i in range(len(off) - 1):
        s, e = int(off[i]), int(off[i + 1])
        if e == s:
            continue
        rs, _ = oracle.runs(keys[s:e])
        if rs_all:
            pw_all.append(np.zeros(1, np.uint8))
        pw_all.append(oracle.powers(rs, k))
        rs_all.append(rs[:-1] + s)
    rs_all.append(np.array([off[-1]], np.uint64))
    return ok, op, int(omc.sum()), np.concatenate(rs_all), np.concatenate(pw_all)


@pytest.mark.parametrize("tile,lane_slice", mps.TILE_CONFIGS)
@pytest.mark.parametrize("k", [4, 2, 8])
def test_tile_configs_vs_oracle(tile, lane_slice, k):
    """Every merge tile configuration on a run-structured int64 input (many tiles,
    ragged tail) and on a ties-heavy int32 input (stability)."""
    for name, n, seed in (("runs_i64", (1 << 17) + 4321, 31), ("ties_i32", (1 << 17) + 99, 32)):
        say(f"[gpu] tile {tile}/{lane_slice} k={k} {name} n={n}")
        keys, pay = workloads.WORKLOADS[name](n=n, seed=seed)
        ok, op, ot = oracle.sort(keys, pay, k=k)
        kd, pd = to_dev(keys), pay_dev(pay)
        tr = mps.sort(kd, pd, k=k, trace=True, tile=tile, lane_slice=lane_slice)
        assert np.array_equal(bits(kd.cpu().numpy()), bits(ok))
        assert np.array_equal(pd.cpu().numpy().view(np.uint32), op)
        assert np.array_equal(tr.run_start, ot.run_start)
        assert np.array_equal(tr.power, ot.power)
        assert tr.merge_cost == ot.merge_cost
        kd, pd = to_dev(keys), pay_dev(pay)     # without a trace
        mps.sort(kd, pd, k=k, tile=tile, lane_slice=lane_slice)
        assert np.array_equal(bits(kd.cpu().numpy()), bits(ok))
        assert np.array_equal(pd.cpu().numpy().view(np.uint32), op)


def test_bad_tile_config_rejected():
    kd = to_dev(np.arange(100, dtype=np.int32)[::-1].copy())
    with pytest.raises(mps.MpsError):
        mps.sort(kd, tile=1024, lane_slice=8)
    with pytest.raises(mps.MpsError):
        mps.sort(kd, tile=3000)


def uneven_batch(m, seed, lo, hi):
    keys, pay, off = workloads.batch_i32(m=m, seed=seed, lo_exp=lo, hi_exp=hi)
    return keys, pay, off


@pytest.mark.parametrize("tile,lane_slice", [(2048, 8), (1024, 4), (4096, 8)])
def test_batched_uneven_vs_oracle(tile, lane_slice):
    """Many arrays with log-uniform sizes (the batched workload's shape, scaled
    down), a few of them empty, through one batched call."""
    say(f"[gpu] batched uneven tile {tile}/{lane_slice}")
    keys, pay, off = uneven_batch(400, 41, 4.0, 16.0)
    sizes = np.diff(off.astype(np.int64))
    sizes[[3, 4, 200]] = 0
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys, pay = keys[: int(off[-1])], pay[: int(off[-1])]
    ok, op, M, rs, pw = batch_truth(keys, pay, off, 4)
    kd, pd = to_dev(keys), pay_dev(pay)
    od = torch.from_numpy(off.view(np.int64)).to(DEV)
    tr = mps.sort_batched(kd, pd, od, k=4, trace=True, host_offsets=off, tile=tile,
                          lane_slice=lane_slice)
    assert np.array_equal(kd.cpu().numpy(), ok)
    assert np.array_equal(pd.cpu().numpy().view(np.uint32), op)
    assert tr.merge_cost == M
    assert np.array_equal(tr.run_start, rs)
    assert np.array_equal(tr.power, pw)
    kd, pd = to_dev(keys), pay_dev(pay)     # without a trace; the trace fetched afterwards
    mps.sort_batched(kd, pd, od, k=4, host_offsets=off, tile=tile, lane_slice=lane_slice)
    assert np.array_equal(kd.cpu().numpy(), ok)
    assert np.array_equal(pd.cpu().numpy().view(np.uint32), op)
    lt = mps.last_trace(DEV)
    assert lt.merge_cost == M and lt.n_nodes == tr.n_nodes and lt.n_levels == tr.n_levels
    assert np.array_equal(lt.leaf_depth, tr.leaf_depth)
    assert np.array_equal(lt.node_depth, tr.node_depth)
    assert np.array_equal(lt.node_arity, tr.node_arity)


def test_graph_replay_matches_eager():
    """A graph-captured batched sort replayed on fresh copies of the input, with
    eager work and synchronisations between the replays: every replay equals the
    eager result, and so does a replay after the offsets' contents change."""
    say("[gpu] graph replay")
    keys, pay, off = uneven_batch(300, 43, 6.0, 15.0)
    kd0, pd0 = to_dev(keys), pay_dev(pay)
    od = torch.from_numpy(off.view(np.int64)).to(DEV)
    ek, ep = kd0.clone(), pd0.clone()
    mps.sort_batched(ek, ep, od, k=4)
    torch.cuda.synchronize()
    ek, ep = ek.cpu().numpy(), ep.cpu().numpy()
    kd, pd = torch.empty_like(kd0), torch.empty_like(pd0)
    for rep in range(4):
        kd.copy_(kd0)
        pd.copy_(pd0)
        mps.sort_batched(kd, pd, od, k=4, graph=True)
        junk = torch.randn(1 << 16, device=DEV).sum()       # eager work between replays
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert np.array_equal(kd.cpu().numpy(), ek), f"replay {rep}"
        assert np.array_equal(pd.cpu().numpy(), ep), f"replay {rep}"
    # same pointers and sizes, different array boundaries: the graph reads them on the device
    sizes = np.diff(off.astype(np.int64))
    perm = np.random.default_rng(5).permutation(sizes.size)
    off2 = np.concatenate([[0], np.cumsum(sizes[perm])]).astype(np.uint64)
    od.copy_(torch.from_numpy(off2.view(np.int64)))
    ok2, op2, _ = oracle.sort_many(keys, pay, off2, k=4)
    kd.copy_(kd0)
    pd.copy_(pd0)
    mps.sort_batched(kd, pd, od, k=4, graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(kd.cpu().numpy(), ok2)
    assert np.array_equal(pd.cpu().numpy().view(np.uint32), op2)


def test_graph_single_array_and_trace():
    say("[gpu] graph single")
    keys, pay = workloads.runs_i32(n=(1 << 16) + 5, seed=8)
    ok, op, ot = oracle.sort(keys, pay, k=4)
    for rep in range(3):
        kd, pd = to_dev(keys), pay_dev(pay)
        tr = mps.sort(kd, pd, k=4, graph=True, trace=(rep == 2))
        torch.cuda.synchronize()
        assert np.array_equal(kd.cpu().numpy(), ok)
        assert np.array_equal(pd.cpu().numpy().view(np.uint32), op)
        if tr is not None:
            assert np.array_equal(tr.run_start, ot.run_start)
            assert tr.merge_cost == ot.merge_cost


def test_graph_rejects_level_timing():
    kd = to_dev(np.arange(1000, dtype=np.int32))
    with pytest.raises(mps.MpsError):
        mps.sort(kd, graph=True, time_levels=True)


def test_autotune_picks_a_candidate_and_sorts():
    say("[gpu] autotune small")
    keys, pay, off = uneven_batch(200, 47, 6.0, 14.0)
    kd, pd = to_dev(keys), pay_dev(pay)
    od = torch.from_numpy(off.view(np.int64)).to(DEV)
    best = mps.autotune(kd, pd, off, sample_keys=1 << 18, graph=True, with_times=True)
    cands = best["candidates"]
    assert len(cands) == len(mps.TUNE_CANDIDATES) and all(np.isfinite(c["ms"]) and c["ms"] > 0 for c in cands)
    fastest = min(cands, key=lambda c: c["ms"])
    assert (best["k"], best["tile"], best["lane_slice"]) == (fastest["k"], fastest["tile"],
                                                             fastest["lane_slice"])
    # the input was only sampled, never modified
    assert np.array_equal(kd.cpu().numpy(), keys)
    again = mps.autotune(kd, pd, off, sample_keys=1 << 18, graph=True)   # cached
    assert (again["k"], again["tile"], again["lane_slice"]) == (best["k"], best["tile"],
                                                                best["lane_slice"])
    k = best["k"]
    ok, op, M, rs, pw = batch_truth(keys, pay, off, k)
    tr = mps.sort_batched(kd, pd, od, k=k, tile=best["tile"], lane_slice=best["lane_slice"],
                          trace=True)
    assert np.array_equal(kd.cpu().numpy(), ok)
    assert np.array_equal(pd.cpu().numpy().view(np.uint32), op)
    assert tr.merge_cost == M and np.array_equal(tr.power, pw)


def device_check_sorted_batch(k_in, k_out, p_out, off, chunk=1 << 27):
    """Properties that single out the stable sort of every array, checked with torch
    on the device chunk by chunk: non-decreasing keys, payload a permutation of the
    array's indices, every output key equal to the input key its payload names, and
    equal keys in increasing payload order."""
    m = off.size - 1
    i = 0
    while i < m:
        j, n = i, 0
        while j < m and (j == i or n + int(off[j + 1] - off[j]) <= chunk):
            n += int(off[j + 1] - off[j])
            j += 1
        s0 = int(off[i])
        if n:
            sz = torch.as_tensor((off[i + 1:j + 1] - off[i:j]).astype(np.int64), device=DEV)
            starts = torch.cumsum(sz, 0) - sz
            first = torch.zeros(n, dtype=torch.bool, device=DEV)
            first[starts[sz > 0]] = True
            ko = k_out[s0:s0 + n].to(torch.int64)
            po = p_out[s0:s0 + n].to(torch.int64)
            inner = ~first[1:]
            assert bool(((ko[1:] >= ko[:-1]) | ~inner).all())
            loc = torch.repeat_interleave(starts, sz)
            assert bool(((po >= 0) & (po < torch.repeat_interleave(sz, sz))).all())
            g = loc + po
            seen = torch.zeros(n, dtype=torch.bool, device=DEV)
            seen[g] = True
            assert bool(seen.all())
            assert bool((k_in[s0:s0 + n].to(torch.int64)[g] == ko).all())
            eq = (ko[1:] == ko[:-1]) & inner
            assert bool(((po[1:] > po[:-1]) | ~eq).all())
        i = j


def test_batched_full_size():
    """The batched workload at full size (8192 arrays, ~3.5e9 keys) in the autotuned
    graph configuration the benchmark times: every array checked by properties on the
    device, and 12 sampled arrays (the smallest, the largest and 10 seeded picks)
    bit-exact against the oracle."""
    say("[gpu] batched full size: generating")
    mps.release_workspaces()
    torch.cuda.empty_cache()
    kin, pin, off = workloads.batch_i32_device(m=8192, device=DEV)
    od = torch.from_numpy(off.view(np.int64)).to(DEV)
    best = mps.autotune(kin, pin, off, sample_keys=1 << 28, graph=True)
    say(f"[gpu] batched full size: total {int(off[-1])}, tuned {best}")
    kd, pd = kin.clone(), pin.clone()
    mps.sort_batched(kd, pd, od, graph=True, **best)
    torch.cuda.synchronize()
    say("[gpu] batched full size: device property checks")
    device_check_sorted_batch(kin, kd, pd, off)
    sizes = np.diff(off.astype(np.int64))
    pick = set(np.random.default_rng(3).choice(sizes.size, 10, replace=False).tolist())
    pick |= {int(sizes.argmin()), int(sizes.argmax())}
    say(f"[gpu] batched full size: oracle on arrays {sorted(pick)}")
    for i in sorted(pick):
        s, e = int(off[i]), int(off[i + 1])
        keys = kin[s:e].cpu().numpy()
        pay = pin[s:e].cpu().numpy().view(np.uint32)
        ok, op, _ = oracle.sort(keys, pay, k=best["k"])
        assert np.array_equal(kd[s:e].cpu().numpy(), ok), f"array {i}"
        assert np.array_equal(pd[s:e].cpu().numpy().view(np.uint32), op), f"array {i}"
    del kin, pin, kd, pd
    mps.release_workspaces()
    torch.cuda.empty_cache()


def test_batched_large_arrays_vs_oracle():
    """Arrays of 2^23 to 2^26 keys in one batch (with small ones between them):
    every array equals the oracle's sort of it alone, keys and payload."""
    say("[gpu] batched large arrays vs oracle")
    big, pb, ob = workloads.batch_i32(m=3, seed=62, lo_exp=23.0, hi_exp=26.0)
    small, ps, os_ = workloads.batch_i32(m=5, seed=63, lo_exp=8.0, hi_exp=12.0)
    keys = np.concatenate([small[: int(os_[2])], big, small[int(os_[2]):]])
    pay = np.concatenate([ps[: int(os_[2])], pb, ps[int(os_[2]):]])
    sizes = np.concatenate([np.diff(os_)[:2], np.diff(ob), np.diff(os_)[2:]]).astype(np.uint64)
    off = np.zeros(sizes.size + 1, np.uint64)
    off[1:] = np.cumsum(sizes)
    assert int(off[-1]) == keys.size and int(np.diff(ob).max()) >= 1 << 23
    kd = torch.from_numpy(keys).to(DEV)
    pd = torch.from_numpy(pay.view(np.int32)).to(DEV)
    od = torch.from_numpy(off.view(np.int64)).to(DEV)
    mps.sort_batched(kd, pd, od, host_offsets=off)
    gk, gp = kd.cpu().numpy(), pd.cpu().numpy().view(np.uint32)
    ok, op, _ = oracle.sort_many(keys, pay, off, k=4)
    assert np.array_equal(gk, ok)
    assert np.array_equal(gp, op)
