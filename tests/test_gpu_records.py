"""GPU parity for records with an 8-byte payload (mps_sort_kv64).

The stable order of the records is the oracle's: sorting the keys with an
index payload gives the stable permutation p, and the expected output
payload is the input payload taken in that order, payload[p].  Keys, the
payload and the trace (runs, powers, tree, merge cost) must match bit for
bit.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2209_06909_amd as mps  # noqa: E402

from test_gpu_parity import bits, check_stable_sort_properties, check_trace, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def payload64(n, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, np.iinfo(np.int64).max, size=n, dtype=np.int64) ^ (
        rng.integers(0, 2, size=n, dtype=np.int64) << 63)


def check_records(keys, pay64, k=4, min_run=1):
    idx = np.arange(keys.size, dtype=np.uint32)
    ok, op, ot = oracle.sort(keys, idx, k=k, min_run=min_run)
    kd = to_dev(keys)
    pd = to_dev(pay64)
    tr = mps.sort(kd, pd, k=k, trace=True, min_run=min_run)
    torch.cuda.synchronize()
    assert np.array_equal(bits(kd.cpu().numpy()), bits(ok))
    assert np.array_equal(pd.cpu().numpy(), pay64[op.astype(np.int64)])
    check_trace(tr, ot)
    kd, pd = to_dev(keys), to_dev(pay64)      # without a trace, as the benchmark runs it
    mps.sort(kd, pd, k=k, min_run=min_run)
    torch.cuda.synchronize()
    assert np.array_equal(bits(kd.cpu().numpy()), bits(ok))
    assert np.array_equal(pd.cpu().numpy(), pay64[op.astype(np.int64)])


CASES = [("runs_i64", (1 << 17) + 3), ("perm_i64", (1 << 16) + 5), ("ties_i32", (1 << 17) + 1),
         ("runs_i32", 50001)]


@pytest.mark.parametrize("k", [4, 2])
@pytest.mark.parametrize("name,n", CASES)
def test_records_vs_oracle(name, n, k):
    keys, _ = workloads.WORKLOADS[name](n=n)
    say(f"[gpu] records {name} n={n} k={k}")
    check_records(keys, payload64(n, 71), k=k)


def test_records_float_keys_and_min_run():
    rng = np.random.default_rng(72)
    keys = (rng.standard_normal(70001) * 3).astype(np.float32)
    keys[rng.integers(0, keys.size, 500)] = np.float32(-0.0)
    say("[gpu] records f32 min_run=24")
    check_records(keys, payload64(keys.size, 73), k=4, min_run=24)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 2049])
def test_records_small(n):
    rng = np.random.default_rng(n + 80)
    keys = rng.integers(-5, 5, size=n).astype(np.int64)
    pay = payload64(n, n + 81)
    kd, pd = to_dev(keys), to_dev(pay)
    mps.sort(kd, pd, k=4)
    torch.cuda.synchronize()
    perm = np.argsort(keys, kind="stable")
    assert np.array_equal(kd.cpu().numpy(), keys[perm])
    assert np.array_equal(pd.cpu().numpy(), pay[perm])


def test_records_full_size():
    """2^28 int64 keys (random runs, the headline input) with an 8-byte payload
    holding each record's index: stable-sort properties of the output."""
    n = 1 << 28
    say("[gpu] records full runs_i64: generating")
    keys, _ = workloads.WORKLOADS["runs_i64"](n=n)
    kd = to_dev(keys)
    pd = torch.arange(n, dtype=torch.int64, device="cuda:0")
    say("[gpu] records full runs_i64: sorting")
    mps.sort(kd, pd, k=4)
    torch.cuda.synchronize()
    say("[gpu] records full runs_i64: checking")
    check_stable_sort_properties(keys, kd.cpu().numpy(), pd.cpu().numpy().astype(np.int64))


def test_wide_payload_only_in_sort():
    """An 8-byte payload goes through mps_sort_kv64 only; the batched call,
    whose ABI takes a u32 payload, rejects it before any launch."""
    kd = torch.arange(100, dtype=torch.int32, device="cuda:0")
    pd = torch.arange(100, dtype=torch.int64, device="cuda:0")
    off = torch.tensor([0, 50, 100], dtype=torch.int64, device="cuda:0")
    with pytest.raises(TypeError):
        mps.sort_batched(kd, pd, off)
