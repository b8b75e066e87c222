"""GPU tests of the error path and of workspace safety.

- A device-side check that fails reaches the caller without a trace: through
  mps_sort_status (C ABI), the binding's check=True, and the caller's device
  error word (mps_opts.error_out).  The failure is forced from the host
  (MPS_OPT_TEST_DEVICE_ERROR) on valid input, so every kernel runs and exits
  normally; the output is still the stable sort.
- Sorts on two streams at once use separate library-managed workspaces.
- A caller-supplied workspace filled with a byte pattern before the sort gives
  the same result as a clean one: no kernel reads scratch memory it has not
  written in the same sort (the plan is cleared by the first kernel).
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2209_06909_amd as mps  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
E_DEVICE = -6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev_arrays(keys, pay):
    kd = torch.from_numpy(np.ascontiguousarray(keys)).to(DEV)
    pd = torch.from_numpy(np.ascontiguousarray(pay).view(np.int32)).to(DEV) if pay is not None else None
    return kd, pd


def check_sorted_like_oracle(kd, pd, keys, pay, k=4, **kw):
    ok, op, _ = oracle.sort(keys, pay, k=k, **kw)
    assert np.array_equal(kd.cpu().numpy().view(np.uint8), ok.view(np.uint8))
    if pay is not None:
        assert np.array_equal(pd.cpu().numpy().view(np.uint32), op)


def test_forced_device_error_raises_with_check():
    say("[gpu] forced device error, binding check")
    keys, pay = workloads.runs_i64(n=200_003, seed=41)
    kd, pd = dev_arrays(keys, pay)
    with pytest.raises(mps.MpsError) as ei:
        mps.sort(kd, pd, test_device_error=True)
    assert ei.value.code == E_DEVICE
    torch.cuda.synchronize()
    check_sorted_like_oracle(kd, pd, keys, pay)       # every kernel ran normally
    # the next sort on the same workspace starts with a clean error word
    kd, pd = dev_arrays(keys, pay)
    mps.sort(kd, pd)
    check_sorted_like_oracle(kd, pd, keys, pay)


def test_forced_device_error_through_c_abi_status():
    """mps_sort_ex with the library-managed workspace, then mps_sort_status on the
    same stream: MPS_E_DEVICE, then MPS_OK after a clean sort."""
    say("[gpu] forced device error, mps_sort_status")
    lib = mps.lib()
    keys, pay = workloads.runs_i32(n=150_001, seed=42)
    kd, pd = dev_arrays(keys, pay)
    s = torch.cuda.current_stream()
    sp = ctypes.c_void_p(s.cuda_stream)
    opts = mps._Opts(k=4, flags=mps.OPT_TEST_DEVICE_ERROR)
    assert lib.mps_sort_ex(ctypes.c_void_p(kd.data_ptr()), mps.KEY_I32, ctypes.c_void_p(pd.data_ptr()),
                           kd.numel(), ctypes.byref(opts), None, sp) == 0
    assert lib.mps_sort_status(None, sp) == E_DEVICE
    assert b"error word" in lib.mps_last_error()
    check_sorted_like_oracle(kd, pd, keys, pay)
    kd, pd = dev_arrays(keys, pay)
    assert lib.mps_sort(ctypes.c_void_p(kd.data_ptr()), mps.KEY_I32, ctypes.c_void_p(pd.data_ptr()),
                        kd.numel(), sp) == 0
    assert lib.mps_sort_status(None, sp) == 0
    check_sorted_like_oracle(kd, pd, keys, pay)


def test_error_word_is_sticky_and_async():
    """mps_opts.error_out: no synchronisation by the library; the word collects
    the forced bit and stays 0 for clean sorts (also through graph replays)."""
    say("[gpu] error_out word")
    keys, pay = workloads.ties_i32(n=120_007, seed=43)
    word = torch.zeros(1, dtype=torch.int32, device=DEV)
    kd, pd = dev_arrays(keys, pay)
    mps.sort(kd, pd, check=False, error_out=word)
    torch.cuda.synchronize()
    assert int(word.item()) == 0
    check_sorted_like_oracle(kd, pd, keys, pay)
    kd, pd = dev_arrays(keys, pay)
    mps.sort(kd, pd, check=False, error_out=word, test_device_error=True)
    torch.cuda.synchronize()
    assert int(word.item()) & (1 << 30)
    check_sorted_like_oracle(kd, pd, keys, pay)
    # graph replays: clean replays leave a cleared word at 0
    word.zero_()
    kg, pg = dev_arrays(keys, pay)
    for rep in range(3):
        kg.copy_(torch.from_numpy(keys).to(DEV))
        pg.copy_(torch.from_numpy(pay.view(np.int32)).to(DEV))
        mps.sort(kg, pg, graph=True, check=False, error_out=word)
        torch.cuda.synchronize()
        assert int(word.item()) == 0, rep
        check_sorted_like_oracle(kg, pg, keys, pay)


def test_forced_device_error_batched():
    say("[gpu] forced device error, batched")
    keys, pay, off = workloads.batch_i32(m=40, lo_exp=8.0, hi_exp=14.0, seed=44)
    kd, pd = dev_arrays(keys, pay)
    od = torch.from_numpy(off.view(np.int64)).to(DEV)
    with pytest.raises(mps.MpsError) as ei:
        mps.sort_batched(kd, pd, od, test_device_error=True)
    assert ei.value.code == E_DEVICE
    kd, pd = dev_arrays(keys, pay)
    mps.sort_batched(kd, pd, od)                   # clean: no error
    gk, gp = kd.cpu().numpy(), pd.cpu().numpy().view(np.uint32)
    for i in range(0, 40, 7):
        a, b = int(off[i]), int(off[i + 1])
        ok, op, _ = oracle.sort(keys[a:b], pay[a:b], k=4)
        assert np.array_equal(gk[a:b], ok) and np.array_equal(gp[a:b], op)


def test_two_streams_library_workspaces():
    """Sorts enqueued on two streams at once, each with the library-managed
    workspace of its stream (C ABI, workspace NULL), both come out right."""
    say("[gpu] two streams, library workspaces")
    lib = mps.lib()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ins = [workloads.runs_i64(n=(1 << 21) + 5, seed=45), workloads.ties_i32(n=(1 << 21) + 9, seed=46)]
    devs = [dev_arrays(k, p) for k, p in ins]
    torch.cuda.synchronize()
    kts = [mps.KEY_I64, mps.KEY_I32]
    for rep in range(3):
        for (kd, pd), (k, p) in zip(devs, ins):
            kd.copy_(torch.from_numpy(k).to(DEV))
            pd.copy_(torch.from_numpy(p.view(np.int32)).to(DEV))
        torch.cuda.synchronize()
        for (kd, pd), kt, s in zip(devs, kts, (s1, s2)):
            assert lib.mps_sort(ctypes.c_void_p(kd.data_ptr()), kt, ctypes.c_void_p(pd.data_ptr()),
                                kd.numel(), ctypes.c_void_p(s.cuda_stream)) == 0
        for s in (s1, s2):
            assert lib.mps_sort_status(None, ctypes.c_void_p(s.cuda_stream)) == 0
        for (kd, pd), (k, p) in zip(devs, ins):
            check_sorted_like_oracle(kd, pd, k, p)


def test_two_streams_binding_workspaces():
    """The binding keys its workspaces by (device, stream): two streams sorting at
    once, without waiting for each other."""
    say("[gpu] two streams, binding workspaces")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ins = [workloads.runs_i32(n=(1 << 20) + 3, seed=47), workloads.perm_i64(n=(1 << 20) + 1, seed=48)]
    devs = [dev_arrays(k, p) for k, p in ins]
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        mps.sort(*devs[0], check=False)
    with torch.cuda.stream(s2):
        mps.sort(*devs[1], check=False)
    mps.check_last(DEV, s1)
    mps.check_last(DEV, s2)
    for (kd, pd), (k, p) in zip(devs, ins):
        check_sorted_like_oracle(kd, pd, k, p)


POISON_CASES = [
    ("runs_i64", 300_007, dict(k=4)),
    ("perm_i64", 200_003, dict(k=8)),
    ("ties_i32", 250_001, dict(k=2)),
    ("runs_i32", 180_001, dict(k=4, min_run=24)),
    ("perm_i64", 220_001, dict(k=4, merge_down=True)),
]


@pytest.mark.parametrize("byte", [0x00, 0xFF, 0xA5])
@pytest.mark.parametrize("name,n,kw", POISON_CASES)
def test_poisoned_workspace(name, n, kw, byte):
    """Parity with the oracle on a caller-supplied workspace filled with a byte
    pattern before every sort (the C ABI, twice in a row on the same buffer)."""
    say(f"[gpu] poisoned workspace {name} n={n} {kw} byte={byte:#x}")
    lib = mps.lib()
    keys, pay = workloads.WORKLOADS[name](n=n, seed=49 + n % 13)
    kt = mps.KEY_I64 if keys.dtype == np.int64 else mps.KEY_I32
    k = kw.get("k", 4)
    need = lib.mps_workspace_bytes(n, 1, kt, 1, k)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=DEV)
    flags = mps.OPT_MERGE_DOWN if kw.get("merge_down") else 0
    opts = mps._Opts(k=k, flags=flags, workspace=ws.data_ptr(), workspace_bytes=ws.numel(),
                     min_run=kw.get("min_run", 1))
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    okw = {kk: v for kk, v in kw.items() if kk != "k"}
    ok, op, _ = oracle.sort(keys, pay, k=k, **okw)
    for rep in range(2):
        ws.fill_(byte)
        kd, pd = dev_arrays(keys, pay)
        assert lib.mps_sort_ex(ctypes.c_void_p(kd.data_ptr()), kt, ctypes.c_void_p(pd.data_ptr()), n,
                               ctypes.byref(opts), None, sp) == 0
        assert lib.mps_sort_status(ctypes.c_void_p(ws.data_ptr()), sp) == 0
        assert np.array_equal(kd.cpu().numpy(), ok)
        assert np.array_equal(pd.cpu().numpy().view(np.uint32), op)


@pytest.mark.parametrize("byte", [0x00, 0xFF, 0xA5])
def test_poisoned_workspace_batched(byte):
    say(f"[gpu] poisoned workspace batched byte={byte:#x}")
    lib = mps.lib()
    keys, pay, off = workloads.batch_i32(m=64, lo_exp=8.0, hi_exp=16.0, seed=50)
    n, m = keys.size, 64
    need = lib.mps_workspace_bytes(n, m, mps.KEY_I32, 1, 4)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=DEV)
    ws.fill_(byte)
    opts = mps._Opts(k=4, workspace=ws.data_ptr(), workspace_bytes=ws.numel())
    kd, pd = dev_arrays(keys, pay)
    od = torch.from_numpy(off.view(np.int64)).to(DEV)
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.mps_sort_batched(ctypes.c_void_p(kd.data_ptr()), mps.KEY_I32, ctypes.c_void_p(pd.data_ptr()),
                                ctypes.c_void_p(od.data_ptr()), None, m, n, ctypes.byref(opts), None,
                                sp) == 0
    assert lib.mps_sort_status(ctypes.c_void_p(ws.data_ptr()), sp) == 0
    gk, gp = kd.cpu().numpy(), pd.cpu().numpy().view(np.uint32)
    ok, op = oracle.sort_many(keys, pay, off, k=4)[:2]
    assert np.array_equal(gk, ok) and np.array_equal(gp, op)
