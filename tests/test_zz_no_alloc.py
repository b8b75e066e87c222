"""GPU test of the allocation-free entry point, mps_sort_noalloc, through the C ABI.

Its workspace is the library's fixed device scratch.  Each call's output must be
bit-identical to mps_sort_ex (the same sort with a library-managed workspace) on a
copy of the same input, for two calls in a row on one device, the second with a
smaller input (the scratch still holds the first call's contents then).
"""
import ctypes
import sys

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
import paper_2209_06909_amd as mps  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(keys, pay):
    kd = torch.from_numpy(np.ascontiguousarray(keys)).to(DEV)
    pd = torch.from_numpy(np.ascontiguousarray(pay).view(np.int32)).to(DEV) if pay is not None else None
    return kd, pd


def ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def sort_both(keys, pay, kt, opts_kw):
    """Sort one copy with mps_sort_noalloc and one with mps_sort_ex; return both."""
    lib = mps.lib()
    s = torch.cuda.current_stream()
    sp = ctypes.c_void_p(s.cuda_stream)
    ka, pa = to_dev(keys, pay)
    kb, pb = to_dev(keys, pay)
    err = torch.zeros(1, dtype=torch.int32, device=DEV)
    o1 = mps._Opts(error_out=err.data_ptr(), **opts_kw)
    rc = lib.mps_sort_noalloc(ptr(ka), kt, ptr(pa), ka.numel(), ctypes.byref(o1), sp)
    assert rc == 0, lib.mps_last_error()
    o2 = mps._Opts(**opts_kw)
    rc = lib.mps_sort_ex(ptr(kb), kt, ptr(pb), kb.numel(), ctypes.byref(o2), None, sp)
    assert rc == 0, lib.mps_last_error()
    assert lib.mps_sort_status(None, sp) == 0, lib.mps_last_error()
    torch.cuda.synchronize()
    assert int(err.item()) == 0, "device-side check failed in mps_sort_noalloc"
    return (ka, pa), (kb, pb)


def assert_same(a, b):
    (ka, pa), (kb, pb) = a, b
    assert torch.equal(ka.view(torch.uint8) if ka.dtype == torch.float32 else ka,
                       kb.view(torch.uint8) if kb.dtype == torch.float32 else kb)
    if pa is not None:
        assert torch.equal(pa, pb)


CASES = [
    # (name, generator, key type, first n, second n, options)
    ("i64_payload_k4", workloads.runs_i64, mps.KEY_I64, 1_000_003, 65_537, dict(k=4)),
    ("i32_payload_k8", workloads.runs_i32, mps.KEY_I32, 1_200_001, 3_001, dict(k=8)),
    ("i32_payload_k2_minrun", workloads.runs_i32, mps.KEY_I32, 700_001, 90_001,
     dict(k=2, min_run=24)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_sort_ex_twice(case):
    name, gen, kt, n1, n2, kw = case
    scratch = mps.noalloc_scratch_bytes()
    for call, n in enumerate((n1, n2)):
        need = mps.workspace_bytes(n, 1, kt, 1, kw.get("k", 4))
        assert 0 < need <= scratch, (n, need, scratch)
        say(f"[gpu] noalloc {name} call {call + 1}: n={n}")
        keys, pay = gen(n=n, seed=700 + 10 * call + len(name))
        a, b = sort_both(keys, pay, kt, kw)
        assert_same(a, b)
        ka = a[0].cpu().numpy()
        assert np.all(ka[:-1] <= ka[1:])


def test_noalloc_keys_only_float():
    """float32 keys without payload (the IEEE-754 total order), two calls."""
    for call, n in enumerate((900_001, 40_000)):
        say(f"[gpu] noalloc f32 keys only call {call + 1}: n={n}")
        rng = np.random.default_rng(810 + call)
        keys = rng.standard_normal(n).astype(np.float32)
        keys[::97] = -0.0
        keys[5::101] = 0.0
        a, b = sort_both(keys, None, mps.KEY_F32, dict(k=4))
        assert_same(a, b)


def test_noalloc_binding_and_limits():
    """The binding's sort_noalloc, and a request beyond the scratch: MPS_E_NOMEM
    from the host, with the scratch's contents still usable by the next call."""
    say("[gpu] noalloc binding and limit")
    scratch = mps.noalloc_scratch_bytes()
    big = 1 << 22
    assert mps.workspace_bytes(big, 1, mps.KEY_I64, 1, 4) > scratch
    kd = torch.zeros(big, dtype=torch.int64, device=DEV)
    pd = torch.zeros(big, dtype=torch.int32, device=DEV)
    with pytest.raises(mps.MpsError) as ei:
        mps.sort_noalloc(kd, pd)
    assert ei.value.code == -2
    keys, pay = workloads.runs_i64(n=300_007, seed=77)
    ka, pa = to_dev(keys, pay)
    kb, pb = to_dev(keys, pay)
    mps.sort_noalloc(ka, pa)
    mps.sort(kb, pb)
    torch.cuda.synchronize()
    assert torch.equal(ka, kb) and torch.equal(pa, pb)
