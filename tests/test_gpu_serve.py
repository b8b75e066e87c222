"""GPU tests of the continuous-batching server (mps_serve_*): every served
result is bit-identical to the same request sorted alone (and to the oracle on
samples), batches overlap while requests keep arriving, admission respects the
HBM budget, and host-forced failures and shutdown behave as documented.
"""
import ctypes
import sys
import time

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


def mixed_requests(seed, count, lo, hi):
    """float32 serving-style requests plus a few int32 / int64 ones (other batches)."""
    pool = workloads.serve_pool_device(count=count, seed=seed, lo_exp=lo, hi_exp=hi, device=DEV)
    out = [(x, p) for x, p in pool]
    rng = np.random.default_rng(seed)
    for i in range(4):
        n = int(rng.integers(1000, 60000))
        k32, p32 = workloads.runs_i32(n=n, seed=seed * 10 + i)
        out.insert(3 * i + 1, (torch.from_numpy(k32).to(DEV),
                               torch.from_numpy(p32.view(np.int32)).to(DEV)))
    k64, p64 = workloads.runs_i64(n=50000, seed=seed)
    out.append((torch.from_numpy(k64).to(DEV), torch.from_numpy(p64.view(np.int32)).to(DEV)))
    return out


def alone(keys, pay):
    k, p = keys.clone(), pay.clone()
    mps.sort(k, p)
    torch.cuda.synchronize()
    return k.cpu().numpy(), p.cpu().numpy()


def test_serve_alone_vs_mix():
    say("[gpu] serve alone vs mix")
    reqs = mixed_requests(11, 24, 8.0, 17.0)
    outs = [(torch.empty_like(k), torch.empty_like(p)) for k, p in reqs]
    with mps.Server(hbm_budget_bytes=2 << 30, n_streams=3, max_batch=8) as srv:
        ids = [srv.submit(k, p, ko, po) for (k, p), (ko, po) in zip(reqs, outs)]
        infos = [srv.wait(i, timeout=60) for i in ids]
        st = srv.stats()
    assert st["batches"] >= 4        # max_batch 8 and three key types force several batches
    for (k, p), (ko, po) in zip(reqs, outs):
        ak, ap = alone(k, p)
        assert np.array_equal(ko.cpu().numpy().view(np.uint8), ak.view(np.uint8))
        assert np.array_equal(po.cpu().numpy(), ap)
    # inputs untouched (out of place)
    for idx in (0, 5, len(reqs) - 1):
        k, p = reqs[idx]
        ok_, op_, _ = oracle.sort(k.cpu().numpy(), p.cpu().numpy().view(np.uint32), k=4)
        assert np.array_equal(outs[idx][0].cpu().numpy().view(np.uint8), ok_.view(np.uint8))
        assert np.array_equal(outs[idx][1].cpu().numpy().view(np.uint32), op_)
    assert all(i["t_done_ns"] >= i["t_admit_ns"] >= i["t_submit_ns"] > 0 for i in infos)


def test_serve_continuous_batching_overlaps():
    """Requests submitted while earlier batches are still running are admitted
    before those batches finish (their batches overlap on the device)."""
    say("[gpu] serve overlap")
    pool = workloads.serve_pool_device(count=12, seed=12, lo_exp=20.0, hi_exp=22.0, device=DEV)
    with mps.Server(hbm_budget_bytes=8 << 30, n_streams=4, max_batch=2) as srv:
        ids = []
        for x, p in pool:
            ids.append(srv.submit(x, p, torch.empty_like(x), torch.empty_like(p)))
            time.sleep(0.0005)
        infos = [srv.wait(i, timeout=60) for i in ids]
    batches = {}
    for inf in infos:
        b = batches.setdefault(inf["batch"], [inf["t_admit_ns"], inf["t_done_ns"]])
        b[1] = max(b[1], inf["t_done_ns"])
    spans = sorted(batches.values())
    overlapping = sum(1 for a, b in zip(spans, spans[1:]) if b[0] < a[1])
    assert len(spans) >= 6 and overlapping >= 1


def test_serve_budget_and_bad_requests():
    say("[gpu] serve budget")
    x = torch.from_numpy(np.arange(1 << 16, dtype=np.int32)[::-1].copy()).to(DEV)
    need_one = mps.workspace_bytes(1 << 16, 1, mps.KEY_I32, False, 4) + (1 << 16) * 4
    budget = 2 * need_one + (4 << 20)
    with mps.Server(hbm_budget_bytes=budget, n_streams=4, max_batch=64) as srv:
        big = torch.zeros(1 << 22, dtype=torch.int32, device=DEV)
        with pytest.raises(mps.MpsError) as e:
            srv.submit(big)                       # more than the whole budget
        assert e.value.code == -2
        with pytest.raises(mps.MpsError) as e:
            srv.poll(12345)
        assert e.value.code == -5
        ins = [x.clone() for _ in range(10)]
        outs = [torch.empty_like(t) for t in ins]
        ids = [srv.submit(a, None, b) for a, b in zip(ins, outs)]
        st = srv.stats()
        assert st["arena_used"] <= st["arena_bytes"]
        for i in ids:
            srv.wait(i, timeout=60)
        with pytest.raises(mps.MpsError):
            srv.release(999999)
        srv.release(ids[0])
        with pytest.raises(mps.MpsError):
            srv.poll(ids[0])
    want = np.arange(1 << 16, dtype=np.int32)
    for b in outs:
        assert np.array_equal(b.cpu().numpy(), want)
    # argument errors through the C ABI
    lib = mps.lib()
    h = ctypes.c_void_p()
    cfg = mps._ServeCfg(hbm_budget_bytes=1 << 10)
    assert lib.mps_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == -1     # budget < 1 MiB
    cfg = mps._ServeCfg(hbm_budget_bytes=64 << 20, k=3)
    assert lib.mps_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == -4
    cfg = mps._ServeCfg(hbm_budget_bytes=64 << 20)
    assert lib.mps_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
    rid = ctypes.c_uint64()
    r = mps._Request(keys=None, keys_out=None, n=10, kt=0)
    assert lib.mps_serve_submit(h, ctypes.byref(r), ctypes.byref(rid)) == -1
    r = mps._Request(keys=x.data_ptr(), keys_out=x.data_ptr(), payload=x.data_ptr(), n=10, kt=0)
    assert lib.mps_serve_submit(h, ctypes.byref(r), ctypes.byref(rid)) == -1   # payload_out missing
    assert lib.mps_serve_destroy(h) == 0


def test_serve_forced_failures_do_not_stop_service():
    """fail_every=2 fails every second batch on the host before anything is
    enqueued: its requests report MPS_E_HIP, the others are correct, and the
    server keeps serving."""
    say("[gpu] serve forced failures")
    reqs = [workloads.runs_i32(n=20000 + 1000 * i, seed=70 + i) for i in range(8)]
    dev = [(torch.from_numpy(k).to(DEV), torch.from_numpy(p.view(np.int32)).to(DEV)) for k, p in reqs]
    outs = [(torch.empty_like(k), torch.empty_like(p)) for k, p in dev]
    with mps.Server(hbm_budget_bytes=1 << 30, n_streams=1, max_batch=1, fail_every=2) as srv:
        ids = [srv.submit(k, p, ko, po) for (k, p), (ko, po) in zip(dev, outs)]
        results = []
        for i in ids:
            while True:
                try:
                    rc, info = srv.poll(i)
                except mps.MpsError as e:
                    results.append(e.code)
                    break
                if rc == 0:
                    results.append(0)
                    break
                time.sleep(1e-4)
    assert results.count(-3) == 4 and results.count(0) == 4
    for (k, p), (ko, po), rc in zip(reqs, outs, results):
        if rc == 0:
            ok_, op_, _ = oracle.sort(k, p, k=4)
            assert np.array_equal(ko.cpu().numpy(), ok_)
            assert np.array_equal(po.cpu().numpy().view(np.uint32), op_)


def test_serve_destroy_drains():
    say("[gpu] serve destroy drains")
    reqs = [workloads.runs_i64(n=30000 + 777 * i, seed=90 + i) for i in range(6)]
    dev = [(torch.from_numpy(k).to(DEV), torch.from_numpy(p.view(np.int32)).to(DEV)) for k, p in reqs]
    srv = mps.Server(hbm_budget_bytes=1 << 30, n_streams=2, max_batch=2)
    for k, p in dev:
        srv.submit(k, p)                   # in place
    srv.close()                            # returns after every request finished
    torch.cuda.synchronize()
    for (k0, p0), (k, p) in zip(reqs, dev):
        ok_, op_, _ = oracle.sort(k0, p0, k=4)
        assert np.array_equal(k.cpu().numpy(), ok_)
        assert np.array_equal(p.cpu().numpy().view(np.uint32), op_)


def test_serve_large_f32_alone_vs_mix():
    """Served float32 requests from the top of the serving size range (2^22 to 2^26
    keys, normal values with about 1% duplicated keys, random runs) mixed with
    small ones: every result equals the request sorted alone, and the large ones
    equal the oracle bit for bit (keys and payload permutation)."""
    say("[gpu] serve large f32 alone vs mix")
    rng = np.random.default_rng(61)
    sizes = [1 << 22, int(2 ** 23.4), int(2 ** 24.7), 1 << 26, 1500, 9000, 70000, 1 << 14]
    host = [workloads.serve_request_f32(s, rng) for s in sizes]
    reqs = [(torch.from_numpy(x).to(DEV), torch.from_numpy(p.view(np.int32)).to(DEV)) for x, p in host]
    outs = [(torch.empty_like(k), torch.empty_like(p)) for k, p in reqs]
    with mps.Server(hbm_budget_bytes=16 << 30, n_streams=3, max_batch=4) as srv:
        ids = []
        for i, ((k, p), (ko, po)) in enumerate(zip(reqs, outs)):
            ids.append(srv.submit(k, p, ko, po))
            if i % 3 == 2:
                time.sleep(0.002)                 # later requests arrive while batches run
        for i in ids:
            srv.wait(i, timeout=120)
    for (k, p), (ko, po) in zip(reqs, outs):
        ak, ap = alone(k, p)
        assert np.array_equal(ko.cpu().numpy().view(np.uint8), ak.view(np.uint8))
        assert np.array_equal(po.cpu().numpy(), ap)
    for idx in range(4):
        x, p = host[idx]
        ok_, op_, _ = oracle.sort(x, p, k=4)
        say(f"[gpu]   oracle check of request {idx} ({x.size} keys)")
        assert np.array_equal(outs[idx][0].cpu().numpy().view(np.uint8), ok_.view(np.uint8))
        assert np.array_equal(outs[idx][1].cpu().numpy().view(np.uint32), op_)
