#!/usr/bin/env python
"""Benchmark of the gfx950 multiway-Powersort library on one MI355X.

Workload (the single-GPU headline configuration): n = 2^28 int64 keys drawn
uniformly over the full int64 range with a uint32 index payload, laid out as
random runs whose lengths are uniform in [1, 2*sqrt(n)], each run sorted
ascending (the paper's "random runs" inputs, Section 4.3).  Synthetic and
seeded (workloads.runs_i64, seed 2).

A step is one full sort: run detection, powers, merge tree, leaf placement
and every merge level.  Before each step the input is restored from a
pristine device copy (the restore is outside the sort's own timing; the K
steps including restores are bracketed by synchronisations as a whole).

Printed: one JSON line with keys/s (whole job, one GPU), the roofline of the
dominant kernel (the level merge) from HIP events recorded by the library
around every merge launch in the timed steps, the sort-level HBM fraction,
and the CPU oracle timed on a bounded prefix of the same input.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

METRIC = "GKeys/s + % HBM roofline per sort; batched vs per-array; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
ROOT = os.path.dirname(os.path.abspath(__file__))


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the level-merge kernel sources; traffic figures measured on other
    sources are not reported."""
    h = hashlib.sha256()
    for name in ("mps_merge.h", "mps_internal.h"):
        with open(os.path.join(ROOT, "paper_2209_06909_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(tag: str):
    """HBM bytes per merged element of the level merges, from the rocprofv3
    FETCH_SIZE / WRITE_SIZE summary kept in profiles/ (calibrated against a copy
    of known size); None if the merge kernel changed since it was measured."""
    p = os.path.join(ROOT, "profiles", f"merge_traffic_{tag}.txt")
    try:
        with open(p) as f:
            kv = dict(line.split(": ", 1) for line in f.read().splitlines() if ": " in line
                      and not line.startswith(("|", "#", " ")))
    except OSError:
        return None
    if kv.get("source_hash", "").strip() != source_hash():
        return None
    return {"bytes_per_merged_element": float(kv["bytes_per_merged_element"]),
            "ratio_to_algorithmic": float(kv["ratio_to_algorithmic"])}


def _timed(fn):
    t0 = time.perf_counter()
    out = fn()
    return out, time.perf_counter() - t0


def cpu_baseline(keys: np.ndarray, pay: np.ndarray, sample_n: int, k: int, full: bool = False):
    """The oracle (single-threaded C multiway Powersort) on the host cores, beside a
    library stable sort (C++ std::stable_sort of (key, payload) records, one thread),
    on a bounded sample of the headline input; with full=True also every config at
    its own size (see cpu_full_configs)."""
    import oracle
    sk, sp = keys[:sample_n].copy(), pay[:sample_n].copy()
    (ok_, op_, _), dt = _timed(lambda: oracle.sort(sk, sp, k=k))
    (rk, rp), dr = _timed(lambda: oracle.stable_sort_ref(sk, sp))
    if not (np.array_equal(rk, ok_) and np.array_equal(rp, op_)):
        raise RuntimeError("std::stable_sort and the oracle disagree on the CPU sample")

    def npref():
        order = np.argsort(sk, kind="stable")
        return sk[order], sp[order]
    _, dn = _timed(npref)
    out = {"value": round(sample_n / dt / 1e9, 6), "unit": "GKeys/s", "cores": 1, "kind": "oracle",
           "sample": f"first {sample_n} keys (2^{int(np.log2(sample_n))}) of the same runs_i64 input, "
                     f"single-threaded C oracle, {dt:.2f} s",
           "host_cpu": host_cpu(), "nproc": os.cpu_count(),
           "cores_available": len(os.sched_getaffinity(0)),
           "library_reference": {"what": "C++ std::stable_sort of (int64 key, u32 payload) records, "
                                         "one thread, g++ -O2",
                                 "value": round(sample_n / dr / 1e9, 6), "seconds": round(dr, 2)},
           "numpy_reference": {"what": "numpy.argsort(kind='stable') + gather, one thread",
                               "value": round(sample_n / dn / 1e9, 6), "seconds": round(dn, 2)}}
    if full:
        out["per_config"] = cpu_full_configs(k)
    return out


def cpu_full_configs(k: int):
    """The oracle and std::stable_sort, one thread each, on every config at its full
    size (configs 1, 2a, 2b, 3); config 4 on a size-stratified sample of its arrays
    (the rate extrapolated to all of them); config 5 per request over a size-stratified
    sample of the request pool (the distribution of the oracle's per-request time)."""
    import math
    import oracle
    import workloads
    res = []
    for cfg, name, n in (("1", "runs_i32", 1 << 20), ("2a", "runs_i64", 1 << 28),
                         ("2b", "perm_i64", 1 << 28), ("3", "ties_i32", 1 << 27)):
        log(f"cpu baseline: config {cfg} ({name}, n={n}) at full size")
        kh, ph = workloads.WORKLOADS[name](n=n)
        (ok_, op_, _), dt = _timed(lambda: oracle.sort(kh, ph, k=k))
        (rk, rp), dr = _timed(lambda: oracle.stable_sort_ref(kh, ph))
        same = bool(np.array_equal(rk, ok_) and np.array_equal(rp, op_))
        res.append({"config": cfg, "workload": name, "n": n,
                    "oracle_s": round(dt, 2), "oracle_gkeys_s": round(n / dt / 1e9, 5),
                    "std_stable_sort_s": round(dr, 2), "std_stable_sort_gkeys_s": round(n / dr / 1e9, 5),
                    "outputs_equal": same})
        del kh, ph, ok_, op_, rk, rp
    # config 4: m = 8192 int32 arrays, sizes floor(2^U), U ~ U[8, 22] (seed 5); every
    # 128th array in size order, each generated with the recipe of the batched workload
    sizes = workloads.serve_sizes(8192, seed=5, lo_exp=8.0, hi_exp=22.0)
    pick = np.sort(sizes)[64::128]
    rng = np.random.default_rng(55)
    t_or = t_ref = 0.0
    for sz in pick.tolist():
        mr = max(1, int(2 * math.isqrt(sz)))
        kh, ph, _ = workloads.batch_i32(m=1, seed=int(rng.integers(1 << 30)), lo_exp=math.log2(sz),
                                        hi_exp=math.log2(sz) + 1e-12)
        t_or += _timed(lambda: oracle.sort(kh, ph, k=k))[1]
        t_ref += _timed(lambda: oracle.stable_sort_ref(kh, ph))[1]
    keys_s = float(pick.sum())
    res.append({"config": "4", "workload": "batch_i32 (m=8192)",
                "sample": f"{pick.size} arrays, every 128th by size (sizes {int(pick.min())}.."
                          f"{int(pick.max())})",
                "oracle_gkeys_s": round(keys_s / t_or / 1e9, 5),
                "std_stable_sort_gkeys_s": round(keys_s / t_ref / 1e9, 5),
                "oracle_s_all_8192_extrapolated": round(float(sizes.sum()) / (keys_s / t_or), 1)})
    # config 5: the request pool (512 sizes floor(2^U), U ~ U[10, 26], seed 6); every 8th
    # request in size order, float32 keys generated by the serving recipe
    psz = workloads.serve_sizes(512, seed=6)
    pick = np.sort(psz)[4::8]
    rng = np.random.default_rng(66)
    per = []
    for sz in pick.tolist():
        x, p = workloads.serve_request_f32(int(sz), rng)
        per.append(_timed(lambda: oracle.sort(x, p, k=k))[1] * 1e3)
    per = np.array(per)
    res.append({"config": "5", "workload": "serve pool (512 float32 requests)",
                "sample": f"{pick.size} requests, every 8th by size",
                "oracle_ms_per_request_p50_p99": [round(float(np.percentile(per, q)), 3) for q in (50, 99)],
                "oracle_ms_per_request_mean": round(float(per.mean()), 3),
                "oracle_gkeys_s": round(float(pick.sum()) / (per.sum() * 1e-3) / 1e9, 5)})
    return res


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_reps(torch, reps, restore, run):
    """Median and all times (ms) of `run` over reps, each after `restore` (untimed)."""
    ts = []
    for _ in range(reps):
        restore()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), ts


def bench_batched(args, torch, mps, workloads):
    """Batched workload: m int32 arrays with log-uniform sizes in [2^8, 2^22] and random
    runs, index payload.  One batched call (autotuned configuration, graph replay)
    against one mps_sort call per array through the C ABI on the same stream."""
    import ctypes
    dev = torch.device("cuda:0")
    m = args.batched_m
    log(f"batched: generating m={m} arrays on the GPU")
    keys0, pay0, off_h = workloads.batch_i32_device(m=m, device="cuda:0")
    total = int(off_h[-1])
    off_d = torch.from_numpy(off_h.view(np.int64)).to(dev)
    keys, pay = torch.empty_like(keys0), torch.empty_like(pay0)

    def restore():
        keys.copy_(keys0)
        pay.copy_(pay0)

    log(f"batched: total {total} keys; autotuning")
    t0 = time.perf_counter()
    tuned = mps.autotune(keys0, pay0, off_h, sample_keys=1 << 28, graph=True, with_times=True)
    tune_s = time.perf_counter() - t0
    cfg = dict(k=tuned["k"], tile=tuned["tile"], lane_slice=tuned["lane_slice"])
    log(f"batched: tuned {cfg} in {tune_s:.1f} s")
    reps = args.batched_reps

    def batched(**c):
        return lambda: mps.sort_batched(keys, pay, off_d, graph=True, check=False, **c)

    restore()
    mps.sort_batched(keys, pay, off_d, graph=True, **cfg)          # warm-up + capture
    t_tuned, all_tuned = _time_reps(torch, reps, restore, batched(**cfg))
    restore()
    mps.sort_batched(keys, pay, off_d, graph=True, k=4)
    t_def, _ = _time_reps(torch, reps, restore, batched(k=4))
    # merge cost and placement of the batch (for the HBM fraction)
    restore()
    tr = mps.sort_batched(keys, pay, off_d, trace=True, **cfg)
    rs = tr.run_start.astype(np.int64)
    moved = (tr.leaf_depth & 1).astype(bool) | tr.run_desc.astype(bool)
    placed = int(np.diff(rs)[moved].sum())
    KV = 4 + 4
    sort_bytes = total * 4 + 2 * KV * placed + 2 * KV * tr.merge_cost

    # one launch sequence per array through the C ABI (library-managed workspace)
    lib = mps.lib()
    kp, pp = keys.data_ptr(), pay.data_ptr()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    offs = off_h.astype(np.int64).tolist()

    def per_array():
        for i in range(m):
            a, b = offs[i], offs[i + 1]
            rc = lib.mps_sort(ctypes.c_void_p(kp + 4 * a), mps.KEY_I32, ctypes.c_void_p(pp + 4 * a),
                              b - a, stream)
            if rc < 0:
                raise RuntimeError(lib.mps_last_error().decode())
    log("batched: per-array loop")
    restore()
    per_array()                                                       # warm-up
    t_loop, _ = _time_reps(torch, max(1, reps - 1), restore, per_array)
    gk = lambda ms: round(total / (ms * 1e-3) / 1e9, 4)
    return {
        "workload": f"batch_i32: m={m} int32 arrays, sizes floor(2^U) U~U[8,22], random runs "
                    f"U{{1..2*sqrt(size)}} ascending, index payload (sizes/runs seed 5, keys drawn "
                    f"on the GPU)",
        "total_keys": total, "bytes": total * KV,
        "batched_value": gk(t_tuned), "batched_ms": round(t_tuned, 3),
        "batched_ms_all": [round(x, 3) for x in all_tuned],
        "batched_default_value": gk(t_def), "batched_default_ms": round(t_def, 3),
        "per_array_value": gk(t_loop), "per_array_ms": round(t_loop, 3),
        "speedup_vs_per_array": round(t_loop / t_tuned, 3),
        "unit": "GKeys/s",
        "tuned": cfg, "tune_seconds": round(tune_s, 2), "tune_sample_keys": 1 << 28,
        "tune_candidates": tuned["candidates"],
        "merge_cost": int(tr.merge_cost), "runs": int(tr.r),
        "sort_hbm": {"algorithmic_bytes": int(sort_bytes),
                     "achieved_GBs": round(sort_bytes / (t_tuned * 1e-3) / 1e9, 1),
                     "frac": round(sort_bytes / (t_tuned * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "per_array_launch": "one mps_sort call per array via the C ABI, same stream, default "
                            "configuration, library-managed workspace",
    }


def bench_perm(args, torch, mps, workloads, tcfg):
    """The second variant of the headline size: a uniform random permutation of
    n int64 keys (no presortedness), index payload, same arity and tile."""
    n = 1 << args.log2n
    log(f"perm variant: generating a random permutation of 2^{args.log2n}")
    kh, ph = workloads.perm_i64(n=n)
    keys0 = torch.from_numpy(kh).cuda()
    pay0 = torch.from_numpy(ph.view(np.int32)).cuda()
    del kh, ph
    keys, pay = keys0.clone(), pay0.clone()
    tr = mps.sort(keys, pay, k=args.k, trace=True, trace_arrays=False, **tcfg)
    ms, all_ms = _time_reps(torch, 3, lambda: (keys.copy_(keys0), pay.copy_(pay0)),
                            lambda: mps.sort(keys, pay, k=args.k, check=False, **tcfg))
    out = {"workload": f"perm_i64: uniform random permutation of 0..n-1 as int64 keys, n=2^{args.log2n}, "
                       "uint32 index payload (seed 3)",
           "ms": round(ms, 3), "gkeys_s": round(n / (ms * 1e-3) / 1e9, 3),
           "runs": int(tr.r), "tree_levels": int(tr.n_levels),
           "merge_cost_per_key": round(tr.merge_cost / n, 4)}
    if args.perm_min_run > 1:
        # the paper's own setting: natural runs extended to a minimal length (Appendix A.3)
        mr = args.perm_min_run
        keys.copy_(keys0)
        pay.copy_(pay0)
        tm = mps.sort(keys, pay, k=args.k, trace=True, trace_arrays=False, min_run=mr, **tcfg)
        ms_m, _ = _time_reps(torch, 3, lambda: (keys.copy_(keys0), pay.copy_(pay0)),
                             lambda: mps.sort(keys, pay, k=args.k, min_run=mr, check=False, **tcfg))
        out[f"min_run_{mr}"] = {
            "ms": round(ms_m, 3), "gkeys_s": round(n / (ms_m * 1e-3) / 1e9, 3),
            "runs": int(tm.r), "tree_levels": int(tm.n_levels),
            "merge_cost_per_key": round(tm.merge_cost / n, 4),
            "speedup_vs_natural_runs": round(ms / ms_m, 3)}
    del keys0, pay0, keys, pay
    mps.release_workspaces()
    torch.cuda.empty_cache()
    return out


def bench_records(args, torch, mps, keys0, tcfg):
    """16-byte records, the paper's key-and-pointer records (Section 4): the headline's
    int64 keys with an 8-byte payload (each record's index), sorted with k = 4 and k = 2
    (mps_sort_kv64: the merges carry a 4-byte record index, the payload is gathered once)."""
    n = keys0.numel()
    pay0 = torch.arange(n, dtype=torch.int64, device=keys0.device)
    keys, pay = keys0.clone(), pay0.clone()
    res = {"workload": f"the headline keys (runs_i64, n=2^{args.log2n}) with an int64 payload "
                       "holding each record's index", "record_bytes": 16}
    for kk in (4, 2):
        t, _ = _time_reps(torch, 3, lambda: (keys.copy_(keys0), pay.copy_(pay0)),
                          lambda: mps.sort(keys, pay, k=kk, check=False, **tcfg))
        res[f"k{kk}"] = {"ms": round(t, 3), "gkeys_s": round(n / (t * 1e-3) / 1e9, 3)}
    res["time_ratio_k4_over_k2"] = round(res["k4"]["ms"] / res["k2"]["ms"], 4)
    res["output_checked"] = bool((keys[1:] >= keys[:-1]).all().item()) and \
        bool((keys0[pay] == keys).all().item())
    del pay0, keys, pay
    torch.cuda.empty_cache()
    return res


def bench_serving(args, torch, mps, workloads):
    """Serving: a pool of float32 requests (sizes log-uniform in [2^10, 2^26], random runs,
    ~1% duplicate keys, index payload) resident on the GPU.  (1) Closed loop: every pool
    entry submitted at once -> the server's capacity, against one mps_sort per request on
    one stream.  (2) Open loop: Poisson arrivals at 0.7 x capacity for --serve-seconds,
    each request drawing a pool entry that the server copies into its admitted slot; the
    latency of a request runs from submit to the scheduler seeing its batch complete."""
    import ctypes
    dev = torch.device("cuda:0")
    log(f"serving: generating a pool of {args.serve_pool} requests on the GPU")
    pool = workloads.serve_pool_device(count=args.serve_pool, device="cuda:0")
    sizes = np.array([x.numel() for x, _ in pool], np.int64)
    mean_size = float(sizes.mean())
    budget = int(args.serve_budget_gib * (1 << 30))
    srv = mps.Server(hbm_budget_bytes=budget, n_streams=args.serve_streams,
                     max_batch=args.serve_max_batch)
    try:
        # closed loop (also warms up the server and the allocator)
        outs = [(torch.empty_like(x), torch.empty_like(p)) for x, p in pool]
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ids = [srv.submit(x, p, ko, po) for (x, p), (ko, po) in zip(pool, outs)]
            infos = [srv.wait(i, timeout=120) for i in ids]
            closed_s = time.perf_counter() - t0
            for i in ids:
                srv.release(i)
        capacity = float(sizes.sum()) / closed_s
        # one mps_sort per request (copy into the output, sort it there), same stream
        lib = mps.lib()
        stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)

        def per_request():
            for (x, p), (ko, po) in zip(pool, outs):
                ko.copy_(x)
                po.copy_(p)
                rc = lib.mps_sort(ctypes.c_void_p(ko.data_ptr()), mps.KEY_F32,
                                  ctypes.c_void_p(po.data_ptr()), ko.numel(), stream)
                if rc < 0:
                    raise RuntimeError(lib.mps_last_error().decode())
        per_request()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_request()
        torch.cuda.synchronize()
        loop_s = time.perf_counter() - t0
        del outs
        # open loop: Poisson arrivals
        rate = 0.7 * capacity / mean_size
        arrivals = workloads.poisson_arrivals(rate, args.serve_seconds, seed=7)
        pick = np.random.default_rng(8).integers(0, len(pool), size=arrivals.size)
        log(f"serving: capacity {capacity / 1e9:.2f} GKeys/s closed loop; offered "
            f"{rate:.1f} req/s for {args.serve_seconds} s ({arrivals.size} requests)")
        lat, keys_done, batch_sizes = [], 0, []
        outstanding = {}
        t0 = time.perf_counter()
        i = 0
        next_note = 10.0
        while i < arrivals.size or outstanding:
            now = time.perf_counter() - t0
            while i < arrivals.size and arrivals[i] <= now:
                x, p = pool[int(pick[i])]
                ko, po = torch.empty_like(x), torch.empty_like(p)
                outstanding[srv.submit(x, p, ko, po)] = (ko, po)
                i += 1
            for rid in list(outstanding):
                rc, info = srv.poll(rid)
                if rc == 0:
                    lat.append((info["t_done_ns"] - info["t_submit_ns"]) * 1e-6)
                    batch_sizes.append(info["batch_requests"])
                    keys_done += outstanding[rid][0].numel()
                    srv.release(rid)
                    del outstanding[rid]
            if now > next_note:
                log(f"serving: t={now:.0f} s, submitted {i}, in flight {len(outstanding)}")
                next_note += 10.0
            if i < arrivals.size:
                time.sleep(max(0.0, min(1e-4, arrivals[i] - (time.perf_counter() - t0))))
            else:
                time.sleep(5e-5)
        wall = time.perf_counter() - t0
        st = srv.stats()
    finally:
        srv.close()
    lat = np.array(lat)
    return {
        "workload": "serve_f32: pool of %d float32 requests, sizes floor(2^U) U~U[10,26] (seed 6), "
                    "N(0,1) keys in random runs U{1..2*sqrt(size)} ascending, ~1%% duplicates, int32 "
                    "index payload, drawn on the GPU; Poisson arrivals (seed 7), pool entry per "
                    "arrival (seed 8)" % len(pool),
        "pool_keys": int(sizes.sum()), "mean_request_keys": round(mean_size, 1),
        "server": {"hbm_budget_bytes": budget, "n_streams": args.serve_streams,
                   "max_batch": args.serve_max_batch},
        "closed_loop_value": round(capacity / 1e9, 4),
        "per_request_loop_value": round(float(sizes.sum()) / loop_s / 1e9, 4),
        "speedup_vs_per_request": round(loop_s / closed_s, 3),
        "offered_rate_rps": round(rate, 2), "offered_load": "0.7 x closed-loop capacity",
        "seconds": args.serve_seconds, "requests": int(arrivals.size), "completed": int(lat.size),
        "served_value": round(keys_done / wall / 1e9, 4), "unit": "GKeys/s",
        "latency_ms_p50": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
        "latency_ms_p99": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
        "latency_ms_mean": round(float(lat.mean()), 3) if lat.size else None,
        "mean_batch_requests": round(float(np.mean(batch_sizes)), 2) if batch_sizes else None,
        "batches": int(st["batches"]),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--tile", type=int, default=2048, help="merge tile (outputs)")
    ap.add_argument("--lane-slice", type=int, default=4, help="outputs per thread per LDS stage")
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--cpu-sample-log2n", type=int, default=26)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle and std::stable_sort on every config at full size "
                         "(several minutes of CPU work)")
    ap.add_argument("--no-k-sweep", action="store_true")
    ap.add_argument("--no-perm", action="store_true", help="skip the random-permutation variant")
    ap.add_argument("--no-records", action="store_true",
                    help="skip the 16-byte-record variant (8-byte payload)")
    ap.add_argument("--perm-min-run", type=int, default=24,
                    help="also time the permutation with this minimal run length (<= 1: skip)")
    ap.add_argument("--batched-m", type=int, default=8192, help="arrays in the batched workload")
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="Poisson run length")
    ap.add_argument("--serve-pool", type=int, default=512, help="request pool size")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-streams", type=int, default=3)
    ap.add_argument("--serve-max-batch", type=int, default=64)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--only", choices=["perm", "records"],
                    help="run just the random-permutation or the 16-byte-record variant and print "
                         "its figures (for profiling them on their own)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library sorts on one device and has no "
              "multi-GPU path (how the sort would shard is a design note)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2209_06909_amd as mps
    import workloads

    n = 1 << args.log2n
    tcfg = dict(tile=args.tile, lane_slice=args.lane_slice)
    if args.only == "perm":
        torch.cuda.set_device(0)
        print(json.dumps({"perm_variant": bench_perm(args, torch, mps, workloads, tcfg)}), flush=True)
        return
    log(f"generating runs_i64 n=2^{args.log2n}")
    keys_h, pay_h = workloads.runs_i64(n=n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    keys0 = torch.from_numpy(keys_h).to(dev)
    pay0 = torch.from_numpy(pay_h.view(np.int32)).to(dev)
    keys = torch.empty_like(keys0)
    pay = torch.empty_like(pay0)
    KV = 8 + 4
    if args.only == "records":
        del pay0, pay
        print(json.dumps({"records16": bench_records(args, torch, mps, keys0, tcfg)}), flush=True)
        return

    # one untimed traced sort: runs, merge cost and placement volume
    keys.copy_(keys0)
    pay.copy_(pay0)
    tr = mps.sort(keys, pay, k=args.k, trace=True, **tcfg)
    rs = tr.run_start.astype(np.int64)
    lens = np.diff(rs)
    moved = (tr.leaf_depth & 1).astype(bool) | tr.run_desc.astype(bool)
    placed = int(lens[moved].sum())
    log(f"r={tr.r} nodes={tr.n_nodes} levels={tr.n_levels} merge_cost={tr.merge_cost} "
        f"(M/n={tr.merge_cost / n:.3f}) placed={placed}")

    for _ in range(args.warmup):
        keys.copy_(keys0)
        pay.copy_(pay0)
        mps.sort(keys, pay, k=args.k, **tcfg)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    merge_bytes = 0.0
    merge_ms = 0.0
    corank_ms = 0.0
    merge_launches = 0
    per_level = None
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    for i in range(args.steps):
        keys.copy_(keys0)
        pay.copy_(pay0)
        ev[i][0].record()
        mps.sort(keys, pay, k=args.k, time_levels=True, check=False, **tcfg)
        ev[i][1].record()
        elems, cms, mms = mps.level_stats()
        live = elems > 0
        merge_bytes += float((elems[live].astype(np.float64) * 2 * KV).sum())
        merge_ms += float(mms[live].sum())
        corank_ms += float(cms[live].sum())
        merge_launches += int(live.sum())
        per_level = (elems, cms, mms)
        ev[i][1].synchronize()
        log(f"step {i}: sort {ev[i][0].elapsed_time(ev[i][1]):.3f} ms, merge levels "
            f"{float(mms[live].sum()):.3f} ms, co-rank {float(cms[live].sum()):.3f} ms")
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    mps.check_last(dev)     # the last timed sort passed every device-side check
    sort_ms = np.array([a.elapsed_time(b) for a, b in ev])
    ms = float(sort_ms.mean())
    gkeys = n / (ms * 1e-3) / 1e9

    # roofline of the dominant kernel: algorithmic bytes (2 x (key + payload) per merged
    # element) per launch over the average launch duration
    achieved = merge_bytes / merge_launches / (merge_ms / merge_launches * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_merge (per-level k-way merge)",
            "bytes_per_unit": 2 * KV, "unit_of_work": "merged element (key+payload read and written)",
            "avg_launch_ms": round(merge_ms / merge_launches, 4),
            "launches": merge_launches}
    tr_d = committed_traffic(f"runs_i64_2p{args.log2n}") if args.k == 4 and args.tile == 2048 \
        and args.lane_slice == 4 else None
    if tr_d is not None:
        # per launch like `achieved`: the measured bytes per merged element times the
        # merged elements of an average launch
        per_launch = merge_bytes / merge_launches / (2 * KV)
        roof["traffic"] = round(tr_d["bytes_per_merged_element"] * per_launch)
        roof["traffic_per_merged_element"] = tr_d["bytes_per_merged_element"]
        roof["traffic_ratio_to_algorithmic"] = tr_d["ratio_to_algorithmic"]
    # measured copy ceiling: the library's streaming copy kernel (mps_stream_copy) over
    # the same key and payload arrays, every byte read once and written once
    cp_ms = []
    for _ in range(5):
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        mps.stream_copy(keys, keys0)
        mps.stream_copy(pay, pay0)
        c1.record()
        c1.synchronize()
        cp_ms.append(c0.elapsed_time(c1))
    copy_gbs = 2 * n * KV / (min(cp_ms[1:]) * 1e-3) / 1e9
    roof["copy_ceiling_GBs"] = round(copy_gbs, 1)
    roof["copy_ceiling_kernel"] = "mps_stream_copy (16-byte loads/stores, 1024 x 256 threads)"
    roof["frac_of_copy_ceiling"] = round(achieved / copy_gbs, 4)
    levels_all = merge_bytes / ((merge_ms + corank_ms) * 1e-3) / 1e9
    sort_bytes = n * 8 + 2 * KV * placed + 2 * KV * tr.merge_cost
    sort_gbs = sort_bytes / (ms * 1e-3) / 1e9

    out = {
        "metric": METRIC, "value": round(gkeys, 4), "unit": "GKeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "runs_i64: n=2^%d int64 keys uniform over the full range, uint32 "
                               "index payload, random runs of length U{1..2*sqrt(n)} each sorted "
                               "ascending (seed 2)" % args.log2n,
                   "n": n, "k": args.k, "key": "int64", "payload": "uint32",
                   "tile": args.tile, "lane_slice": args.lane_slice},
        "roofline": roof,
        "merge_levels_incl_corank": {"achieved_GBs": round(levels_all, 1),
                                     "frac": round(levels_all / HBM_PEAK_GBS, 4),
                                     "corank_ms_per_sort": round(corank_ms / args.steps, 4),
                                     "merge_ms_per_sort": round(merge_ms / args.steps, 4)},
        "sort_hbm": {"algorithmic_bytes": int(sort_bytes), "achieved_GBs": round(sort_gbs, 1),
                     "frac": round(sort_gbs / HBM_PEAK_GBS, 4)},
        "sort_ms_p10_p50_p90": [round(float(np.percentile(sort_ms, q)), 4) for q in (10, 50, 90)],
        "step_wall_ms_incl_restore": round(t_wall / args.steps * 1e3, 4),
        "runs": int(tr.r), "merge_cost": int(tr.merge_cost), "tree_levels": int(tr.n_levels),
        "levels": [{"d": d, "elems": int(per_level[0][d]), "corank_ms": round(float(per_level[1][d]), 4),
                    "merge_ms": round(float(per_level[2][d]), 4)} for d in range(len(per_level[0]))],
    }
    if not args.no_k_sweep:
        # the paper's central comparison (Section 4, Table 1): the same input sorted with
        # 2-way, 4-way and 8-way merging -- merge cost and time
        sweep = []
        for kk in (2, 4, 8):
            keys.copy_(keys0)
            pay.copy_(pay0)
            trk = mps.sort(keys, pay, k=kk, trace=True, trace_arrays=False, **tcfg)
            t_k, _ = _time_reps(torch, 3, lambda: (keys.copy_(keys0), pay.copy_(pay0)),
                                lambda: mps.sort(keys, pay, k=kk, check=False, **tcfg))
            sweep.append({"k": kk, "ms": round(t_k, 3), "gkeys_s": round(n / (t_k * 1e-3) / 1e9, 3),
                          "merge_cost": int(trk.merge_cost),
                          "merge_cost_per_key": round(trk.merge_cost / n, 4),
                          "tree_levels": int(trk.n_levels)})
        m4 = next(x["merge_cost"] for x in sweep if x["k"] == 4)
        m2 = next(x["merge_cost"] for x in sweep if x["k"] == 2)
        t4 = next(x["ms"] for x in sweep if x["k"] == 4)
        t2 = next(x["ms"] for x in sweep if x["k"] == 2)
        out["k_sweep"] = {"runs": sweep, "merge_cost_ratio_k4_over_k2": round(m4 / m2, 4),
                          "time_ratio_k4_over_k2": round(t4 / t2, 4)}
        # the paper reports relative figures only (no absolute times); quoted as context
        out["paper_context"] = {
            "hardware": "Intel Core i7-4790 (Haswell) at 3.6 GHz, one thread, g++ -Ofast",
            "four_way_vs_two_way_time": "4-way about 20% faster than 2-way on int32 random runs "
                                        "(Section 4.3)",
            "merge_cost_ratio_k4_over_k2": 0.522,
            "merge_cost_workload": "n=10^8 int32, random runs of mean length 10^4 (Table 1)",
            "this_gpu": {"time_ratio_k4_over_k2": round(t4 / t2, 4),
                         "merge_cost_ratio_k4_over_k2": round(m4 / m2, 4)}}
    if not args.no_k_sweep:
        # Appendix A.3's merge-down final phase on the same input (k-way merges along the
        # right spine): merge cost and time against the pure tree
        keys.copy_(keys0)
        pay.copy_(pay0)
        trm = mps.sort(keys, pay, k=args.k, trace=True, trace_arrays=False, merge_down=True, **tcfg)
        t_md, _ = _time_reps(torch, 3, lambda: (keys.copy_(keys0), pay.copy_(pay0)),
                             lambda: mps.sort(keys, pay, k=args.k, merge_down=True, check=False, **tcfg))
        out["merge_down"] = {"ms": round(t_md, 3), "merge_cost": int(trm.merge_cost),
                             "merge_cost_pure": int(tr.merge_cost),
                             "tree_levels": int(trm.n_levels)}
    if not args.no_records:
        out["records16"] = bench_records(args, torch, mps, keys0, tcfg)
    if not args.no_perm:
        out["perm_variant"] = bench_perm(args, torch, mps, workloads, tcfg)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(keys_h, pay_h, 1 << args.cpu_sample_log2n, args.k,
                                           full=args.cpu_full)
    del keys_h, pay_h, keys0, pay0, keys, pay
    mps.release_workspaces()
    torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = bench_batched(args, torch, mps, workloads)
        mps.release_workspaces()
        torch.cuda.empty_cache()
    if not args.no_serve:
        out["serving"] = bench_serving(args, torch, mps, workloads)
        mps.release_workspaces()
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
