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


def cpu_baseline(keys: np.ndarray, pay: np.ndarray, sample_n: int, k: int):
    import oracle
    sk, sp = keys[:sample_n].copy(), pay[:sample_n].copy()
    t0 = time.perf_counter()
    oracle.sort(sk, sp, k=k)
    dt = time.perf_counter() - t0
    return {"value": round(sample_n / dt / 1e9, 6), "unit": "GKeys/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample_n} keys (2^{int(np.log2(sample_n))}) of the same runs_i64 input, "
                      f"single-threaded C oracle, {dt:.2f} s"}


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
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sort runs on one device; see the sharding notes in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2209_06909_amd as mps
    import workloads

    n = 1 << args.log2n
    log(f"generating runs_i64 n=2^{args.log2n}")
    keys_h, pay_h = workloads.runs_i64(n=n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    keys0 = torch.from_numpy(keys_h).to(dev)
    pay0 = torch.from_numpy(pay_h.view(np.int32)).to(dev)
    keys = torch.empty_like(keys0)
    pay = torch.empty_like(pay0)
    KV = 8 + 4

    # one untimed traced sort: runs, merge cost and placement volume
    keys.copy_(keys0)
    pay.copy_(pay0)
    tcfg = dict(tile=args.tile, lane_slice=args.lane_slice)
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
        mps.sort(keys, pay, k=args.k, time_levels=True, **tcfg)
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
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(keys_h, pay_h, 1 << args.cpu_sample_log2n, args.k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
