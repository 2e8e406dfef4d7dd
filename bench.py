#!/usr/bin/env python3
"""Throughput benchmark of the MI355X frequent-itemset miner.

One step = one ``fim_mine`` call over the resident database: item supports,
bitmap build, sample-based estimate, root-class pair kernel, persistent DFS,
result copy and canonical ordering (the whole hot path).  The database is
uploaded once before the timed region.  Default workload: ``sparse-200k``
(200,000 basket transactions over 5,000 items, minimum support 0.1 %).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  ``value`` is candidate supports per second (pairs of
extensions whose support was computed, summed over all classes) of the whole
call.  ``roofline`` describes the dominant kernel, timed with HIP events on
the library's stream inside the timed region: the root-class pair kernel is
bound by the integer vector ALU (two 32-bit operations per AND-popcounted
word pair), the depth-first kernel by HBM bandwidth (algorithmic bytes:
every class's sibling bitmaps written once and read once).  ``cpu_baseline``
is the CPU oracle (plain Eclat over sorted tid-lists) timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "candidate supports/s + HBM GB/s; served p50/p99 latency, batched vs plain"
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit integer VALU operations per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sparse-200k",
                    choices=["sparse-200k", "basket-10k", "dense-50k"])
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--flags", type=int, default=0, help="fim_options.flags")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import oracle
    import paper_2108_05038_amd as F
    import synth

    db = synth.make(args.workload)
    ctx = F.Context(0)
    d = F.Database(ctx, db.offsets, db.items, db.n_items)
    gold_path = os.path.join(ROOT, "tests", "golden", "%s.json" % args.workload)
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else None

    verified = None
    for i in range(args.warmup):
        r = F.mine(ctx, d, db.minsup, flags=args.flags)
        if i == 0 and gold is not None:
            verified = (oracle.digest(r.offsets, r.items, r.supports) == gold["digest"]
                        and r.stats["candidates"] == gold["candidates_ascending_support"])
            log("warmup result matches the oracle's golden digest:", verified)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = F.mine(ctx, d, db.minsup, flags=args.flags)
        stats.append(r.stats)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    st = stats[-1]
    cands = st["candidates"]
    value = cands / dt

    root_ns = float(np.mean([s["root_kernel_ns"] for s in stats]))
    dfs_ns = float(np.mean([s["dfs_kernel_ns"] for s in stats]))
    root_tops = 2.0 * st["root_pair_words"] / root_ns / 1e3 if root_ns else 0.0
    dfs_gbs = st["dfs_bytes_algorithmic"] / dfs_ns if dfs_ns else 0.0
    kernels = {
        "k_root_pairs": {"ms": root_ns / 1e6, "bound": "alu", "achieved_TOPs": root_tops,
                         "frac": root_tops / VALU_PEAK_TOPS,
                         "ops_per_launch": 2 * st["root_pair_words"]},
        "k_dfs": {"ms": dfs_ns / 1e6, "bound": "hbm", "achieved_GBs": dfs_gbs,
                  "frac": dfs_gbs / HBM_PEAK_GBS, "bytes_per_launch": st["dfs_bytes_algorithmic"]},
    }
    if root_ns >= dfs_ns:
        roofline = {"kernel": "k_root_pairs", "bound": "alu", "achieved": root_tops,
                    "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": root_tops / VALU_PEAK_TOPS,
                    "traffic": None}
    else:
        roofline = {"kernel": "k_dfs", "bound": "hbm", "achieved": dfs_gbs, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": dfs_gbs / HBM_PEAK_GBS, "traffic": None}

    cpu = None
    if not args.no_cpu:
        threads = max(1, min(args.cpu_threads, os.cpu_count() or 1))
        log("timing the CPU oracle with %d threads ..." % threads)
        c0 = time.perf_counter()
        o = oracle.mine_db(db, threads=threads)
        c1 = time.perf_counter()
        cpu = {"value": o.candidates / (c1 - c0), "unit": "candidate supports/s",
               "cores": threads, "kind": "oracle",
               "sample": "the full %s workload, one run (%d candidate pairs, %.1f s)"
                         % (args.workload, o.candidates, c1 - c0),
               "matches_gpu": bool(o.digest() == oracle.digest(r.offsets, r.items, r.supports))}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "candidate supports/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_tx": db.n_tx, "n_items": db.n_items,
                   "minsup": db.minsup, "n_itemsets": st["n_itemsets"],
                   "candidates": cands, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "hbm_GBs_dfs": dfs_gbs,
        "verified_vs_oracle": verified,
    }
    print(json.dumps(out), flush=True)
    d.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
