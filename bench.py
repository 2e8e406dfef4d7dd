#!/usr/bin/env python3
"""Throughput benchmark of the MI355X frequent-itemset miner.

One step = one ``fim_mine`` call over the resident database: item supports,
bitmap build, sample-based estimate, root-class pair kernel, persistent DFS,
result copy and canonical ordering (the whole hot path).  The database is
uploaded once before the timed region.  Default workload: ``sparse-200k``
(200,000 basket transactions over 5,000 items, minimum support 0.1 %).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-batch] [--no-serve] [--no-cpu]

Prints one JSON line.  ``value`` is candidate supports per second (pairs of
extensions whose support was computed, summed over all classes) of the whole
call.  ``roofline`` describes the dominant kernel, timed with HIP events on
the library's stream inside the timed region: the root-class pair kernels
are bound by the integer vector ALU (two 32-bit operations per
AND-popcounted word pair), the depth-first kernel by HBM bandwidth
(algorithmic bytes: every class's sibling bitmaps written once and read
once).  ``cpu_baseline`` is the CPU oracle (plain Eclat over sorted
tid-lists) timed on this host.

Two more legs go into the same line:
  ``batched``  256 independent basket instances (log-uniform sizes) mined by
               one ``fim_mine_batch`` call with autotuned tile width and
               classes per workgroup, against the plain miner called once per
               instance; every instance's result is checked against its
               stored digest.
  ``served``   a seeded Poisson stream of requests (basket instances like the
               batch, one in ten dense) offered to the continuous-batching
               server, against the plain miner serving the same stream one
               request at a time; p50/p99 latency and throughput per rate.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "candidate supports/s + HBM GB/s; served p50/p99 latency, batched vs plain"
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit integer VALU operations per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_2108_05038_amd", "csrc", "fim_kernels.hip")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def digest(r) -> str:
    """SHA-256 of a result's canonical binary CSR (little-endian u64 offsets,
    u32 items, u32 supports), the format the stored expected values use."""
    import numpy as np
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(r.offsets, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(r.items, dtype="<u4").tobytes())
    h.update(np.ascontiguousarray(r.supports, dtype="<u4").tobytes())
    return h.hexdigest()


def kernel_source_sha() -> str:
    """SHA-256 (first 16 hex digits) of the kernel source file: a profile's
    counters describe the kernels only while this matches the value the
    profile records."""
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the rocprofv3
    counter summary ``profiles/<kernel>.<workload>.txt`` (FETCH_SIZE and
    WRITE_SIZE scaled by the plain-copy calibration), or None when there is
    no summary or it was taken with other kernel sources."""
    p = os.path.join(PROFILES, "%s.%s.txt" % (kernel, workload))
    if not os.path.exists(p):
        return None
    sha, traffic = None, None
    for line in open(p):
        if line.startswith("kernel_source_sha256_16:"):
            sha = line.split(":", 1)[1].strip()
        if line.startswith("hbm_bytes_per_launch:"):
            traffic = float(line.split(":", 1)[1].strip())
    return traffic if sha == kernel_source_sha() else None


def load_golden(name):
    p = os.path.join(GOLDEN, name)
    return json.load(open(p)) if os.path.exists(p) else None


# ---------------------------------------------------------------- one workload, whole calls

def mine_leg(F, ctx, db, workload, steps, warmup, flags, estimate_leg=False):
    """Times `steps` whole ``fim_mine`` calls over the resident database and
    describes the dominant kernel against its roofline (HIP-event times the
    library records on the stream it launches on)."""
    import numpy as np
    import torch
    # the upload (validation, set semantics, host-to-device copy) is outside
    # the timed loop; timed here for the host-inclusive rate
    upload_ms = None
    for _ in range(2):
        t_up = time.perf_counter()
        d = F.Database(ctx, db.offsets, db.items, db.n_items)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t_up) * 1e3
        upload_ms = ms if upload_ms is None else min(upload_ms, ms)
        if _ == 0:
            d.close()
    log("%s: database upload %.2f ms" % (workload, upload_ms))
    gold = load_golden("%s.json" % workload)
    verified = None
    for i in range(warmup):
        r = F.mine(ctx, d, db.minsup, flags=flags)
        if i == 0 and gold is not None:
            verified = (digest(r) == gold["digest"]
                        and r.stats["candidates"] == gold["candidates_ascending_support"])
            log("%s: warm-up result matches the oracle's golden digest: %s" % (workload, verified))
    torch.cuda.synchronize()
    stats, ends = [], []
    # Python's cyclic garbage collector is run before the timed calls and
    # kept out of them (as timeit does): a full collection inside one call
    # would be charged to the library
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = F.mine(ctx, d, db.minsup, flags=flags)
        stats.append(r.stats)
        ends.append(time.perf_counter())
    torch.cuda.synchronize()
    gc.enable()
    dt = (time.perf_counter() - t0) / steps
    step_ms = np.diff([t0] + ends) * 1e3  # per call (each call returns a finished result)
    log("%s: %.3f ms/step" % (workload, dt * 1e3))
    est_leg = None
    if estimate_leg:
        # The same step with the sample-based class-size estimate forced (the
        # library draws it by default only where it pays): the cost of that
        # row of the path where the default policy replaces it.
        est_steps = max(3, steps // 4)
        re_ = F.mine(ctx, d, db.minsup, flags=flags | F.FIM_FLAG_ALWAYS_ESTIMATE)
        torch.cuda.synchronize()
        te = time.perf_counter()
        for _ in range(est_steps):
            re_ = F.mine(ctx, d, db.minsup, flags=flags | F.FIM_FLAG_ALWAYS_ESTIMATE)
        torch.cuda.synchronize()
        est_leg = {"ms_per_step": (time.perf_counter() - te) / est_steps * 1e3, "steps": est_steps,
                   "estimate_ms": re_.stats["estimate_ns"] / 1e6,
                   "dfs_ms": re_.stats["dfs_kernel_ns"] / 1e6,
                   "candidates": re_.stats["candidates"],
                   "verified_vs_oracle": (digest(re_) == gold["digest"]) if gold else None}
        del re_
        log("%s: with the sample estimate forced %.3f ms/step" % (workload, est_leg["ms_per_step"]))
    d.close()
    st = stats[-1]
    root_ns = float(np.mean([s_["root_kernel_ns"] for s_ in stats]))
    dfs_ns = float(np.mean([s_["dfs_kernel_ns"] for s_ in stats]))
    root_name = ("k_root_pairs", "k_root_sparse", "k_root_project")[st["root_kernel"]]
    dfs_bytes = st["dfs_bytes_algorithmic"]
    root_bytes = st["bytes_algorithmic"] - dfs_bytes
    dfs_gbs = dfs_bytes / dfs_ns if dfs_ns else 0.0
    if st["root_kernel"] == 0:
        # whole rows: two integer operations (AND, popcount-add) per pair-word
        root_ops = 2.0 * st["root_pair_words"]
        root_k = {"ms": root_ns / 1e6, "bound": "alu",
                  "achieved": root_ops / root_ns / 1e3 if root_ns else 0.0,
                  "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "algorithmic": root_ops}
    else:
        # covers / projected transactions: the bytes the kernel must read
        root_k = {"ms": root_ns / 1e6, "bound": "hbm",
                  "achieved": root_bytes / root_ns if root_ns else 0.0,
                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "algorithmic": root_bytes}
    root_k["frac"] = root_k["achieved"] / root_k["peak"]
    dfs_k = {"ms": dfs_ns / 1e6, "bound": "hbm", "achieved": dfs_gbs, "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": dfs_gbs / HBM_PEAK_GBS, "algorithmic": dfs_bytes}
    kernels = {root_name: root_k, "k_dfs": dfs_k}
    name, k = (root_name, root_k) if root_ns >= dfs_ns else ("k_dfs", dfs_k)
    for kn, kk in kernels.items():
        kk["traffic"] = measured_traffic(kn, workload)
    roofline = {"kernel": name, "bound": k["bound"], "achieved": k["achieved"], "peak": k["peak"],
                "unit": k["unit"], "frac": k["frac"], "traffic": k["traffic"],
                "traffic_GBs": k["traffic"] / (k["ms"] * 1e6) if k["traffic"] else None}
    return {
        "workload": workload, "n_tx": db.n_tx, "n_items": db.n_items, "minsup": db.minsup,
        "steps": steps, "warmup": warmup, "ms_per_step": dt * 1e3,
        "ms_per_step_min_median_max": [float(step_ms.min()), float(np.median(step_ms)),
                                       float(step_ms.max())],
        "step_ms": [round(float(x), 3) for x in step_ms],
        "value": st["candidates"] / dt, "unit": "candidate supports/s",
        "n_itemsets": st["n_itemsets"], "candidates": st["candidates"],
        "upload_ms": upload_ms, "with_sample_estimate": est_leg,
        "roofline": roofline, "kernels": kernels, "verified_vs_oracle": verified,
        "stats": st, "result": r,
    }


# ---------------------------------------------------------------- batched leg

def batch_leg(F, ctx, args):
    import numpy as np
    import torch

    import synth
    g = load_golden("batch-256.json")
    n = args.batch
    subs = [g["instances"][i]["substream"] for i in range(n)] if g else list(range(n))
    log("batched: generating %d instances ..." % n)
    t0 = time.perf_counter()
    params = [synth.batch_params(s) for s in subs]
    handles, minsups = [], []
    for p in params:
        d = synth.batch_instance(p)
        handles.append(F.Database(ctx, d.offsets, d.items, d.n_items))
        minsups.append(d.minsup)
        del d
    log("batched: generated and uploaded in %.1f s" % (time.perf_counter() - t0))

    t0 = time.perf_counter()
    tuned = F.autotune(ctx, handles, minsups, reps=1)
    tune_s = time.perf_counter() - t0
    log("batched: autotuned in %.1f s:" % tune_s, tuned)
    opts = dict(tile_words=tuned["tile_words"], classes_per_wg=tuned["classes_per_wg"])

    res = F.mine_batch(ctx, handles, minsups, **opts)
    verified = None
    if g:
        bad = [i for i, r in enumerate(res)
               if digest(r) != g["instances"][i]["digest"]
               or r.stats["candidates"] != g["instances"][i]["candidates_ascending_support"]]
        verified = not bad
        log("batched: %d of %d instances match their digests" % (n - len(bad), n))
    cands = sum(r.stats["candidates"] for r in res)
    n_sets = sum(len(r) for r in res)
    dfs_ns = res[0].stats["dfs_kernel_ns"]
    del res

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        res = F.mine_batch(ctx, handles, minsups, **opts)
        del res
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / args.batch_steps

    # plain: the one-instance-per-launch miner over the same instances
    for i in range(min(4, n)):
        F.mine(ctx, handles[i], minsups[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h, m in zip(handles, minsups):
        F.mine(ctx, h, m)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    for h in handles:
        h.close()
    ctx.release_cached()
    return {
        "instances": n, "n_itemsets": n_sets, "candidates": cands,
        "ms_per_batch": batch_s * 1e3, "value": cands / batch_s,
        "plain_ms": plain_s * 1e3, "plain_value": cands / plain_s,
        "speedup_vs_plain": plain_s / batch_s,
        "dfs_kernel_ms": dfs_ns / 1e6,
        "tile_words": tuned["tile_words"], "classes_per_wg": tuned["classes_per_wg"],
        "autotune_s": tune_s, "verified_vs_oracle": verified,
        "unit": "candidate supports/s",
    }


# ---------------------------------------------------------------- served leg

def _trace(rate, seconds, pool_n):
    """Seeded Poisson arrival times and the pool request each one is."""
    import numpy as np

    import synth
    base = synth.substream(synth.SERVE_BASE, 1_000_000 + int(rate))
    n = int(rate * seconds * 1.5) + 16
    gaps = synth.exponentials(base, n, 1.0 / rate)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    u = synth.uniforms(synth.substream(base, 1), len(t))
    return t, np.minimum((u * pool_n).astype(np.int64), pool_n - 1)


def _stats(lat, censored, seconds, done):
    import numpy as np
    a = np.maximum(np.array(lat), 0.0) if lat else np.zeros(1)
    return {"p50_ms": float(np.percentile(a, 50) * 1e3), "p99_ms": float(np.percentile(a, 99) * 1e3),
            "mean_ms": float(a.mean() * 1e3), "completed": done, "censored": censored,
            "throughput_rps": done / seconds}


class Checker:
    """Checks served results against the oracle's stored values: every
    result's itemset and candidate counts (cheap enough for the serving
    loop), and the full digest of the first result of each pool request."""

    def __init__(self, gold):
        self.gold = gold
        self.first = {}
        self.checked = 0
        self.bad = []

    def __call__(self, k, r):
        if self.gold is None:
            return
        e = self.gold["instances"][k]
        self.checked += 1
        if len(r) != e["n_itemsets"] or r.stats["candidates"] != e["candidates_ascending_support"]:
            self.bad.append(k)
        self.first.setdefault(int(k), r)

    def digests(self):
        if self.gold is None:
            return None
        bad = [k for k, r in self.first.items() if self.gold["instances"][k]["digest"] != digest(r)]
        self.first = {k: None for k in self.first}
        return bad


def serve_served(F, ctx, handles, minsups, arr, idx, seconds, lanes, check):
    srv = F.Server(ctx, lanes=lanes)
    deadline = 2 * seconds + 10
    pending, lat = {}, []
    k, n = 0, len(arr)
    t0 = time.perf_counter()
    while k < n or pending:
        now = time.perf_counter() - t0
        if now > deadline:
            break
        while k < n and arr[k] <= now:
            pending[srv.submit(handles[idx[k]], minsups[idx[k]])] = k
            k += 1
        # block until a request finishes or the next one arrives
        wait = min(arr[k] - now, 0.05) if k < n else 0.05
        t, r = srv.next(max(wait, 0.0))
        if t:
            q = pending.pop(t)
            lat.append(time.perf_counter() - t0 - arr[q])
            check(int(idx[q]), r)
    end = time.perf_counter() - t0
    # requests still open at the deadline count with their waiting time so
    # far (a lower bound), so that overload shows in the percentiles
    censored = len(pending) + (n - k)
    lat += [end - arr[q] for q in pending.values()] + [end - a for a in arr[k:]]
    for t in pending:
        srv.cancel(t)
    st = srv.stats()
    srv.close()
    out = _stats(lat, censored, max(seconds, end), n - censored)
    out["server"] = {"lanes": st["lanes"], "steps": st["steps"], "peak_active": st["peak_active"]}
    return out


def serve_plain(F, ctx, handles, minsups, arr, idx, seconds, check):
    deadline = 2 * seconds + 10
    lat = []
    t0 = time.perf_counter()
    k = 0
    for k in range(len(arr)):
        now = time.perf_counter() - t0
        if now > deadline:
            break
        if arr[k] > now:
            time.sleep(arr[k] - now)
        r = F.mine(ctx, handles[idx[k]], minsups[idx[k]])
        lat.append(time.perf_counter() - t0 - arr[k])
        check(int(idx[k]), r)
        del r
    end = time.perf_counter() - t0
    done = len(lat)
    lat += [end - a for a in arr[done:]]  # open at the deadline: lower bounds
    return _stats(lat, len(arr) - done, max(seconds, end), done)


def serve_leg(F, ctx, args, seconds):
    import synth
    g = load_golden("serve-pool.json")
    pool_n = args.serve_pool
    log("served: generating a pool of %d requests ..." % pool_n)
    t0 = time.perf_counter()
    handles, minsups, kinds = [], [], []
    for k in range(pool_n):
        p = synth.serve_params(k, g["instances"][k].get("substream", k) if g else None)
        d = synth.serve_instance(p)
        handles.append(F.Database(ctx, d.offsets, d.items, d.n_items))
        minsups.append(d.minsup)
        kinds.append(p.get("kind", "basket"))
        del d
    log("served: pool ready in %.1f s (%d dense)" % (time.perf_counter() - t0, kinds.count("dense")))
    # warm both paths on a few requests
    for k in range(min(8, pool_n)):
        F.mine(ctx, handles[k], minsups[k])
    rates = [float(x) for x in args.serve_rates.split(",") if x]
    out = {"seconds": seconds, "configured_seconds": 60.0, "pool": pool_n, "rates": {}}
    check = Checker(g)
    for rate in rates:
        arr, idx = _trace(rate, seconds, pool_n)
        t1 = time.perf_counter()
        log("served: %g req/s for %.0f s, %d requests ..." % (rate, seconds, len(arr)))
        s = serve_served(F, ctx, handles, minsups, arr, idx, seconds, args.lanes, check)
        log("served: continuous batching", s)
        p = serve_plain(F, ctx, handles, minsups, arr, idx, seconds, check)
        log("served: plain per request", p)
        out["rates"]["%g" % rate] = {"requests": len(arr), "batched": s, "plain": p,
                                     "wall_s": time.perf_counter() - t1}
    bad = check.digests()
    if g:
        out["verified_vs_oracle"] = not bad and not check.bad
        out["verified_requests"] = len(check.first)  # distinct pool requests, full digest
        out["checked_results"] = check.checked       # every result: itemset and candidate counts
        out["mismatches"] = sorted(set(bad) | set(check.bad))[:20]
        log("served: %d distinct requests verified by digest, %d results by counts, %d bad"
            % (len(check.first), check.checked, len(out["mismatches"])))
    for h in handles:
        h.close()
    ctx.release_cached()
    return out


# ---------------------------------------------------------------- estimator study

def share_errors(F, n_atoms, weights, actual, n_workers, alpha=0.3):
    """The thesis's experiment on each processor's share of the work, for a
    static plan: the classes are split by Partition and scheduled by LPT on
    n_workers workers with the given per-row weights; returns the largest
    and mean |estimated share - actual share| over the workers (the actual
    share from the rows' real candidate pairs) and the actual makespan over
    the mean load (1.0 = perfect balance)."""
    import numpy as np
    tasks, _ = F.fim_partition_lpt(n_atoms, weights, alpha, n_workers)
    start = np.concatenate([[0], np.cumsum(np.asarray(n_atoms, dtype=np.int64))])
    cw = np.concatenate([[0.0], np.cumsum(np.asarray(weights, dtype=np.float64))])
    ca = np.concatenate([[0.0], np.cumsum(np.asarray(actual, dtype=np.float64))])
    est = np.array([cw[start[c] + r1] - cw[start[c] + r0] for c, r0, r1 in tasks])
    act = np.array([ca[start[c] + r1] - ca[start[c] + r0] for c, r0, r1 in tasks])
    if len(tasks) == 0 or est.sum() <= 0 or act.sum() <= 0:
        return None
    worker, _ = F.fim_lpt_schedule(est, n_workers)
    e = np.bincount(worker, weights=est, minlength=n_workers) / est.sum()
    a = np.bincount(worker, weights=act, minlength=n_workers) / act.sum()
    return {"max_abs_err": float(np.abs(e - a).max()), "mean_abs_err": float(np.abs(e - a).mean()),
            "actual_makespan_over_mean": float(a.max() * n_workers), "tasks": int(len(tasks))}


def study(F, ctx, args):
    """The sample-based class-size estimate against the actual work, the
    thesis's experiment on each processor's share carried over to the waves
    of one GPU.  Per workload: (1) call and kernel times with the estimate
    (counted in the run, or the reservoir variant), with the bitonic
    scheduling's C(n, 2) weight in its place and without splitting; (2) from
    one class profile (per second-level class: the sample's frequent
    itemsets, the sample's candidate pairs, the run's own candidate pairs),
    the static plan's share error and balance for P = 10, 20 (the thesis's
    processor counts) and 1024 (the waves) under three weights: the
    estimate (sampled frequent itemsets), sampled candidate pairs, and
    C(n, 2) of the class's n atoms."""
    import numpy as np

    import synth
    policies = {
        "estimate": F.FIM_FLAG_ALWAYS_ESTIMATE,
        "estimate_reservoir": F.FIM_FLAG_ALWAYS_ESTIMATE | F.FIM_FLAG_RESERVOIR,
        "proxy": F.FIM_FLAG_NO_ESTIMATE,
        "proxy_no_split": F.FIM_FLAG_NO_ESTIMATE | F.FIM_FLAG_NO_SPLIT,
    }
    loads = [("dense-50k", synth.make("dense-50k")), ("sparse-200k", synth.make("sparse-200k"))]
    o, it, ni = synth.dense(synth.SEED_BASE + 6, 200000, 120)
    loads.append(("dense-200k", synth.Database(o, it, ni, 80000, "dense-200k")))
    out = {}
    for name, db in loads:
        d = F.Database(ctx, db.offsets, db.items, db.n_items)
        row = {"policies": {}}
        for pol, flags in policies.items():
            walls, st = [], None
            for rep in range(4):
                t0 = time.perf_counter()
                r = F.mine(ctx, d, db.minsup, flags=flags)
                walls.append(time.perf_counter() - t0)
                st = r.stats
            row["policies"][pol] = {
                "wall_ms": float(np.median(walls[1:]) * 1e3),
                "dfs_ms": st["dfs_kernel_ns"] / 1e6, "estimate_ms": st["estimate_ns"] / 1e6,
                "imbalance": st["dfs_busy_max_ns"] / max(st["dfs_busy_mean_ns"], 1),
                "tasks": st["n_tasks"]}
            log("study", name, pol, row["policies"][pol])
        prof = F.class_profile(ctx, d, db.minsup)
        na = prof["n_atoms"]
        later = np.concatenate([np.arange(int(k) - 1, -1, -1) for k in na]) if len(na) else np.zeros(0)
        weights = {"estimate_fi": prof["est_fi"], "estimate_candidates": prof["est_cand"],
                   "pairs_C(n,2)": later * (later - 1) / 2.0}
        act = prof["act_cand"].astype(np.float64)
        row["share_error"] = {}
        for wname, w in weights.items():
            row["share_error"][wname] = {str(P): share_errors(F, na, w, act, P) for P in (10, 20, 1024)}
            log("study", name, wname, row["share_error"][wname])
        row["classes"] = {"first_level": int(len(na)), "second_level": int(len(act)),
                          "candidates_below_root": float(act.sum())}
        out[name] = row
        d.close()
    return out


# ---------------------------------------------------------------- CPU baseline

def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(db, r, args):
    """The oracle (plain Eclat over sorted tid-lists) on this host's cores:
    the median of three runs on the full workload with up to 16 threads (the
    host share of one GPU), and one single-thread run when the budget
    leaves time for it."""
    import numpy as np

    import oracle
    nproc = os.cpu_count() or 1
    threads = max(1, min(args.cpu_threads, nproc))
    log("timing the CPU oracle with %d threads (median of 3) ..." % threads)
    walls, o = [], None
    for _ in range(3):
        c0 = time.perf_counter()
        o = oracle.mine_db(db, threads=threads)
        walls.append(time.perf_counter() - c0)
    med = float(np.median(walls))
    out = {"value": o.candidates / med, "unit": "candidate supports/s", "cores": threads,
           "kind": "oracle", "nproc": nproc, "cpu_model": cpu_model(),
           "sample": "the full %s workload, median of 3 runs (%d candidate pairs; %s s)"
                     % (args.workload, o.candidates, ", ".join("%.2f" % w for w in walls)),
           "matches_gpu": bool(o.digest() == digest(r)), "one_thread": None}
    left = args.budget_s - (time.perf_counter() - T_START)
    est1 = med * threads * 1.3  # a single thread takes about threads x as long
    if args.cpu_one_thread and est1 < left - 20:
        log("timing the CPU oracle with 1 thread (about %.0f s) ..." % est1)
        c0 = time.perf_counter()
        o1 = oracle.mine_db(db, threads=1)
        w1 = time.perf_counter() - c0
        out["one_thread"] = {"value": o1.candidates / w1, "seconds": w1, "runs": 1,
                             "matches_gpu": bool(o1.digest() == digest(r))}
    else:
        log("CPU oracle, 1 thread: skipped (about %.0f s needed, %.0f s left)" % (est1, left))
    return out


# ---------------------------------------------------------------- main

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
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch", type=int, default=256, help="instances of the batched leg")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rates", default="50,100,200,400", help="request rates (req/s)")
    ap.add_argument("--serve-seconds", type=float, default=0.0,
                    help="arrival window per rate and mode (0 = what the time budget leaves, "
                         "at most 60 s)")
    ap.add_argument("--serve-pool", type=int, default=512, help="distinct requests (<= 512)")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-50k leg")
    ap.add_argument("--dense-steps", type=int, default=10)
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-clock budget of the whole run; the served leg and the "
                         "single-thread CPU run are sized to stay inside it")
    ap.add_argument("--no-cpu-one-thread", dest="cpu_one_thread", action="store_false")
    ap.add_argument("--lanes", type=int, default=0, help="server lanes (0 = default)")
    ap.add_argument("--study", action="store_true",
                    help="only run the estimator study and print its JSON line")
    ap.add_argument("--batch-only", action="store_true",
                    help="only mine the batch instances --batch-steps times with default "
                         "options, after one untimed call (for kernel traces of the batched "
                         "path), and print their times")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (the "
                         "reference for scaling the HBM byte counters) and exit")
    args = ap.parse_args(argv)

    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.calibrate_copy, "copies": 3}), flush=True)
        return 0

    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2108_05038_amd as F
    import synth

    if args.study:
        ctx = F.Context(0)
        print(json.dumps({"study": "estimator", "results": study(F, ctx, args)}), flush=True)
        ctx.close()
        return 0

    if args.batch_only:
        ctx = F.Context(0)
        g = load_golden("batch-256.json")
        subs = [g["instances"][i]["substream"] for i in range(args.batch)] if g else list(range(args.batch))
        handles, minsups = [], []
        for sub in subs:
            d = synth.batch_instance(synth.batch_params(sub))
            handles.append(F.Database(ctx, d.offsets, d.items, d.n_items))
            minsups.append(d.minsup)
        res = F.mine_batch(ctx, handles, minsups)
        ok = None if not g else all(digest(r_) == g["instances"][i]["digest"] for i, r_ in enumerate(res))
        del res
        torch.cuda.synchronize()
        times = []
        for _ in range(args.batch_steps):
            t0 = time.perf_counter()
            res = F.mine_batch(ctx, handles, minsups)
            times.append((time.perf_counter() - t0) * 1e3)
            del res
        print(json.dumps({"batch_only": args.batch, "calls": args.batch_steps, "ms": times,
                          "verified_vs_oracle": ok}), flush=True)
        return 0

    ctx = F.Context(0)
    db = synth.make(args.workload)
    main = mine_leg(F, ctx, db, args.workload, args.steps, args.warmup, args.flags,
                    estimate_leg=True)
    dense = None
    if not args.no_dense and args.workload != "dense-50k":
        dense = mine_leg(F, ctx, synth.make("dense-50k"), "dense-50k", args.dense_steps, 2, args.flags)
        dense.pop("result", None)
    r = main.pop("result")
    st = main["stats"]
    batched = None if args.no_batch else batch_leg(F, ctx, args)
    served = None
    if not args.no_serve:
        # the served leg gets the time left of the budget (the CPU baseline
        # runs after it), at most the configuration's 60 s per rate and mode
        n_rates = len([x for x in args.serve_rates.split(",") if x])
        left = args.budget_s - (time.perf_counter() - T_START) - (0 if args.no_cpu else 90) - 40
        secs = args.serve_seconds or max(10.0, min(60.0, left / max(1, 2 * n_rates)))
        served = serve_leg(F, ctx, args, secs)

    cpu = None if args.no_cpu else cpu_leg(db, r, args)

    value = main["value"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "candidate supports/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "ms_per_step_min_median_max": main["ms_per_step_min_median_max"],
        "upload_ms": main["upload_ms"],
        "with_sample_estimate": main["with_sample_estimate"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_tx": db.n_tx, "n_items": db.n_items,
                   "minsup": db.minsup, "n_itemsets": st["n_itemsets"],
                   "candidates": st["candidates"], "parallelism": "single GPU"},
        "roofline": main["roofline"],
        "cpu_baseline": cpu,
        "kernels": main["kernels"],
        "hbm_GBs_dfs": main["kernels"]["k_dfs"]["achieved"],
        "verified_vs_oracle": main["verified_vs_oracle"],
        "dense": None if dense is None else {k: v for k, v in dense.items() if k != "stats"},
        "batched": batched,
        "served": served,
        "wall_s": time.perf_counter() - T_START,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
