"""Write the expected results of the full-size workloads with the CPU oracle.

Only ``oracle`` and ``synth`` are used: every stored value is the oracle's
Eclat result on the seeded synthetic input (canonical CSR digest, counts,
candidate pairs under the ascending-support order).

    python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

NAMES = ["basket-10k", "sparse-200k", "dense-50k"]


def golden(name: str, threads: int) -> dict:
    db = synth.make(name)
    t0 = time.time()
    res = oracle.mine_db(db, threads=threads)
    dt = time.time() - t0
    lens = np.diff(res.offsets.astype(np.int64))
    return {
        "workload": name,
        "n_tx": db.n_tx,
        "n_items": db.n_items,
        "nnz": int(len(db.items)),
        "minsup": db.minsup,
        "n_itemsets": len(res),
        "n_items_total": int(len(res.items)),
        "by_length": np.bincount(lens).tolist() if len(lens) else [],
        "candidates_ascending_support": res.candidates,
        "digest": res.digest(),
        "oracle_seconds": round(dt, 2),
        "oracle_threads": threads,
    }


def _instance_golden(db, threads):
    t0 = time.time()
    res = oracle.mine_db(db, threads=threads, max_sets=synth.GUARD_LIMIT)
    return res, time.time() - t0


def golden_batch(threads: int, n: int = 256) -> dict:
    """Oracle results of the batch instances, with the explosion guard: an
    instance with more than GUARD_LIMIT itemsets is redrawn from substream
    index + GUARD_STRIDE (repeatedly) and the substream used is recorded."""
    out = []
    for i in range(n):
        sub = i
        while True:
            p = synth.batch_params(sub)
            res, dt = _instance_golden(synth.batch_instance(p), threads)
            if not res.overflow:
                break
            print("instance", i, "substream", sub, "exceeds the guard; redrawn", flush=True)
            sub += synth.GUARD_STRIDE
        out.append({"index": i, "substream": sub, "n_tx": p["n_tx"], "n_items": p["n_items"],
                    "minsup": p["minsup"], "n_itemsets": len(res),
                    "candidates_ascending_support": res.candidates, "digest": res.digest(),
                    "oracle_seconds": round(dt, 2)})
        print("batch", i, len(res), round(dt, 2), flush=True)
    return {"workload": "batch-%d" % n, "guard_limit": synth.GUARD_LIMIT, "instances": out}


def golden_serve(threads: int, n: int = 512) -> dict:
    """Oracle results of the serving pool, with the same explosion guard as
    the batch (redraws recorded as the substream used)."""
    out = []
    for k in range(n):
        sub = k
        while True:
            p = synth.serve_params(k, sub)
            res, dt = _instance_golden(synth.serve_instance(p), threads)
            if not res.overflow:
                break
            print("request", k, "substream", sub, "exceeds the guard; redrawn", flush=True)
            sub += synth.GUARD_STRIDE
        out.append({"index": k, "substream": sub, "kind": p.get("kind", "basket"),
                    "n_tx": p["n_tx"], "minsup": p["minsup"], "n_itemsets": len(res),
                    "candidates_ascending_support": res.candidates, "digest": res.digest(),
                    "oracle_seconds": round(dt, 2)})
        print("serve", k, out[-1]["kind"], len(res), round(dt, 2), flush=True)
    return {"workload": "serve-pool-%d" % n, "guard_limit": synth.GUARD_LIMIT, "instances": out}


def main(argv):
    threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    if argv and argv[0] in ("batch-256", "serve-pool"):
        g = golden_batch(threads) if argv[0] == "batch-256" else golden_serve(threads)
        with open(os.path.join(HERE, "%s.json" % argv[0]), "w") as f:
            json.dump(g, f, indent=0)
        return
    names = argv or NAMES
    for name in names:
        g = golden(name, threads)
        path = os.path.join(HERE, "%s.json" % name)
        with open(path, "w") as f:
            json.dump(g, f, indent=1)
        print(name, g["n_itemsets"], g["digest"][:16], "%.1fs" % g["oracle_seconds"], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
