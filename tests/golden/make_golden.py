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


def main(argv):
    names = argv or NAMES
    threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    for name in names:
        g = golden(name, threads)
        path = os.path.join(HERE, "%s.json" % name)
        with open(path, "w") as f:
            json.dump(g, f, indent=1)
        print(name, g["n_itemsets"], g["digest"][:16], "%.1fs" % g["oracle_seconds"], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
