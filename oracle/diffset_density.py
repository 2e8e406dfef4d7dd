"""Diffset density of a workload's classes, measured on the oracle's result.

Test infrastructure (it runs the CPU oracle); it prints the figures that
decide whether a list-form diffset representation would pay on the GPU.

For every frequent itemset X of two or more items, with P its prefix in the
depth-first order (X minus its last item in ascending-support order), the
diffset d(X) = T(P) minus T(X) has supp(P) - supp(X) transactions (appendix
on sequential algorithms, the concept of diffsets: the support of a class
member follows from its parent's support minus the size of its diffset).
The script reports, over all such X:

* the density |d(X)| / |T(P)| (median and quantiles, and by length);
* the share of X whose diffset, stored as a list of 32-bit transaction ids,
  is smaller than the bitmap the GPU path stores for X's row (a full-width
  row of ceil(n_tx / 32) words when the cover is not projected, or a row
  projected on T(P) of ceil(supp(P) / 32) words when it is);
* total list words against total bitmap words.

    python oracle/diffset_density.py [workload]     (default dense-50k)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, _ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def measure(db, res):
    n_tx = db.n_tx
    off = res.offsets.astype(np.int64)
    items = res.items
    sup = res.supports.astype(np.int64)
    lens = np.diff(off)
    # ascending (support, item id) order of the frequent items: the class order
    single = lens == 1
    s_item = items[off[:-1][single]]
    s_sup = sup[single]
    order = np.lexsort((s_item, s_sup))
    rank = np.full(db.n_items, -1, np.int64)
    rank[s_item[order]] = np.arange(len(order))
    # every itemset's items in class order, as a tuple key
    key_of = {}
    keys = []
    for i in range(len(sup)):
        its = items[off[i]:off[i + 1]]
        t = tuple(sorted(its.tolist(), key=lambda x: rank[x]))
        keys.append(t)
        key_of[t] = sup[i]
    dens, d_abs, p_sup, L = [], [], [], []
    for i, t in enumerate(keys):
        if len(t) < 2:
            continue
        sp = key_of[t[:-1]]
        dens.append((sp - sup[i]) / sp)
        d_abs.append(sp - sup[i])
        p_sup.append(sp)
        L.append(len(t))
    dens = np.array(dens)
    d_abs = np.array(d_abs)
    p_sup = np.array(p_sup)
    L = np.array(L)
    W = (n_tx + 31) // 32
    proj = (p_sup + 31) // 32
    # the GPU path projects a row on its prefix's cover when that cover is at
    # most a quarter of the database
    bitmap_words = np.where(4 * proj <= W, proj, W)
    return {
        "n_tx": n_tx, "itemsets_ge2": int(len(dens)),
        "density_median": float(np.median(dens)), "density_mean": float(dens.mean()),
        "density_q10_q90": [float(np.quantile(dens, 0.1)), float(np.quantile(dens, 0.9))],
        "share_below_1_32": float((dens < 1 / 32).mean()),
        "share_list_smaller_than_row": float((d_abs < bitmap_words).mean()),
        "list_words": int(d_abs.sum()), "bitmap_words": int(bitmap_words.sum()),
        "median_by_length": {int(k): float(np.median(dens[L == k])) for k in np.unique(L)},
    }


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "dense-50k"
    db = synth.make(name)
    t0 = time.perf_counter()
    res = oracle.mine_db(db)
    print("%s: %d itemsets mined by the oracle in %.1f s" % (name, len(res), time.perf_counter() - t0))
    for k, v in measure(db, res).items():
        print("  %s: %s" % (k, v))


if __name__ == "__main__":
    main()
