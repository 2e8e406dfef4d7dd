"""GPU parity: libfim.so (through the C ABI) against the CPU oracle.

Integer work, so the bar is bit-exact: identical itemsets and supports in
canonical order, and the same number of candidate pairs when both sides use
the same extension order.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fim():
    import paper_2108_05038_amd as F
    F.lib()
    return F


@pytest.fixture(scope="module")
def ctx(fim):
    c = fim.Context(0)
    yield c
    c.close()


def gpu_mine(fim, ctx, db, minsup=None, **opts):
    d = fim.Database(ctx, db.offsets, db.items, db.n_items)
    try:
        return fim.mine(ctx, d, minsup if minsup is not None else db.minsup, **opts)
    finally:
        d.close()


def assert_same(g, o, what=""):
    assert len(g) == len(o), (what, len(g), len(o))
    assert np.array_equal(g.offsets, o.offsets), what
    assert np.array_equal(g.items, o.items), what
    assert np.array_equal(g.supports, o.supports), what


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- thesis examples

def test_paper_eclat_example(fim, ctx):
    g = _load("eclat_example.json")
    db = synth.from_lists(g["transactions"], minsup=g["minsup"])
    say("eclat example")
    r = gpu_mine(fim, ctx, db)
    want = {tuple(t["itemset"]): len(t["tids"]) for t in g["tidlists"] if t["frequent"]}
    assert r.as_dict() == want
    assert r.stats["candidates"] == 19  # hand-counted, ascending-support order
    r = gpu_mine(fim, ctx, db, flags=fim.FIM_FLAG_ORDER_BY_ID)
    assert r.as_dict() == want and r.stats["candidates"] == 20


def test_paper_apriori_example(fim, ctx):
    g = _load("apriori_example.json")
    db = synth.from_lists(g["transactions"], minsup=g["minsup"])
    say("apriori example")
    want = {tuple(int(x) for x in k.split(",")): v for k, v in g["frequent"].items()}
    assert gpu_mine(fim, ctx, db).as_dict() == want


# ---------------------------------------------------------------- random inputs

def test_tiny_random_vs_bruteforce(fim, ctx):
    rng = np.random.default_rng(2024)
    for case in range(150):
        n_items = int(rng.integers(1, 14))
        n_tx = int(rng.integers(0, 70))
        dens = float(rng.uniform(0.1, 0.9))
        T = [[i for i in range(n_items) if rng.random() < dens] for _ in range(n_tx)]
        m = int(rng.integers(1, max(2, n_tx // 2 + 2)))
        db = synth.from_lists(T, n_items=n_items, minsup=m)
        if case % 25 == 0:
            say("tiny", case)
        o = oracle.mine_db(db, "bruteforce")
        g = gpu_mine(fim, ctx, db)
        assert_same(g, o, ("tiny", case))


@pytest.mark.parametrize("n_tx,n_items,mlen,minsup", [
    (3001, 150, 10.0, 12),    # ragged word tail, two row tiles
    (4097, 400, 12.0, 9),     # more than 64 frequent items, deep classes
    (777, 90, 20.0, 25),      # long transactions
    (10000, 1000, 10.0, 20),  # basket shape at a lower minimum support
])
def test_medium_vs_oracle(fim, ctx, n_tx, n_items, mlen, minsup):
    o_, it, ni = synth.basket(n_tx * 7 + n_items, n_tx, n_items, mlen, 2 * n_items, 4.0)
    db = synth.Database(o_, it, ni, minsup)
    say("medium", n_tx, n_items, minsup)
    o = oracle.mine_db(db, threads=4)
    g = gpu_mine(fim, ctx, db)
    assert len(o) > 200
    assert_same(g, o)
    assert g.stats["candidates"] == o.candidates
    oi = oracle.mine_db(db, order=oracle.ORDER_ID, threads=4)
    gi = gpu_mine(fim, ctx, db, flags=fim.FIM_FLAG_ORDER_BY_ID)
    assert_same(gi, oi)
    assert gi.stats["candidates"] == oi.candidates


def test_dense_reduced_vs_oracle(fim, ctx):
    o_, it, ni = synth.dense(synth.SEED_BASE + 3, 2500, 120)
    db = synth.Database(o_, it, ni, 1000)  # 40 % as in the full dense workload
    say("dense reduced")
    o = oracle.mine_db(db, threads=8)
    assert len(o) > 100000
    # default, estimate counted in the run, the thesis's reservoir, and none
    for flags in (0, fim.FIM_FLAG_ALWAYS_ESTIMATE,
                  fim.FIM_FLAG_RESERVOIR | fim.FIM_FLAG_ALWAYS_ESTIMATE, fim.FIM_FLAG_NO_ESTIMATE):
        g = gpu_mine(fim, ctx, db, flags=flags)
        assert_same(g, o, flags)
        assert g.stats["candidates"] == o.candidates
        # the waves' busy times are reported (busiest >= mean > 0)
        assert g.stats["dfs_busy_max_ns"] >= g.stats["dfs_busy_mean_ns"] > 0
        if flags & fim.FIM_FLAG_ALWAYS_ESTIMATE:
            assert g.stats["estimate_ns"] > 0


# ---------------------------------------------------------------- options do not change F

def test_options_invariance(fim, ctx):
    o_, it, ni = synth.basket(77, 5000, 300, 14.0, 600, 5.0)
    db = synth.Database(o_, it, ni, 15)
    o = oracle.mine_db(db, threads=4)
    variants = [
        dict(workers=4), dict(workers=64, classes_per_wg=3), dict(flags=fim.FIM_FLAG_NO_ESTIMATE),
        dict(flags=fim.FIM_FLAG_NO_SPLIT), dict(alpha=1.0), dict(alpha=0.05, seed=99),
        dict(flags=fim.FIM_FLAG_DENSE_ROOT), dict(flags=fim.FIM_FLAG_ALWAYS_ESTIMATE),
        dict(flags=fim.FIM_FLAG_NO_PROJECT), dict(flags=fim.FIM_FLAG_NO_PROJECT, workers=8),
        dict(flags=fim.FIM_FLAG_RESERVOIR | fim.FIM_FLAG_ALWAYS_ESTIMATE),
        dict(flags=fim.FIM_FLAG_ALWAYS_ESTIMATE, workers=8, alpha=0.1),
        dict(sample_tx=500, sample_fi=1000),
    ]
    for v in variants:
        say("variant", v)
        g = gpu_mine(fim, ctx, db, **v)
        assert_same(g, o, v)
        assert g.stats["candidates"] == o.candidates, v


@pytest.mark.parametrize("n_tx,n_items,mlen,minsup", [
    (20000, 800, 10.0, 40),   # sparse rows: covers or projected transactions by default
    (9000, 300, 25.0, 60),    # denser rows
    (40000, 20000, 6.0, 4),   # more frequent items than one LDS tile of counters
    (60000, 150, 8.0, 300),   # few row tiles over long rows: whole-row words split over blocks
])
def test_root_kernels_agree(fim, ctx, n_tx, n_items, mlen, minsup):
    # the three exact root-class kernels, forced in turn and by default,
    # against the oracle
    o_, it, ni = synth.basket(n_tx + n_items, n_tx, n_items, mlen, 2 * n_items, 4.0)
    db = synth.Database(o_, it, ni, minsup)
    say("root kernels", n_tx, n_items)
    o = oracle.mine_db(db, threads=4)
    runs = {"default": gpu_mine(fim, ctx, db)}
    for name, flag, kind in (("rows", fim.FIM_FLAG_DENSE_ROOT, 0),
                             ("covers", fim.FIM_FLAG_ROOT_COVERS, 1),
                             ("project", fim.FIM_FLAG_ROOT_PROJECT, 2)):
        r = gpu_mine(fim, ctx, db, flags=flag)
        if n_items <= 65535 or kind != 1:
            assert r.stats["root_kernel"] == kind, name
        runs[name] = r
    for name, r in runs.items():
        assert_same(r, o, name)
        assert r.stats["candidates"] == o.candidates, name
    # covers skip words of whole rows
    assert runs["covers"].stats["root_pair_words"] < runs["rows"].stats["root_pair_words"]
    # classes below the root on rows projected on their prefix's cover, or not
    full = gpu_mine(fim, ctx, db, flags=fim.FIM_FLAG_NO_PROJECT)
    assert_same(full, o, "no projection")
    assert full.stats["candidates"] == o.candidates
    d, f = runs["default"].stats, full.stats
    if f["pair_words"] > f["root_pair_words"]:  # there is work below the root
        assert d["pair_words"] - d["root_pair_words"] < f["pair_words"] - f["root_pair_words"]


def test_projected_root_long_transactions(fim, ctx):
    # transactions of more than one wave of items (up to 127) with infrequent
    # items among them: the ranked transactions are built 64 items at a time
    o_, it, ni = synth.basket(3600, 3000, 600, 90.0, 1200, 4.0)
    db = synth.Database(o_, it, ni, 300)
    assert max(np.diff(np.asarray(o_))) > 64
    say("projected root, long transactions")
    o = oracle.mine_db(db, threads=4)
    assert max(len(u) for u in o.itemsets()) >= 3
    for flags in (fim.FIM_FLAG_ROOT_PROJECT, fim.FIM_FLAG_ROOT_PROJECT | fim.FIM_FLAG_NO_PROJECT, 0):
        g = gpu_mine(fim, ctx, db, flags=flags)
        if flags & fim.FIM_FLAG_ROOT_PROJECT:
            assert g.stats["root_kernel"] == 2
        assert_same(g, o, flags)
        assert g.stats["candidates"] == o.candidates, flags


def test_projection_with_work_sharing(fim, ctx):
    # few workers and a skewed database: donated classes (prefixes of two or
    # more items) are rebuilt projected on their own covers
    o_, it, ni = synth.basket(99, 30000, 400, 18.0, 300, 7.0)
    db = synth.Database(o_, it, ni, 60)
    say("projection + donations")
    o = oracle.mine_db(db, threads=8)
    assert len(o) > 20000
    for v in (dict(workers=4), dict(workers=16, flags=fim.FIM_FLAG_NO_SPLIT), dict()):
        g = gpu_mine(fim, ctx, db, **v)
        assert_same(g, o, v)
        assert g.stats["candidates"] == o.candidates, v


def test_long_itemsets_over_wide_ids(fim, ctx):
    # 2^20 item ids need 21-bit codes: itemsets of more than 6 items do not fit
    # a 128-bit key, so the call falls back to variable-length records
    big = [5, 77, 1000, 65535, 99999, 400000, 777777, 1048575]
    T = [big] * 3 + [big[:3]] * 2 + [[1, 2]] * 4 + [[2, 3, 4]] * 2
    db = synth.from_lists(T, n_items=1 << 20, minsup=2)
    say("long itemsets, wide ids")
    o = oracle.mine_db(db, "bruteforce")
    assert max(len(u) for u in o.itemsets()) == 8
    assert_same(gpu_mine(fim, ctx, db), o)
    # short enough for keys with wide ids
    db6 = synth.from_lists([big[:6]] * 3 + [[1, 2]] * 4, n_items=1 << 20, minsup=2)
    assert_same(gpu_mine(fim, ctx, db6), oracle.mine_db(db6, "bruteforce"))


def test_max_len(fim, ctx):
    o_, it, ni = synth.basket(5, 3000, 100, 12.0, 200, 5.0)
    db = synth.Database(o_, it, ni, 10)
    full = oracle.mine_db(db)
    for L in (1, 2, 3, 4):
        say("max_len", L)
        g = gpu_mine(fim, ctx, db, max_len=L)
        want = {u: s for u, s in full.as_dict().items() if len(u) <= L}
        assert g.as_dict() == want


def test_result_views_outlive_the_result_object(fim, ctx):
    # the binding hands out views of the library's result arrays (no copy):
    # they stay valid after the Result object is gone and its handle would
    # otherwise be released, and they are read-only; the pooled host memory
    # of released results is reused by later calls without disturbing them
    import gc
    o_, it, ni = synth.basket(77, 4000, 300, 12.0, 600, 4.0)
    db = synth.Database(o_, it, ni, 40)
    say("result views")
    o = oracle.mine_db(db, threads=4)
    r = gpu_mine(fim, ctx, db)
    off, items, supp = r.offsets, r.items, r.supports
    del r
    gc.collect()
    for _ in range(3):  # later results reuse released pool blocks
        gpu_mine(fim, ctx, db)
        gc.collect()
    assert oracle.digest(off, items, supp) == oracle.digest(o.offsets, o.items, o.supports)
    with pytest.raises(ValueError):
        items[0] = 0


# ---------------------------------------------------------------- edge cases and errors

def test_edge_cases(fim, ctx):
    say("edge cases")
    assert len(gpu_mine(fim, ctx, synth.from_lists([], n_items=4, minsup=1))) == 0
    assert len(gpu_mine(fim, ctx, synth.from_lists([[], [], []], n_items=4, minsup=1))) == 0
    T = [[0, 1], [1, 2], [0, 1, 2]]
    assert len(gpu_mine(fim, ctx, synth.from_lists(T, n_items=3, minsup=4))) == 0
    assert gpu_mine(fim, ctx, synth.from_lists(T, n_items=3, minsup=1)).as_dict() == \
        oracle.mine_db(synth.from_lists(T, n_items=3, minsup=1), "bruteforce").as_dict()
    dup = synth.from_lists([[3, 1, 3, 2], [2, 2], [1, 3], [3, 3, 3]], n_items=5, minsup=2)
    assert gpu_mine(fim, ctx, dup).as_dict() == {(1,): 2, (2,): 2, (3,): 3, (1, 3): 2}
    one = synth.from_lists([[7]] * 40, n_items=8, minsup=40)
    assert gpu_mine(fim, ctx, one).as_dict() == {(7,): 40}
    # every transaction identical: all 2^12 - 1 subsets are frequent
    full = synth.from_lists([list(range(12))] * 33, n_items=12, minsup=33)
    r = gpu_mine(fim, ctx, full)
    assert len(r) == 4095 and set(r.supports.tolist()) == {33}


def test_errors(fim, ctx):
    say("errors")
    with pytest.raises(fim.FimError) as e:
        fim.Database(ctx, np.array([0, 2], np.uint64), np.array([1, 9], np.uint32), 5)
    assert e.value.status == fim.FIM_E_ITEM_RANGE
    with pytest.raises(fim.FimError) as e:
        fim.Database(ctx, np.array([0, 2, 1], np.uint64), np.array([1, 2], np.uint32), 5)
    assert e.value.status == fim.FIM_E_INVALID_ARG
    d = fim.Database(ctx, np.array([0, 2], np.uint64), np.array([1, 2], np.uint32), 5)
    with pytest.raises(fim.FimError) as e:
        fim.mine(ctx, d, 0)
    assert e.value.status == fim.FIM_E_INVALID_ARG
    full = synth.from_lists([list(range(10))] * 5, n_items=10, minsup=1)
    with pytest.raises(fim.FimError) as e:
        gpu_mine(fim, ctx, full, max_itemsets=100)
    assert e.value.status == fim.FIM_E_OUTPUT_LIMIT
    d.close()


# ---------------------------------------------------------------- full workloads

@pytest.mark.parametrize("name", ["basket-10k", "dense-50k", "sparse-200k"])
def test_full_workload_vs_golden(fim, ctx, name):
    g = _load("%s.json" % name)
    db = synth.make(name)
    say("full", name)
    r = gpu_mine(fim, ctx, db)
    assert len(r) == g["n_itemsets"]
    assert oracle.digest(r.offsets, r.items, r.supports) == g["digest"]
    assert r.stats["candidates"] == g["candidates_ascending_support"]
    # sampled supports recounted by the oracle's scan
    rng = np.random.default_rng(1)
    for i in rng.choice(len(r), min(40, len(r)), replace=False):
        u = r.items[r.offsets[i]:r.offsets[i + 1]]
        assert oracle.support(db.offsets, db.items, u) == r.supports[i]


# ---------------------------------------------------------------- batch and serving

def _batch_dbs(k, scale=0.25):
    out = []
    for i in range(k):
        p = synth.batch_params(i)
        p["n_tx"] = max(1000, int(p["n_tx"] * scale))
        p["minsup"] = synth.minsup_abs(p["rel_minsup"], p["n_tx"])
        out.append(synth.batch_instance(p, "b%d" % i))
    return out


def test_batch_equals_solo_and_oracle(fim, ctx):
    dbs = _batch_dbs(6)
    handles = [fim.Database(ctx, d.offsets, d.items, d.n_items) for d in dbs]
    say("batch of", len(dbs))
    res = fim.mine_batch(ctx, handles, [d.minsup for d in dbs])
    for d, h, r in zip(dbs, handles, res):
        o = oracle.mine_db(d, threads=4, max_sets=3_000_000)
        assert not o.overflow
        assert_same(r, o, d.name)
        solo = fim.mine(ctx, h, d.minsup)
        assert_same(solo, o, d.name)
        assert solo.stats["candidates"] == r.stats["candidates"] == o.candidates
    for h in handles:
        h.close()


def test_exploding_estimate_sample_is_abandoned(fim, ctx):
    # Small instances at a low minimum support: the estimate's sample, drawn
    # with replacement at the scaled support (at least 2), makes every subset
    # of a long transaction drawn twice frequent.  Its search must be cut off
    # (no estimate for that instance) and the real result stay exact.
    g = _load("batch-256.json")
    picks = [227, 56, 90, 131]
    dbs = [synth.batch_instance(synth.batch_params(g["instances"][i]["substream"])) for i in picks]
    handles = [fim.Database(ctx, d.offsets, d.items, d.n_items) for d in dbs]
    for i, d, h in zip(picks, dbs, handles):
        say("exploding sample", i)
        r = fim.mine(ctx, h, d.minsup, flags=fim.FIM_FLAG_ALWAYS_ESTIMATE)
        assert oracle.digest(r.offsets, r.items, r.supports) == g["instances"][i]["digest"], i
    say("exploding samples, batched")
    res = fim.mine_batch(ctx, handles, [d.minsup for d in dbs], flags=fim.FIM_FLAG_ALWAYS_ESTIMATE)
    for i, r in zip(picks, res):
        assert oracle.digest(r.offsets, r.items, r.supports) == g["instances"][i]["digest"], i
    for h in handles:
        h.close()


def test_max_itemsets_stops_early(fim, ctx):
    # the whole powerset of 26 items (67 M itemsets) is never enumerated:
    # the kernel stops once the limit is certain to be exceeded
    db = synth.from_lists([list(range(26))] * 3, n_items=26, minsup=2)
    say("max_itemsets early stop")
    with pytest.raises(fim.FimError) as e:
        gpu_mine(fim, ctx, db, max_itemsets=100000)
    assert e.value.status == fim.FIM_E_OUTPUT_LIMIT


def test_autotune_settings_do_not_change_results(fim, ctx):
    dbs = _batch_dbs(4, scale=0.1)
    handles = [fim.Database(ctx, d.offsets, d.items, d.n_items) for d in dbs]
    ms = [d.minsup for d in dbs]
    say("autotune")
    t = fim.autotune(ctx, handles, ms, reps=1)
    assert t["tile_words"] in (256, 512, 1024, 2048) and t["classes_per_wg"] in (1, 2, 4)
    ref = fim.mine_batch(ctx, handles, ms)
    oracles = [oracle.mine_db(d, threads=4) for d in dbs]
    for r, o, d in zip(ref, oracles, dbs):
        assert_same(r, o, d.name)
        assert r.stats["candidates"] == o.candidates
    for tw in (256, 512, 1024, 2048, 3000):
        for c in (1, 4):
            got = fim.mine_batch(ctx, handles, ms, tile_words=tw, classes_per_wg=c)
            for a, o in zip(got, oracles):
                assert_same(a, o, (tw, c))
                assert a.stats["candidates"] == o.candidates
    for h in handles:
        h.close()


@pytest.mark.parametrize("lanes,max_active,budget", [(1, 3, 0), (3, 4, 0), (2, 64, 1)])
def test_server_results_same_alone_and_mixed(fim, ctx, lanes, max_active, budget):
    dbs = _batch_dbs(5, scale=0.1)
    dbs.append(synth.dense_instance(synth.dense_params(9, synth.SERVE_BASE, 1000, 4000)))
    handles = [fim.Database(ctx, d.offsets, d.items, d.n_items) for d in dbs]
    alone = [fim.mine(ctx, h, d.minsup) for d, h in zip(dbs, handles)]
    # every request alone against the oracle, so that mixed = alone = oracle
    for k, (d, r) in enumerate(zip(dbs, alone)):
        o = oracle.mine_db(d, threads=4)
        assert_same(r, o, ("alone", k))
        assert r.stats["candidates"] == o.candidates
    say("server", lanes, max_active, budget)
    srv = fim.Server(ctx, max_active=max_active, lanes=lanes, hbm_budget_bytes=budget)
    tickets = [srv.submit(h, d.minsup) for d, h in zip(dbs, handles)]
    tickets += [srv.submit(h, d.minsup) for d, h in zip(dbs[::-1], handles[::-1])]
    got = [srv.wait(t) for t in tickets]
    for k, r in enumerate(got):
        i = k if k < len(dbs) else len(dbs) - 1 - (k - len(dbs))
        assert_same(r, alone[i], k)
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["peak_active"] <= max_active
    if budget == 1:  # every request is admitted alone
        assert st["peak_active"] == 1 and st["steps"] == len(tickets)
    # the same requests again, taken in completion order
    tickets = {srv.submit(h, d.minsup): i for i, (d, h) in enumerate(zip(dbs, handles))}
    seen = 0
    while seen < len(tickets):
        t, r = srv.next(30.0)
        assert t in tickets
        assert_same(r, alone[tickets[t]], ("next", t))
        seen += 1
    assert srv.next(0.01) == (0, None)
    srv.close()
    for h in handles:
        h.close()


# ---------------------------------------------------------------- full-size batch and serving pool

def test_batch_256_full_size_vs_golden(fim, ctx):
    # all 256 batch instances at their full sizes in one batched call, and
    # each one alone, against the oracle's stored digests and candidate counts
    g = _load("batch-256.json")
    say("batch-256: generating")
    dbs = [synth.batch_instance(synth.batch_params(e["substream"])) for e in g["instances"]]
    handles = [fim.Database(ctx, d.offsets, d.items, d.n_items) for d in dbs]
    ms = [d.minsup for d in dbs]
    assert ms == [e["minsup"] for e in g["instances"]]
    say("batch-256: one batched call")
    res = fim.mine_batch(ctx, handles, ms)
    bad = [i for i, (r, e) in enumerate(zip(res, g["instances"]))
           if oracle.digest(r.offsets, r.items, r.supports) != e["digest"]
           or r.stats["candidates"] != e["candidates_ascending_support"]]
    assert not bad, bad
    del res
    say("batch-256: each instance alone")
    for i, (h, m, e) in enumerate(zip(handles, ms, g["instances"])):
        r = fim.mine(ctx, h, m)
        assert oracle.digest(r.offsets, r.items, r.supports) == e["digest"], i
        assert r.stats["candidates"] == e["candidates_ascending_support"], i
    for h in handles:
        h.close()
    ctx.release_cached()


def test_serve_pool_512_vs_golden(fim, ctx):
    # every request of the 512-request serving pool (one in ten dense)
    # submitted to the server at once, results against the stored digests;
    # then a second round in reverse order while the first is still running
    g = _load("serve-pool.json")
    say("serve pool: generating")
    handles, ms = [], []
    for k, e in enumerate(g["instances"]):
        d = synth.serve_instance(synth.serve_params(k, e["substream"]))
        assert d.minsup == e["minsup"], k
        handles.append(fim.Database(ctx, d.offsets, d.items, d.n_items))
        ms.append(d.minsup)
        del d
    say("serve pool: 2 x 512 requests")
    srv = fim.Server(ctx)
    first = [srv.submit(h, m) for h, m in zip(handles, ms)]
    second = [srv.submit(h, m) for h, m in zip(handles[::-1], ms[::-1])][::-1]
    for k, e in enumerate(g["instances"]):
        for t in (first[k], second[k]):
            r = srv.wait(t)
            assert oracle.digest(r.offsets, r.items, r.supports) == e["digest"], k
            assert len(r) == e["n_itemsets"], k
    st = srv.stats()
    assert st["completed"] == 2 * len(handles)
    srv.close()
    for h in handles:
        h.close()
    ctx.release_cached()


def test_context_closed_before_its_databases(fim):
    # closing a context first closes the databases and servers made on it
    # (the library frees a database through its context); closing them again
    # afterwards does nothing
    say("context closed before its database and server")
    c = fim.Context(0)
    d = fim.Database(c, np.array([0, 2, 3], np.uint64), np.array([0, 1, 1], np.uint32), 2)
    r = fim.mine(c, d, 1)
    assert len(r) == 3  # {0}, {1}, {0, 1}
    srv = fim.Server(c)
    c.close()
    assert d.handle is None and not srv.handle
    d.close()
    srv.close()
    del r
