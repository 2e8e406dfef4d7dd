"""Pins of the CPU oracle against what the thesis and the mathematics fix.

The oracle is checked against
  * the values the thesis prints for its worked examples (Eclat bottom-up
    example, Apriori example with its errata),
  * brute-force enumeration of all subsets on tiny inputs,
  * closed forms: singleton supports are the item histogram and pair supports
    are the co-occurrence Gram matrix X^T X of the 0/1 incidence matrix,
    computed here with numpy from Python sets,
  * invariants: downward closure and monotonicity of support, a sampled
    negative border, independence of item order and thread count,
  * hand-counted candidate numbers on the Eclat example.
None of these re-types the oracle's own formulas.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _db(transactions, minsup, n_items=None):
    return synth.from_lists(transactions, n_items=n_items, minsup=minsup)


def _set_support(transactions, itemset):
    u = set(itemset)
    return sum(1 for t in transactions if u <= set(t))


# ---------------------------------------------------------------- worked examples

def test_eclat_example_fixture_is_consistent():
    g = _load("eclat_example.json")
    T = g["transactions"]
    for row in g["tidlists"]:
        tids = [i + 1 for i, t in enumerate(T) if set(row["itemset"]) <= set(t)]
        assert tids == row["tids"], row
        assert (len(tids) >= g["minsup"]) == row["frequent"], row


@pytest.mark.parametrize("method", ["eclat", "apriori", "bruteforce"])
def test_eclat_example_printed_supports(method):
    g = _load("eclat_example.json")
    db = _db(g["transactions"], g["minsup"])
    kw = {"threads": 3} if method == "eclat" else {}
    got = oracle.mine_db(db, method, **kw).as_dict()
    assert len(got) == g["n_frequent"] == 23
    for row in g["tidlists"]:
        key = tuple(row["itemset"])
        if row["frequent"]:
            assert got[key] == len(row["tids"]), key
        else:
            assert key not in got, key
    # the example's tables cover every frequent itemset
    assert set(got) == {tuple(r["itemset"]) for r in g["tidlists"] if r["frequent"]}


def test_eclat_example_maximal_itemsets():
    # the two longest frequent itemsets of the example
    g = _load("eclat_example.json")
    got = oracle.mine_db(_db(g["transactions"], g["minsup"])).as_dict()
    maximal = [u for u in got if not any(set(u) < set(v) for v in got)]
    assert sorted(maximal) == [(1, 2, 3, 4), (1, 3, 4, 5)]


@pytest.mark.parametrize("method", ["eclat", "apriori", "bruteforce"])
def test_apriori_example_with_errata(method):
    g = _load("apriori_example.json")
    db = _db(g["transactions"], g["minsup"])
    got = oracle.mine_db(db, method).as_dict()
    want = {tuple(int(x) for x in k.split(",")): v for k, v in g["frequent"].items()}
    assert got == want
    # printed candidate supports that are right
    for level in ("C1", "C2", "C3"):
        for k, v in g["printed"][level].items():
            u = tuple(int(x) for x in k.split(","))
            if u == (5,):
                continue  # erratum: printed 5, true 4
            assert _set_support(g["transactions"], u) == v


def test_extensions_example_class_members():
    # [U | E] = { U + Y : Y non-empty subset of E }, the prefix itself excluded
    g = _load("extensions_example.json")
    U, E = g["prefix"], g["extensions"]
    members = []
    for r in range(1, len(E) + 1):
        for Y in itertools.combinations(E, r):
            members.append(sorted(U + list(Y)))
    assert sorted(members) == sorted(g["members"])
    # with every transaction holding the whole base set, the oracle reports
    # exactly these members among the itemsets with prefix U and suffix in E
    db = _db([g["base_set"]] * 3, 1)
    got = oracle.mine_db(db).as_dict()
    in_class = [list(k) for k in got
                if list(k[:len(U)]) == U and len(k) > len(U) and set(k[len(U):]) <= set(E)]
    assert sorted(in_class) == sorted(g["members"])


def test_candidate_counts_hand_counted():
    # Eclat example, counted by hand: 20 intersections with the atoms in id
    # order, 19 with ascending-support order (ties by id).
    g = _load("eclat_example.json")
    db = _db(g["transactions"], g["minsup"])
    assert oracle.mine_db(db, order=oracle.ORDER_ID).candidates == 20
    assert oracle.mine_db(db, order=oracle.ORDER_ASCENDING_SUPPORT).candidates == 19


# ---------------------------------------------------------------- brute force

def _random_tiny(rng, n_tx, n_items, density, dup=False):
    T = []
    for _ in range(n_tx):
        t = [i for i in range(n_items) if rng.random() < density]
        if dup and t:
            t = t + [t[int(rng.integers(len(t)))]]
            rng.shuffle(t)
        T.append(t)
    return T


def test_three_way_agreement_on_tiny_inputs():
    rng = np.random.default_rng(1234)
    for case in range(300):
        n_items = int(rng.integers(1, 13))
        n_tx = int(rng.integers(0, 40))
        T = _random_tiny(rng, n_tx, n_items, float(rng.uniform(0.1, 0.9)), dup=case % 3 == 0)
        m = int(rng.integers(1, max(2, n_tx + 2)))
        db = _db(T, m, n_items=n_items)
        bf = oracle.mine_db(db, "bruteforce")
        e1 = oracle.mine_db(db, "eclat", order=oracle.ORDER_ID)
        e2 = oracle.mine_db(db, "eclat", order=oracle.ORDER_ASCENDING_SUPPORT, threads=4)
        ap = oracle.mine_db(db, "apriori")
        d = bf.digest()
        assert e1.digest() == d and e2.digest() == d and ap.digest() == d, (case, T, m)
        # spot-check supports against a Python set count
        for u, s in list(bf.as_dict().items())[:5]:
            assert _set_support(T, u) == s


def test_bruteforce_against_python_definition():
    rng = np.random.default_rng(7)
    for _ in range(40):
        n_items = int(rng.integers(1, 8))
        T = _random_tiny(rng, int(rng.integers(1, 15)), n_items, 0.5)
        m = int(rng.integers(1, 5))
        want = {}
        for r in range(1, n_items + 1):
            for u in itertools.combinations(range(n_items), r):
                s = _set_support(T, u)
                if s >= m:
                    want[u] = s
        db = _db(T, m, n_items)
        assert oracle.bruteforce(db.offsets, db.items, n_items, m).as_dict() == want


# ---------------------------------------------------------------- closed forms

def _incidence(db):
    X = np.zeros((db.n_tx, db.n_items), np.float64)
    for t, items in enumerate(db.transactions()):
        X[t, list(set(items))] = 1.0
    return X


@pytest.mark.parametrize("seed", [11, 12])
def test_singletons_and_pairs_are_the_gram_matrix(seed):
    o, it, ni = synth.basket(seed, 3000, 60, 8.0, 80, 3.0)
    m = 30
    db = synth.Database(o, it, ni, m)
    G = _incidence(db).T @ _incidence(db)  # float64, exact for counts < 2**53
    got = oracle.mine_db(db).as_dict()
    singles = {u: s for u, s in got.items() if len(u) == 1}
    pairs = {u: s for u, s in got.items() if len(u) == 2}
    assert singles == {(i,): int(G[i, i]) for i in range(ni) if G[i, i] >= m}
    want_pairs = {(i, j): int(G[i, j]) for i in range(ni) for j in range(i + 1, ni)
                  if G[i, j] >= m and G[i, i] >= m and G[j, j] >= m}
    assert pairs == want_pairs
    assert len(pairs) > 20  # the case is not trivial


def test_duplicates_collapse_like_sets():
    T = [[3, 1, 3, 2], [2, 2], [1, 3], [3, 3, 3]]
    got = oracle.mine_db(_db(T, 2, 4)).as_dict()
    assert got == {(1,): 2, (2,): 2, (3,): 3, (1, 3): 2}


# ---------------------------------------------------------------- invariants

@pytest.fixture(scope="module")
def medium():
    o, it, ni = synth.basket(99, 4000, 150, 12.0, 120, 5.0)
    db = synth.Database(o, it, ni, 25)
    return db, oracle.mine_db(db)


def test_downward_closure_and_monotonicity(medium):
    db, res = medium
    got = res.as_dict()
    assert len(got) == len(res)  # no duplicates
    assert max(len(u) for u in got) >= 4
    for u, s in got.items():
        assert s >= db.minsup
        if len(u) > 1:
            for v in itertools.combinations(u, len(u) - 1):
                assert v in got and got[v] >= s, (u, v)


def test_sampled_supports_and_negative_border(medium):
    db, res = medium
    got = res.as_dict()
    rng = np.random.default_rng(5)
    keys = list(got)
    for idx in rng.choice(len(keys), 60, replace=False):
        u = keys[int(idx)]
        assert oracle.support(db.offsets, db.items, u) == got[u]
    # negative border: frequent U plus one more item that is not reported
    checked = 0
    for idx in rng.choice(len(keys), 400, replace=True):
        u = keys[int(idx)]
        b = int(rng.integers(db.n_items))
        if b in u:
            continue
        v = tuple(sorted(u + (b,)))
        if v in got:
            continue
        assert oracle.support(db.offsets, db.items, v) < db.minsup
        checked += 1
    assert checked > 100


def test_order_and_threads_do_not_change_the_result(medium):
    db, res = medium
    a = oracle.mine_db(db, order=oracle.ORDER_ID, threads=1)
    b = oracle.mine_db(db, order=oracle.ORDER_ASCENDING_SUPPORT, threads=5)
    assert a.digest() == b.digest() == res.digest()
    c = oracle.mine_db(db, order=oracle.ORDER_ASCENDING_SUPPORT, threads=1)
    assert c.candidates == b.candidates  # same classes, same work


def test_canonical_order_is_lexicographic(medium):
    _, res = medium
    sets = res.itemsets()
    assert all(list(u) == sorted(u) for u in sets)
    assert sets == sorted(sets)  # Python tuple order: prefix first, then by items


# ---------------------------------------------------------------- edge cases

def test_edge_cases():
    empty = synth.from_lists([], n_items=5, minsup=1)
    assert len(oracle.mine_db(empty)) == 0
    blank = synth.from_lists([[], [], []], n_items=5, minsup=1)
    assert len(oracle.mine_db(blank)) == 0
    T = [[0, 1], [1, 2], [0, 1, 2]]
    assert len(oracle.mine_db(_db(T, 4, 3))) == 0  # minsup above |D|
    every = oracle.mine_db(_db(T, 1, 3)).as_dict()  # minsup 1: every subset of a transaction
    assert set(every) == {(0,), (1,), (2,), (0, 1), (0, 2), (1, 2), (0, 1, 2)}
    with pytest.raises(RuntimeError):
        oracle.eclat(np.array([0, 1], np.uint64), np.array([0], np.uint32), 1, 0)


def test_output_cap_sets_overflow():
    T = [[0, 1, 2, 3, 4, 5]] * 3
    db = _db(T, 1, 6)
    r = oracle.eclat(db.offsets, db.items, 6, 1, max_sets=10)
    assert r.overflow
    r = oracle.eclat(db.offsets, db.items, 6, 1)
    assert not r.overflow and len(r) == 63


def test_support_scan_matches_python():
    rng = np.random.default_rng(3)
    T = _random_tiny(rng, 50, 10, 0.4, dup=True)
    db = _db(T, 1, 10)
    for _ in range(30):
        u = tuple(sorted(set(int(x) for x in rng.integers(0, 10, int(rng.integers(1, 4))))))
        assert oracle.support(db.offsets, db.items, u) == _set_support(T, u)
    assert oracle.support(db.offsets, db.items, ()) == 50
