"""CPU oracle for frequent-itemset mining — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the benchmark's ``cpu_baseline`` leg and the smoke check
may import this package. The GPU library never calls it and shares no code
with it; the only thing both sides share is the seeded input generator in
``synth``.

The plain C miners live in ``oracle.c`` (compiled with gcc into
``liboracle.so`` beside this file):

* :func:`bruteforce` — all subsets of the items present, supports by scanning
  (definitions of cover, support and frequent itemset in the chapter on
  mathematical foundations).
* :func:`eclat` — Eclat-DFS over sorted tid-lists (appendix on sequential
  algorithms, the Eclat section: support counting by tid-list intersection and
  the depth-first search over prefix-based classes), with an optional
  ascending-support order of each class's extensions (section on the
  ordering of items in DFS algorithms).
* :func:`apriori` — level-wise Apriori (appendix, the Apriori algorithm).
* :func:`support` — support of one itemset by a full scan.

Every miner returns the canonical result: items ascending inside an itemset
and itemsets in lexicographic order (a prefix before its extensions).
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORDER_ID = 0
ORDER_ASCENDING_SUPPORT = 1


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (always when ``force``)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=gnu99", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Res(ctypes.Structure):
    _fields_ = [("n_sets", ctypes.c_uint64), ("n_items", ctypes.c_uint64),
                ("offsets", ctypes.POINTER(ctypes.c_uint64)),
                ("items", ctypes.POINTER(ctypes.c_uint32)),
                ("supports", ctypes.POINTER(ctypes.c_uint32)),
                ("candidates", ctypes.c_uint64), ("overflow", ctypes.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        u64p, u32p = P(ctypes.c_uint64), P(ctypes.c_uint32)
        lib.orc_bruteforce.argtypes = [ctypes.c_uint64, u64p, u32p, ctypes.c_uint32,
                                       ctypes.c_uint32, P(_Res)]
        lib.orc_eclat.argtypes = [ctypes.c_uint64, u64p, u32p, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_uint64, P(_Res)]
        lib.orc_apriori.argtypes = [ctypes.c_uint64, u64p, u32p, ctypes.c_uint32,
                                    ctypes.c_uint32, P(_Res)]
        lib.orc_support.argtypes = [ctypes.c_uint64, u64p, u32p, u32p, ctypes.c_uint32]
        lib.orc_support.restype = ctypes.c_uint64
        lib.orc_result_free.argtypes = [P(_Res)]
        _lib = lib
    return _lib


@dataclass
class Result:
    """Canonical frequent-itemset result in CSR form."""
    offsets: np.ndarray   # uint64[n + 1]
    items: np.ndarray     # uint32[total items], ascending within each itemset
    supports: np.ndarray  # uint32[n]
    candidates: int = 0   # pair supports computed inside classes (Eclat only)
    overflow: bool = False

    def __len__(self):
        return len(self.supports)

    def itemsets(self):
        o = self.offsets
        return [tuple(self.items[o[i]:o[i + 1]].tolist()) for i in range(len(self))]

    def as_dict(self):
        return dict(zip(self.itemsets(), self.supports.tolist()))

    def digest(self) -> str:
        return digest(self.offsets, self.items, self.supports)


def digest(offsets, items, supports) -> str:
    """SHA-256 of the canonical binary CSR (little-endian uint64/uint32/uint32)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offsets, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(items, dtype="<u4").tobytes())
    h.update(np.ascontiguousarray(supports, dtype="<u4").tobytes())
    return h.hexdigest()


def _args(offsets, items):
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    items = np.ascontiguousarray(items, dtype=np.uint32)
    if len(items) == 0:
        items = np.zeros(1, np.uint32)
    return (offsets, items, len(offsets) - 1,
            offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
            items.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))


def _take(res: _Res) -> Result:
    n, ni = int(res.n_sets), int(res.n_items)
    if res.offsets:
        offs = np.ctypeslib.as_array(res.offsets, shape=(n + 1,)).copy()
    else:
        offs = np.zeros(1, np.uint64)
    items = (np.ctypeslib.as_array(res.items, shape=(ni,)).copy() if ni
             else np.zeros(0, np.uint32))
    sup = (np.ctypeslib.as_array(res.supports, shape=(n,)).copy() if n
           else np.zeros(0, np.uint32))
    out = Result(offs.astype(np.uint64), items.astype(np.uint32), sup.astype(np.uint32),
                 int(res.candidates), bool(res.overflow))
    _load().orc_result_free(ctypes.byref(res))
    return out


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed (%d)" % (what, rc))


def bruteforce(offsets, items, n_items: int, minsup: int) -> Result:
    """All frequent itemsets by enumerating subsets (at most 24 distinct items present)."""
    o, it, n, po, pi = _args(offsets, items)
    res = _Res()
    _check(_load().orc_bruteforce(n, po, pi, n_items, minsup, ctypes.byref(res)), "bruteforce")
    return _take(res)


def eclat(offsets, items, n_items: int, minsup: int, order: int = ORDER_ASCENDING_SUPPORT,
          threads: int = 1, max_sets: int = 0) -> Result:
    """Eclat-DFS over sorted tid-lists."""
    o, it, n, po, pi = _args(offsets, items)
    res = _Res()
    _check(_load().orc_eclat(n, po, pi, n_items, minsup, order, threads, max_sets,
                             ctypes.byref(res)), "eclat")
    return _take(res)


def apriori(offsets, items, n_items: int, minsup: int) -> Result:
    """Level-wise Apriori with per-transaction subset tests."""
    o, it, n, po, pi = _args(offsets, items)
    res = _Res()
    _check(_load().orc_apriori(n, po, pi, n_items, minsup, ctypes.byref(res)), "apriori")
    return _take(res)


def support(offsets, items, itemset) -> int:
    """Support of one itemset by scanning every transaction."""
    o, it, n, po, pi = _args(offsets, items)
    u = np.ascontiguousarray(itemset, dtype=np.uint32)
    if len(u) == 0:
        return n
    return int(_load().orc_support(n, po, pi, u.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                   len(u)))


def mine_db(db, method: str = "eclat", **kw) -> Result:
    """Mine a ``synth.Database`` at its own minimum support."""
    f = {"eclat": eclat, "apriori": apriori, "bruteforce": bruteforce}[method]
    return f(db.offsets, db.items, db.n_items, db.minsup, **kw)
