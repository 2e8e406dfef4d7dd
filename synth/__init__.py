"""Seeded synthetic transaction databases (inputs only, no mining arithmetic).

The C generator in ``synth.c`` is compiled with gcc into ``libsynth.so`` next
to this file. Both the CPU oracle's tests and the GPU library's tests and
benchmarks take their inputs from here.

Workloads (the thesis's IBM-generator databases are not available, so these
stand in for them; see the dataset description of the experimental
evaluation):

* ``basket-10k``   10,000 basket transactions over 1,000 items, Poisson mean
                   length 10, 2,000 latent patterns of mean length 4,
                   minimum support 1 % = 100 transactions.
* ``sparse-200k``  200,000 transactions over 5,000 items, mean length 20,
                   10,000 patterns of mean length 6, minimum support 0.1 % = 200.
* ``dense-50k``    50,000 transactions over 120 items, item probabilities
                   Beta(4, 6) plus 20 planted groups of 8..12 items (group
                   activation uniform in [0, 0.5), each item of an active
                   group kept with probability 0.97), minimum support
                   40 % = 20,000.
* ``batch-256``    256 independent basket instances with log-uniform sizes
                   (see :func:`batch_params`).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

SEED_BASE = 2108050380


def build(force: bool = False) -> str:
    """Compile ``libsynth.so`` with gcc (always when ``force``)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _SynthDb(ctypes.Structure):
    _fields_ = [("n_tx", ctypes.c_uint64), ("nnz", ctypes.c_uint64),
                ("n_items", ctypes.c_uint32),
                ("offsets", ctypes.POINTER(ctypes.c_uint64)),
                ("items", ctypes.POINTER(ctypes.c_uint32))]


class _BasketParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_tx", ctypes.c_uint64),
                ("n_items", ctypes.c_uint32), ("mean_len", ctypes.c_double),
                ("rel_minsup", ctypes.c_double), ("n_patterns", ctypes.c_uint32),
                ("mean_pat_len", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        lib.synth_basket.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_double, ctypes.c_uint32, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     P(P(_SynthDb))]
        lib.synth_dense.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, P(P(_SynthDb))]
        lib.synth_free.argtypes = [P(_SynthDb)]
        lib.synth_substream.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_substream.restype = ctypes.c_uint64
        lib.synth_draw_basket_params.argtypes = [
            ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
            ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, P(_BasketParams)]
        lib.synth_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, P(ctypes.c_double)]
        lib.synth_exponentials.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                           P(ctypes.c_double)]
        lib.synth_raw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, P(ctypes.c_uint64)]
        _lib = lib
    return _lib


@dataclass
class Database:
    """A transaction database in CSR form plus the minimum support to mine it at."""
    offsets: np.ndarray  # uint64[n_tx + 1]
    items: np.ndarray    # uint32[nnz], each transaction sorted, no duplicates
    n_items: int         # item ids are in [0, n_items)
    minsup: int          # absolute minimum support (transactions)
    name: str = ""

    @property
    def n_tx(self) -> int:
        return len(self.offsets) - 1

    def transactions(self):
        o, it = self.offsets, self.items
        return [it[o[t]:o[t + 1]].tolist() for t in range(self.n_tx)]


def _take(ptr) -> tuple[np.ndarray, np.ndarray, int]:
    db = ptr.contents
    n = int(db.n_tx)
    nnz = int(db.nnz)
    offs = np.ctypeslib.as_array(db.offsets, shape=(n + 1,)).copy()
    items = (np.ctypeslib.as_array(db.items, shape=(nnz,)).copy() if nnz
             else np.zeros(0, np.uint32))
    n_items = int(db.n_items)
    _load().synth_free(ptr)
    return offs.astype(np.uint64), items.astype(np.uint32), n_items


def basket(seed, n_tx, n_items, mean_len, n_patterns, mean_pat_len,
           corr_mean=0.5, corrupt_mean=0.5, corrupt_sd=0.1):
    """Basket CSR (offsets, items, n_items) from the IBM-style generator."""
    ptr = ctypes.POINTER(_SynthDb)()
    rc = _load().synth_basket(seed, n_tx, n_items, mean_len, n_patterns, mean_pat_len,
                              corr_mean, corrupt_mean, corrupt_sd, ctypes.byref(ptr))
    if rc:
        raise RuntimeError("synth_basket failed (%d)" % rc)
    return _take(ptr)


def dense(seed, n_tx, n_items, beta_a=4, beta_b=6, n_groups=20, gmin=8, gmax=12,
          act_lo=0.0, act_hi=0.50, keep=0.97):
    """Dense CSR (offsets, items, n_items) with Beta item probabilities and planted groups."""
    ptr = ctypes.POINTER(_SynthDb)()
    rc = _load().synth_dense(seed, n_tx, n_items, beta_a, beta_b, n_groups, gmin, gmax,
                             act_lo, act_hi, keep, ctypes.byref(ptr))
    if rc:
        raise RuntimeError("synth_dense failed (%d)" % rc)
    return _take(ptr)


def minsup_abs(rel: float, n_tx: int) -> int:
    """Absolute minimum support ceil(rel * n_tx), at least 1, in double arithmetic."""
    return max(1, int(math.ceil(rel * n_tx)))


def substream(base: int, index: int) -> int:
    return int(_load().synth_substream(base, index))


def batch_params(index: int, base: int = SEED_BASE + 4, lo_tx=1000, hi_tx=200000,
                 lo_items=200, hi_items=5000, lo_len=8.0, hi_len=30.0,
                 lo_rel=0.002, hi_rel=0.05) -> dict:
    """Parameters of batch instance ``index`` (drawn from its own substream)."""
    p = _BasketParams()
    _load().synth_draw_basket_params(substream(base, index), lo_tx, hi_tx, lo_items, hi_items,
                                     lo_len, hi_len, lo_rel, hi_rel, ctypes.byref(p))
    return dict(seed=int(p.seed), n_tx=int(p.n_tx), n_items=int(p.n_items),
                mean_len=float(p.mean_len), rel_minsup=float(p.rel_minsup),
                n_patterns=int(p.n_patterns), mean_pat_len=float(p.mean_pat_len),
                minsup=minsup_abs(float(p.rel_minsup), int(p.n_tx)))


def batch_instance(params: dict, name: str = "") -> Database:
    o, it, ni = basket(params["seed"], params["n_tx"], params["n_items"], params["mean_len"],
                       params["n_patterns"], params["mean_pat_len"])
    return Database(o, it, ni, params["minsup"], name)


BATCH_BASE = SEED_BASE + 4
SERVE_BASE = SEED_BASE + 5
# a batch instance whose oracle result exceeds this many itemsets is redrawn
# from substream index + GUARD_STRIDE (the redraw is recorded in the manifest)
GUARD_LIMIT = 5_000_000
GUARD_STRIDE = 100_000


def serve_params(k: int, sub: int | None = None) -> dict:
    """Request k of the serving pool: 9 in 10 basket instances drawn like the
    batch instances (from their own substreams), 1 in 10 dense instances with
    log-uniform 1,000..50,000 transactions over 120 items at 40 % support.
    ``sub`` is the substream drawn from (default k; a request whose result
    exceeds GUARD_LIMIT itemsets is redrawn from k + GUARD_STRIDE, ...)."""
    sub = k if sub is None else sub
    if k % 10 == 9:
        return dense_params(sub, SERVE_BASE)
    p = batch_params(sub, base=SERVE_BASE)
    p["kind"] = "basket"
    return p


def serve_instance(params: dict, name: str = "") -> Database:
    if params.get("kind") == "dense":
        return dense_instance(params, name)
    return batch_instance(params, name)


def dense_params(index: int, base: int, lo_tx=1000, hi_tx=50000) -> dict:
    """Parameters of a dense request instance: log-uniform n_tx, 120 items, minsup 40 %."""
    u = uniforms(substream(base, index), 1)[0]
    n_tx = int(round(math.exp(math.log(lo_tx) + (math.log(hi_tx) - math.log(lo_tx)) * u)))
    return dict(kind="dense", seed=substream(base, index + 7777777), n_tx=n_tx, n_items=120,
                minsup=minsup_abs(0.4, n_tx))


def dense_instance(params: dict, name: str = "") -> Database:
    o, it, ni = dense(params["seed"], params["n_tx"], params["n_items"])
    return Database(o, it, ni, params["minsup"], name)


def uniforms(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, np.float64)
    _load().synth_uniforms(seed, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def exponentials(seed: int, n: int, mean: float) -> np.ndarray:
    out = np.zeros(n, np.float64)
    _load().synth_exponentials(seed, n, mean,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def raw(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, np.uint64)
    _load().synth_raw(seed, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def make(name: str) -> Database:
    """One of the named single-instance workloads."""
    if name == "basket-10k":
        o, it, ni = basket(SEED_BASE + 1, 10_000, 1_000, 10.0, 2_000, 4.0)
        return Database(o, it, ni, 100, name)
    if name == "sparse-200k":
        o, it, ni = basket(SEED_BASE + 2, 200_000, 5_000, 20.0, 10_000, 6.0)
        return Database(o, it, ni, 200, name)
    if name == "dense-50k":
        o, it, ni = dense(SEED_BASE + 3, 50_000, 120)
        return Database(o, it, ni, 20_000, name)
    raise KeyError(name)


def from_lists(transactions, n_items=None, minsup=1, name="") -> Database:
    """CSR from a list of item lists (duplicates kept as given, for input tests)."""
    offs = np.zeros(len(transactions) + 1, np.uint64)
    flat = []
    for i, t in enumerate(transactions):
        flat.extend(int(x) for x in t)
        offs[i + 1] = len(flat)
    items = np.asarray(flat, np.uint32)
    if n_items is None:
        n_items = int(items.max()) + 1 if len(items) else 1
    return Database(offs, items, n_items, minsup, name)
