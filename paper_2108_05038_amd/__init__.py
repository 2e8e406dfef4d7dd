"""Python binding of ``libfim.so``, the MI355X frequent-itemset miner.

The binding only marshals arguments: every step of mining runs in the HIP
kernels and the C++ runtime of the library (``include/fim.h`` documents the
ABI).  PyTorch, when present, supplies device memory (its caching
allocator) and the HIP stream; without it the library uses hipMalloc and
the null stream.  There is no CPU fallback: if the library or a gfx950 GPU
is missing, the calls raise.

Low level: functions named like the C entry points (``fim_ctx_create`` ...)
taking and returning opaque handles.  High level: :class:`Context`,
:class:`Database`, :func:`mine`, :func:`mine_batch`, :class:`Server`.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfim.so")

FIM_OK = 0
FIM_E_INVALID_ARG = -1
FIM_E_ITEM_RANGE = -2
FIM_E_OOM_HOST = -3
FIM_E_OOM_DEVICE = -4
FIM_E_DEVICE = -5
FIM_E_OUTPUT_LIMIT = -6
FIM_E_BUSY = -7
FIM_E_CANCELLED = -8
FIM_E_NOT_FOUND = -9
FIM_E_NO_DEVICE = -10

FIM_FLAG_NO_ESTIMATE = 0x1
FIM_FLAG_ORDER_BY_ID = 0x2
FIM_FLAG_NO_SPLIT = 0x4
FIM_FLAG_ALWAYS_ESTIMATE = 0x8
FIM_FLAG_DENSE_ROOT = 0x10
FIM_FLAG_ROOT_COVERS = 0x20
FIM_FLAG_ROOT_PROJECT = 0x40
FIM_FLAG_NO_PROJECT = 0x80
FIM_FLAG_RESERVOIR = 0x100

EXPORTED = [
    "fim_status_str", "fim_last_error", "fim_version", "fim_ctx_create", "fim_ctx_destroy",
    "fim_ctx_release_cached",
    "fim_db_create", "fim_db_destroy", "fim_db_sizes", "fim_minsup_from_relative", "fim_mine",
    "fim_mine_batch", "fim_autotune", "fim_result_sizes", "fim_result_copy", "fim_result_view",
    "fim_result_stats",
    "fim_result_destroy", "fim_server_create", "fim_server_submit", "fim_server_poll",
    "fim_server_wait", "fim_server_next", "fim_server_cancel", "fim_server_stats_get", "fim_server_destroy",
    "fim_estimate_sample_sizes", "fim_reservoir_sample", "fim_partition_lpt", "fim_lpt_schedule",
    "fim_mine_noalloc", "fim_class_profile",
]

FIM_NOALLOC_SCRATCH_BYTES = 256 << 20


class FimError(RuntimeError):
    def __init__(self, status: int, name: str, message: str):
        super().__init__("%s (%d): %s" % (name, status, message))
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class fim_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class fim_options(ctypes.Structure):
    _fields_ = [("max_len", ctypes.c_uint32), ("max_itemsets", ctypes.c_uint64),
                ("seed", ctypes.c_uint64), ("alpha", ctypes.c_double),
                ("sample_tx", ctypes.c_uint32), ("sample_fi", ctypes.c_uint32),
                ("tile_words", ctypes.c_uint32), ("classes_per_wg", ctypes.c_uint32),
                ("workers", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class fim_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "candidates", "pair_words", "item_supports", "n_frequent_items", "bytes_algorithmic",
        "kernel_ns", "total_ns", "estimate_ns", "n_tasks", "retries", "root_candidates",
        "root_pair_words", "root_kernel_ns", "dfs_kernel_ns", "dfs_bytes_algorithmic",
        "n_itemsets", "root_kernel", "dfs_busy_max_ns", "dfs_busy_mean_ns")]


class fim_server_config(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_uint32), ("max_queue", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("lanes", ctypes.c_uint32),
                ("opts", fim_options)]


class fim_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "completed", "cancelled", "steps", "peak_active", "peak_bytes", "lanes")]


_lib = None


def lib():
    """The loaded ``libfim.so`` (built first if it does not exist yet)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .build import build
        build()
    # PyTorch ships its own HIP runtime.  Loading it first makes libfim.so
    # bind to that same runtime (matched by soname), so the process holds one
    # runtime and torch's memory and streams are valid for the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, V = ctypes.POINTER, ctypes.c_void_p
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    sig = {
        "fim_status_str": (ctypes.c_char_p, [i32]),
        "fim_last_error": (ctypes.c_char_p, []),
        "fim_version": (ctypes.c_char_p, []),
        "fim_ctx_create": (i32, [ctypes.c_int, V, P(fim_allocator), P(V)]),
        "fim_ctx_destroy": (None, [V]),
        "fim_ctx_release_cached": (i32, [V]),
        "fim_db_create": (i32, [V, u64, P(u64), P(u32), u32, P(V)]),
        "fim_db_destroy": (None, [V]),
        "fim_db_sizes": (i32, [V, P(u64), P(u64)]),
        "fim_minsup_from_relative": (i32, [u64, ctypes.c_double, P(u32)]),
        "fim_mine": (i32, [V, V, u32, P(fim_options), P(V)]),
        "fim_mine_batch": (i32, [V, u32, P(V), P(u32), P(fim_options), P(V)]),
        "fim_autotune": (i32, [V, u32, P(V), P(u32), P(fim_options), u32, P(fim_options), P(u64)]),
        "fim_result_sizes": (i32, [V, P(u64), P(u64)]),
        "fim_result_copy": (i32, [V, P(u64), P(u32), P(u32)]),
        "fim_result_view": (i32, [V, P(P(u64)), P(P(u32)), P(P(u32))]),
        "fim_result_stats": (i32, [V, P(fim_stats)]),
        "fim_result_destroy": (None, [V]),
        "fim_server_create": (i32, [V, P(fim_server_config), P(V)]),
        "fim_server_submit": (i32, [V, V, u32, P(u64)]),
        "fim_server_poll": (i32, [V, u64, P(V)]),
        "fim_server_wait": (i32, [V, u64, P(V)]),
        "fim_server_next": (i32, [V, u64, P(u64), P(V)]),
        "fim_server_cancel": (i32, [V, u64]),
        "fim_server_stats_get": (i32, [V, P(fim_server_stats)]),
        "fim_server_destroy": (None, [V]),
        "fim_estimate_sample_sizes": (i32, [ctypes.c_double] * 5 + [P(u32), P(u32)]),
        "fim_reservoir_sample": (i32, [u64, u64, u64, P(u64)]),
        "fim_partition_lpt": (i32, [u32, P(u32), P(ctypes.c_double), ctypes.c_double, u32, u32,
                                    P(u32), u32, P(u32), P(ctypes.c_double)]),
        "fim_lpt_schedule": (i32, [P(ctypes.c_double), u64, u32, P(u32), P(ctypes.c_double)]),
        "fim_mine_noalloc": (i32, [V, V, u32, P(fim_options), u64, u64, P(u64), P(u32), P(u32),
                                   P(u64), P(u64)]),
        "fim_class_profile": (i32, [V, V, u32, P(fim_options), P(u32), P(u32), u32, P(u64),
                                    P(ctypes.c_double), P(ctypes.c_double), P(u64), u64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != FIM_OK:
        L = lib()
        raise FimError(status, L.fim_status_str(status).decode(), L.fim_last_error().decode())


def _u64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _u32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


# ---------------------------------------------------------------- C-named calls

def fim_version() -> str:
    return lib().fim_version().decode()


def fim_ctx_create(device: int = 0, hip_stream: int | None = None, allocator=None):
    h = ctypes.c_void_p()
    _check(lib().fim_ctx_create(device, hip_stream, ctypes.byref(allocator) if allocator else None,
                                ctypes.byref(h)))
    return h


def fim_ctx_destroy(ctx):
    lib().fim_ctx_destroy(ctx)


def fim_db_create(ctx, offsets, items, n_item_ids: int):
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    items = np.ascontiguousarray(items, dtype=np.uint32)
    h = ctypes.c_void_p()
    _check(lib().fim_db_create(ctx, len(offsets) - 1, _u64p(offsets),
                               _u32p(items) if len(items) else None, n_item_ids, ctypes.byref(h)))
    return h


def fim_db_destroy(db):
    lib().fim_db_destroy(db)


def fim_minsup_from_relative(n_tx: int, rel: float) -> int:
    out = ctypes.c_uint32()
    _check(lib().fim_minsup_from_relative(n_tx, rel, ctypes.byref(out)))
    return out.value


def make_options(**kw) -> fim_options:
    o = fim_options()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def fim_mine(ctx, db, minsup: int, opts: fim_options | None = None):
    h = ctypes.c_void_p()
    _check(lib().fim_mine(ctx, db, minsup, ctypes.byref(opts) if opts else None, ctypes.byref(h)))
    return h


def fim_mine_batch(ctx, dbs, minsups, opts: fim_options | None = None):
    n = len(dbs)
    arr = (ctypes.c_void_p * n)(*[d.value for d in dbs])
    ms = np.ascontiguousarray(minsups, dtype=np.uint32)
    outs = (ctypes.c_void_p * n)()
    _check(lib().fim_mine_batch(ctx, n, arr, _u32p(ms), ctypes.byref(opts) if opts else None,
                                outs))
    return [ctypes.c_void_p(outs[i]) for i in range(n)]


def fim_autotune(ctx, dbs, minsups, base: fim_options | None = None, reps: int = 0):
    """Returns (tuned options, best depth-first kernel ns)."""
    n = len(dbs)
    arr = (ctypes.c_void_p * n)(*[d.value for d in dbs])
    ms = np.ascontiguousarray(minsups, dtype=np.uint32)
    out, ns = fim_options(), ctypes.c_uint64()
    _check(lib().fim_autotune(ctx, n, arr, _u32p(ms), ctypes.byref(base) if base else None, reps,
                              ctypes.byref(out), ctypes.byref(ns)))
    return out, ns.value


class _ResultHandle:
    """Owns a result handle; destroyed when the last array viewing it goes."""

    def __init__(self, res):
        self.res = res

    def __del__(self):
        L = _lib
        if self.res is not None and L is not None:
            L.fim_result_destroy(self.res)
            self.res = None


def _view(addr, n, ctype, dtype, owner):
    if n == 0 or not addr:
        return np.zeros(0, dtype)
    buf = (ctype * n).from_address(addr)
    buf._owner = owner  # the arrays keep the handle alive
    return np.frombuffer(buf, dtype=dtype)


def fim_result_take(res) -> "Result":
    """Numpy views of a result handle's arrays (no copy); the handle is
    destroyed when the last of them is garbage-collected.  The views are
    read-only."""
    L = lib()
    n, ni = ctypes.c_uint64(), ctypes.c_uint64()
    _check(L.fim_result_sizes(res, ctypes.byref(n), ctypes.byref(ni)))
    st = fim_stats()
    _check(L.fim_result_stats(res, ctypes.byref(st)))
    stats = {name: int(getattr(st, name)) for name, _ in fim_stats._fields_}
    po, pi, ps = ctypes.POINTER(ctypes.c_uint64)(), ctypes.POINTER(ctypes.c_uint32)(), \
        ctypes.POINTER(ctypes.c_uint32)()
    _check(L.fim_result_view(res, ctypes.byref(po), ctypes.byref(pi), ctypes.byref(ps)))
    owner = _ResultHandle(res)
    addr = lambda p: ctypes.cast(p, ctypes.c_void_p).value or 0
    off = _view(addr(po), n.value + 1, ctypes.c_uint64, np.uint64, owner)
    items = _view(addr(pi), ni.value, ctypes.c_uint32, np.uint32, owner)
    supp = _view(addr(ps), n.value, ctypes.c_uint32, np.uint32, owner)
    for a in (off, items, supp):
        a.flags.writeable = False
    return Result(off, items, supp, stats)


def fim_estimate_sample_sizes(eps_db=0.02, delta_db=0.05, rho=0.001, eps_fi=0.0005,
                              delta_fi=0.05):
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().fim_estimate_sample_sizes(eps_db, delta_db, rho, eps_fi, delta_fi,
                                           ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def fim_reservoir_sample(stream_len: int, n: int, seed: int) -> np.ndarray:
    out = np.zeros(max(1, min(n, stream_len)), np.uint64)
    _check(lib().fim_reservoir_sample(stream_len, n, seed, _u64p(out)))
    return out[:min(n, stream_len)]


def fim_lpt_schedule(weights, n_workers: int):
    w = np.ascontiguousarray(weights, dtype=np.float64)
    wk = np.zeros(max(1, len(w)), np.uint32)
    ms = ctypes.c_double()
    _check(lib().fim_lpt_schedule(w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(w),
                                  n_workers, _u32p(wk), ctypes.byref(ms)))
    return wk[:len(w)], ms.value


def fim_partition_lpt(n_atoms, row_weights, alpha: float, n_workers: int, flags: int = 0):
    na = np.ascontiguousarray(n_atoms, dtype=np.uint32)
    rw = np.ascontiguousarray(row_weights, dtype=np.float64)
    cap = int(na.sum()) + 1
    tasks = np.zeros(3 * cap, np.uint32)
    nt, ms = ctypes.c_uint32(), ctypes.c_double()
    _check(lib().fim_partition_lpt(len(na), _u32p(na),
                                   rw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), alpha,
                                   n_workers, flags, _u32p(tasks), cap, ctypes.byref(nt),
                                   ctypes.byref(ms)))
    return tasks[:3 * nt.value].reshape(-1, 3), ms.value


# ---------------------------------------------------------------- high level

@dataclass
class Result:
    """Frequent itemsets in canonical order (CSR) and run statistics."""
    offsets: np.ndarray
    items: np.ndarray
    supports: np.ndarray
    stats: dict = field(default_factory=dict)

    def __len__(self):
        return len(self.supports)

    def itemsets(self):
        o = self.offsets
        return [tuple(self.items[o[i]:o[i + 1]].tolist()) for i in range(len(self))]

    def as_dict(self):
        return dict(zip(self.itemsets(), self.supports.tolist()))


class Context:
    """A GPU, a HIP stream and a device allocator (PyTorch's when available)."""

    def __init__(self, device: int = 0, use_torch: bool = True):
        self.device = device
        self._keep = []
        # databases and servers on this context: closed before it (the
        # library frees a database through its context)
        self._deps = weakref.WeakSet()
        stream, alloc = None, None
        if use_torch:
            try:
                import torch
            except ImportError:
                torch = None
            if torch is not None and torch.cuda.is_available():
                torch.cuda.set_device(device)
                self.stream = torch.cuda.Stream(device)  # default priority
                stream = self.stream.cuda_stream

                def _alloc(nbytes, strm, user):
                    try:
                        return torch.cuda.caching_allocator_alloc(int(nbytes), device,
                                                                  int(strm or 0))
                    except Exception:
                        return None

                def _free(ptr, strm, user):
                    try:
                        torch.cuda.caching_allocator_delete(ptr)
                    except Exception:  # interpreter shutdown
                        pass

                fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
                alloc = fim_allocator(fa, ff, None)
                self._keep += [fa, ff, alloc]
        self.handle = fim_ctx_create(device, stream, alloc)

    def release_cached(self):
        """Give the device blocks the library keeps for reuse back to the allocator."""
        _check(lib().fim_ctx_release_cached(self.handle))

    def close(self):
        if self.handle:
            deps = list(self._deps)
            for d in deps:  # servers first: they mine the databases
                if isinstance(d, Server):
                    d.close()
            for d in deps:
                d.close()
            fim_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Database:
    """A transaction database resident on the context's GPU."""

    def __init__(self, ctx: Context, offsets, items, n_item_ids: int):
        self.ctx = ctx
        self.handle = fim_db_create(ctx.handle, offsets, items, n_item_ids)
        ctx._deps.add(self)
        n, nnz = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().fim_db_sizes(self.handle, ctypes.byref(n), ctypes.byref(nnz)))
        self.n_tx, self.nnz = n.value, nnz.value

    def close(self):
        if self.handle:
            fim_db_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mine(ctx: Context, db: Database, minsup: int, **opts) -> Result:
    o = make_options(**opts) if opts else None
    return fim_result_take(fim_mine(ctx.handle, db.handle, minsup, o))


def fim_mine_noalloc(ctx, db, minsup: int, cap_itemsets: int, cap_items: int,
                     opts: fim_options | None = None):
    """``fim_mine_noalloc`` into caller arrays of the given capacities:
    returns (status, offsets, items, supports, n_itemsets, n_items_total);
    the arrays hold the result when status is FIM_OK."""
    off = np.zeros(cap_itemsets + 1, np.uint64)
    items = np.zeros(max(cap_items, 1), np.uint32)
    supp = np.zeros(max(cap_itemsets, 1), np.uint32)
    n, ni = ctypes.c_uint64(), ctypes.c_uint64()
    st = lib().fim_mine_noalloc(ctx, db, minsup, ctypes.byref(opts) if opts else None, cap_itemsets,
                                cap_items, _u64p(off), _u32p(items), _u32p(supp), ctypes.byref(n),
                                ctypes.byref(ni))
    return st, off, items, supp, n.value, ni.value


def mine_noalloc(ctx: Context, db: Database, minsup: int, cap_itemsets: int, cap_items: int,
                 **opts):
    """Mining without device allocation (``fim_mine_noalloc``) into arrays of
    the given capacities; returns (offsets, items, supports) trimmed to the
    result."""
    o = make_options(**opts) if opts else None
    st, off, items, supp, n, ni = fim_mine_noalloc(ctx.handle, db.handle, minsup, cap_itemsets,
                                                   cap_items, o)
    _check(st)
    return off[:n + 1], items[:ni], supp[:n]


def class_profile(ctx: Context, db: Database, minsup: int, **opts) -> dict:
    """``fim_class_profile``: atoms per first-level class and, per
    second-level class, the sample's frequent itemsets and candidate pairs
    and the run's own candidate pairs."""
    o = make_options(**opts) if opts else None
    cap_c, cap_r = 1 << 16, 1 << 22
    while True:
        nc, nr = ctypes.c_uint32(), ctypes.c_uint64()
        atoms = np.zeros(cap_c, np.uint32)
        efi = np.zeros(cap_r, np.float64)
        ecand = np.zeros(cap_r, np.float64)
        act = np.zeros(cap_r, np.uint64)
        st = lib().fim_class_profile(ctx.handle, db.handle, minsup, ctypes.byref(o) if o else None,
                                     ctypes.byref(nc), _u32p(atoms), cap_c, ctypes.byref(nr),
                                     efi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     ecand.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     _u64p(act), cap_r)
        if st == FIM_E_OUTPUT_LIMIT and (nc.value > cap_c or nr.value > cap_r):
            cap_c, cap_r = max(cap_c, nc.value), max(cap_r, nr.value)
            continue
        _check(st)
        n, k = nc.value, nr.value
        return {"n_atoms": atoms[:n], "est_fi": efi[:k], "est_cand": ecand[:k], "act_cand": act[:k]}


def mine_batch(ctx: Context, dbs, minsups, **opts):
    o = make_options(**opts) if opts else None
    return [fim_result_take(h) for h in fim_mine_batch(ctx.handle, [d.handle for d in dbs],
                                                       minsups, o)]


def autotune(ctx: Context, dbs, minsups, reps: int = 0, **opts) -> dict:
    """Tile width and classes per workgroup for this batch, by measurement;
    returns the options to pass to ``mine_batch`` (``tile_words``,
    ``classes_per_wg``) and the winner's kernel time."""
    o, ns = fim_autotune(ctx.handle, [d.handle for d in dbs], minsups,
                         make_options(**opts) if opts else None, reps)
    return {"tile_words": o.tile_words, "classes_per_wg": o.classes_per_wg, "dfs_kernel_ns": ns}


class Server:
    """Continuous-batching request loop on one GPU."""

    def __init__(self, ctx: Context, max_active: int = 0, max_queue: int = 0,
                 hbm_budget_bytes: int = 0, lanes: int = 0, **opts):
        cfg = fim_server_config()
        cfg.max_active, cfg.max_queue, cfg.hbm_budget_bytes = max_active, max_queue, hbm_budget_bytes
        cfg.lanes = lanes
        if opts:
            cfg.opts = make_options(**opts)
        self.ctx = ctx
        self.handle = ctypes.c_void_p()
        _check(lib().fim_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(self.handle)))
        ctx._deps.add(self)

    def submit(self, db: Database, minsup: int) -> int:
        t = ctypes.c_uint64()
        _check(lib().fim_server_submit(self.handle, db.handle, minsup, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        h = ctypes.c_void_p()
        _check(lib().fim_server_poll(self.handle, ticket, ctypes.byref(h)))
        return fim_result_take(h) if h.value else None

    def wait(self, ticket: int) -> Result:
        h = ctypes.c_void_p()
        _check(lib().fim_server_wait(self.handle, ticket, ctypes.byref(h)))
        return fim_result_take(h)

    def next(self, timeout_s: float):
        """(ticket, Result) of the next finished request in completion order,
        or (0, None) if none finishes within timeout_s seconds."""
        t, h = ctypes.c_uint64(), ctypes.c_void_p()
        _check(lib().fim_server_next(self.handle, max(0, int(timeout_s * 1e6)), ctypes.byref(t),
                                     ctypes.byref(h)))
        return (t.value, fim_result_take(h)) if t.value else (0, None)

    def cancel(self, ticket: int):
        _check(lib().fim_server_cancel(self.handle, ticket))

    def stats(self) -> dict:
        st = fim_server_stats()
        _check(lib().fim_server_stats_get(self.handle, ctypes.byref(st)))
        return {name: int(getattr(st, name)) for name, _ in fim_server_stats._fields_}

    def close(self):
        if self.handle:
            lib().fim_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
