// Host runtime of libfim.so: contexts, databases, the mining pipeline, the
// sample-based class-size estimate, results.  Every step of the mining path
// runs in the HIP kernels of fim_kernels.hip; the host decides the order of
// work, moves data and puts the result into canonical order.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <numeric>
#include <thread>

#include "fim_host.h"
#include "fim_plan.h"
#include "fim_canon.h"

using fim::DevBuf;

namespace fim {

static thread_local std::string g_error;
thread_local ClassProfile *g_profile = nullptr;

fim_status set_error(fim_status s, const std::string &msg) {
    g_error = msg;
    return s;
}

bool DevBuf::ensure(fim_ctx *ctx, size_t bytes) {
    if (p_ && bytes_ >= bytes && ctx_ == ctx) return true;
    reset();
    ctx_ = ctx;
    if (bytes == 0) bytes = 256;
    p_ = ctx->dalloc(bytes);
    if (!p_) return false;
    bytes_ = bytes;
    return true;
}

void DevBuf::reset() {
    if (p_ && ctx_) ctx_->dfree(p_);
    p_ = nullptr;
    bytes_ = 0;
}

}  // namespace fim

void *fim_ctx::raw_alloc(size_t bytes) {
    if (user_alloc) return alloc.alloc(bytes, (void *)stream, alloc.user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void fim_ctx::raw_free(void *p) {
    if (!p) return;
    if (user_alloc) alloc.free(p, (void *)stream, alloc.user);
    else (void)hipFree(p);
}

// size class: at least 256 bytes, then within 1/8 of the next power of two
static size_t size_class(size_t bytes) {
    if (bytes <= 256) return 256;
    size_t p = 1;
    while (p < bytes) p <<= 1;
    const size_t step = std::max<size_t>(256, p / 8);
    return (bytes + step - 1) / step * step;
}

void fim_ctx::release_cached() {
    std::lock_guard<std::mutex> lk(cache_mu);
    for (auto &kv : cache)
        for (void *p : kv.second) {
            block_class.erase(p);
            raw_free(p);
        }
    cache.clear();
    cached_bytes = 0;
}

void *fim_ctx::dalloc(size_t bytes) {
    if (arena) {
        const size_t b = (std::max<size_t>(bytes, 256) + 255) & ~size_t(255);
        if (b > arena_cap - arena_used) return nullptr;
        void *p = arena + arena_used;
        last_piece_at = arena_used;
        arena_used += b;
        return p;
    }
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        auto it = cache.find(cls);
        if (it != cache.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            cached_bytes -= cls;
            return p;
        }
    }
    void *p = raw_alloc(cls);
    if (!p && cached_bytes) {  // give the cached blocks back and try again
        release_cached();
        p = raw_alloc(cls);
    }
    if (p) {
        std::lock_guard<std::mutex> lk(cache_mu);
        block_class[p] = cls;
    }
    return p;
}

void fim_ctx::dfree(void *p) {
    if (!p) return;
    if (arena && (char *)p >= arena && (char *)p < arena + arena_cap) {
        // only the most recent piece can be taken back; the others stay
        // used until the arena is released at the end of the call
        if ((char *)p < arena + arena_used) {
            const size_t at = (size_t)((char *)p - arena);
            if (last_piece_at == at) arena_used = at;
        }
        return;
    }
    std::unique_lock<std::mutex> lk(cache_mu);
    auto it = block_class.find(p);
    if (it == block_class.end()) {
        lk.unlock();
        raw_free(p);
        return;
    }
    // keep it for the next call unless the cache already holds a quarter of
    // the device (a server runs several contexts on one device)
    if (cached_bytes + it->second > total_mem / 4) {
        block_class.erase(it);
        lk.unlock();
        raw_free(p);
        return;
    }
    cache[it->second].push_back(p);
    cached_bytes += it->second;
}

#define HIPCHK(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fim::set_error(FIM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define ENSURE(buf, ctx, bytes)                                                               \
    do {                                                                                      \
        if (!(buf).ensure((ctx), (bytes)))                                                    \
            return fim::set_error(FIM_E_OOM_DEVICE,                                           \
                                  "device allocation of " + std::to_string((size_t)(bytes)) + \
                                      " bytes failed");                                       \
    } while (0)

// ====================================================================== status

extern "C" const char *fim_status_str(fim_status s) {
    switch (s) {
        case FIM_OK: return "FIM_OK";
        case FIM_E_INVALID_ARG: return "FIM_E_INVALID_ARG";
        case FIM_E_ITEM_RANGE: return "FIM_E_ITEM_RANGE";
        case FIM_E_OOM_HOST: return "FIM_E_OOM_HOST";
        case FIM_E_OOM_DEVICE: return "FIM_E_OOM_DEVICE";
        case FIM_E_DEVICE: return "FIM_E_DEVICE";
        case FIM_E_OUTPUT_LIMIT: return "FIM_E_OUTPUT_LIMIT";
        case FIM_E_BUSY: return "FIM_E_BUSY";
        case FIM_E_CANCELLED: return "FIM_E_CANCELLED";
        case FIM_E_NOT_FOUND: return "FIM_E_NOT_FOUND";
        case FIM_E_NO_DEVICE: return "FIM_E_NO_DEVICE";
        default: return "FIM_E_UNKNOWN";
    }
}

extern "C" const char *fim_last_error(void) { return fim::g_error.c_str(); }

extern "C" const char *fim_version(void) { return "fim 1.0 gfx950"; }

// ====================================================================== context

extern "C" fim_status fim_ctx_create(int device, void *hip_stream, const fim_allocator *alloc,
                                     fim_ctx **out) {
    if (!out) return fim::set_error(FIM_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return fim::set_error(FIM_E_NO_DEVICE, "no HIP device " + std::to_string(device));
    }
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    std::string arch = prop.gcnArchName;
    if (arch.rfind("gfx950", 0) != 0)
        return fim::set_error(FIM_E_NO_DEVICE, "device " + std::to_string(device) + " is " + arch +
                                                   ", this library is built for gfx950");
    if (alloc && (!alloc->alloc || !alloc->free))
        return fim::set_error(FIM_E_INVALID_ARG, "allocator without alloc/free");
    HIPCHK(hipSetDevice(device));
    fim_ctx *c = new (std::nothrow) fim_ctx();
    if (!c) return fim::set_error(FIM_E_OOM_HOST, "ctx");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (!c->stream) {  // a caller capturing work into a graph needs a stream other than the null one
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fim::set_error(FIM_E_DEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    if (alloc) {
        c->alloc = *alloc;
        c->user_alloc = true;
    }
    c->n_cu = prop.multiProcessorCount;
    c->total_mem = prop.totalGlobalMem;
    c->lds_per_block = prop.sharedMemPerBlock;
    c->arch = arch;
    *out = c;
    return FIM_OK;
}

fim_ctx *fim_ctx::aux_ctx() {
    if (!aux) {
        fim_ctx *c = nullptr;
        if (fim_ctx_create(device, nullptr, user_alloc ? &alloc : nullptr, &c) != FIM_OK) return nullptr;
        aux = c;
    }
    return aux;
}

uint32_t *fim_ctx::stage(size_t words) {
    if (words <= pinned_words && pinned) return pinned;
    if (pinned) {
        if (pinned_heap) free(pinned);
        else (void)hipHostFree(pinned);
    }
    pinned = nullptr;
    pinned_words = 0;
    const size_t want = std::max<size_t>(words + words / 4, 1u << 20);
    pinned_heap = fim::g_no_pinned;
    if (pinned_heap) {
        pinned = static_cast<uint32_t *>(malloc(want * 4));
        if (pinned) pinned_words = want;
        return pinned;
    }
    if (hipHostMalloc((void **)&pinned, want * 4, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        pinned = nullptr;
        return nullptr;
    }
    pinned_words = want;
    return pinned;
}

fim_ctx::~fim_ctx() {
    delete aux;
    for (hipEvent_t e : timing_events) (void)hipEventDestroy(e);
    for (hipEvent_t e : sync_events)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t x : side_streams) {
        (void)hipStreamSynchronize(x);
        (void)hipStreamDestroy(x);
    }
    release_cached();
    if (pinned) {
        if (pinned_heap) free(pinned);
        else (void)hipHostFree(pinned);
    }
    if (up) {
        if (stream) (void)hipStreamSynchronize(stream);
        (void)hipHostFree(up);
    }
    if (own_stream && stream) {
        (void)hipStreamSynchronize(stream);
        (void)hipStreamDestroy(stream);
    }
}

namespace fim {

hipError_t ctx_side_streams(fim_ctx *ctx, std::vector<hipStream_t> &out) {
    constexpr size_t kSide = 4;
    while (ctx->side_streams.size() < kSide) {
        hipStream_t x = nullptr;
        const hipError_t e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        ctx->side_streams.push_back(x);
    }
    out = ctx->side_streams;
    return hipSuccess;
}

hipError_t ctx_timing_events(fim_ctx *ctx, size_t n) {
    while (ctx->timing_events.size() < n) {
        hipEvent_t e = nullptr;
        const hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ctx->timing_events.push_back(e);
    }
    return hipSuccess;
}

hipError_t h2d(fim_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const size_t b = (bytes + 255) & ~size_t(255);
    ctx->up_need += b;
    if (ctx->up && ctx->up_used + b <= ctx->up_cap) {
        char *p = ctx->up + ctx->up_used;
        ctx->up_used += b;
        memcpy(p, src, bytes);
        return hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, s);
    }
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
}

hipError_t h2d_pieces(fim_ctx *ctx, void *dst, const H2DPiece *pieces, size_t n, hipStream_t s) {
    size_t total = 0;
    for (size_t i = 0; i < n; i++) total += (pieces[i].bytes + 7) & ~size_t(7);
    if (total == 0) return hipSuccess;
    const size_t b = (total + 255) & ~size_t(255);
    ctx->up_need += b;
    size_t at = 0;
    if (ctx->up && ctx->up_used + b <= ctx->up_cap) {
        char *p = ctx->up + ctx->up_used;
        ctx->up_used += b;
        for (size_t i = 0; i < n; i++) {
            if (pieces[i].bytes) memcpy(p + at, pieces[i].src, pieces[i].bytes);
            at += (pieces[i].bytes + 7) & ~size_t(7);
        }
        return hipMemcpyAsync(dst, p, total, hipMemcpyHostToDevice, s);
    }
    for (size_t i = 0; i < n; i++) {
        if (pieces[i].bytes) {
            const hipError_t e = hipMemcpyAsync(static_cast<char *>(dst) + at, pieces[i].src, pieces[i].bytes,
                                                hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return e;
        }
        at += (pieces[i].bytes + 7) & ~size_t(7);
    }
    return hipSuccess;
}

hipError_t stream_wait(hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t k = 0;; k++) {
        const hipError_t e = hipStreamQuery(s);
        if (e != hipErrorNotReady) return e;
        if ((k & 63u) == 63u && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20))
            return hipStreamSynchronize(s);
    }
}

StageRun::StageRun(fim_ctx *ctx) : ctx_(ctx) {
    if (ctx_->up_depth++ > 0) return;
    // copies of an earlier run that ended early may still read the staging
    // (from the call's stream or from its side streams)
    (void)hipStreamSynchronize(ctx_->stream);
    for (hipStream_t x : ctx_->side_streams) (void)hipStreamSynchronize(x);
    if (ctx_->up_need > ctx_->up_cap && !g_no_pinned) {
        if (ctx_->up) (void)hipHostFree(ctx_->up);
        ctx_->up = nullptr;
        ctx_->up_cap = 0;
        const size_t want = std::max<size_t>(1u << 20, (ctx_->up_need + ctx_->up_need / 4 + 0xFFFFF) & ~size_t(0xFFFFF));
        void *p = nullptr;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) == hipSuccess) {
            ctx_->up = static_cast<char *>(p);
            ctx_->up_cap = want;
        } else {
            (void)hipGetLastError();
        }
    }
    ctx_->up_used = 0;
    ctx_->up_need = 0;
}

StageRun::~StageRun() { ctx_->up_depth--; }

}  // namespace fim

extern "C" void fim_ctx_destroy(fim_ctx *ctx) { delete ctx; }

extern "C" fim_status fim_ctx_release_cached(fim_ctx *ctx) {
    if (!ctx) return fim::set_error(FIM_E_INVALID_ARG, "ctx is NULL");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->release_cached();
    if (ctx->aux) ctx->aux->release_cached();
    return FIM_OK;
}

// ====================================================================== database

extern "C" fim_status fim_db_create(fim_ctx *ctx, uint64_t n_tx, const uint64_t *tx_offsets,
                                    const uint32_t *items, uint32_t n_item_ids, fim_db **out) {
    if (!out) return fim::set_error(FIM_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx || !tx_offsets || n_item_ids == 0)
        return fim::set_error(FIM_E_INVALID_ARG, "ctx/tx_offsets NULL or n_item_ids == 0");
    if (n_tx >= (1ull << 31)) return fim::set_error(FIM_E_INVALID_ARG, "n_tx must be < 2^31");
    if (tx_offsets[0] != 0) return fim::set_error(FIM_E_INVALID_ARG, "tx_offsets[0] != 0");
    for (uint64_t t = 0; t < n_tx; t++)
        if (tx_offsets[t + 1] < tx_offsets[t])
            return fim::set_error(FIM_E_INVALID_ARG,
                                  "tx_offsets not monotone at " + std::to_string(t));
    const uint64_t nnz_in = tx_offsets[n_tx];
    if (nnz_in && !items) return fim::set_error(FIM_E_INVALID_ARG, "items is NULL");
    fim_db *db = new (std::nothrow) fim_db();
    if (!db) return fim::set_error(FIM_E_OOM_HOST, "db");
    try {
        db->h_off.resize(n_tx + 1);
        db->h_items.resize(nnz_in);
    } catch (...) {
        delete db;
        return fim::set_error(FIM_E_OOM_HOST, "db arrays");
    }
    // a1: transactions are sets: sort each one and drop repeated items
    uint64_t pos = 0;
    db->h_off[0] = 0;
    for (uint64_t t = 0; t < n_tx; t++) {
        const uint64_t a = tx_offsets[t], b = tx_offsets[t + 1];
        uint32_t *dst = db->h_items.data() + pos;
        for (uint64_t p = a; p < b; p++) {
            if (items[p] >= n_item_ids) {
                delete db;
                return fim::set_error(FIM_E_ITEM_RANGE, "item " + std::to_string(items[p]) +
                                                            " >= n_item_ids at position " +
                                                            std::to_string(p));
            }
            dst[p - a] = items[p];
        }
        std::sort(dst, dst + (b - a));
        uint64_t n = std::unique(dst, dst + (b - a)) - dst;
        pos += n;
        db->h_off[t + 1] = pos;
        db->pairs_in_tx += n * (n ? n - 1 : 0) / 2;
        db->max_tx_len = std::max(db->max_tx_len, n);
    }
    db->h_items.resize(pos);
    db->ctx = ctx;
    db->n_tx = n_tx;
    db->nnz = pos;
    db->n_item_ids = n_item_ids;
    if (!db->d_off.ensure(ctx, (n_tx + 1) * sizeof(uint64_t)) ||
        !db->d_items.ensure(ctx, std::max<uint64_t>(pos, 1) * sizeof(uint32_t))) {
        delete db;
        return fim::set_error(FIM_E_OOM_DEVICE, "db device arrays");
    }
    hipError_t e = hipMemcpyAsync(db->d_off.as<void>(), db->h_off.data(), (n_tx + 1) * 8,
                                  hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess && pos)
        e = hipMemcpyAsync(db->d_items.as<void>(), db->h_items.data(), pos * 4,
                           hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        delete db;
        return fim::set_error(FIM_E_DEVICE, std::string("db upload: ") + hipGetErrorString(e));
    }
    *out = db;
    return FIM_OK;
}

extern "C" void fim_db_destroy(fim_db *db) { delete db; }

extern "C" fim_status fim_db_sizes(const fim_db *db, uint64_t *n_tx, uint64_t *nnz) {
    if (!db) return fim::set_error(FIM_E_INVALID_ARG, "db is NULL");
    if (n_tx) *n_tx = db->n_tx;
    if (nnz) *nnz = db->nnz;
    return FIM_OK;
}

extern "C" fim_status fim_minsup_from_relative(uint64_t n_tx, double rel, uint32_t *out_abs) {
    if (!out_abs || !(rel > 0.0) || rel > 1.0)
        return fim::set_error(FIM_E_INVALID_ARG, "relative minimum support must be in (0, 1]");
    double v = ceil(rel * (double)n_tx);
    if (v < 1.0) v = 1.0;
    if (v > 4294967295.0) return fim::set_error(FIM_E_INVALID_ARG, "minimum support overflows");
    *out_abs = (uint32_t)v;
    return FIM_OK;
}

// ====================================================================== results

extern "C" fim_status fim_result_sizes(const fim_result *r, uint64_t *n_itemsets,
                                       uint64_t *n_items_total) {
    if (!r) return fim::set_error(FIM_E_INVALID_ARG, "result is NULL");
    if (n_itemsets) *n_itemsets = r->n_itemsets();
    if (n_items_total) *n_items_total = r->n_items();
    return FIM_OK;
}

extern "C" fim_status fim_result_copy(const fim_result *r, uint64_t *offsets, uint32_t *items,
                                      uint32_t *supports) {
    if (!r) return fim::set_error(FIM_E_INVALID_ARG, "result is NULL");
    if (offsets) memcpy(offsets, r->off.data(), r->off.size() * sizeof(uint64_t));
    if (items && r->n_items()) memcpy(items, r->items_data(), r->n_items() * 4);
    if (supports && r->n_itemsets()) memcpy(supports, r->supp_data(), r->n_itemsets() * 4);
    return FIM_OK;
}

extern "C" fim_status fim_result_view(const fim_result *r, const uint64_t **offsets,
                                      const uint32_t **items, const uint32_t **supports) {
    if (!r || !offsets || !items || !supports) return fim::set_error(FIM_E_INVALID_ARG, "NULL argument");
    *offsets = r->off.data();
    *items = r->n_items() ? r->items_data() : nullptr;
    *supports = r->n_itemsets() ? r->supp_data() : nullptr;
    return FIM_OK;
}

extern "C" fim_status fim_result_stats(const fim_result *r, fim_stats *out) {
    if (!r || !out) return fim::set_error(FIM_E_INVALID_ARG, "NULL argument");
    *out = r->stats;
    return FIM_OK;
}

extern "C" void fim_result_destroy(fim_result *r) { delete r; }

// ====================================================================== mining

namespace fim {

fim_options resolve_options(const fim_options *o) {
    fim_options r{};
    if (o) r = *o;
    if (r.seed == 0) r.seed = 0x2108050380ull;
    if (!(r.alpha > 0.0) || r.alpha > 1.0) r.alpha = 0.3;
    return r;
}

namespace {

using clk = std::chrono::steady_clock;

uint64_t ns_since(clk::time_point t0) {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - t0).count();
}

// FIM_TRACE=1 prints the wall time of every phase of a run to stderr
struct Tracer {
    bool on;
    clk::time_point t0, last;
    const char *tag;
    explicit Tracer(const char *t) : on(getenv("FIM_TRACE") != nullptr), t0(clk::now()), last(t0), tag(t) {}
    void mark(const char *what) {
        if (!on) return;
        const auto now = clk::now();
        fprintf(stderr, "[fim %s] %-24s %8.3f ms (total %8.3f ms)\n", tag, what,
                std::chrono::duration<double, std::milli>(now - last).count(),
                std::chrono::duration<double, std::milli>(now - t0).count());
        last = now;
    }
};

// per-instance state of one run
struct Inst {
    const fim_db *db = nullptr;
    uint32_t minsup = 0;
    uint32_t W = 0, Wp = 0, n_freq = 0;
    std::vector<uint32_t> counts, item_of_rank, rank_of_item, supp_of_rank;
    uint64_t n_pairs = 0;
    std::vector<uint32_t> l2_off, l2_atom, l2_supp;
    DevBuf d_counts, d_rank_of_item, d_rows, d_pairs, d_npairs;
    uint32_t *p_counts = nullptr;  // item supports on the device (d_counts or a batch's shared array)
    DevBuf d_l2_off, d_l2_atom, d_l2_supp;
    bool l2_on_device = false;  // the l2 arrays above hold l2_off, l2_atom, l2_supp
    // root-class kernel: 0 whole rows, 1 covers, 2 projected transactions
    uint32_t root_kind = 0;
    // covers: non-zero words per row and the transposed arena
    std::vector<uint64_t> nz_off;
    std::vector<uint32_t> nz_cnt;
    DevBuf d_nz_off, d_nz_w, d_nz_m, d_nz_cnt, d_bt;
    // projected: ranked transactions, tid lists and the lists' pointers into
    // the ranked transactions, pair increments
    std::vector<uint64_t> tl_off;
    DevBuf d_rk, d_tlp, d_suf, d_tl;
    // inside d_rank_of_item (one upload): item_of_rank and tl_off
    uint32_t *p_item_of_rank = nullptr;
    uint64_t *p_tl_off = nullptr;
    bool lists_built = false;  // d_tl holds the transaction lists
    unsigned long long project_work = 0;
    fim_stats st{};
    uint64_t first_class_rows = 0;  // sum of atoms over first-level classes with >= 2 atoms
};

}  // namespace

// Page-locked host memory for one run's device-to-host copies: a copy into
// it does not stall the host, so every instance's copy is queued before one
// wait.
struct PinnedBlock {
    void *p = nullptr;
    size_t bytes = 0;
    explicit PinnedBlock(size_t b) : bytes(std::max<size_t>(b, 8)) { p = host_pool_alloc(bytes); }
    ~PinnedBlock() { host_pool_free(p, bytes); }
    PinnedBlock(const PinnedBlock &) = delete;
    PinnedBlock &operator=(const PinnedBlock &) = delete;
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

uint32_t max_supp_of(const Inst &I) {
    uint32_t m = 0;
    for (uint32_t r = 0; r < I.n_freq; r++) m = std::max(m, I.supp_of_rank[r]);
    return m;
}

// item order key: ascending support, ties by item id (or item id alone)
static void rank_items(Inst &I, bool by_id) {
    const uint32_t ni = I.db->n_item_ids;
    I.item_of_rank.clear();
    if (by_id) {
        for (uint32_t it = 0; it < ni; it++)
            if (I.counts[it] >= I.minsup) I.item_of_rank.push_back(it);
    } else {
        // frequent ids (ascending) sorted by support with a stable LSD radix
        // sort, 11 bits a pass: ties keep the id order
        std::vector<uint32_t> a, b;
        a.reserve(ni);
        uint32_t top = 0;
        for (uint32_t it = 0; it < ni; it++)
            if (I.counts[it] >= I.minsup) {
                a.push_back(it);
                top = std::max(top, I.counts[it]);
            }
        b.resize(a.size());
        for (uint32_t sh = 0; sh < 32 && (top >> sh); sh += 11) {
            uint32_t h[2049] = {0};
            for (uint32_t it : a) h[((I.counts[it] >> sh) & 2047u) + 1]++;
            for (uint32_t d = 0; d < 2048; d++) h[d + 1] += h[d];
            for (uint32_t it : a) b[h[(I.counts[it] >> sh) & 2047u]++] = it;
            a.swap(b);
        }
        I.item_of_rank.swap(a);
    }
    I.n_freq = (uint32_t)I.item_of_rank.size();
    I.rank_of_item.assign(ni, kNone);
    I.supp_of_rank.resize(I.n_freq);
    for (uint32_t r = 0; r < I.n_freq; r++) {
        I.rank_of_item[I.item_of_rank[r]] = r;
        I.supp_of_rank[r] = I.counts[I.item_of_rank[r]];
    }
}

// atoms of every first-level class: frequent pairs (i, j) bucketed by i and
// ordered ascending by (support, item id of j), or by j (= id order)
static void build_level2(Inst &I, bool by_id, const uint32_t *pairs) {
    const uint32_t n = I.n_freq;
    I.l2_off.assign(n + 1, 0);
    for (uint64_t p = 0; p < I.n_pairs; p++) I.l2_off[pairs[3 * p] + 1]++;
    for (uint32_t i = 0; i < n; i++) I.l2_off[i + 1] += I.l2_off[i];
    I.l2_atom.resize(I.n_pairs);
    I.l2_supp.resize(I.n_pairs);
    std::vector<uint32_t> fill(I.l2_off.begin(), I.l2_off.end() - 1);
    for (uint64_t p = 0; p < I.n_pairs; p++) {
        const uint32_t i = pairs[3 * p], q = fill[i]++;
        I.l2_atom[q] = pairs[3 * p + 1];
        I.l2_supp[q] = pairs[3 * p + 2];
    }
    // every bucket sorted by its key in one array (no allocation per bucket;
    // insertion sort for the many short buckets)
    struct E {
        uint64_t key;
        uint32_t atom, supp;
    };
    std::vector<E> e(I.n_pairs);
    for (uint64_t q = 0; q < I.n_pairs; q++)
        e[q] = E{by_id ? I.l2_atom[q] : ((uint64_t)I.l2_supp[q] << 32) | I.item_of_rank[I.l2_atom[q]],
                 I.l2_atom[q], I.l2_supp[q]};
    for (uint32_t i = 0; i < n; i++) {
        const uint32_t a = I.l2_off[i], b = I.l2_off[i + 1];
        if (b - a < 2) continue;
        if (b - a <= 16) {
            for (uint32_t q = a + 1; q < b; q++) {
                const E v = e[q];
                uint32_t j = q;
                while (j > a && e[j - 1].key > v.key) {
                    e[j] = e[j - 1];
                    j--;
                }
                e[j] = v;
            }
        } else {
            std::sort(e.begin() + a, e.begin() + b, [](const E &x, const E &y) { return x.key < y.key; });
        }
    }
    for (uint64_t q = 0; q < I.n_pairs; q++) {
        I.l2_atom[q] = e[q].atom;
        I.l2_supp[q] = e[q].supp;
    }
}

// One persistent depth-first launch over `tasks`, rerun with a larger
// per-wave stack or output arena when the kernel's flags ask for it.
struct DfsLaunch {
    uint64_t frame0 = 0;  // words of the largest first frame
    uint32_t variant = 0, n_workers = 0, claim = 1, nap_max = 64;
    bool cap_output = false;     // a full output arena ends the run (internal sample runs)
    bool stop_is_error = true;   // an instance over its record budget is an error
    uint64_t out_cap = 1ull << 24;
    // words placed at the start of the arena before the launch (key mode:
    // the records of the itemsets found before the persistent kernel)
    // key records of the 1- and 2-itemsets, written before the launch
    const std::vector<PrefixSrc> *prefix = nullptr;
    uint64_t prefix_rec = 0, prefix_max = 0;  // records in all, most of one instance
    DfsCounters ctr{};
    std::vector<InstCounters> ictr;
    float ms = 0.f;
    uint32_t retries = 0;
    bool truncated = false;
    uint64_t busy_max_ns = 0, busy_mean_ns = 0;  // per wave
};

static fim_status run_persistent(fim_ctx *ctx, hipStream_t s, Tracer &tr,
                                 const std::vector<InstDesc> &desc, const std::vector<Task> &tasks,
                                 DevBuf &d_out, DfsLaunch &L) {
    const uint32_t n_inst = (uint32_t)desc.size();
    DevBuf d_in(ctx), d_stack(ctx), d_cnt(ctx), d_heap(ctx), d_trace(ctx);
    hipEvent_t ev0, ev1;
    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } evg{ev0, ev1};
    // descriptors, tasks and the prefix-record sources in one upload (pieces
    // at 8-byte multiples, as h2d_pieces lays them out)
    const size_t b_desc = desc.size() * sizeof(InstDesc), b_tasks = tasks.size() * sizeof(Task);
    const size_t b_pre = L.prefix ? L.prefix->size() * sizeof(PrefixSrc) : 0;
    const size_t at_tasks = (b_desc + 7) & ~size_t(7), at_pre = at_tasks + ((b_tasks + 7) & ~size_t(7));
    ENSURE(d_in, ctx, at_pre + b_pre + 8);
    {
        const H2DPiece up[3] = {{desc.data(), b_desc}, {tasks.data(), b_tasks},
                                {L.prefix ? L.prefix->data() : nullptr, b_pre}};
        HIPCHK(h2d_pieces(ctx, d_in.as<void>(), up, 3, s));
    }
    const InstDesc *p_desc = d_in.as<InstDesc>();
    const Task *p_tasks = reinterpret_cast<const Task *>(d_in.as<char>() + at_tasks);
    const PrefixSrc *p_pre = reinterpret_cast<const PrefixSrc *>(d_in.as<char>() + at_pre);
    L.ictr.assign(n_inst, InstCounters{});
    // per-worker stack: room for the largest first frame and its subtree,
    // within a quarter of device memory in total
    uint64_t S = (std::max<uint64_t>(4 * L.frame0, 1ull << 18) + 63) & ~63ull;
    const uint64_t kMaxStack = 0xFFFFFFF0ull;  // frame offsets are 32-bit
    // stacks and arena within what the run may plan with (half of an
    // arena's free part: the output arena and its ordering need the rest)
    const uint64_t budget_words = (uint64_t)(ctx->arena ? ctx->plan_bytes() / 2 : ctx->plan_bytes()) / 4;
    // work sharing between waves
    const uint64_t n_slots = 1ull << 16;
    const uint64_t heap_words = 1ull << 24;
    // a wave gives up waiting for donated work after 60 s of wall clock
    int clk_khz = 0;
    (void)hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, ctx->device);
    const uint64_t wait_ticks = (uint64_t)(clk_khz > 0 ? clk_khz : 100000) * 60000ull;
    // a busy wave checks for idle waves (loads of shared counters) at most
    // every 50 us (measured on dense-50k, persistent kernel: 9.7 ms polling
    // every 2 us, 8.4 ms every 20, 7.9 ms every 50, 8.1 ms every 100, 9.6 ms
    // every 300, 14.8 ms every 1000)
    uint64_t poll_ticks = (uint64_t)(clk_khz > 0 ? clk_khz : 100000) / 20;
    if (const char *e = getenv("FIM_POLL_US")) poll_ticks = (uint64_t)(clk_khz > 0 ? clk_khz : 100000) * std::max(1, atoi(e)) / 1000;  // tuning
    uint32_t nap_max = L.nap_max;
    if (const char *e = getenv("FIM_NAP_MAX")) nap_max = (uint32_t)std::max(1, atoi(e));  // tuning
    for (;;) {
        uint32_t workers = L.n_workers;
        if ((uint64_t)workers * S > budget_words)
            workers = (uint32_t)std::max<uint64_t>(4, budget_words / S / 4 * 4);
        if (((uint64_t)workers * S > budget_words && S > budget_words / 4) || S > kMaxStack)
            return set_error(FIM_E_OOM_DEVICE, "a first-level class does not fit on the device");
        ENSURE(d_stack, ctx, (size_t)workers * S * 4);
        if (L.prefix && 8 * L.prefix_rec + 8 > L.out_cap) L.out_cap = 16 * L.prefix_rec + 4096;
        ENSURE(d_out, ctx, (size_t)L.out_cap * 4);
        // the launch's counters, the instances' counters and the donation
        // slots in one block, set by one kernel (the output position past
        // the prefix records, zeros elsewhere)
        const size_t b_ictr = (sizeof(InstCounters) * n_inst + 255) & ~size_t(255);
        const size_t cnt_bytes = sizeof(DfsCounters) + b_ictr + n_slots * 8;
        ENSURE(d_cnt, ctx, cnt_bytes);
        DfsCounters *p_ctr = d_cnt.as<DfsCounters>();
        InstCounters *p_ictr = reinterpret_cast<InstCounters *>(d_cnt.as<char>() + sizeof(DfsCounters));
        unsigned long long *p_slots =
            reinterpret_cast<unsigned long long *>(d_cnt.as<char>() + sizeof(DfsCounters) + b_ictr);
        if (tr.on) {
            ENSURE(d_trace, ctx, (size_t)workers * 64);
            HIPCHK(launch_fill_u32(d_trace.as<uint32_t>(), (uint64_t)workers * 16, 0u, s));
        }
        ENSURE(d_heap, ctx, heap_words * 4);
        const unsigned long long start = (L.prefix && L.prefix_rec) ? 8 * L.prefix_rec : 0;
        HIPCHK(launch_fill_words(d_cnt.as<uint32_t>(), cnt_bytes / 4, offsetof(DfsCounters, out_used) / 4, start, s));
        if (start)
            HIPCHK(launch_prefix_keys(p_pre, (uint32_t)L.prefix->size(), L.prefix_max, d_out.as<uint32_t>(), s));
        if (L.cap_output) HIPCHK(launch_fill_u32(d_out.as<uint32_t>(), L.out_cap, 0u, s));
        tr.mark("  (dfs inputs queued)");
        HIPCHK(hipEventRecord(ev0, s));
        // at most one worker per CU: one wave per block, so that the waves
        // spread over all CUs instead of filling a quarter of them
        uint32_t wpb = workers <= (uint32_t)std::max(ctx->n_cu, 1) ? 1u : 4u;
        if (const char *e = getenv("FIM_WPB")) wpb = (uint32_t)std::max(1, std::min(4, atoi(e)));  // tuning
        if (workers % wpb != 0) wpb = 1;
        auto launch = [&]() {
            return launch_dfs(p_desc, p_tasks, tasks.size(),
                              d_stack.as<uint32_t>(), S, workers, L.claim, d_out.as<uint32_t>(),
                              L.out_cap, p_ctr, p_ictr, p_slots, n_slots, d_heap.as<uint32_t>(),
                              heap_words, wait_ticks,
                              tr.on ? d_trace.as<unsigned long long>() : nullptr, L.variant, nap_max,
                              poll_ticks, wpb, s);
        };
        HIPCHK(launch());
        HIPCHK(hipEventRecord(ev1, s));
        // both kinds of counters in one copy
        std::vector<char> h_cnt(sizeof(DfsCounters) + sizeof(InstCounters) * n_inst);
        HIPCHK(hipMemcpyAsync(h_cnt.data(), d_cnt.as<void>(), h_cnt.size(), hipMemcpyDeviceToHost, s));
        tr.mark("  (dfs queued)");
        HIPCHK(stream_wait(s));
        memcpy(&L.ctr, h_cnt.data(), sizeof(DfsCounters));
        memcpy(L.ictr.data(), h_cnt.data() + sizeof(DfsCounters), sizeof(InstCounters) * n_inst);
        tr.mark("  (dfs done)");
        HIPCHK(hipEventElapsedTime(&L.ms, ev0, ev1));
        const DfsCounters &ctr = L.ctr;
        if (clk_khz > 0) {
            L.busy_max_ns = (uint64_t)((double)ctr.busy_max * 1e6 / clk_khz);
            L.busy_mean_ns = (uint64_t)((double)ctr.busy_sum / workers * 1e6 / clk_khz);
        }
        if (tr.on) {
            const double mean = (double)ctr.busy_sum / workers;
            std::vector<unsigned long long> wt((size_t)workers * 8);
            if (hipMemcpy(wt.data(), d_trace.as<void>(), wt.size() * 8, hipMemcpyDeviceToHost) == hipSuccess) {
                std::vector<uint32_t> ord(workers);
                std::iota(ord.begin(), ord.end(), 0u);
                std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return wt[8 * a] > wt[8 * b]; });
                for (uint32_t x = 0; x < std::min<uint32_t>(5, workers); x++) {
                    const unsigned long long *v = &wt[8 * ord[x]];
                    fprintf(stderr, "[fim %s]   wave %u busy %.3f ms pieces %llu given %llu cands %llu max_k %llu max_depth %llu (%llu %llu)\n",
                            tr.tag, ord[x], clk_khz ? v[0] / (double)clk_khz : 0.0, v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
                }
            }
            fprintf(stderr, "[fim %s] dfs kernel %.3f ms, %zu tasks, %llu donations, %u workers, busiest %.3f ms, mean %.3f ms, imbalance %.1f, flags %u\n",
                    tr.tag, L.ms, tasks.size(), (unsigned long long)ctr.donations, workers,
                    clk_khz ? ctr.busy_max / (double)clk_khz : 0.0,
                    clk_khz ? mean / clk_khz : 0.0, mean > 0 ? ctr.busy_max / mean : 0.0, ctr.flags);
        }
        if (ctr.flags & kFlagSpin)
            return set_error(FIM_E_DEVICE, "work sharing between waves timed out");
        if (ctr.flags & kFlagDepthOverflow)
            return set_error(FIM_E_OUTPUT_LIMIT, "an itemset is longer than " +
                                                     std::to_string(kMaxDepth + 2) + " items");
        bool again = false;
        if (ctr.flags & kFlagStackOverflow) {
            // a multiple of 64 words keeps every wave's region 256-byte aligned
            S = (std::max<uint64_t>(2 * S, ctr.stack_need + ctr.stack_need / 4) + 63) & ~63ull;
            again = true;
        }
        if (L.stop_is_error)
            for (uint32_t q = 0; q < n_inst; q++)
                if (L.ictr[q].stop)
                    return set_error(FIM_E_OUTPUT_LIMIT, "instance " + std::to_string(q) +
                                                             ": more frequent itemsets than max_itemsets");
        if ((ctr.flags & kFlagOutOverflow) || ctr.out_used.v > L.out_cap) {
            // grow the arena (work sharing varies the need between runs);
            // a sample run past a hard cap is cut short instead
            const uint64_t want = ctr.out_used.v + ctr.out_used.v / 2 + 4096;
            if (L.cap_output && want > kSampleOutCap) {
                L.truncated = true;
            } else {
                L.out_cap = want;
                again = true;
            }
        }
        if (!again) break;
        L.retries++;
        if (L.retries > 12) return set_error(FIM_E_DEVICE, "persistent kernel did not converge");
    }
    return FIM_OK;
}

// Longest itemset of the sample the estimate counts (see count_estimate):
// the sample is searched to itemsets of four items, so that its cost stays
// a fraction of the run's (measured on dense-50k: searched to the bottom it
// took 5.7 ms against 1.4 ms, for a plan that saved 1.1 ms more of kernel
// time).
static constexpr uint32_t kSampleMaxLen = 4;

// Phase 1 inside the run: for every instance to estimate, a sample of
// |D~| transactions drawn with replacement is turned into bitmaps over the
// instance's own frequent items, and the persistent kernel mines it on the
// instance's own first-level classes (the same atoms, in the same order) at
// the relative minimum support, counting every frequent itemset of 3 to
// kSampleMaxLen items into its second-level class instead of reporting it;
// one task per second-level class.  row_w[q] gets
// count x words per row for every second-level class of instance q (empty
// when the instance has no estimate); out_words the sample's record words.
static fim_status count_estimate(fim_ctx *ctx, hipStream_t s, Tracer &tr, std::vector<Inst> &insts,
                                 const std::vector<PlanInput> &pin, const fim_options &opts,
                                 std::vector<std::vector<double>> &row_w, uint64_t &out_words) {
    const uint32_t n_inst = (uint32_t)insts.size();
    row_w.assign(n_inst, {});
    out_words = 0;
    const uint32_t want_tx = opts.sample_tx ? opts.sample_tx : default_sample_tx(0.02, 0.05);
    std::vector<InstDesc> desc(n_inst);
    std::vector<Task> tasks;
    std::vector<DevBuf> s_off, s_items, s_rows;
    for (uint32_t q = 0; q < n_inst; q++) {
        s_off.emplace_back(ctx);
        s_items.emplace_back(ctx);
        s_rows.emplace_back(ctx);
    }
    std::vector<std::vector<uint64_t>> h_off(n_inst);  // kept until the copies are done
    std::vector<std::vector<uint32_t>> h_items(n_inst);
    std::vector<uint64_t> count_at(n_inst + 1, 0);
    std::vector<bool> used(n_inst, false);
    uint64_t frame0 = 0;
    uint32_t max_chunks = 0;
    auto sample_size = [&](uint32_t q) -> uint64_t {
        const Inst &I = insts[q];
        const uint64_t nd = std::min<uint64_t>(want_tx, I.db->n_tx / 4);
        return (!pin[q].estimate || nd < 256 || I.n_freq < 3 || I.l2_atom.empty()) ? 0 : nd;
    };
    // the instances' samples are independent: drawn side by side
    parallel_for(n_inst, host_threads((uint64_t)n_inst * want_tx * 8), [&](uint64_t q) {
        const uint64_t nd = sample_size((uint32_t)q);
        if (nd)
            draw_sample(insts[q].db, insts[q].rank_of_item, nd,
                        opts.seed ^ (0x51ED270B1DE0ull * (q + 1)), h_off[q], h_items[q]);
    });
    for (uint32_t q = 0; q < n_inst; q++) {
        Inst &I = insts[q];
        count_at[q + 1] = count_at[q] + I.l2_atom.size();
        const uint64_t N = I.db->n_tx;
        const uint64_t nd = sample_size(q);
        if (nd == 0) continue;
        std::vector<uint64_t> &off = h_off[q];
        std::vector<uint32_t> &items = h_items[q];
        const uint32_t Ws = (uint32_t)((nd + 31) / 32);
        const uint32_t Wps = std::max<uint32_t>(kRowAlign, (Ws + kRowAlign - 1) / kRowAlign * kRowAlign);
        ENSURE(s_off[q], ctx, off.size() * 8);
        ENSURE(s_items[q], ctx, std::max<size_t>(items.size(), 1) * 4);
        ENSURE(s_rows[q], ctx, (size_t)I.n_freq * Wps * 4);
        HIPCHK(hipMemcpyAsync(s_off[q].as<void>(), off.data(), off.size() * 8, hipMemcpyHostToDevice, s));
        if (!items.empty())
            HIPCHK(hipMemcpyAsync(s_items[q].as<void>(), items.data(), items.size() * 4,
                                  hipMemcpyHostToDevice, s));
        HIPCHK(launch_fill_u32(s_rows[q].as<uint32_t>(), (uint64_t)I.n_freq * Wps, 0u, s));
        HIPCHK(launch_bitmap_build(s_off[q].as<uint64_t>(), s_items[q].as<uint32_t>(), nd,
                                   I.d_rank_of_item.as<uint32_t>(), s_rows[q].as<uint32_t>(), Wps, s));
        InstDesc &D = desc[q];
        D.rows = s_rows[q].as<uint32_t>();
        D.item_of_rank = I.p_item_of_rank;
        D.l2_off = I.d_l2_off.as<uint32_t>();
        D.l2_atom = I.d_l2_atom.as<uint32_t>();
        D.l2_supp = I.d_l2_supp.as<uint32_t>();
        D.Wp = Wps;
        D.n_freq = I.n_freq;
        // relative minimum support carried over to the sample, at least 2
        D.minsup = std::max<uint32_t>(2, (uint32_t)ceil((double)I.minsup * (double)nd / (double)N));
        D.max_len = kSampleMaxLen;
        D.order_by_id = (opts.flags & FIM_FLAG_ORDER_BY_ID) ? 1u : 0u;
        D.project = (opts.flags & FIM_FLAG_NO_PROJECT) ? 0u : 1u;
        D.rec_budget = kSampleRecordBudget;
        used[q] = true;
        max_chunks = std::max(max_chunks, Wps / 4);
        // one task per second-level class (row of a first-level class), so
        // that the sample's wide classes spread over the waves
        for (uint32_t i = 0; i < I.n_freq; i++) {
            const uint32_t f = I.l2_off[i + 1] - I.l2_off[i];
            if (f < 2) continue;
            for (uint32_t r = 0; r + 1 < f; r++) tasks.push_back(Task{q, i, r, r + 1});
            frame0 = std::max<uint64_t>(frame0, (uint64_t)f * Wps + 3ull * f);
        }
    }
    if (tasks.empty()) return FIM_OK;
    // most later atoms first
    std::stable_sort(tasks.begin(), tasks.end(), [&](const Task &a, const Task &b) {
        return insts[a.inst].l2_off[a.node + 1] - insts[a.inst].l2_off[a.node] - a.r0 >
               insts[b.inst].l2_off[b.node + 1] - insts[b.inst].l2_off[b.node] - b.r0;
    });
    DevBuf d_count(ctx), d_out(ctx);
    ENSURE(d_count, ctx, std::max<uint64_t>(count_at[n_inst], 1) * 8);
    HIPCHK(launch_fill_u32(d_count.as<uint32_t>(), std::max<uint64_t>(count_at[n_inst], 1) * 2, 0u, s));
    for (uint32_t q = 0; q < n_inst; q++)
        if (used[q]) desc[q].class_count = d_count.as<unsigned long long>() + count_at[q];
    DevBuf d_pcand(ctx);  // a class profile: the sample's candidate pairs per class
    if (g_profile) {
        ENSURE(d_pcand, ctx, std::max<uint64_t>(count_at[n_inst], 1) * 8);
        HIPCHK(launch_fill_u32(d_pcand.as<uint32_t>(), std::max<uint64_t>(count_at[n_inst], 1) * 2, 0u, s));
        for (uint32_t q = 0; q < n_inst; q++)
            if (used[q]) desc[q].row_cand = d_pcand.as<unsigned long long>() + count_at[q];
    }
    DfsLaunch L;
    L.frame0 = frame0;
    L.variant = dfs_variant(max_chunks);
    L.n_workers = std::max<uint32_t>(4, dfs_resident_workers(ctx->n_cu, L.variant) / 4 * 4);
    // about one wave per eight small tasks, as in the main run
    L.n_workers = std::min<uint32_t>(L.n_workers, std::max<uint32_t>(256, (uint32_t)(tasks.size() / 8 + 3) / 4 * 4));
    L.nap_max = 64;
    L.cap_output = true;
    L.stop_is_error = false;
    L.out_cap = 1024;  // nothing is reported
    Tracer sub("sample");
    sub.on = tr.on;
    fim_status st = run_persistent(ctx, s, sub, desc, tasks, d_out, L);
    if (st != FIM_OK) return st;
    std::vector<unsigned long long> cnt(count_at[n_inst]), pcand;
    if (!cnt.empty())
        HIPCHK(hipMemcpyAsync(cnt.data(), d_count.as<void>(), cnt.size() * 8, hipMemcpyDeviceToHost, s));
    if (g_profile && !cnt.empty()) {
        pcand.resize(cnt.size());
        HIPCHK(hipMemcpyAsync(pcand.data(), d_pcand.as<void>(), pcand.size() * 8, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(stream_wait(s));
    if (g_profile && n_inst == 1 && used[0]) {
        g_profile->est_fi.assign(cnt.begin(), cnt.begin() + count_at[1]);
        g_profile->est_cand.assign(pcand.begin(), pcand.begin() + count_at[1]);
    }
    for (uint32_t q = 0; q < n_inst; q++) {
        if (!used[q] || L.ictr[q].stop) continue;  // exploded sample: no estimate
        const Inst &I = insts[q];
        row_w[q].assign(I.l2_atom.size(), 0.0);
        uint64_t any = 0;
        for (size_t k = 0; k < I.l2_atom.size(); k++) {
            row_w[q][k] = (double)cnt[count_at[q] + k] * (double)I.W;
            any += cnt[count_at[q] + k];
        }
        if (!any) row_w[q].clear();
        out_words += L.ictr[q].out_words;
    }
    return FIM_OK;
}

fim_status mine_many(fim_ctx *ctx, const std::vector<MineRequest> &reqs, const fim_options &opts_in,
                     std::vector<fim_result *> &results) {
    const auto t_start = clk::now();
    const fim_options opts = resolve_options(&opts_in);
    const bool sample_run = (opts.flags & kFlagInternalSample) != 0;
    Tracer tr(sample_run ? "sample" : "mine");
    const bool by_id = (opts.flags & FIM_FLAG_ORDER_BY_ID) != 0;
    const uint32_t n_inst = (uint32_t)reqs.size();
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    StageRun stage_run(ctx);
    std::vector<Inst> insts(n_inst);

    // ---------------- a2: item supports (all instances, one sync). Several
    // instances spread over the context's side streams, forked from and
    // joined back into s by events; each side stream has its own slice of
    // the block-histogram scratch, used in that stream's order.
    std::vector<hipStream_t> side;
    hipEvent_t ev_fork = nullptr;
    if (n_inst > 1) {
        HIPCHK(ctx_side_streams(ctx, side));
        HIPCHK(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    }
    struct ForkGuard {
        hipEvent_t e;
        ~ForkGuard() {
            if (e) (void)hipEventDestroy(e);
        }
    } fork_guard{ev_fork};
    // side streams start after everything queued on s so far
    auto fork = [&]() -> hipError_t {
        if (side.empty()) return hipSuccess;
        hipError_t e = hipEventRecord(ev_fork, s);
        for (size_t i = 0; e == hipSuccess && i < side.size(); i++) e = hipStreamWaitEvent(side[i], ev_fork, 0);
        return e;
    };
    // s continues after everything queued on the side streams
    auto join = [&]() -> hipError_t {
        for (hipStream_t x : side) {
            hipEvent_t ej = nullptr;
            hipError_t e = hipEventCreateWithFlags(&ej, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(ej, x);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, ej, 0);
            if (ej) (void)hipEventDestroy(ej);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const uint32_t n_lanes = side.empty() ? 1u : (uint32_t)side.size();
    std::vector<uint64_t> count_at(n_inst + 1, 0);
    for (uint32_t q = 0; q < n_inst; q++) count_at[q + 1] = count_at[q] + reqs[q].db->n_item_ids;
    PinnedBlock h_counts(count_at[n_inst] * 4);
    DevBuf d_part(ctx), d_counts_all(ctx), d_count_src(ctx);
    if (n_inst > 1) {
        // every instance's item supports in one launch into one array, and
        // one copy back
        std::vector<CountSrc> src(n_inst);
        uint32_t blocks = 0, max_ids = 0;
        for (uint32_t q = 0; q < n_inst; q++) {
            Inst &I = insts[q];
            I.db = reqs[q].db;
            I.minsup = reqs[q].minsup;
            src[q] = CountSrc{I.db->d_items.as<uint32_t>(), I.db->nnz, count_at[q], I.db->n_item_ids, blocks};
            blocks += count_many_blocks(I.db->nnz);
            max_ids = std::max(max_ids, I.db->n_item_ids);
        }
        ENSURE(d_counts_all, ctx, std::max<uint64_t>(count_at[n_inst], 1) * 4);
        ENSURE(d_count_src, ctx, n_inst * sizeof(CountSrc));
        HIPCHK(h2d(ctx, d_count_src.as<void>(), src.data(), n_inst * sizeof(CountSrc), s));
        HIPCHK(launch_fill_u32(d_counts_all.as<uint32_t>(), count_at[n_inst], 0u, s));
        HIPCHK(launch_item_count_many(d_count_src.as<CountSrc>(), n_inst, blocks, max_ids,
                                      d_counts_all.as<uint32_t>(), s));
        if (count_at[n_inst])
            HIPCHK(hipMemcpyAsync(h_counts.as<uint32_t>(), d_counts_all.as<void>(), count_at[n_inst] * 4,
                                  hipMemcpyDeviceToHost, s));
        for (uint32_t q = 0; q < n_inst; q++) insts[q].p_counts = d_counts_all.as<uint32_t>() + count_at[q];
    } else {
        Inst &I = insts[0];
        I.db = reqs[0].db;
        I.minsup = reqs[0].minsup;
        const uint32_t ni = I.db->n_item_ids;
        const uint64_t part_words = item_count_scratch_words(I.db->nnz, ni);
        if (part_words) ENSURE(d_part, ctx, part_words * 4);
        ENSURE(I.d_counts, ctx, (size_t)ni * 4);
        HIPCHK(launch_item_count(I.db->d_items.as<uint32_t>(), I.db->nnz, I.d_counts.as<uint32_t>(), ni,
                                 part_words ? d_part.as<uint32_t>() : nullptr, s));
        HIPCHK(hipMemcpyAsync(h_counts.as<uint32_t>(), I.d_counts.as<void>(), (size_t)ni * 4,
                              hipMemcpyDeviceToHost, s));
        I.p_counts = I.d_counts.as<uint32_t>();
    }
    HIPCHK(stream_wait(s));
    for (uint32_t q = 0; q < n_inst; q++)
        insts[q].counts.assign(h_counts.as<uint32_t>() + count_at[q], h_counts.as<uint32_t>() + count_at[q + 1]);
    tr.mark("item supports");

    // ---------------- a3 + root class: bitmaps and frequent pairs
    hipEvent_t ev0, ev1;
    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } evg{ev0, ev1};
    float root_ms = 0.f;
    // one event pair per instance around its root-class kernel
    HIPCHK(ctx_timing_events(ctx, 2ull * n_inst));
    const std::vector<hipEvent_t> &rev = ctx->timing_events;
    // per instance: frequent pairs found, pair increments (projected root)
    PinnedBlock h_small(16ull * n_inst);
    memset(h_small.p, 0, 16ull * n_inst);
    // several instances: their root work spread over the side streams so
    // that the small kernels of different instances overlap (joined below)
    HIPCHK(fork());
    DevBuf d_rsplit(ctx);
    tr.mark("  (events)");
    // item ranks of every instance (independent host work, so several
    // instances are ranked on several threads)
    parallel_for(n_inst, n_inst > 1 ? host_threads(count_at[n_inst]) : 1u,
                 [&](uint64_t q) { rank_items(insts[q], by_id); });
    tr.mark("  (ranks)");
    for (uint32_t q = 0; q < n_inst; q++) {
        Inst &I = insts[q];
        const hipStream_t sq = side.empty() ? s : side[q % side.size()];
        I.W = (uint32_t)((I.db->n_tx + 31) / 32);
        I.Wp = std::max<uint32_t>(kRowAlign, (I.W + kRowAlign - 1) / kRowAlign * kRowAlign);
        I.st.item_supports = I.db->n_item_ids;
        I.st.n_frequent_items = I.n_freq;
        if (I.n_freq == 0) continue;
        const uint32_t ni = I.db->n_item_ids;
        const uint32_t n = I.n_freq;
        // offsets of the ranks' transaction lists (used if lists are built)
        I.tl_off.assign(n + 1, 0);
        for (uint32_t r = 0; r < n; r++) I.tl_off[r + 1] = I.tl_off[r] + I.supp_of_rank[r];
        // rank_of_item, item_of_rank and tl_off in one device block, one copy
        const size_t b_rank = ((size_t)ni * 4 + 7) & ~size_t(7);
        const size_t b_item = ((size_t)n * 4 + 7) & ~size_t(7);
        ENSURE(I.d_rank_of_item, ctx, b_rank + b_item + (size_t)(n + 1) * 8);
        ENSURE(I.d_rows, ctx, (size_t)I.n_freq * I.Wp * 4);
        I.p_item_of_rank = reinterpret_cast<uint32_t *>(I.d_rank_of_item.as<char>() + b_rank);
        I.p_tl_off = reinterpret_cast<uint64_t *>(I.d_rank_of_item.as<char>() + b_rank + b_item);
        const H2DPiece up[3] = {{I.rank_of_item.data(), (size_t)ni * 4},
                                {I.item_of_rank.data(), (size_t)n * 4},
                                {I.tl_off.data(), (size_t)(n + 1) * 8}};
        HIPCHK(h2d_pieces(ctx, I.d_rank_of_item.as<void>(), up, 3, sq));
        tr.mark("  (rank uploads)");
        // positions in the ranked transactions are 32-bit, ranks and suffix
        // lengths 16-bit
        const bool fits = I.db->nnz + I.db->n_tx + 8 < (1ull << 32) && I.db->max_tx_len < (1u << 16) &&
                          n < 0xFFFFu;
        const bool pairs_needed = n >= 2 && opts.max_len != 1;
        if (pairs_needed) {
            // Root-class kernel by estimated time (picoseconds per unit measured
            // on MI355X): whole rows cost all * W pair-words; covers at most
            // sum_i min(supp_i, W)(n - 1 - i) pair-words (row i has at most
            // min(supp_i, W) non-zero words), each a cached 4-byte load; the
            // projected count one LDS increment per pair inside a transaction
            // (bounded by the pairs over all items) plus its set-up.
            const uint64_t all = (uint64_t)n * (n - 1) / 2;
            double bound = 0.0;
            for (uint32_t r = 0; r < n; r++)
                bound += (double)std::min<uint32_t>(I.supp_of_rank[r], I.W) * (double)(n - 1 - r);
            const double t_rows = 0.075 * (double)all * (double)I.W;
            const double t_covers = n >= 64 && n <= 65535 ? 0.75 * bound + 1.5e5 : 1e300;
            const double t_project =
                fits ? 20.0 * (double)I.db->pairs_in_tx + 6.0 * (double)I.db->nnz + 1.5e5 : 1e300;
            if (opts.flags & FIM_FLAG_DENSE_ROOT) I.root_kind = 0;
            else if (opts.flags & FIM_FLAG_ROOT_COVERS) I.root_kind = n <= 65535 ? 1 : 0;
            else if (opts.flags & FIM_FLAG_ROOT_PROJECT) I.root_kind = fits ? 2 : 0;
            else if (t_project <= t_covers && t_project < t_rows) I.root_kind = 2;
            else if (t_covers < t_rows) I.root_kind = 1;
            else I.root_kind = 0;
        }
        // One instance with the projected root: its transactions are ranked
        // on a side stream while the rows and lists are built on sq (the
        // ranking reads only the transactions and the ranks just uploaded).
        hipEvent_t ev_ranked = nullptr;
        if (n_inst == 1 && I.root_kind == 2 && pairs_needed) {
            std::vector<hipStream_t> rs;
            HIPCHK(ctx_side_streams(ctx, rs));
            for (hipEvent_t &e : ctx->sync_events)
                if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            ENSURE(I.d_rk, ctx, (I.db->nnz + I.db->n_tx + 48) * 2);
            HIPCHK(hipEventRecord(ctx->sync_events[0], sq));
            HIPCHK(hipStreamWaitEvent(rs[0], ctx->sync_events[0], 0));
            HIPCHK(launch_rank_only(I.db->d_off.as<uint64_t>(), I.db->d_items.as<uint32_t>(), I.db->n_tx,
                                    I.d_rank_of_item.as<uint32_t>(), I.d_rk.as<uint16_t>(), rs[0]));
            ev_ranked = ctx->sync_events[1];
            HIPCHK(hipEventRecord(ev_ranked, rs[0]));
            tr.mark("  (ranking queued)");
        }
        // rows from LDS tiles (a column window of a group of rows) when the
        // device's LDS allows, else zero fill and global atomics
        if (bitmap_tiles_fit(ctx->lds_per_block)) {
            HIPCHK(launch_bitmap_tiles(I.db->d_off.as<uint64_t>(), I.db->d_items.as<uint32_t>(),
                                       I.db->n_tx, I.d_rank_of_item.as<uint32_t>(), n,
                                       I.d_rows.as<uint32_t>(), I.Wp, ctx->lds_per_block, sq));
        } else {
            HIPCHK(launch_fill_u32(I.d_rows.as<uint32_t>(), (uint64_t)n * I.Wp, 0u, sq));
            HIPCHK(launch_bitmap_build(I.db->d_off.as<uint64_t>(), I.db->d_items.as<uint32_t>(),
                                       I.db->n_tx, I.d_rank_of_item.as<uint32_t>(),
                                       I.d_rows.as<uint32_t>(), I.Wp, sq));
        }
        tr.mark("  (bitmap queued)");
        // Ascending transaction lists of the ranks (the set bits of their
        // rows), used by the projected root kernel and by pieces of work
        // whose rows are projected on a one-item prefix's cover
        uint32_t min_supp = ~0u;
        for (uint32_t r = 0; r < n; r++) min_supp = std::min(min_supp, I.supp_of_rank[r]);
        const bool lists = (I.root_kind == 2 && pairs_needed) ||
                           (!(opts.flags & FIM_FLAG_NO_PROJECT) && n >= 3 &&
                            (opts.max_len == 0 || opts.max_len >= 3) &&
                            4ull * min_supp <= I.db->n_tx && I.db->n_tx < (1ull << 32));
        if (lists) {
            I.lists_built = true;
            ENSURE(I.d_tl, ctx, std::max<uint64_t>(I.tl_off[n], 1) * 4);
            const bool ranked = I.root_kind == 2 && pairs_needed;
            if (ranked) ENSURE(I.d_suf, ctx, std::max<uint64_t>(I.tl_off[n], 1) * 2);
            // the ranks of the entries go to suf, which k_tl_slots then
            // overwrites with the suffix lengths
            HIPCHK(launch_tidlist(I.d_rows.as<uint32_t>(), n, I.Wp, I.p_tl_off, I.d_tl.as<uint32_t>(),
                                  ranked ? I.d_suf.as<uint16_t>() : nullptr, sq));
            if (ranked) {
                ENSURE(I.d_rk, ctx, (I.db->nnz + I.db->n_tx + 48) * 2);
                ENSURE(I.d_tlp, ctx, std::max<uint64_t>(I.tl_off[n], 1) * 4);
                if (ev_ranked) {
                    HIPCHK(hipStreamWaitEvent(sq, ev_ranked, 0));
                    HIPCHK(launch_tl_slots(I.db->d_off.as<uint64_t>(), I.db->n_tx, I.d_rk.as<uint16_t>(),
                                           I.d_tl.as<uint32_t>(), I.tl_off[n], I.d_tlp.as<uint32_t>(),
                                           I.d_suf.as<uint16_t>(), sq));
                } else {
                    HIPCHK(launch_rank_tx(I.db->d_off.as<uint64_t>(), I.db->d_items.as<uint32_t>(),
                                          I.db->n_tx, I.d_rank_of_item.as<uint32_t>(),
                                          I.d_tl.as<uint32_t>(), I.tl_off[n], I.d_rk.as<uint16_t>(),
                                          I.d_tlp.as<uint32_t>(), I.d_suf.as<uint16_t>(), sq));
                }
            }
        }
        if (ev_ranked) HIPCHK(hipStreamWaitEvent(sq, ev_ranked, 0));  // joined in every case
        tr.mark("  (lists queued)");
        if (!pairs_needed) continue;
        const uint64_t all = (uint64_t)n * (n - 1) / 2;
        const uint64_t cap = std::min<uint64_t>(all, std::max<uint64_t>(1u << 16, 64ull * n));
        ENSURE(I.d_pairs, ctx, cap * 12);
        // the frequent pairs found and (projected root) the pair increments,
        // side by side: one fill, one copy back
        ENSURE(I.d_npairs, ctx, 16);
        HIPCHK(launch_fill_u32(I.d_npairs.as<uint32_t>(), 4, 0u, sq));
        if (I.root_kind == 2) {
            HIPCHK(hipEventRecord(rev[2 * q], sq));
            HIPCHK(launch_root_project(I.d_rk.as<uint16_t>(), I.d_tlp.as<uint32_t>(),
                                       I.d_suf.as<uint16_t>(), I.p_tl_off, n,
                                       max_supp_of(I), I.minsup,
                                       I.d_pairs.as<uint32_t>(), cap,
                                       I.d_npairs.as<unsigned long long>(),
                                       I.d_npairs.as<unsigned long long>() + 1, sq));
            HIPCHK(hipEventRecord(rev[2 * q + 1], sq));
        } else if (I.root_kind == 1) {
            I.nz_off.assign(n + 1, 0);
            for (uint32_t r = 0; r < n; r++)
                I.nz_off[r + 1] = I.nz_off[r] + std::min<uint32_t>(I.supp_of_rank[r], I.W);
            const uint64_t np = (n + 3) / 4 * 4;
            ENSURE(I.d_nz_off, ctx, (n + 1) * 8);
            ENSURE(I.d_nz_w, ctx, std::max<uint64_t>(I.nz_off[n], 1) * 4);
            ENSURE(I.d_nz_m, ctx, std::max<uint64_t>(I.nz_off[n], 1) * 4);
            ENSURE(I.d_nz_cnt, ctx, (size_t)n * 4);
            ENSURE(I.d_bt, ctx, (size_t)I.W * np * 4);
            HIPCHK(h2d(ctx, I.d_nz_off.as<void>(), I.nz_off.data(), (n + 1) * 8, sq));
            HIPCHK(launch_row_nonzero(I.d_rows.as<uint32_t>(), n, I.Wp, I.d_nz_off.as<uint64_t>(),
                                      I.d_nz_w.as<uint32_t>(), I.d_nz_m.as<uint32_t>(),
                                      I.d_nz_cnt.as<uint32_t>(), sq));
            HIPCHK(launch_transpose(I.d_rows.as<uint32_t>(), n, I.Wp, I.W, I.d_bt.as<uint32_t>(),
                                    (uint32_t)np, sq));
            HIPCHK(hipEventRecord(rev[2 * q], sq));
            HIPCHK(launch_root_sparse(I.d_bt.as<uint32_t>(), (uint32_t)np, I.d_nz_off.as<uint64_t>(),
                                      I.d_nz_cnt.as<uint32_t>(), I.d_nz_w.as<uint32_t>(),
                                      I.d_nz_m.as<uint32_t>(), n, I.minsup,
                                      I.d_pairs.as<uint32_t>(), cap,
                                      I.d_npairs.as<unsigned long long>(), sq));
            HIPCHK(hipEventRecord(rev[2 * q + 1], sq));
            I.nz_cnt.resize(n);
            HIPCHK(hipMemcpyAsync(I.nz_cnt.data(), I.d_nz_cnt.as<void>(), (size_t)n * 4,
                                  hipMemcpyDeviceToHost, sq));
        } else {
            // word-range split scratch: one slice per stream, sized once
            ENSURE(d_rsplit, ctx, root_pairs_scratch_words() * n_lanes * 4);
            HIPCHK(hipEventRecord(rev[2 * q], sq));
            HIPCHK(launch_root_pairs(I.d_rows.as<uint32_t>(), I.n_freq, I.Wp, I.minsup,
                                     I.d_pairs.as<uint32_t>(), cap,
                                     I.d_npairs.as<unsigned long long>(),
                                     d_rsplit.as<uint32_t>() + (q % n_lanes) * root_pairs_scratch_words(),
                                     sq));
            HIPCHK(hipEventRecord(rev[2 * q + 1], sq));
        }
        HIPCHK(hipMemcpyAsync(h_small.as<unsigned long long>() + 2 * q, I.d_npairs.as<void>(), 16,
                              hipMemcpyDeviceToHost, sq));
    }
    HIPCHK(join());
    const bool deep = opts.max_len == 0 || opts.max_len >= 3;
    tr.mark("  (root work queued)");
    HIPCHK(stream_wait(s));
    tr.mark("  (root work done)");
    for (uint32_t q = 0; q < n_inst; q++) {
        Inst &I = insts[q];
        if (I.n_freq < 2 || opts.max_len == 1) continue;
        I.n_pairs = h_small.as<unsigned long long>()[2 * q];
        if (I.root_kind == 2) I.project_work = h_small.as<unsigned long long>()[2 * q + 1];
    }
    // every instance's frequent pairs into one page-locked block, one wait
    std::vector<uint64_t> pair_at(n_inst + 1, 0);
    for (uint32_t q = 0; q < n_inst; q++) {
        const Inst &I = insts[q];
        pair_at[q + 1] = pair_at[q] + ((I.n_freq < 2 || opts.max_len == 1) ? 0 : I.n_pairs);
    }
    PinnedBlock h_pairs(pair_at[n_inst] * 12);
    auto h_pairs_of = [&](uint32_t q) { return h_pairs.as<uint32_t>() + 3 * pair_at[q]; };
    for (uint32_t q = 0; q < n_inst; q++) {
        const Inst &I = insts[q];
        if (I.n_freq < 2 || opts.max_len == 1) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, rev[2 * q], rev[2 * q + 1]));
        root_ms += ms;
    }
    for (uint32_t q = 0; q < n_inst; q++) {
        Inst &I = insts[q];
        if (I.n_freq < 2 || opts.max_len == 1) continue;
        const uint64_t all = (uint64_t)I.n_freq * (I.n_freq - 1) / 2;
        const uint64_t cap = I.d_pairs.bytes() / 12;
        if (I.n_pairs > cap) {  // rerun with room for every frequent pair
            ENSURE(I.d_pairs, ctx, I.n_pairs * 12);
            HIPCHK(launch_fill_u32(I.d_npairs.as<uint32_t>(), 4, 0u, s));
            if (I.root_kind == 2)
                HIPCHK(launch_root_project(I.d_rk.as<uint16_t>(), I.d_tlp.as<uint32_t>(),
                                           I.d_suf.as<uint16_t>(), I.p_tl_off,
                                           I.n_freq, max_supp_of(I), I.minsup,
                                           I.d_pairs.as<uint32_t>(), I.n_pairs,
                                           I.d_npairs.as<unsigned long long>(),
                                           I.d_npairs.as<unsigned long long>() + 1, s));
            else if (I.root_kind == 1)
                HIPCHK(launch_root_sparse(I.d_bt.as<uint32_t>(), (uint32_t)((I.n_freq + 3) / 4 * 4),
                                          I.d_nz_off.as<uint64_t>(), I.d_nz_cnt.as<uint32_t>(),
                                          I.d_nz_w.as<uint32_t>(), I.d_nz_m.as<uint32_t>(),
                                          I.n_freq, I.minsup, I.d_pairs.as<uint32_t>(), I.n_pairs,
                                          I.d_npairs.as<unsigned long long>(), s));
            else
                HIPCHK(launch_root_pairs(I.d_rows.as<uint32_t>(), I.n_freq, I.Wp, I.minsup,
                                         I.d_pairs.as<uint32_t>(), I.n_pairs,
                                         I.d_npairs.as<unsigned long long>(),
                                         d_rsplit.bytes() ? d_rsplit.as<uint32_t>() : nullptr, s));
            I.st.retries++;
        }
        if (I.n_pairs)
            HIPCHK(hipMemcpyAsync(h_pairs_of(q), I.d_pairs.as<void>(), I.n_pairs * 12,
                                  hipMemcpyDeviceToHost, s));
        I.st.candidates = all;
        I.st.root_candidates = all;
        I.st.root_kernel = I.root_kind;
        if (I.root_kind == 2) {
            // increments: the pairs inside the transactions; bytes: a 16-bit
            // rank per increment, and per tid-list entry its 32-bit pointer
            // and 16-bit suffix length
            I.st.root_pair_words = I.project_work;
            I.st.bytes_algorithmic = 2 * I.project_work + 6 * I.tl_off[I.n_freq];
        } else if (I.root_kind == 1) {
            // words counted: row i's cover words against every later row;
            // bytes: each row's non-zero words (word + mask) and the
            // transposed arena read once
            uint64_t pw = 0, nzt = 0;
            for (uint32_t r = 0; r < I.n_freq; r++) {
                pw += (uint64_t)I.nz_cnt[r] * (I.n_freq - 1 - r);
                nzt += I.nz_cnt[r];
            }
            I.st.root_pair_words = pw;
            I.st.bytes_algorithmic = 8 * nzt + (uint64_t)I.n_freq * I.W * 4;
        } else {
            I.st.root_pair_words = all * I.W;
            I.st.bytes_algorithmic = (uint64_t)I.n_freq * I.W * 4;
        }
        I.st.pair_words = I.st.root_pair_words;
    }
    HIPCHK(stream_wait(s));
    tr.mark("  (pairs copied)");
    parallel_for(n_inst, host_threads((uint64_t)n_inst << 14), [&](uint64_t q) {
        Inst &I = insts[q];
        I.st.root_kernel_ns = (uint64_t)(root_ms * 1e6);
        I.st.kernel_ns = I.st.root_kernel_ns;
        // straight from the page-locked copy of the pairs
        if (I.n_pairs) build_level2(I, by_id, h_pairs_of((uint32_t)q));
        else I.l2_off.assign(I.n_freq + 1, 0);
    });

    tr.mark("bitmaps + root pairs");
    // ---------------- a4: class-size estimate, Partition, LPT order
    uint32_t max_chunks = 0;
    for (const Inst &I : insts) max_chunks = std::max(max_chunks, I.Wp / 4);
    const uint32_t variant = opts.tile_words ? tile_variant(opts.tile_words) : dfs_variant(max_chunks);
    uint32_t n_workers = opts.workers ? opts.workers : dfs_resident_workers(ctx->n_cu, variant);
    n_workers = std::max<uint32_t>(4, (n_workers + 3) / 4 * 4);
    std::vector<Task> tasks;
    uint64_t est_out_words = 0;
    bool deep_work = false;  // some instance has much work below its root class
    if (deep) {
        const auto t_plan = clk::now();
        std::vector<PlanInput> pin(n_inst);
        for (uint32_t q = 0; q < n_inst; q++) {
            Inst &I = insts[q];
            pin[q].db = I.db;
            pin[q].minsup = I.minsup;
            pin[q].n_freq = I.n_freq;
            pin[q].W = I.W;
            pin[q].item_of_rank = &I.item_of_rank;
            pin[q].rank_of_item = &I.rank_of_item;
            pin[q].l2_off = &I.l2_off;
            pin[q].l2_atom = &I.l2_atom;
            pin[q].supp_of_rank = &I.supp_of_rank;
            pin[q].Wp = I.Wp;
            pin[q].project = !(opts.flags & FIM_FLAG_NO_PROJECT);
            // The sample-based estimate balances the work below the root
            // class.  Its first level holds sum f_i (f_i - 1) / 2 candidate
            // pairs (f_i atoms of first-level class i), known exactly now;
            // when that is under 1/20 of the root class's pairs there is
            // nothing worth balancing and no sample is drawn.
            uint64_t below = 0;
            for (uint32_t i = 0; i < I.n_freq; i++) {
                const uint64_t f = I.l2_off[i + 1] - I.l2_off[i];
                below += f * (f ? f - 1 : 0) / 2;
            }
            const uint64_t root = (uint64_t)I.n_freq * (I.n_freq ? I.n_freq - 1 : 0) / 2;
            // The sample is searched to itemsets of kSampleMaxLen items, one
            // task per second-level class; its cost is then a few times the
            // time of a sample-sized search, and it pays where the database
            // is much longer than the sample (measured: dense-200k = 43 |D~|
            // 54.8 ms with it against 62.8 ms without; dense-50k = 11 |D~|
            // 12.1 ms with it against 11.1 ms without).  It is drawn for at
            // least 16 |D~| transactions, and only for a launch of one
            // instance: in a batch the other instances' classes fill the
            // waves that one instance's imbalance leaves idle (measured: 256
            // basket instances of log-uniform sizes, 113 ms with samples
            // drawn against 75 ms without).
            const uint64_t want_tx = opts.sample_tx ? opts.sample_tx : default_sample_tx(0.02, 0.05);
            pin[q].estimate = (opts.flags & FIM_FLAG_ALWAYS_ESTIMATE) ||
                              (20 * below >= root && n_inst == 1 && I.db->n_tx >= 16 * want_tx);
            deep_work = deep_work || 20 * below >= root;
        }
        fim_status ps = FIM_OK;
        if (opts.flags & (FIM_FLAG_RESERVOIR | FIM_FLAG_NO_ESTIMATE)) {
            ps = plan_tasks(ctx, pin, opts, n_workers, tasks, nullptr, &est_out_words);
        } else {
            // l2 arrays on the device for the sample's persistent run (only
            // the instances that draw a sample; kept for the main run)
            bool any_estimate = false;
            for (uint32_t q = 0; q < n_inst; q++) {
                Inst &I = insts[q];
                if (!pin[q].estimate || I.l2_atom.empty()) continue;
                any_estimate = true;
                ENSURE(I.d_l2_off, ctx, I.l2_off.size() * 4);
                ENSURE(I.d_l2_atom, ctx, I.l2_atom.size() * 4);
                ENSURE(I.d_l2_supp, ctx, I.l2_supp.size() * 4);
                HIPCHK(h2d(ctx, I.d_l2_off.as<void>(), I.l2_off.data(), I.l2_off.size() * 4, s));
                HIPCHK(h2d(ctx, I.d_l2_atom.as<void>(), I.l2_atom.data(), I.l2_atom.size() * 4, s));
                HIPCHK(h2d(ctx, I.d_l2_supp.as<void>(), I.l2_supp.data(), I.l2_supp.size() * 4, s));
                I.l2_on_device = true;
            }
            // no sample drawn: every instance planned by the proxy
            std::vector<std::vector<double>> row_w(n_inst);
            uint64_t sample_words = 0;
            if (any_estimate) ps = count_estimate(ctx, s, tr, insts, pin, opts, row_w, sample_words);
            if (ps != FIM_OK) return ps;
            // the sample has about as many frequent itemsets as the database
            // at the same relative support: room for twice its records
            est_out_words = 2 * sample_words;
            ps = plan_tasks(ctx, pin, opts, n_workers, tasks, nullptr, nullptr, nullptr, &row_w);
        }
        if (ps != FIM_OK) return ps;
        const uint64_t plan_ns = ns_since(t_plan);
        for (auto &I : insts) I.st.estimate_ns = plan_ns;
    }
    for (uint32_t q = 0; q < n_inst; q++) {
        Inst &I = insts[q];
        for (uint32_t i = 0; i < I.n_freq; i++) {
            const uint32_t f = I.l2_off[i + 1] - I.l2_off[i];
            if (f >= 2) I.first_class_rows += f;
        }
    }

    // With little work below the root class (small classes, no estimate
    // wanted) a launch with every resident wave mostly makes the waves
    // contend for the shared counters and caches: about one wave per eight
    // tasks is faster (measured on sparse-200k: 0.26 ms with 256 waves,
    // 0.48 ms with 2048).
    if (!opts.workers && !deep_work && !tasks.empty())
        n_workers = std::min<uint32_t>(n_workers, std::max<uint32_t>(256, (uint32_t)(tasks.size() / 8 + 3) / 4 * 4));
    tr.mark("estimate + plan");
    // ---------------- a5-a8: one persistent launch over every task
    DevBuf d_out(ctx);
    struct Span {
        const uint32_t *p = nullptr;
        size_t n = 0;
        uint32_t operator[](size_t i) const { return p[i]; }
        size_t size() const { return n; }
        bool empty() const { return n == 0; }
    } out_host;
    std::vector<InstCounters> ictr(n_inst);
    DfsCounters ctr{};
    float dfs_ms = 0.f;
    bool truncated = false;
    // Key mode: the persistent kernel writes fixed key records that the GPU
    // sorts into canonical order (fim_order.hip).  Item codes of instance q
    // take bits_of[q] bits (ids 0 .. n_item_ids - 1 as 1 .. n_item_ids).
    const bool key_mode = !(opts.flags & (kFlagInternalSample | kFlagInternalRecords)) &&
                          deep && !tasks.empty();
    std::vector<uint32_t> bits_of(n_inst, 1);
    for (uint32_t q = 0; q < n_inst; q++)
        while ((uint64_t)insts[q].db->n_item_ids >> bits_of[q]) bits_of[q]++;
    bool keys_done = false;
    std::vector<PrefixSrc> key_prefix;  // sources of the 1- and 2-itemsets' records
    // the packed second-level arrays (below) live until the call has waited
    // for its stream
    DevBuf d_l2_all(ctx);
    std::unique_ptr<PinnedBlock> h_l2;
    if (deep && !tasks.empty()) {
        std::vector<InstDesc> desc(n_inst);
        uint64_t frame0 = 0;
        // second-level arrays (l2_off, l2_atom, l2_supp) of the instances not
        // on the device yet, packed into one page-locked block, one copy
        std::vector<uint64_t> l2_at(n_inst, ~0ull);
        uint64_t l2_words = 0;
        for (uint32_t q = 0; q < n_inst; q++) {
            const Inst &I = insts[q];
            if (I.l2_atom.empty() || I.l2_on_device) continue;
            l2_at[q] = l2_words;
            l2_words += I.l2_off.size() + 2 * I.l2_atom.size();
        }
        if (l2_words) {
            ENSURE(d_l2_all, ctx, l2_words * 4);
            h_l2.reset(new PinnedBlock(l2_words * 4));
            uint32_t *h = h_l2->as<uint32_t>();
            parallel_for(n_inst, host_threads(l2_words), [&](uint64_t q) {
                if (l2_at[q] == ~0ull) return;
                const Inst &I = insts[q];
                uint32_t *d = h + l2_at[q];
                memcpy(d, I.l2_off.data(), I.l2_off.size() * 4);
                memcpy(d + I.l2_off.size(), I.l2_atom.data(), I.l2_atom.size() * 4);
                memcpy(d + I.l2_off.size() + I.l2_atom.size(), I.l2_supp.data(), I.l2_supp.size() * 4);
            });
            HIPCHK(hipMemcpyAsync(d_l2_all.as<void>(), h, l2_words * 4, hipMemcpyHostToDevice, s));
        }
        for (uint32_t q = 0; q < n_inst; q++) {
            Inst &I = insts[q];
            InstDesc &D = desc[q];
            D.rows = I.d_rows.as<uint32_t>();
            D.item_of_rank = I.p_item_of_rank;
            if (l2_at[q] != ~0ull) {
                const uint32_t *b = d_l2_all.as<uint32_t>() + l2_at[q];
                D.l2_off = b;
                D.l2_atom = b + I.l2_off.size();
                D.l2_supp = b + I.l2_off.size() + I.l2_atom.size();
            } else {
                D.l2_off = I.d_l2_off.as<uint32_t>();
                D.l2_atom = I.d_l2_atom.as<uint32_t>();
                D.l2_supp = I.d_l2_supp.as<uint32_t>();
            }
            D.Wp = I.Wp;
            D.n_freq = I.n_freq;
            D.minsup = I.minsup;
            D.max_len = opts.max_len;
            D.order_by_id = by_id ? 1u : 0u;
            D.project = (opts.flags & FIM_FLAG_NO_PROJECT) ? 0u : 1u;
            const bool lists = D.project && I.lists_built;
            D.tl = lists ? I.d_tl.as<uint32_t>() : nullptr;
            D.tl_off = lists ? I.p_tl_off : nullptr;
            // A sample drawn with replacement at a small scaled support can
            // make every subset of a repeatedly drawn long transaction
            // frequent; its search is abandoned past a fixed budget (the
            // instance then has no estimate).  A real run stops early once
            // it is certain to exceed max_itemsets.
            D.rec_budget = sample_run ? kSampleRecordBudget : opts.max_itemsets;
            D.key_bits = key_mode ? bits_of[q] : 0u;
        }
        for (const Task &T : tasks) {
            const Inst &I = insts[T.inst];
            const uint64_t k = I.l2_off[T.node + 1] - I.l2_off[T.node] - T.r0;
            // the width the piece's rows will have: projected on the item's
            // cover when that is at most a quarter of the row
            const uint32_t s1 = I.supp_of_rank[T.node];
            const uint64_t wq = std::max<uint64_t>(kRowAlign, ((s1 + 31) / 32 + kRowAlign - 1) / kRowAlign * kRowAlign);
            const bool proj = !(opts.flags & FIM_FLAG_NO_PROJECT) && 4 * wq <= I.Wp;
            frame0 = std::max<uint64_t>(frame0, k * (proj ? wq : I.Wp) + 3 * k);
        }
        DfsLaunch L;
        L.frame0 = frame0;
        L.variant = variant;
        L.n_workers = n_workers;
        L.claim = opts.classes_per_wg ? opts.classes_per_wg : 1;
        // Longest back-off of an idle wave.  Idle waves poll counters the
        // busy waves update; with much work below the root, polling often
        // slows those updates more than it speeds up hand-overs, while a
        // short run mostly waits for its last sleepers to wake.
        L.nap_max = deep_work ? 64 : 16;
        L.cap_output = (opts.flags & kFlagInternalSample) != 0;
        L.stop_is_error = !L.cap_output;
        // a generous arena (kept by the context's block cache between calls):
        // an overflow costs a second run of the whole launch
        L.out_cap = L.cap_output ? (1ull << 24) : std::max<uint64_t>(1ull << 26, est_out_words);
        if (ctx->arena)  // a fixed device block: start small, the overflow check grows it
            L.out_cap = std::max<uint64_t>(1ull << 18, std::min<uint64_t>(est_out_words, ctx->plan_bytes() / 64));
        if (key_mode) {
            // the 1- and 2-itemsets' records come first in the arena,
            // written on the device from the ranks and the root pairs
            uint64_t at = 0;
            for (uint32_t q = 0; q < n_inst; q++) {
                const Inst &I = insts[q];
                const uint64_t np = opts.max_len != 1 ? I.n_pairs : 0;
                if (I.n_freq + np == 0) continue;
                key_prefix.push_back(PrefixSrc{I.p_item_of_rank, I.p_counts,
                                               np ? I.d_pairs.as<uint32_t>() : nullptr, I.n_freq,
                                               bits_of[q], q, 0u, np, at});
                at += I.n_freq + np;
                L.prefix_max = std::max<uint64_t>(L.prefix_max, I.n_freq + np);
            }
            L.prefix = &key_prefix;
            L.prefix_rec = at;
            L.out_cap = std::max<uint64_t>(L.out_cap, 16 * at);
        }
        DevBuf d_act(ctx);  // a class profile: the run's candidate pairs per class
        if (g_profile && n_inst == 1 && !sample_run) {
            const uint64_t nr = std::max<uint64_t>(insts[0].l2_atom.size(), 1);
            ENSURE(d_act, ctx, nr * 8);
            HIPCHK(launch_fill_u32(d_act.as<uint32_t>(), nr * 2, 0u, s));
            desc[0].row_cand = d_act.as<unsigned long long>();
        }
        fim_status ls = run_persistent(ctx, s, tr, desc, tasks, d_out, L);
        if (ls == FIM_OK && g_profile && n_inst == 1 && !sample_run) {
            const Inst &I0 = insts[0];
            g_profile->act_cand.assign(I0.l2_atom.size(), 0);
            if (!I0.l2_atom.empty())
                HIPCHK(hipMemcpy(g_profile->act_cand.data(), d_act.as<void>(), I0.l2_atom.size() * 8,
                                 hipMemcpyDeviceToHost));
            g_profile->n_atoms.assign(I0.n_freq, 0);
            for (uint32_t i = 0; i < I0.n_freq; i++) g_profile->n_atoms[i] = I0.l2_off[i + 1] - I0.l2_off[i];
        }
        if (ls != FIM_OK) return ls;
        if (key_mode && (L.ctr.flags & kFlagKeyOverflow)) {
            // an itemset longer than a key holds: the same call with records
            fim_options ro = opts_in;
            ro.flags |= kFlagInternalRecords;
            return mine_many(ctx, reqs, ro, results);
        }
        ctr = L.ctr;
        ictr = L.ictr;
        dfs_ms = L.ms;
        for (auto &I : insts) {
            I.st.dfs_busy_max_ns = L.busy_max_ns;
            I.st.dfs_busy_mean_ns = L.busy_mean_ns;
        }
        truncated = L.truncated;
        const uint64_t out_cap = L.out_cap;
        for (auto &I : insts) I.st.retries += L.retries;
        out_host.n = key_mode ? 0 : std::min<uint64_t>(ctr.out_used.v, out_cap);
        if (out_host.n) {
            uint32_t *st = ctx->stage(out_host.n);
            if (!st) return set_error(FIM_E_OOM_HOST, "pinned staging buffer");
            out_host.p = st;
            HIPCHK(hipMemcpyAsync(st, d_out.as<void>(), out_host.n * 4, hipMemcpyDeviceToHost, s));
        }
        HIPCHK(stream_wait(s));
    }

    tr.mark("persistent dfs + copy");
    // ---------------- a9: results in canonical order
    std::vector<U32Vec> r_items(n_inst), r_supp(n_inst);
    std::vector<U64Vec> r_off(n_inst);
    // several instances in key mode: items and supports stay in the sorted
    // output, shared by the instances' results (r_at: each one's start)
    std::shared_ptr<SharedArrays> shared;
    std::vector<std::pair<uint64_t, uint64_t>> r_at(n_inst, {0, 0});
    std::vector<uint64_t> r_n(n_inst, 0);  // itemsets of each instance
    if (key_mode) {
        std::vector<uint64_t> first;
        U64Vec all_off;
        U32Vec all_items, all_supp;
        fim_status os = gpu_order(ctx, s, d_out.as<uint32_t>(), ctr.out_used.v / 8, bits_of, first,
                                  all_off, all_items, all_supp);
        if (os != FIM_OK) return os;
        const uint64_t n_all = all_supp.size();
        // instance q's itemsets are the sorted positions [first[q], next first)
        std::vector<uint64_t> lo(n_inst, n_all), hi(n_inst, n_all);
        uint64_t nxt = n_all;
        for (uint32_t q = n_inst; q-- > 0;) {
            if (first[q] != ~0ull) {
                lo[q] = first[q];
                hi[q] = nxt;
                nxt = first[q];
            }
        }
        if (n_inst == 1 && lo[0] == 0 && hi[0] == n_all) {
            // one instance: its result is the whole sorted output, moved as is
            r_off[0].swap(all_off);
            r_items[0].swap(all_items);
            r_supp[0].swap(all_supp);
        } else {
            shared = std::make_shared<SharedArrays>();
            shared->items.swap(all_items);
            shared->supp.swap(all_supp);
            parallel_for(n_inst, host_threads(n_all), [&](uint64_t q) {
                const uint64_t a = lo[q], b = hi[q];
                r_off[q].resize(b - a + 1);
                const uint64_t base = all_off[a];
                for (uint64_t x = a; x <= b; x++) r_off[q][x - a] = all_off[x] - base;
                r_at[q] = {base, a};
            });
        }
        keys_done = true;
    }
    for (uint32_t q = 0; q < n_inst; q++) {
        Inst &I = insts[q];
        if (keys_done) {
            I.st.candidates += ictr[q].candidates;
            I.st.pair_words += ictr[q].pair_words;
            I.st.dfs_bytes_algorithmic = 8 * ictr[q].row_words;
            I.st.bytes_algorithmic += I.st.dfs_bytes_algorithmic;
            I.st.dfs_kernel_ns = (uint64_t)(dfs_ms * 1e6);
            I.st.kernel_ns += I.st.dfs_kernel_ns;
            I.st.n_tasks = 0;
            continue;
        }
        r_off[q].push_back(0);
        for (uint32_t r = 0; r < I.n_freq; r++) {
            r_items[q].push_back(I.item_of_rank[r]);
            r_off[q].push_back(r_items[q].size());
            r_supp[q].push_back(I.supp_of_rank[r]);
        }
        if (opts.max_len != 1 && I.n_pairs)  // in class order: deterministic
            for (uint32_t i = 0; i < I.n_freq; i++)
                for (uint32_t k = I.l2_off[i]; k < I.l2_off[i + 1]; k++) {
                    r_items[q].push_back(I.item_of_rank[i]);
                    r_items[q].push_back(I.item_of_rank[I.l2_atom[k]]);
                    r_off[q].push_back(r_items[q].size());
                    r_supp[q].push_back(I.l2_supp[k]);
                }
        I.st.candidates += ictr[q].candidates;
        I.st.pair_words += ictr[q].pair_words;
        // every sibling row (of a first class or a child class, full width
        // or projected) written once and read once
        I.st.dfs_bytes_algorithmic = 8 * ictr[q].row_words;
        I.st.bytes_algorithmic += I.st.dfs_bytes_algorithmic;
        I.st.dfs_kernel_ns = (uint64_t)(dfs_ms * 1e6);
        I.st.kernel_ns += I.st.dfs_kernel_ns;
        I.st.n_tasks = 0;
    }
    for (const Task &T : tasks) insts[T.inst].st.n_tasks++;
    if (!keys_done) {
        // chunks of the output arena, put back in (task, chunk number) order
        struct Chunk {
            uint32_t task, seq, inst;
            uint64_t off, used;
        };
        std::vector<Chunk> chunks;
        const uint64_t limit = out_host.size();
        for (uint64_t p = 0; p + kChunkHeader <= limit;) {
            const uint32_t size = out_host[p];
            if (size < kChunkHeader || p + size > limit) break;
            const uint32_t used = out_host[p + 3];
            if (used >= kChunkHeader && used <= size && out_host[p + 4] < n_inst)
                chunks.push_back({out_host[p + 1], out_host[p + 2], out_host[p + 4], p, used});
            p += size;
        }
        std::sort(chunks.begin(), chunks.end(), [](const Chunk &a, const Chunk &b) {
            return a.task != b.task ? a.task < b.task : a.seq < b.seq;
        });
        // records and items of every chunk, then each chunk fills its own
        // slice of the preallocated result arrays
        const uint64_t nch = chunks.size();
        std::vector<uint64_t> c_sets(nch, 0), c_items(nch, 0);
        const uint32_t n_thr = host_threads(out_host.size() / 8);
        parallel_for(nch, n_thr, [&](uint64_t k) {
            const Chunk &c = chunks[k];
            for (uint64_t p = c.off + kChunkHeader; p + kRecHeader <= c.off + c.used;) {
                const uint32_t len = out_host[p];
                if (len == 0 || p + kRecHeader + len > c.off + c.used) break;
                c_sets[k]++;
                c_items[k] += len;
                p += kRecHeader + len;
            }
        });
        std::vector<uint64_t> set_at(nch), item_at(nch);
        {
            std::vector<uint64_t> ns(n_inst), ni(n_inst);
            for (uint32_t q = 0; q < n_inst; q++) {
                ns[q] = r_supp[q].size();
                ni[q] = r_items[q].size();
            }
            for (uint64_t k = 0; k < nch; k++) {
                const uint32_t q = chunks[k].inst;
                set_at[k] = ns[q];
                item_at[k] = ni[q];
                ns[q] += c_sets[k];
                ni[q] += c_items[k];
            }
            for (uint32_t q = 0; q < n_inst && !sample_run; q++) {
                r_items[q].resize(ni[q]);
                r_supp[q].resize(ns[q]);
                r_off[q].resize(ns[q] + 1);
            }
        }
        if (sample_run) {
            // a sample run returns only the itemsets the reservoir keeps
            // (Simple-Reservoir-Sampling over the instance's stream: its
            // 1-itemsets, its 2-itemsets, then the records in chunk order)
            const uint32_t n_fi = opts.sample_fi ? opts.sample_fi
                                                 : default_sample_fi(0.001, 0.0005, 0.05);
            std::vector<std::vector<uint64_t>> chunks_of(n_inst);
            for (uint64_t k = 0; k < nch; k++) chunks_of[chunks[k].inst].push_back(k);
            for (uint32_t q = 0; q < n_inst; q++) {
                const Inst &I = insts[q];
                const uint64_t head = r_supp[q].size();
                uint64_t L = head;
                for (uint64_t k : chunks_of[q]) L += c_sets[k];
                std::vector<uint64_t> keep = reservoir_indices(L, n_fi, opts.seed + 7 * q + 1);
                std::sort(keep.begin(), keep.end());
                U32Vec ki, ks;
                U64Vec ko{0};
                size_t j = 0;
                for (; j < keep.size() && keep[j] < head; j++) {
                    const uint64_t i = keep[j];
                    ki.insert(ki.end(), r_items[q].begin() + r_off[q][i],
                              r_items[q].begin() + r_off[q][i + 1]);
                    ko.push_back(ki.size());
                    ks.push_back(r_supp[q][i]);
                }
                // kept records of every chunk, found in parallel, joined in order
                const std::vector<uint64_t> &cq = chunks_of[q];
                std::vector<uint64_t> cpos(cq.size() + 1, head);
                for (size_t x = 0; x < cq.size(); x++) cpos[x + 1] = cpos[x] + c_sets[cq[x]];
                std::vector<U32Vec> pi(cq.size()), ps(cq.size());
                std::vector<std::vector<uint32_t>> pl(cq.size());
                parallel_for(cq.size(), n_thr, [&](uint64_t x) {
                    auto lo = std::lower_bound(keep.begin() + j, keep.end(), cpos[x]);
                    auto hi = std::lower_bound(lo, keep.end(), cpos[x + 1]);
                    if (lo == hi) return;
                    const Chunk &c = chunks[cq[x]];
                    uint64_t pos = cpos[x];
                    for (uint64_t p = c.off + kChunkHeader; p + kRecHeader <= c.off + c.used && lo != hi;) {
                        const uint32_t len = out_host[p];
                        if (len == 0 || p + kRecHeader + len > c.off + c.used) break;
                        if (*lo == pos) {
                            for (uint32_t y = 0; y < len; y++)
                                pi[x].push_back(I.item_of_rank[out_host[p + 2 + y]]);
                            pl[x].push_back(len);
                            ps[x].push_back(out_host[p + 1]);
                            ++lo;
                        }
                        pos++;
                        p += kRecHeader + len;
                    }
                });
                for (size_t x = 0; x < cq.size(); x++) {
                    uint64_t a = 0;
                    for (size_t y = 0; y < pl[x].size(); y++) {
                        ki.insert(ki.end(), pi[x].begin() + a, pi[x].begin() + a + pl[x][y]);
                        a += pl[x][y];
                        ko.push_back(ki.size());
                        ks.push_back(ps[x][y]);
                    }
                }
                r_items[q].swap(ki);
                r_off[q].swap(ko);
                r_supp[q].swap(ks);
                insts[q].st.n_itemsets = L;
            }
        } else {
        parallel_for(nch, n_thr, [&](uint64_t k) {
            const Chunk &c = chunks[k];
            const uint32_t q = c.inst;
            const Inst &I = insts[q];
            uint32_t *ri = r_items[q].data();
            uint64_t *ro = r_off[q].data();
            uint32_t *rs = r_supp[q].data();
            uint64_t si = set_at[k], ii = item_at[k];
            for (uint64_t p = c.off + kChunkHeader; p + kRecHeader <= c.off + c.used;) {
                const uint32_t len = out_host[p];
                if (len == 0 || p + kRecHeader + len > c.off + c.used) break;
                for (uint32_t x = 0; x < len; x++) ri[ii++] = I.item_of_rank[out_host[p + 2 + x]];
                rs[si] = out_host[p + 1];
                ro[++si] = ii;
                p += kRecHeader + len;
            }
        });
        }
    }
    for (uint32_t q = 0; q < n_inst; q++) {
        r_n[q] = r_off[q].empty() ? 0 : r_off[q].size() - 1;
        if (opts.max_itemsets && r_n[q] > opts.max_itemsets && !truncated)
            return set_error(FIM_E_OUTPUT_LIMIT,
                             "instance " + std::to_string(q) + " has " +
                                 std::to_string(r_n[q]) + " frequent itemsets > max_itemsets");
    }
    // canonical order: large instances one after another with all host
    // threads, the others side by side with one thread each (internal
    // sample runs keep the deterministic task order: the reservoir does not
    // need the canonical one)
    if (!(opts.flags & kFlagInternalSample) && !keys_done) {
        uint64_t total_sets = 0;
        for (uint32_t q = 0; q < n_inst; q++) total_sets += r_supp[q].size();
        std::vector<uint32_t> small;
        for (uint32_t q = 0; q < n_inst; q++) {
            if (n_inst == 1 || r_supp[q].size() * 16 > total_sets)
                canonicalize(r_items[q], r_off[q], r_supp[q]);
            else
                small.push_back(q);
        }
        parallel_for(small.size(), host_threads(total_sets), [&](uint64_t k) {
            const uint32_t q = small[k];
            canonicalize(r_items[q], r_off[q], r_supp[q], 1);
        });
    }
    results.assign(n_inst, nullptr);
    for (uint32_t q = 0; q < n_inst; q++) {
        fim_result *R = new (std::nothrow) fim_result();
        if (!R) {
            for (auto *x : results) delete x;
            results.clear();
            return set_error(FIM_E_OOM_HOST, "result");
        }
        R->items.swap(r_items[q]);
        R->off.swap(r_off[q]);
        R->supp.swap(r_supp[q]);
        if (shared) {
            R->shared = shared;
            R->items_at = r_at[q].first;
            R->supp_at = r_at[q].second;
        }
        R->stats = insts[q].st;
        if (!sample_run) R->stats.n_itemsets = R->n_itemsets();
        R->truncated = truncated || (sample_run && ictr[q].stop);
        results[q] = R;
    }
    tr.mark("decode + canonical order");
    const uint64_t total = ns_since(t_start);
    for (auto *R : results) R->stats.total_ns = total;
    return FIM_OK;
}

}  // namespace fim

// ====================================================================== mining ABI

extern "C" fim_status fim_mine(fim_ctx *ctx, const fim_db *db, uint32_t minsup_abs,
                               const fim_options *opts, fim_result **out) {
    if (!out) return fim::set_error(FIM_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx || !db) return fim::set_error(FIM_E_INVALID_ARG, "ctx or db is NULL");
    if (db->ctx != ctx && db->ctx->device != ctx->device)
        return fim::set_error(FIM_E_INVALID_ARG, "db belongs to another device");
    if (minsup_abs == 0) return fim::set_error(FIM_E_INVALID_ARG, "minsup_abs must be >= 1");
    std::vector<fim::MineRequest> reqs{{db, minsup_abs}};
    std::vector<fim_result *> res;
    fim_status st = fim::mine_many(ctx, reqs, fim::resolve_options(opts), res);
    if (st != FIM_OK) return st;
    *out = res[0];
    return FIM_OK;
}

extern "C" fim_status fim_mine_batch(fim_ctx *ctx, uint32_t n, const fim_db *const *dbs,
                                     const uint32_t *minsups, const fim_options *opts,
                                     fim_result **outs) {
    if (!ctx || (n && (!dbs || !minsups || !outs)))
        return fim::set_error(FIM_E_INVALID_ARG, "NULL argument");
    std::vector<fim::MineRequest> reqs(n);
    for (uint32_t q = 0; q < n; q++) {
        outs[q] = nullptr;
        if (!dbs[q] || minsups[q] == 0)
            return fim::set_error(FIM_E_INVALID_ARG, "instance " + std::to_string(q) +
                                                         ": NULL db or minimum support 0");
        if (dbs[q]->ctx->device != ctx->device)
            return fim::set_error(FIM_E_INVALID_ARG, "db belongs to another device");
        reqs[q] = {dbs[q], minsups[q]};
    }
    if (n == 0) return FIM_OK;
    std::vector<fim_result *> res;
    fim_status st = fim::mine_many(ctx, reqs, fim::resolve_options(opts), res);
    if (st != FIM_OK) return st;
    for (uint32_t q = 0; q < n; q++) outs[q] = res[q];
    return FIM_OK;
}

extern "C" fim_status fim_autotune(fim_ctx *ctx, uint32_t n, const fim_db *const *dbs,
                                   const uint32_t *minsups, const fim_options *base, uint32_t reps,
                                   fim_options *out, uint64_t *best_ns) {
    if (!out) return fim::set_error(FIM_E_INVALID_ARG, "out is NULL");
    const fim_options b = fim::resolve_options(base);
    *out = b;
    if (reps == 0) reps = 2;
    std::vector<fim_result *> res(n);
    // least depth-first kernel time of `reps` runs with tile t and claim c
    auto trial = [&](uint32_t t, uint32_t c, uint64_t &ns) -> fim_status {
        fim_options o = b;
        o.tile_words = t;
        o.classes_per_wg = c;
        ns = ~0ull;
        for (uint32_t k = 0; k < reps; k++) {
            fim_status st = fim_mine_batch(ctx, n, dbs, minsups, &o, res.data());
            if (st != FIM_OK) return st;
            fim_stats s0{};
            if (n) (void)fim_result_stats(res[0], &s0);
            ns = std::min<uint64_t>(ns, s0.dfs_kernel_ns);
            for (fim_result *r : res) fim_result_destroy(r);
        }
        return FIM_OK;
    };
    uint32_t best_t = 0, best_c = 1;
    uint64_t best = ~0ull, ns = 0;
    for (uint32_t t : {256u, 512u, 1024u, 2048u}) {
        fim_status st = trial(t, 1, ns);
        if (st != FIM_OK) return st;
        if (ns < best) best = ns, best_t = t;
    }
    for (uint32_t c : {2u, 4u}) {
        fim_status st = trial(best_t, c, ns);
        if (st != FIM_OK) return st;
        if (ns < best) best = ns, best_c = c;
    }
    out->tile_words = best_t;
    out->classes_per_wg = best_c;
    if (best_ns) *best_ns = best;
    return FIM_OK;
}

extern "C" fim_status fim_class_profile(fim_ctx *ctx, const fim_db *db, uint32_t minsup_abs,
                                        const fim_options *opts, uint32_t *n_classes, uint32_t *n_atoms,
                                        uint32_t class_capacity, uint64_t *n_rows, double *est_fi,
                                        double *est_cand, uint64_t *act_cand, uint64_t row_capacity) {
    if (!ctx || !db || !n_classes || !n_rows || minsup_abs == 0)
        return fim::set_error(FIM_E_INVALID_ARG, "NULL argument or minimum support 0");
    fim::ClassProfile prof;
    fim::g_profile = &prof;
    fim_options o = opts ? *opts : fim_options{};
    o.flags = (o.flags | FIM_FLAG_ALWAYS_ESTIMATE) & ~(FIM_FLAG_NO_ESTIMATE | FIM_FLAG_RESERVOIR);
    std::vector<fim_result *> res;
    const fim_status st = fim::mine_many(ctx, {fim::MineRequest{db, minsup_abs}}, o, res);
    fim::g_profile = nullptr;
    for (fim_result *r : res) fim_result_destroy(r);
    if (st != FIM_OK) return st;
    *n_classes = (uint32_t)prof.n_atoms.size();
    *n_rows = prof.act_cand.size();
    if (prof.n_atoms.size() > class_capacity || prof.act_cand.size() > row_capacity)
        return fim::set_error(FIM_E_OUTPUT_LIMIT, "profile arrays too small");
    if (n_atoms) std::copy(prof.n_atoms.begin(), prof.n_atoms.end(), n_atoms);
    for (size_t k = 0; k < prof.act_cand.size(); k++) {
        if (est_fi) est_fi[k] = k < prof.est_fi.size() ? prof.est_fi[k] : 0.0;
        if (est_cand) est_cand[k] = k < prof.est_cand.size() ? prof.est_cand[k] : 0.0;
        if (act_cand) act_cand[k] = prof.act_cand[k];
    }
    return FIM_OK;
}
