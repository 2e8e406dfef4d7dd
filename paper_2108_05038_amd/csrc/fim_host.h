// Host-side internals of libfim.so (not part of the public ABI).
#pragma once

#include <stdint.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fim.h"
#include "fim_internal.h"
#include "fim_canon.h"

struct fim_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;  // created by the library when the caller gave none
    fim_allocator alloc{};
    bool user_alloc = false;
    int n_cu = 256;
    size_t total_mem = 0;
    size_t lds_per_block = 65536;  // largest LDS allocation of one workgroup
    std::string arch;

    // a second context on the same device with a stream of its own, for
    // work that overlaps the main stream (the estimate's sample)
    fim_ctx *aux = nullptr;
    fim_ctx *aux_ctx();

    // pinned host staging buffer for device-to-host copies of results
    uint32_t *pinned = nullptr;
    size_t pinned_words = 0;
    // page-locked staging of one run's host-to-device copies (fim::h2d):
    // bump-allocated during the run, emptied when the next run starts
    char *up = nullptr;
    size_t up_cap = 0, up_used = 0, up_need = 0;
    int up_depth = 0;
    // streams (default priority) that let the instances of a batched call
    // overlap their root-class work; created on first use
    std::vector<hipStream_t> side_streams;
    // timing events of the root-class kernels (two per instance), kept for
    // the next run: a batch of 256 instances spent 0.6 ms creating them
    std::vector<hipEvent_t> timing_events;
    // two events without timing that order a side stream's work within a run
    hipEvent_t sync_events[2] = {nullptr, nullptr};
    uint32_t *stage(size_t words);

    // Device blocks freed by the library are kept by size class for the
    // next call (a call then needs no allocator round trip); released on
    // fim_ctx_release_cached, on an allocation failure and at destruction.
    std::mutex cache_mu;  // databases may be created while a server mines
    std::map<size_t, std::vector<void *>> cache;
    std::unordered_map<void *, size_t> block_class;
    size_t cached_bytes = 0;
    void *raw_alloc(size_t bytes);
    void raw_free(void *p);
    void release_cached();

    void *dalloc(size_t bytes);
    void dfree(void *p);
    ~fim_ctx();

    // While `arena` is set, dalloc hands out pieces of this caller-owned
    // device block (a bump pointer; a free of the most recent piece takes it
    // back) and never calls the allocator; pinned staging is not used.
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0, last_piece_at = ~size_t(0);
    // device memory a run may plan with: a quarter of the device, or the
    // arena's free part
    size_t plan_bytes() const { return arena ? arena_cap - arena_used : total_mem / 4; }
    bool pinned_heap = false;  // `pinned` came from the ordinary heap
};

namespace fim {

// Device buffer released through the context's allocator.
class DevBuf {
   public:
    DevBuf() = default;
    explicit DevBuf(fim_ctx *ctx) : ctx_(ctx) {}
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            reset();
            ctx_ = o.ctx_;
            p_ = o.p_;
            bytes_ = o.bytes_;
            o.p_ = nullptr;
            o.bytes_ = 0;
        }
        return *this;
    }
    ~DevBuf() { reset(); }
    // (re)allocate at least `bytes` (contents are not kept); false on failure
    bool ensure(fim_ctx *ctx, size_t bytes);
    void reset();
    template <class T>
    T *as() const { return reinterpret_cast<T *>(p_); }
    size_t bytes() const { return bytes_; }

   private:
    fim_ctx *ctx_ = nullptr;
    void *p_ = nullptr;
    size_t bytes_ = 0;
};

// The context's side streams (created on first use).
hipError_t ctx_side_streams(fim_ctx *ctx, std::vector<hipStream_t> &out);
// At least n timing events in ctx->timing_events (created on first use,
// reused by later runs on the context).
hipError_t ctx_timing_events(fim_ctx *ctx, size_t n);

// Several host pieces copied to consecutive places of dst, each piece's
// place starting at the sum of the earlier pieces' sizes rounded up to 8
// bytes: one copy through the context's staging when it has room (else one
// plain copy per piece); src may be reused as soon as this returns.
struct H2DPiece {
    const void *src;
    size_t bytes;
};
hipError_t h2d_pieces(fim_ctx *ctx, void *dst, const H2DPiece *pieces, size_t n, hipStream_t s);

// Host-to-device copy of `bytes` from src to dst, queued on s through the
// context's page-locked staging (src may be reused as soon as this returns;
// the copy does not wait for the stream); a plain copy when the staging of
// this run is used up (the next run's staging is then larger).
hipError_t h2d(fim_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t s);

// Wait for the work queued on s: spins on the stream's status (a sleeping
// wait can wake up milliseconds late on a busy host) for up to 20 ms, then
// blocks.
hipError_t stream_wait(hipStream_t s);

// Marks one run on a context: the outermost run starts with an idle stream
// and an emptied (and if need be grown) staging area.
class StageRun {
   public:
    explicit StageRun(fim_ctx *ctx);
    ~StageRun();
    StageRun(const StageRun &) = delete;
    StageRun &operator=(const StageRun &) = delete;

   private:
    fim_ctx *ctx_;
};

// Thread-local error text and status helpers.
fim_status set_error(fim_status s, const std::string &msg);

}  // namespace fim

struct fim_db {
    fim_ctx *ctx = nullptr;
    uint64_t n_tx = 0, nnz = 0;
    uint32_t n_item_ids = 0;
    uint64_t pairs_in_tx = 0;      // sum over transactions of L (L - 1) / 2
    uint64_t max_tx_len = 0;       // longest transaction
    std::vector<uint64_t> h_off;   // canonical CSR (sorted, duplicate-free transactions)
    std::vector<uint32_t> h_items;
    fim::DevBuf d_off, d_items;
};

namespace fim {
// Items and supports of every instance of one batched call, in one pair of
// arrays that the instances' results share (each holds its own offsets).
struct SharedArrays {
    U32Vec items, supp;
};
}  // namespace fim

struct fim_result {
    fim::U64Vec off{0};
    fim::U32Vec items, supp;  // empty when the arrays are shared
    std::shared_ptr<const fim::SharedArrays> shared;
    uint64_t items_at = 0, supp_at = 0;  // this result's start in the shared arrays
    fim_stats stats{};
    bool truncated = false;  // internal sample runs only: output budget exceeded

    uint64_t n_itemsets() const { return off.size() - 1; }
    uint64_t n_items() const { return off.back(); }
    const uint32_t *items_data() const { return shared ? shared->items.data() + items_at : items.data(); }
    const uint32_t *supp_data() const { return shared ? shared->supp.data() + supp_at : supp.data(); }
};

namespace fim {

// Internal option flag: the run mines a database sample for the estimate;
// its output is capped at a fixed budget instead of growing, and an
// exceeded budget marks the results truncated instead of failing.
constexpr uint32_t kFlagInternalSample = 0x80000000u;

// Internal option flag: the persistent kernel reports variable-length
// records that the host puts in canonical order (used when an itemset does
// not fit a 128-bit key of its instance's item codes).
constexpr uint32_t kFlagInternalRecords = 0x40000000u;

// The canonical order of key records (see fim_order.hip): n 8-word records
// at d_rec; bits_of[q] the code width of instance q; first[q] receives the
// position of instance q's first itemset in the sorted result (~0 if none).
fim_status gpu_order(fim_ctx *ctx, hipStream_t s, const uint32_t *d_rec, uint64_t n,
                     const std::vector<uint32_t> &bits_of, std::vector<uint64_t> &first,
                     U64Vec &off, U32Vec &items, U32Vec &supp);

// Limits of an internal sample run: itemsets below the first level per
// instance, and words of the output arena of the whole run.
constexpr unsigned long long kSampleRecordBudget = 1ull << 21;
constexpr uint64_t kSampleOutCap = 1ull << 27;

// One mining instance inside a (possibly batched) run.
struct MineRequest {
    const fim_db *db;
    uint32_t minsup;
};

// Mine every request; results[i] receives the canonical result of request i.
// Used by fim_mine (one request), fim_mine_batch and the server.
fim_status mine_many(fim_ctx *ctx, const std::vector<MineRequest> &reqs, const fim_options &opts,
                     std::vector<fim_result *> &results);

// Resolved option values.
fim_options resolve_options(const fim_options *opts);

// Per second-level class figures of one run, gathered while a caller asks
// for them (fim_class_profile): the first-level classes' atom counts (rank
// order), and per second-level class (row r of first-level class c, rows of
// the classes in order) the sample's frequent itemsets of three or more
// items and its candidate pairs below that class, and the run's own
// candidate pairs below it.
struct ClassProfile {
    std::vector<uint32_t> n_atoms;
    std::vector<double> est_fi, est_cand;
    std::vector<uint64_t> act_cand;
};
extern thread_local ClassProfile *g_profile;

}  // namespace fim
