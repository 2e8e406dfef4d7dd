// fim_mine_noalloc: the miner without device allocation.
//
// Every piece of device memory the call needs (bitmap arenas, per-wave
// stacks, the output arena, the ordering's sort buffers) is carved out of
// one block of FIM_NOALLOC_SCRATCH_BYTES that lives in the library's code
// object on every GPU it runs on (`scratch` below); no allocator and no
// page-locked host memory is used.  The host side only ever sees the
// block's per-device address, taken once per device with
// hipGetSymbolAddress: the array's name in host code is a host-side stand-in,
// not a device address.
#include <map>
#include <mutex>

#include "fim_host.h"

namespace {

static __device__ __align__(256) unsigned char scratch[FIM_NOALLOC_SCRATCH_BYTES];

// one call at a time in this process: they share each GPU's block
std::mutex g_mu;
std::map<int, char *> g_scratch;  // device -> that device's address of `scratch`

// The block's address on `device`, which must be the current device.
fim_status scratch_of(int device, char **out) {
    auto it = g_scratch.find(device);
    if (it != g_scratch.end()) {
        *out = it->second;
        return FIM_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        return fim::set_error(FIM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                                hipGetErrorString(e));
    g_scratch[device] = static_cast<char *>(p);
    *out = static_cast<char *>(p);
    return FIM_OK;
}

}  // namespace

extern "C" fim_status fim_mine_noalloc(fim_ctx *ctx, const fim_db *db, uint32_t minsup_abs,
                                       const fim_options *opts, uint64_t cap_itemsets,
                                       uint64_t cap_items, uint64_t *offsets, uint32_t *items,
                                       uint32_t *supports, uint64_t *n_itemsets,
                                       uint64_t *n_items_total) {
    if (!ctx || !db || !offsets || !n_itemsets || !n_items_total || minsup_abs == 0)
        return fim::set_error(FIM_E_INVALID_ARG, "NULL argument or minimum support 0");
    if (db->ctx && db->ctx->device != ctx->device)
        return fim::set_error(FIM_E_INVALID_ARG, "database of another device");
    if ((cap_items && !items) || (cap_itemsets && !supports))
        return fim::set_error(FIM_E_INVALID_ARG, "NULL result array with a non-zero capacity");
    *n_itemsets = 0;
    *n_items_total = 0;
    std::lock_guard<std::mutex> lk(g_mu);
    const hipError_t se = hipSetDevice(ctx->device);
    if (se != hipSuccess) return fim::set_error(FIM_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(se));
    char *base = nullptr;
    fim_status st = scratch_of(ctx->device, &base);
    if (st != FIM_OK) return st;
    // the context hands out pieces of the block for this call only
    struct Arena {
        fim_ctx *c;
        bool no_pinned;
        ~Arena() {
            c->arena = nullptr;
            c->arena_cap = c->arena_used = 0;
            c->last_piece_at = ~size_t(0);
            fim::g_no_pinned = no_pinned;
        }
    } arena{ctx, fim::g_no_pinned};
    ctx->arena = base;
    ctx->arena_cap = FIM_NOALLOC_SCRATCH_BYTES;
    ctx->arena_used = 0;
    fim::g_no_pinned = true;
    fim_options o = opts ? *opts : fim_options{};
    o.flags |= FIM_FLAG_NO_ESTIMATE;  // the estimate would mine a sample on a second context
    std::vector<fim_result *> res;
    st = fim::mine_many(ctx, {fim::MineRequest{db, minsup_abs}}, o, res);
    if (st != FIM_OK) {
        if (st == FIM_E_OOM_DEVICE)
            fim::set_error(st, std::string(fim_last_error()) + " (the work does not fit the " +
                                   std::to_string(FIM_NOALLOC_SCRATCH_BYTES >> 20) + " MiB scratch block)");
        return st;
    }
    std::unique_ptr<fim_result, void (*)(fim_result *)> r(res.at(0), fim_result_destroy);
    *n_itemsets = r->n_itemsets();
    *n_items_total = r->n_items();
    if (r->n_itemsets() > cap_itemsets || r->n_items() > cap_items)
        return fim::set_error(FIM_E_OUTPUT_LIMIT, "the result (" + std::to_string(r->n_itemsets()) +
                                                      " itemsets, " + std::to_string(r->n_items()) +
                                                      " items) does not fit the arrays");
    return fim_result_copy(r.get(), offsets, items, supports);
}
