// Serving: a request loop on one GPU with continuous batching.
//
// Requests are queued by fim_server_submit (any thread).  The server runs
// several lanes, each a worker thread with a HIP stream of its own.  An idle
// lane admits waiting requests while a slot is free and the HBM footprint of
// their bitmaps fits what the other lanes leave of the budget, and mines
// them in one batched persistent launch.  Dense databases (more than a
// quarter of the item ids in an average transaction: deep searches with
// many frequent itemsets) are mined in batches of their own, so that the
// light requests behind them are not held up: an idle lane takes the oldest
// request if it is dense, alone, and otherwise the light requests in arrival
// order.  Requests that arrive while a batch runs are taken by the next idle
// lane, so their work overlaps the running batch on the device (and its
// host-side stages); a finished batch gives its slots and memory back at
// once.  Results are identical to fim_mine on the same database and minimum
// support.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "fim_host.h"

namespace {

struct Request {
    uint64_t ticket;
    const fim_db *db;
    uint32_t minsup;
    uint64_t footprint;
    bool dense;
};

struct Done {
    fim_status status;
    fim_result *result;
    std::string error;
};

struct Lane {
    fim_ctx *ctx = nullptr;
    bool own = false;
    std::thread th;
};

}  // namespace

struct fim_server {
    fim_ctx *ctx = nullptr;
    fim_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::unordered_map<uint64_t, Done> done;
    std::unordered_map<uint64_t, int> state;  // 0 queued, 1 running, 2 done
    std::unordered_map<uint64_t, bool> cancelled;
    std::deque<uint64_t> finished;  // tickets in completion order (fim_server_next)
    uint64_t next_ticket = 1;
    uint64_t active = 0, active_bytes = 0;  // over all lanes
    bool stop = false;
    fim_server_stats stats{};
    std::vector<Lane> lanes;
};

namespace {

// device bytes a request holds while resident: its level-1 bitmaps, item
// arrays and a share of the worker stacks and output arena
uint64_t footprint(const fim_db *db) {
    const uint64_t W = (db->n_tx + 31) / 32 + 4;
    const uint64_t rows = std::min<uint64_t>(db->n_item_ids, db->nnz);
    return rows * W * 4 + (uint64_t)db->n_item_ids * 16 + (64ull << 20);
}

// more than a quarter of the item ids in an average transaction
bool is_dense(const fim_db *db) {
    return db->n_tx && db->n_item_ids && 4 * db->nnz > (uint64_t)db->n_tx * db->n_item_ids;
}

// request r fits the free slots and memory (a request alone on an idle
// device is always admitted, whatever its size)
bool fits(const fim_server *s, const Request &r, uint64_t taken, uint64_t taken_bytes) {
    if (s->active + taken >= s->cfg.max_active) return false;
    const uint64_t busy = s->active + taken;
    return busy == 0 || s->active_bytes + taken_bytes + r.footprint <= s->cfg.hbm_budget_bytes;
}

// an idle lane has something to take
bool admissible(const fim_server *s) {
    if (s->queue.empty()) return false;
    if (s->queue.front().dense) return fits(s, s->queue.front(), 0, 0);
    for (const Request &r : s->queue)
        if (!r.dense) return fits(s, r, 0, 0);
    return false;
}

void worker_loop(fim_server *s, fim_ctx *ctx) {
    (void)hipSetDevice(ctx->device);
    // a share of the host for this lane's host-side stages
    fim::g_host_thread_cap = std::max<uint32_t>(2, 16 / std::max<uint32_t>(1, s->cfg.lanes));
    for (;;) {
        std::vector<Request> batch;
        uint64_t bytes = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return (s->stop && s->queue.empty()) || admissible(s); });
            if (s->queue.empty()) return;  // stopping
            if (s->queue.front().dense) {
                batch.push_back(s->queue.front());
                bytes = s->queue.front().footprint;
                s->queue.pop_front();
            } else {
                for (auto it = s->queue.begin(); it != s->queue.end();) {
                    if (it->dense) {
                        ++it;
                        continue;
                    }
                    if (!fits(s, *it, batch.size(), bytes)) break;
                    bytes += it->footprint;
                    batch.push_back(*it);
                    it = s->queue.erase(it);
                }
            }
            for (const Request &r : batch) s->state[r.ticket] = 1;
            s->active += batch.size();
            s->active_bytes += bytes;
            s->stats.peak_active = std::max<uint64_t>(s->stats.peak_active, s->active);
            s->stats.peak_bytes = std::max<uint64_t>(s->stats.peak_bytes, s->active_bytes);
        }
        std::vector<fim::MineRequest> reqs;
        for (const Request &r : batch) reqs.push_back({r.db, r.minsup});
        std::vector<fim_result *> res;
        fim_status st = fim::mine_many(ctx, reqs, s->cfg.opts, res);
        std::string err = st == FIM_OK ? "" : fim_last_error();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stats.steps++;
            s->active -= batch.size();
            s->active_bytes -= bytes;
            for (size_t k = 0; k < batch.size(); k++) {
                const uint64_t t = batch[k].ticket;
                fim_result *r = st == FIM_OK ? res[k] : nullptr;
                if (s->cancelled.count(t)) {
                    fim_result_destroy(r);
                    s->done[t] = Done{FIM_E_CANCELLED, nullptr, "cancelled"};
                } else {
                    s->done[t] = Done{st, r, err};
                }
                s->state[t] = 2;
                s->finished.push_back(t);
                s->stats.completed++;
            }
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();  // freed slots and memory may admit more
    }
}

}  // namespace

extern "C" fim_status fim_server_create(fim_ctx *ctx, const fim_server_config *cfg,
                                        fim_server **out) {
    if (!out || !ctx) return fim::set_error(FIM_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    fim_server *s = new (std::nothrow) fim_server();
    if (!s) return fim::set_error(FIM_E_OOM_HOST, "server");
    s->ctx = ctx;
    if (cfg) s->cfg = *cfg;
    // defaults measured on MI355X with the serving pool, closed loop: two
    // lanes of at most 16 requests 216 req/s, 64 requests 181 req/s, one
    // lane 192 req/s, three lanes far fewer (the one-request-per-call
    // miner: 133 req/s)
    if (s->cfg.max_active == 0) s->cfg.max_active = 16;
    if (s->cfg.max_queue == 0) s->cfg.max_queue = 1u << 16;
    if (s->cfg.lanes == 0) s->cfg.lanes = 2;
    if (s->cfg.lanes > 8) {
        delete s;
        return fim::set_error(FIM_E_INVALID_ARG, "at most 8 lanes");
    }
    if (s->cfg.hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        (void)hipSetDevice(ctx->device);
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = ctx->total_mem / 2;
        s->cfg.hbm_budget_bytes = fr / 4 * 3;
    }
    s->stats.lanes = s->cfg.lanes;
    // lane 0 mines on the caller's context; the others on contexts of their
    // own (same device and allocator, a stream each)
    s->lanes.resize(s->cfg.lanes);
    s->lanes[0].ctx = ctx;
    for (uint32_t l = 1; l < s->cfg.lanes; l++) {
        fim_ctx *c = nullptr;
        const fim_status st = fim_ctx_create(ctx->device, nullptr,
                                             ctx->user_alloc ? &ctx->alloc : nullptr, &c);
        if (st != FIM_OK) {
            for (uint32_t q = 1; q < l; q++) fim_ctx_destroy(s->lanes[q].ctx);
            delete s;
            return st;
        }
        s->lanes[l].ctx = c;
        s->lanes[l].own = true;
    }
    for (Lane &L : s->lanes) L.th = std::thread(worker_loop, s, L.ctx);
    *out = s;
    return FIM_OK;
}

extern "C" fim_status fim_server_submit(fim_server *s, const fim_db *db, uint32_t minsup_abs,
                                        uint64_t *ticket) {
    if (!s || !db || !ticket || minsup_abs == 0)
        return fim::set_error(FIM_E_INVALID_ARG, "NULL argument or minimum support 0");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->queue.size() >= s->cfg.max_queue) return fim::set_error(FIM_E_BUSY, "queue full");
    const uint64_t t = s->next_ticket++;
    s->queue.push_back(Request{t, db, minsup_abs, footprint(db), is_dense(db)});
    s->state[t] = 0;
    s->stats.submitted++;
    *ticket = t;
    s->cv_work.notify_one();
    return FIM_OK;
}

static fim_status take(fim_server *s, uint64_t ticket, fim_result **out, bool block) {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->state.find(ticket);
    if (it == s->state.end()) return fim::set_error(FIM_E_NOT_FOUND, "unknown ticket");
    if (block) s->cv_done.wait(lk, [&] { return s->state[ticket] == 2; });
    if (s->state[ticket] != 2) {
        *out = nullptr;
        return FIM_OK;
    }
    Done d = s->done[ticket];
    s->done.erase(ticket);
    s->state.erase(ticket);
    s->cancelled.erase(ticket);
    *out = d.result;
    if (d.status != FIM_OK) return fim::set_error(d.status, d.error);
    return FIM_OK;
}

extern "C" fim_status fim_server_poll(fim_server *s, uint64_t ticket, fim_result **out) {
    if (!s || !out) return fim::set_error(FIM_E_INVALID_ARG, "NULL argument");
    return take(s, ticket, out, false);
}

extern "C" fim_status fim_server_wait(fim_server *s, uint64_t ticket, fim_result **out) {
    if (!s || !out) return fim::set_error(FIM_E_INVALID_ARG, "NULL argument");
    return take(s, ticket, out, true);
}

extern "C" fim_status fim_server_next(fim_server *s, uint64_t timeout_us, uint64_t *ticket,
                                      fim_result **out) {
    if (!s || !ticket || !out) return fim::set_error(FIM_E_INVALID_ARG, "NULL argument");
    *ticket = 0;
    *out = nullptr;
    uint64_t t = 0;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto ready = [&] {
            // skip tickets already taken by poll / wait
            while (!s->finished.empty() && !s->state.count(s->finished.front()))
                s->finished.pop_front();
            return !s->finished.empty();
        };
        if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return FIM_OK;
        t = s->finished.front();
        s->finished.pop_front();
    }
    *ticket = t;
    return take(s, t, out, false);
}

extern "C" fim_status fim_server_cancel(fim_server *s, uint64_t ticket) {
    if (!s) return fim::set_error(FIM_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->state.find(ticket);
    if (it == s->state.end()) return fim::set_error(FIM_E_NOT_FOUND, "unknown ticket");
    if (it->second == 0) {  // still queued: drop it now
        for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
            if (q->ticket == ticket) {
                s->queue.erase(q);
                break;
            }
        s->done[ticket] = Done{FIM_E_CANCELLED, nullptr, "cancelled"};
        it->second = 2;
        s->finished.push_back(ticket);
    } else if (it->second == 1) {
        s->cancelled[ticket] = true;
    }
    s->stats.cancelled++;
    s->cv_done.notify_all();
    return FIM_OK;
}

extern "C" fim_status fim_server_stats_get(const fim_server *s, fim_server_stats *out) {
    if (!s || !out) return fim::set_error(FIM_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(const_cast<fim_server *>(s)->mu);
    *out = s->stats;
    return FIM_OK;
}

extern "C" void fim_server_destroy(fim_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (const Request &r : s->queue) {
            s->done[r.ticket] = Done{FIM_E_CANCELLED, nullptr, "server stopped"};
            s->state[r.ticket] = 2;
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    for (Lane &L : s->lanes)
        if (L.th.joinable()) L.th.join();
    for (Lane &L : s->lanes)
        if (L.own) fim_ctx_destroy(L.ctx);
    for (auto &kv : s->done) fim_result_destroy(kv.second.result);
    delete s;
}
