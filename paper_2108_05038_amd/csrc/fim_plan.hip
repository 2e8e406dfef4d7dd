// Work planning of the persistent kernel (host side).
//
// The thesis balances its distributed miner statically: it samples the
// database, mines the sample, keeps a uniform reservoir sample S of the
// sample's frequent itemsets, estimates the size of every prefix-based class
// as the number of S's itemsets it holds, splits classes whose estimate
// exceeds alpha * |S| / P (the Partition algorithm) and assigns the classes
// to the P processors by LPT-Schedule (chapter on the new parallel method,
// Phase 1 reservoir variant and Phase 2).  Here the processors are the waves
// of one persistent kernel; the sample is mined by the same GPU miner; the
// classes are first-level classes [a_i | later items] and, for large ones,
// contiguous ranges of their second-level classes [a_i, a_j | later atoms];
// the global task queue is filled in LPT order, so that every idle wave
// takes the largest remaining class, and the static LPT assignment is
// computed as well to report its estimated makespan.
#include <math.h>

#include <algorithm>
#include <numeric>
#include <queue>

#include "fim_plan.h"

namespace fim {

namespace {

uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double u01(uint64_t &x) { return (double)(splitmix64(x) >> 11) * 0x1.0p-53; }

}  // namespace

uint32_t default_sample_tx(double eps, double delta) {
    return (uint32_t)ceil(log(2.0 / delta) / (2.0 * eps * eps));
}

double bernoulli_kl(double x, double y) {
    double r = 0.0;
    if (x > 0.0) r += x * log(x / y);
    if (x < 1.0) r += (1.0 - x) * log((1.0 - x) / (1.0 - y));
    return r;
}

uint32_t default_sample_fi(double rho, double eps, double delta) {
    return (uint32_t)ceil(-log(delta / 2.0) / bernoulli_kl(rho + eps, rho));
}

std::vector<uint64_t> reservoir_indices(uint64_t len, uint64_t n, uint64_t seed) {
    std::vector<uint64_t> R;
    uint64_t x = seed;
    for (uint64_t j = 0; j < n && j < len; j++) R.push_back(j);
    uint64_t t = R.size();
    for (uint64_t idx = t; idx < len; idx++) {
        t = t + 1;
        const uint64_t m = (uint64_t)floor((double)t * u01(x));
        if (m < n) R[m] = idx;
    }
    return R;
}

double lpt_schedule(const std::vector<double> &w, uint32_t p, std::vector<uint32_t> &worker) {
    std::vector<uint32_t> order(w.size());
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return w[a] > w[b]; });
    typedef std::pair<double, uint32_t> Load;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (uint32_t k = 0; k < p; k++) heap.push(Load(0.0, k));
    worker.assign(w.size(), 0);
    double makespan = 0.0;
    for (uint32_t j : order) {
        Load l = heap.top();
        heap.pop();
        worker[j] = l.second;
        l.first += w[j];
        makespan = std::max(makespan, l.first);
        heap.push(l);
    }
    return makespan;
}

// Row weights of every first-level class from the sample, or empty when no
// usable estimate exists for that instance.
static fim_status estimate_rows(fim_ctx *ctx, const std::vector<PlanInput> &in,
                                const fim_options &opts,
                                std::vector<std::vector<double>> &row_w) {
    const uint32_t n_inst = (uint32_t)in.size();
    row_w.assign(n_inst, {});
    const uint32_t want_tx = opts.sample_tx ? opts.sample_tx : default_sample_tx(0.02, 0.05);
    const uint32_t n_fi = opts.sample_fi ? opts.sample_fi : default_sample_fi(0.001, 0.0005, 0.05);

    // Phase 1: draw |D~| transactions uniformly with replacement
    std::vector<fim_db *> sdb(n_inst, nullptr);
    std::vector<MineRequest> reqs;
    std::vector<uint32_t> req_inst;
    struct DbGuard {
        std::vector<fim_db *> &v;
        ~DbGuard() {
            for (auto *d : v) fim_db_destroy(d);
        }
    } guard{sdb};
    for (uint32_t q = 0; q < n_inst; q++) {
        const PlanInput &P = in[q];
        const uint64_t N = P.db->n_tx;
        const uint64_t nd = std::min<uint64_t>(want_tx, N / 4);
        if (nd < 256 || P.n_freq < 3) continue;
        uint64_t x = opts.seed ^ (0x51ED270B1DE0ull * (q + 1));
        std::vector<uint64_t> off{0};
        std::vector<uint32_t> items;
        for (uint64_t d = 0; d < nd; d++) {
            const uint64_t t = std::min<uint64_t>(N - 1, (uint64_t)(u01(x) * (double)N));
            for (uint64_t p = P.db->h_off[t]; p < P.db->h_off[t + 1]; p++) {
                const uint32_t it = P.db->h_items[p];
                if ((*P.rank_of_item)[it] != kNone) items.push_back(it);
            }
            off.push_back(items.size());
        }
        fim_status s = fim_db_create(ctx, nd, off.data(), items.empty() ? nullptr : items.data(),
                                     P.db->n_item_ids, &sdb[q]);
        if (s != FIM_OK) return s;
        // relative minimum support carried over to the sample, at least 2
        uint32_t ms = (uint32_t)ceil((double)P.minsup * (double)nd / (double)N);
        ms = std::max<uint32_t>(ms, 2);
        reqs.push_back({sdb[q], ms});
        req_inst.push_back(q);
    }
    if (reqs.empty()) return FIM_OK;

    // mine the samples with the same miner (no estimate of their own)
    fim_options so = opts;
    so.flags |= FIM_FLAG_NO_ESTIMATE | kFlagInternalSample;
    so.max_itemsets = 0;
    so.max_len = 0;
    std::vector<fim_result *> res;
    fim_status s = mine_many(ctx, reqs, so, res, false);
    if (s != FIM_OK) return s;
    struct ResGuard {
        std::vector<fim_result *> &v;
        ~ResGuard() {
            for (auto *r : v) fim_result_destroy(r);
        }
    } rguard{res};

    for (size_t k = 0; k < reqs.size(); k++) {
        const uint32_t q = req_inst[k];
        const PlanInput &P = in[q];
        const fim_result *R = res[k];
        if (R->truncated) continue;  // exploded sample: no estimate
        const uint64_t L = R->supp.size();
        if (L == 0) continue;
        std::vector<uint64_t> keep = reservoir_indices(L, n_fi, opts.seed + 7 * q + 1);
        // Phase 2 sizes: every sampled itemset of length >= 3 lies in one
        // second-level class [a, b | ...]: a = its first item in the miner's
        // order, b = the next one in the order of a's atoms
        const std::vector<uint32_t> &l2o = *P.l2_off, &l2a = *P.l2_atom;
        std::vector<std::vector<uint32_t>> by_first(P.n_freq);
        std::vector<uint32_t> ranks;
        for (size_t j = 0; j < keep.size(); j++) {
            const uint64_t i = keep[j];
            const uint64_t a = R->off[i], b = R->off[i + 1];
            if (b - a < 3) continue;
            uint32_t first = kNone;
            for (uint64_t p = a; p < b; p++) {
                const uint32_t r = (*P.rank_of_item)[R->items[p]];
                if (r == kNone) {  // not frequent in D: not a frequent itemset of D
                    first = kNone;
                    break;
                }
                first = std::min(first, r);
            }
            if (first == kNone || l2o[first + 1] - l2o[first] < 2) continue;
            by_first[first].push_back((uint32_t)i);
        }
        row_w[q].assign(l2a.size(), 0.0);
        std::vector<uint32_t> pos(P.n_freq, kNone);
        uint64_t used = 0;
        for (uint32_t f = 0; f < P.n_freq; f++) {
            if (by_first[f].empty()) continue;
            const uint32_t a0 = l2o[f], a1 = l2o[f + 1];
            for (uint32_t q2 = a0; q2 < a1; q2++) pos[l2a[q2]] = q2 - a0;
            for (uint32_t i : by_first[f]) {
                uint32_t best = kNone;
                bool ok = true;
                for (uint64_t p = R->off[i]; p < R->off[i + 1]; p++) {
                    const uint32_t r = (*P.rank_of_item)[R->items[p]];
                    if (r == f) continue;
                    if (pos[r] == kNone) {  // {a_f, x} is not frequent in D
                        ok = false;
                        break;
                    }
                    best = std::min(best, pos[r]);
                }
                if (!ok || best == kNone) continue;
                row_w[q][a0 + best] += 1.0;
                used++;
            }
            for (uint32_t q2 = a0; q2 < a1; q2++) pos[l2a[q2]] = kNone;
        }
        // scale sample counts to estimated itemsets times words per row
        const double scale = (double)L / (double)std::max<size_t>(keep.size(), 1) * (double)P.W;
        for (double &w : row_w[q]) w *= scale;
        if (used == 0) row_w[q].clear();
    }
    return FIM_OK;
}

fim_status plan_tasks(fim_ctx *ctx, const std::vector<PlanInput> &in, const fim_options &opts,
                      uint32_t n_workers, std::vector<Task> &tasks,
                      std::vector<PlanClass> *classes_out) {
    tasks.clear();
    const uint32_t n_inst = (uint32_t)in.size();
    std::vector<std::vector<double>> row_w;
    if (!(opts.flags & FIM_FLAG_NO_ESTIMATE)) {
        fim_status s = estimate_rows(ctx, in, opts, row_w);
        if (s != FIM_OK) return s;
    } else {
        row_w.assign(n_inst, {});
    }
    // proxy weight of a second-level class: pairs of its child class times
    // words per row (the weight of a class with k atoms in Zaki's bitonic
    // scheduling is C(k, 2))
    auto proxy = [&](uint32_t q, uint32_t i, uint32_t r) {
        const uint32_t f = (*in[q].l2_off)[i + 1] - (*in[q].l2_off)[i];
        const double k = (double)(f - r - 1);
        return (k * (k + 1.0) / 2.0 + 1.0) * (double)in[q].W;
    };
    // when an instance has no sample estimate, its rows get proxy weights
    double total = 0.0;
    std::vector<std::vector<double>> w(n_inst);
    for (uint32_t q = 0; q < n_inst; q++) {
        const auto &l2o = *in[q].l2_off;
        w[q].assign(in[q].l2_atom->size(), 0.0);
        const bool est = !row_w[q].empty();
        for (uint32_t i = 0; i < in[q].n_freq; i++)
            for (uint32_t r = 0; r + 1 < l2o[i + 1] - l2o[i]; r++) {
                const double v = est ? row_w[q][l2o[i] + r] : proxy(q, i, r);
                w[q][l2o[i] + r] = v;
                total += v;
            }
    }
    // Partition: split a class whose estimate exceeds alpha * total / P into
    // contiguous ranges of its second-level classes
    const double theta = std::max(opts.alpha * total / (double)std::max<uint32_t>(n_workers, 1), 1e-300);
    std::vector<PlanClass> cls;
    for (uint32_t q = 0; q < n_inst; q++) {
        const auto &l2o = *in[q].l2_off;
        for (uint32_t i = 0; i < in[q].n_freq; i++) {
            const uint32_t f = l2o[i + 1] - l2o[i];
            if (f < 2) continue;
            double cw = 0.0, cp = 0.0;
            for (uint32_t r = 0; r + 1 < f; r++) {
                cw += w[q][l2o[i] + r];
                cp += proxy(q, i, r);
            }
            if (cw <= theta || (opts.flags & FIM_FLAG_NO_SPLIT) || f == 2) {
                cls.push_back({q, i, 0, f - 1, cw, cp});
                continue;
            }
            uint32_t r0 = 0;
            double acc = 0.0, accp = 0.0;
            for (uint32_t r = 0; r + 1 < f; r++) {
                const double v = w[q][l2o[i] + r];
                if (r > r0 && acc + v > theta) {
                    cls.push_back({q, i, r0, r, acc, accp});
                    r0 = r;
                    acc = 0.0;
                    accp = 0.0;
                }
                acc += v;
                accp += proxy(q, i, r);
            }
            cls.push_back({q, i, r0, f - 1, acc, accp});
        }
    }
    // LPT order: decreasing estimate, then decreasing proxy, then position
    std::stable_sort(cls.begin(), cls.end(), [](const PlanClass &a, const PlanClass &b) {
        if (a.weight != b.weight) return a.weight > b.weight;
        return a.proxy > b.proxy;
    });
    tasks.reserve(cls.size());
    for (const PlanClass &c : cls) tasks.push_back(Task{c.inst, c.node, c.r0, c.r1});
    if (classes_out) *classes_out = std::move(cls);
    return FIM_OK;
}

}  // namespace fim
