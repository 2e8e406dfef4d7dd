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

#include <cstring>

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

SampleEstimate::~SampleEstimate() {
    for (auto *r : res) fim_result_destroy(r);
}

void draw_sample(const fim_db *db, const std::vector<uint32_t> &rank_of_item, uint64_t nd,
                 uint64_t seed, std::vector<uint64_t> &off, std::vector<uint32_t> &items) {
    const uint64_t N = db->n_tx;
    uint64_t x = seed;
    off.assign(1, 0);
    items.clear();
    for (uint64_t d = 0; d < nd; d++) {
        const uint64_t t = std::min<uint64_t>(N - 1, (uint64_t)(u01(x) * (double)N));
        for (uint64_t p = db->h_off[t]; p < db->h_off[t + 1]; p++) {
            const uint32_t it = db->h_items[p];
            if (rank_of_item[it] != kNone) items.push_back(it);
        }
        off.push_back(items.size());
    }
}

// Phase 1 (reservoir variant): a sample of |D~| transactions drawn
// uniformly with replacement, mined by the same miner at the same relative
// minimum support, its frequent itemsets reservoir-sampled.
fim_status sample_phase(fim_ctx *ctx, const std::vector<PlanInput> &in, const fim_options &opts,
                        SampleEstimate &est) {
    const uint32_t n_inst = (uint32_t)in.size();
    const uint32_t want_tx = opts.sample_tx ? opts.sample_tx : default_sample_tx(0.02, 0.05);
    std::vector<fim_db *> sdb(n_inst, nullptr);
    std::vector<MineRequest> reqs;
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
        if (nd < 256 || P.n_freq < 3 || !P.estimate) continue;
        std::vector<uint64_t> off;
        std::vector<uint32_t> items;
        draw_sample(P.db, *P.rank_of_item, nd, opts.seed ^ (0x51ED270B1DE0ull * (q + 1)), off, items);
        fim_status s = fim_db_create(ctx, nd, off.data(), items.empty() ? nullptr : items.data(),
                                     P.db->n_item_ids, &sdb[q]);
        if (s != FIM_OK) return s;
        // relative minimum support carried over to the sample, at least 2
        uint32_t ms = (uint32_t)ceil((double)P.minsup * (double)nd / (double)N);
        ms = std::max<uint32_t>(ms, 2);
        reqs.push_back({sdb[q], ms});
        est.inst.push_back(q);
    }
    est.done = true;
    if (reqs.empty()) return FIM_OK;
    // mine the samples with the same miner (no estimate of their own)
    fim_options so = opts;
    so.flags |= FIM_FLAG_NO_ESTIMATE | kFlagInternalSample;
    so.max_itemsets = 0;
    so.max_len = 0;
    return mine_many(ctx, reqs, so, est.res);
}

// Row weights of every first-level class from the sample, or empty when no
// usable estimate exists for that instance.
static fim_status estimate_rows(fim_ctx *ctx, const std::vector<PlanInput> &in,
                                const fim_options &opts,
                                std::vector<std::vector<double>> &row_w, uint64_t &out_words,
                                SampleEstimate *pre) {
    out_words = 0;
    const uint32_t n_inst = (uint32_t)in.size();
    row_w.assign(n_inst, {});
    SampleEstimate own;
    SampleEstimate &est = pre && pre->done ? *pre : own;
    if (!est.done) {
        fim_status s = sample_phase(ctx, in, opts, est);
        if (s != FIM_OK) return s;
    }
    const std::vector<fim_result *> &res = est.res;
    const std::vector<uint32_t> &req_inst = est.inst;
    struct Reqs {
        size_t n;
        size_t size() const { return n; }
    } reqs{res.size()};

    for (size_t k = 0; k < reqs.size(); k++) {
        const uint32_t q = req_inst[k];
        const PlanInput &P = in[q];
        const fim_result *R = res[k];
        if (R->truncated) continue;  // exploded sample: no estimate
        // the sample run returns the reservoir's itemsets and the length of
        // its whole stream of frequent itemsets
        const uint64_t L = R->stats.n_itemsets;
        if (L == 0 || R->supp.empty()) continue;
        const double avg_len = (double)R->items.size() / (double)R->supp.size();
        // the sample's output, with room to spare, sizes the real output
        out_words += (uint64_t)((avg_len + kRecHeader + 1.0) * (double)L * 2.0);
        std::vector<uint64_t> keep(R->supp.size());
        for (uint64_t j = 0; j < keep.size(); j++) keep[j] = j;
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

// Partition + LPT order over classes given by their row weights.
// cls_in: one entry per first-level class with >= 2 atoms (inst, node,
// r0 = 0, r1 = n_atoms - 1); rw[k] the row weights of class k; rp[k] the
// row proxies.  Output classes in LPT order.
void lpt_order(std::vector<PlanClass> &out);

void partition_lpt_order(const std::vector<PlanClass> &cls_in,
                         const std::vector<const double *> &rw,
                         const std::vector<const double *> &rp, double alpha, uint32_t n_workers,
                         bool no_split, std::vector<PlanClass> &out) {
    out.clear();
    double total = 0.0;
    for (size_t k = 0; k < cls_in.size(); k++)
        for (uint32_t r = 0; r < cls_in[k].r1; r++) total += rw[k][r];
    const double theta = std::max(alpha * total / (double)std::max<uint32_t>(n_workers, 1), 1e-300);
    for (size_t k = 0; k < cls_in.size(); k++) {
        const PlanClass &c = cls_in[k];
        const uint32_t rows = c.r1;  // rows with a later atom
        double cw = 0.0, cp = 0.0;
        for (uint32_t r = 0; r < rows; r++) {
            cw += rw[k][r];
            cp += rp[k][r];
        }
        if (cw <= theta || no_split || rows == 1) {
            out.push_back({c.inst, c.node, 0, rows, cw, cp});
            continue;
        }
        uint32_t r0 = 0;
        double acc = 0.0, accp = 0.0;
        for (uint32_t r = 0; r < rows; r++) {
            const double v = rw[k][r];
            if (r > r0 && acc + v > theta) {
                out.push_back({c.inst, c.node, r0, r, acc, accp});
                r0 = r;
                acc = 0.0;
                accp = 0.0;
            }
            acc += v;
            accp += rp[k][r];
        }
        out.push_back({c.inst, c.node, r0, rows, acc, accp});
    }
    lpt_order(out);
}

// LPT order: decreasing estimate, then decreasing proxy, then position.
// One counting pass puts the tasks into 1,024 buckets of decreasing
// weight (sixteenths of an octave), then each bucket, a few tasks, is
// sorted exactly: the same order as a full sort of the 64-bit keys, whose
// radix passes cost the host about 0.1 ms for 2,000 tasks.
void lpt_order(std::vector<PlanClass> &out) {
    const size_t m = out.size();
    auto bucket = [](double w) -> uint32_t {  // 0 .. 1023, ascending in w
        if (!(w > 0.0)) return 0u;
        uint64_t b;
        memcpy(&b, &w, 8);
        const int e = (int)((b >> 52) & 2047u) - 1023 + 32;
        if (e < 0) return 0u;
        if (e >= 64) return 1023u;
        return (uint32_t)e * 16u + (uint32_t)((b >> 48) & 15u);
    };
    std::vector<uint32_t> idx(m), key(m);
    uint32_t h[1025] = {0};
    for (size_t i = 0; i < m; i++) {
        key[i] = 1023u - bucket(out[i].weight);
        h[key[i] + 1]++;
    }
    for (uint32_t d = 0; d < 1024; d++) h[d + 1] += h[d];
    {
        std::vector<uint32_t> pos(h, h + 1024);
        for (size_t i = 0; i < m; i++) idx[pos[key[i]]++] = (uint32_t)i;
    }
    auto before = [&](uint32_t a, uint32_t b) {
        if (out[a].weight != out[b].weight) return out[a].weight > out[b].weight;
        if (out[a].proxy != out[b].proxy) return out[a].proxy > out[b].proxy;
        return a < b;
    };
    for (uint32_t d = 0; d < 1024; d++)
        if (h[d + 1] - h[d] > 1) std::sort(idx.begin() + h[d], idx.begin() + h[d + 1], before);
    std::vector<PlanClass> sorted(m);
    for (size_t i = 0; i < m; i++) sorted[i] = out[idx[i]];
    out.swap(sorted);
}

fim_status plan_tasks(fim_ctx *ctx, const std::vector<PlanInput> &in, const fim_options &opts,
                      uint32_t n_workers, std::vector<Task> &tasks,
                      std::vector<PlanClass> *classes_out, uint64_t *est_out_words,
                      SampleEstimate *est, const std::vector<std::vector<double>> *given) {
    tasks.clear();
    const uint32_t n_inst = (uint32_t)in.size();
    std::vector<std::vector<double>> row_w;
    uint64_t ow = 0;
    if (given) {
        row_w = *given;
    } else if (!(opts.flags & FIM_FLAG_NO_ESTIMATE)) {
        fim_status s = estimate_rows(ctx, in, opts, row_w, ow, est);
        if (est_out_words) *est_out_words = ow;
        if (s != FIM_OK) return s;
    } else {
        row_w.assign(n_inst, {});
    }
    // proxy weight of a second-level class: pairs of its child class times
    // words per row (the weight of a class with k atoms in Zaki's bitonic
    // scheduling is C(k, 2)); instances without a sample estimate use it.
    // The rows of first-level class i are ceil(supp(i) / 32) words wide when
    // they are projected on its cover (a quarter of the stored width or
    // less, as the persistent kernel decides), else W.
    auto width_of = [&](uint32_t q, uint32_t i) {
        double width = (double)in[q].W;
        if (in[q].project && in[q].supp_of_rank) {
            const uint32_t s = (*in[q].supp_of_rank)[i];
            const uint32_t Wq = std::max<uint32_t>(4, ((s + 31) / 32 + 3) / 4 * 4);
            if (4ull * Wq <= in[q].Wp) width = (double)((s + 31) / 32);
        }
        return width;
    };
    bool any_est = false;
    for (const auto &v : row_w) any_est = any_est || !v.empty();
    if (!any_est && !classes_out) {
        // Proxy weights alone, in closed form: row r of a class of f atoms
        // weighs (k (k + 1) / 2 + 1) width with k = f - 1 - r, the class
        // width ((f - 1) f (f + 1) / 6 + f - 1); only the classes above the
        // Partition threshold are walked row by row.  The tasks are those of
        // partition_lpt_order over arrays of these weights (whole numbers,
        // so the sums agree wherever they stay below 2^53), without filling
        // a weight per second-level class (millions in a batch).
        std::vector<PlanClass> cls;
        double total = 0.0;
        for (uint32_t q = 0; q < n_inst; q++) {
            const auto &l2o = *in[q].l2_off;
            for (uint32_t i = 0; i < in[q].n_freq; i++) {
                const uint32_t f = l2o[i + 1] - l2o[i];
                if (f < 2) continue;
                const double fd = (double)f;
                const double cw = width_of(q, i) * ((fd - 1.0) * fd * (fd + 1.0) / 6.0 + fd - 1.0);
                cls.push_back({q, i, 0, f - 1, cw, cw});
                total += cw;
            }
        }
        const double theta =
            std::max(opts.alpha * total / (double)std::max<uint32_t>(n_workers, 1), 1e-300);
        const bool no_split = (opts.flags & FIM_FLAG_NO_SPLIT) != 0;
        std::vector<PlanClass> out;
        out.reserve(cls.size());
        for (const PlanClass &c : cls) {
            const uint32_t rows = c.r1;
            if (c.weight <= theta || no_split || rows == 1) {
                out.push_back(c);
                continue;
            }
            const double width = width_of(c.inst, c.node);
            const uint32_t f = rows + 1;
            uint32_t r0 = 0;
            double acc = 0.0;
            for (uint32_t r = 0; r < rows; r++) {
                const double k = (double)(f - r - 1);
                const double v = (k * (k + 1.0) / 2.0 + 1.0) * width;
                if (r > r0 && acc + v > theta) {
                    out.push_back({c.inst, c.node, r0, r, acc, acc});
                    r0 = r;
                    acc = 0.0;
                }
                acc += v;
            }
            out.push_back({c.inst, c.node, r0, rows, acc, acc});
        }
        lpt_order(out);
        tasks.reserve(out.size());
        for (const PlanClass &c : out) tasks.push_back(Task{c.inst, c.node, c.r0, c.r1});
        return FIM_OK;
    }
    std::vector<std::vector<double>> w(n_inst), px(n_inst);
    std::vector<PlanClass> cls_in;
    std::vector<const double *> rw, rp;
    for (uint32_t q = 0; q < n_inst; q++) {
        const auto &l2o = *in[q].l2_off;
        const size_t na = in[q].l2_atom->size();
        px[q].assign(na, 0.0);
        const bool est = !row_w[q].empty();
        if (est) w[q].assign(na, 0.0);  // else the proxy is the weight
        for (uint32_t i = 0; i < in[q].n_freq; i++) {
            const uint32_t f = l2o[i + 1] - l2o[i];
            const double width = width_of(q, i);
            for (uint32_t r = 0; r + 1 < f; r++) {
                const double k = (double)(f - r - 1);
                px[q][l2o[i] + r] = (k * (k + 1.0) / 2.0 + 1.0) * width;
                if (est) w[q][l2o[i] + r] = row_w[q][l2o[i] + r];
            }
        }
    }
    for (uint32_t q = 0; q < n_inst; q++) {
        const auto &l2o = *in[q].l2_off;
        for (uint32_t i = 0; i < in[q].n_freq; i++) {
            const uint32_t f = l2o[i + 1] - l2o[i];
            if (f < 2) continue;
            cls_in.push_back({q, i, 0, f - 1, 0.0, 0.0});
            rw.push_back((w[q].empty() ? px[q] : w[q]).data() + l2o[i]);
            rp.push_back(px[q].data() + l2o[i]);
        }
    }
    std::vector<PlanClass> cls;
    partition_lpt_order(cls_in, rw, rp, opts.alpha, n_workers,
                        (opts.flags & FIM_FLAG_NO_SPLIT) != 0, cls);
    tasks.reserve(cls.size());
    for (const PlanClass &c : cls) tasks.push_back(Task{c.inst, c.node, c.r0, c.r1});
    if (classes_out) *classes_out = std::move(cls);
    return FIM_OK;
}

}  // namespace fim

// ====================================================================== ABI

extern "C" fim_status fim_estimate_sample_sizes(double eps_db, double delta_db, double rho,
                                                double eps_fi, double delta_fi,
                                                uint32_t *sample_tx, uint32_t *sample_fi) {
    auto in01 = [](double x) { return x > 0.0 && x < 1.0; };
    if (!in01(eps_db) || !in01(delta_db) || !in01(rho) || !in01(eps_fi) || !in01(delta_fi) ||
        rho + eps_fi >= 1.0)
        return fim::set_error(FIM_E_INVALID_ARG, "sample-size parameters out of range");
    if (sample_tx) *sample_tx = fim::default_sample_tx(eps_db, delta_db);
    if (sample_fi) *sample_fi = fim::default_sample_fi(rho, eps_fi, delta_fi);
    return FIM_OK;
}

extern "C" fim_status fim_reservoir_sample(uint64_t stream_len, uint64_t n, uint64_t seed,
                                           uint64_t *out) {
    if (!out && n && stream_len) return fim::set_error(FIM_E_INVALID_ARG, "out is NULL");
    std::vector<uint64_t> r = fim::reservoir_indices(stream_len, n, seed);
    std::copy(r.begin(), r.end(), out);
    return FIM_OK;
}

extern "C" fim_status fim_lpt_schedule(const double *weights, uint64_t n_jobs, uint32_t n_workers,
                                       uint32_t *worker_of_job, double *makespan) {
    if ((n_jobs && (!weights || !worker_of_job)) || n_workers == 0)
        return fim::set_error(FIM_E_INVALID_ARG, "NULL argument or no workers");
    std::vector<double> w(weights, weights + n_jobs);
    std::vector<uint32_t> wk;
    const double ms = fim::lpt_schedule(w, n_workers, wk);
    std::copy(wk.begin(), wk.end(), worker_of_job);
    if (makespan) *makespan = ms;
    return FIM_OK;
}

extern "C" fim_status fim_partition_lpt(uint32_t n_classes, const uint32_t *n_atoms,
                                        const double *row_weights, double alpha,
                                        uint32_t n_workers, uint32_t flags, uint32_t *tasks,
                                        uint32_t capacity, uint32_t *n_tasks, double *makespan) {
    if ((n_classes && (!n_atoms || !row_weights)) || !n_tasks || n_workers == 0 ||
        !(alpha > 0.0) || alpha > 1.0)
        return fim::set_error(FIM_E_INVALID_ARG, "invalid argument");
    std::vector<fim::PlanClass> cls_in;
    std::vector<const double *> rw, rp;
    std::vector<double> zeros;
    uint64_t off = 0, maxa = 0;
    for (uint32_t c = 0; c < n_classes; c++) maxa = std::max<uint64_t>(maxa, n_atoms[c]);
    zeros.assign(maxa + 1, 0.0);
    for (uint32_t c = 0; c < n_classes; c++) {
        if (n_atoms[c] >= 2) {
            cls_in.push_back({0, c, 0, n_atoms[c] - 1, 0.0, 0.0});
            rw.push_back(row_weights + off);
            rp.push_back(zeros.data());
        }
        off += n_atoms[c];
    }
    std::vector<fim::PlanClass> out;
    fim::partition_lpt_order(cls_in, rw, rp, alpha, n_workers, (flags & FIM_FLAG_NO_SPLIT) != 0,
                             out);
    *n_tasks = (uint32_t)out.size();
    if (makespan) {
        std::vector<double> w;
        for (auto &c : out) w.push_back(c.weight);
        std::vector<uint32_t> wk;
        *makespan = fim::lpt_schedule(w, n_workers, wk);
    }
    if (out.size() > capacity)
        return fim::set_error(FIM_E_OUTPUT_LIMIT, "task capacity too small");
    if (!tasks && !out.empty()) return fim::set_error(FIM_E_INVALID_ARG, "tasks is NULL");
    for (size_t k = 0; k < out.size(); k++) {
        tasks[3 * k] = out[k].node;
        tasks[3 * k + 1] = out[k].r0;
        tasks[3 * k + 2] = out[k].r1;
    }
    return FIM_OK;
}
