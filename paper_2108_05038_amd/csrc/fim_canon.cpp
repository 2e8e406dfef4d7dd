// Canonical order of a frequent-itemset result (host).
#include "fim_canon.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>

namespace fim {

thread_local uint32_t g_host_thread_cap = 16;
thread_local bool g_no_pinned = false;

// ---------------------------------------------------------------- host pool
// Blocks are sized in powers of two; released blocks wait in per-size lists
// (up to kPoolCacheBytes in all) for the next request of their size.  Blocks
// are page-locked while the page-locked total stays below kPinnedBudget,
// ordinary heap memory beyond it (or when page-locking fails).
namespace {

constexpr size_t kPoolCacheBytes = size_t(2) << 30;
constexpr size_t kPinnedBudget = size_t(16) << 30;

struct HostPool {
    std::mutex mu;
    std::map<size_t, std::vector<void *>> free_lists;
    std::unordered_map<void *, bool> pinned;  // every live or cached block
    size_t cached = 0, pinned_total = 0;
};

HostPool &host_pool() {
    static HostPool *p = new HostPool();  // never destroyed: blocks may outlive static teardown
    return *p;
}

size_t pool_class(size_t bytes) {
    size_t c = kHostPoolMin;
    while (c < bytes) c <<= 1;
    return c;
}

}  // namespace

void *host_pool_alloc(size_t bytes) {
    const size_t c = pool_class(bytes);
    HostPool &P = host_pool();
    {
        std::lock_guard<std::mutex> g(P.mu);
        auto it = P.free_lists.find(c);
        if (it != P.free_lists.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            P.cached -= c;
            return p;
        }
    }
    void *p = nullptr;
    bool pin = false;
    {
        std::lock_guard<std::mutex> g(P.mu);
        pin = !g_no_pinned && P.pinned_total + c <= kPinnedBudget;
        if (pin) P.pinned_total += c;
    }
    if (pin && hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        std::lock_guard<std::mutex> g(P.mu);
        P.pinned_total -= c;
        pin = false;
    }
    if (!p) {
        p = std::malloc(c);
        if (!p) throw std::bad_alloc();
    }
    std::lock_guard<std::mutex> g(P.mu);
    P.pinned[p] = pin;
    return p;
}

void host_pool_free(void *p, size_t bytes) {
    if (!p) return;
    const size_t c = pool_class(bytes);
    HostPool &P = host_pool();
    bool pin = false;
    {
        std::lock_guard<std::mutex> g(P.mu);
        // (a call that allocates nothing may exceed the cache rather than
        // give page-locked memory back)
        if (P.cached + c <= kPoolCacheBytes || (g_no_pinned && P.pinned.count(p) && P.pinned[p])) {
            P.free_lists[c].push_back(p);
            P.cached += c;
            return;
        }
        auto it = P.pinned.find(p);
        pin = it != P.pinned.end() && it->second;
        if (it != P.pinned.end()) P.pinned.erase(it);
        if (pin) P.pinned_total -= c;
    }
    if (pin) (void)hipHostFree(p);
    else std::free(p);
}


namespace {

typedef unsigned __int128 u128;

// exclusive prefix sums of blocks of v computed in parallel
void block_scan(const std::vector<uint64_t> &block_sum, std::vector<uint64_t> &block_start) {
    block_start.resize(block_sum.size() + 1);
    block_start[0] = 0;
    for (size_t b = 0; b < block_sum.size(); b++) block_start[b + 1] = block_start[b] + block_sum[b];
}

// items of one itemset ascending (insertion sort: itemsets are short)
inline void sort_small(uint32_t *a, uint64_t n) {
    if (n > 24) {
        std::sort(a, a + n);
        return;
    }
    for (uint64_t i = 1; i < n; i++) {
        const uint32_t v = a[i];
        uint64_t j = i;
        while (j > 0 && a[j - 1] > v) {
            a[j] = a[j - 1];
            j--;
        }
        a[j] = v;
    }
}

// Sort record: the key alone when the support fits in its unused low bits
// (Packed), else the key and the support.
template <bool Packed>
struct KeyRec;
template <>
struct KeyRec<true> {
    u128 key;
    uint32_t supp() const { return (uint32_t)key; }
};
template <>
struct KeyRec<false> {
    u128 key;
    uint32_t s;
    uint32_t supp() const { return s; }
};

// Itemsets as keys of (item + 1) codes of `bits` bits, most significant
// first: a prefix has zero codes where its extensions continue, so it sorts
// first, and two itemsets compare like their item sequences.  Each
// itemset's items are sorted while its key is built, and the sorted result
// is read back from the keys.
template <bool Packed>
void canonical_by_keys(U32Vec &items, U64Vec &off, U32Vec &supp, uint32_t bits, uint32_t n_thr) {
    typedef KeyRec<Packed> Rec;
    const uint64_t n = supp.size();
    const uint32_t *it = items.data();
    const uint64_t *o = off.data();
    std::unique_ptr<Rec[]> kv(new Rec[n]), kb(new Rec[n]);
    const uint32_t T = std::max(1u, n_thr);
    const uint64_t per = (n + T - 1) / T;
    // radix partition on the top B bits (about the first two items)
    const uint32_t B = std::min<uint32_t>(16, 2 * bits);
    const uint32_t NB = 1u << B;
    std::vector<std::vector<uint64_t>> hist(T, std::vector<uint64_t>(NB, 0));
    parallel_for(T, T, [&](uint64_t t) {
        const uint64_t a = t * per, e = std::min(n, a + per);
        auto &h = hist[t];
        uint32_t buf[128];
        for (uint64_t q = a; q < e; q++) {
            const uint64_t len = o[q + 1] - o[q];
            for (uint64_t k = 0; k < len; k++) buf[k] = it[o[q] + k];
            sort_small(buf, len);
            u128 key = 0;
            uint32_t sh = 128;
            for (uint64_t k = 0; k < len; k++) {
                sh -= bits;
                key |= (u128)(buf[k] + 1) << sh;
            }
            if constexpr (Packed) {
                kv[q].key = key | supp[q];
            } else {
                kv[q].key = key;
                kv[q].s = supp[q];
            }
            h[(uint32_t)(key >> (128 - B))]++;
        }
    });
    std::vector<uint64_t> bstart(NB + 1, 0);
    for (uint32_t b = 0; b < NB; b++) {
        uint64_t sum = 0;
        for (uint32_t t = 0; t < T; t++) sum += hist[t][b];
        bstart[b + 1] = bstart[b] + sum;
    }
    parallel_for(T, T, [&](uint64_t t) {
        // this thread's first slot in every bucket
        std::vector<uint64_t> pos(NB);
        for (uint32_t b = 0; b < NB; b++) {
            uint64_t p = bstart[b];
            for (uint32_t u = 0; u < t; u++) p += hist[u][b];
            pos[b] = p;
        }
        const uint64_t a = t * per, e = std::min(n, a + per);
        for (uint64_t q = a; q < e; q++) kb[pos[(uint32_t)(kv[q].key >> (128 - B))]++] = kv[q];
    });
    std::vector<uint32_t> big;
    for (uint32_t b = 0; b < NB; b++)
        if (bstart[b + 1] - bstart[b] > 1) big.push_back(b);
    std::sort(big.begin(), big.end(), [&](uint32_t x, uint32_t y) {
        return bstart[x + 1] - bstart[x] > bstart[y + 1] - bstart[y];
    });
    parallel_for(big.size(), T, [&](uint64_t k) {
        const uint32_t b = big[k];
        std::sort(kb.get() + bstart[b], kb.get() + bstart[b + 1],
                  [](const Rec &x, const Rec &y) { return x.key < y.key; });
    });
    // lengths (non-zero codes) per block, block starts, then every block
    // decodes its keys in parallel
    const uint64_t blk = 1u << 14, nblk = (n + blk - 1) / blk;
    const uint64_t mask = (1ull << bits) - 1;
    const uint32_t per_key = 128 / bits;
    std::vector<uint64_t> bsum(nblk, 0), bst;
    auto code = [&](const u128 &key, uint32_t k) {
        return (uint64_t)(key >> (128 - bits * (k + 1))) & mask;
    };
    parallel_for(nblk, T, [&](uint64_t b) {
        uint64_t s = 0;
        for (uint64_t q = b * blk; q < std::min(n, (b + 1) * blk); q++) {
            uint32_t k = 0;
            while (k < per_key && code(kb[q].key, k)) k++;
            s += k;
        }
        bsum[b] = s;
    });
    block_scan(bsum, bst);
    U32Vec ni(items.size()), ns(n);
    U64Vec no(n + 1);
    parallel_for(nblk, T, [&](uint64_t b) {
        uint64_t w = bst[b];
        for (uint64_t q = b * blk; q < std::min(n, (b + 1) * blk); q++) {
            const u128 key = kb[q].key;
            for (uint32_t k = 0; k < per_key; k++) {
                const uint64_t c = code(key, k);
                if (!c) break;
                ni[w++] = (uint32_t)c - 1;
            }
            no[q + 1] = w;
            ns[q] = kb[q].supp();
        }
    });
    no[0] = 0;
    items.swap(ni);
    off.swap(no);
    supp.swap(ns);
}

// general case: itemsets bucketed by their first item, buckets sorted by
// comparing item sequences
void canonical_by_compare(U32Vec &items, U64Vec &off, U32Vec &supp, uint32_t max_item,
                          uint32_t n_thr) {
    const uint64_t n = supp.size();
    const uint32_t *it = items.data();
    const uint64_t *o = off.data();
    std::vector<uint64_t> start(max_item + 2, 0);
    for (uint64_t i = 0; i < n; i++) start[it[o[i]] + 1]++;
    for (uint32_t b = 0; b <= max_item; b++) start[b + 1] += start[b];
    std::vector<uint64_t> idx(n);
    {
        std::vector<uint64_t> fill(start.begin(), start.end() - 1);
        for (uint64_t i = 0; i < n; i++) idx[fill[it[o[i]]]++] = i;
    }
    std::vector<uint32_t> order;
    for (uint32_t b = 0; b <= max_item; b++)
        if (start[b + 1] - start[b] > 1) order.push_back(b);
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return start[a + 1] - start[a] > start[b + 1] - start[b];
    });
    auto less = [&](uint64_t a, uint64_t b) {
        const uint32_t *x = it + o[a], *y = it + o[b];
        const uint64_t nx = o[a + 1] - o[a], ny = o[b + 1] - o[b];
        const uint64_t m = std::min(nx, ny);
        for (uint64_t k = 1; k < m; k++)  // item 0 is the bucket
            if (x[k] != y[k]) return x[k] < y[k];
        return nx < ny;
    };
    parallel_for(order.size(), n_thr, [&](uint64_t k) {
        const uint32_t b = order[k];
        std::sort(idx.begin() + start[b], idx.begin() + start[b + 1], less);
    });
    U64Vec no(n + 1);
    no[0] = 0;
    for (uint64_t q = 0; q < n; q++) no[q + 1] = no[q] + (o[idx[q] + 1] - o[idx[q]]);
    U32Vec ni(items.size()), ns(n);
    const uint64_t blk = 8192, nblk = (n + blk - 1) / blk;
    parallel_for(nblk, n_thr, [&](uint64_t b) {
        for (uint64_t q = b * blk; q < std::min(n, (b + 1) * blk); q++) {
            const uint64_t a = idx[q];
            std::copy(it + o[a], it + o[a + 1], ni.begin() + no[q]);
            ns[q] = supp[a];
        }
    });
    items.swap(ni);
    off.swap(no);
    supp.swap(ns);
}

}  // namespace

// Items ascending inside every itemset, then the itemsets in lexicographic
// order: as 128-bit integer keys when every itemset fits (radix partition on
// the top bits, buckets sorted in parallel), otherwise by comparison.
void canonicalize(U32Vec &items, U64Vec &off, U32Vec &supp, uint32_t threads) {
    const uint64_t n = supp.size();
    if (n == 0) return;
    const uint32_t n_thr = threads ? threads : host_threads(n);
    uint32_t *it = items.data();
    const uint64_t *o = off.data();
    // largest item and longest itemset
    const uint64_t blk = 8192, nblk = (n + blk - 1) / blk;
    std::vector<uint32_t> bmax(nblk, 0);
    std::vector<uint64_t> blen(nblk, 0);
    parallel_for(nblk, n_thr, [&](uint64_t b) {
        uint32_t mi = 0;
        uint64_t ml = 0;
        for (uint64_t i = b * blk; i < std::min(n, (b + 1) * blk); i++) {
            for (uint64_t k = o[i]; k < o[i + 1]; k++) mi = std::max(mi, it[k]);
            ml = std::max<uint64_t>(ml, o[i + 1] - o[i]);
        }
        bmax[b] = mi;
        blen[b] = ml;
    });
    const uint32_t max_item = *std::max_element(bmax.begin(), bmax.end());
    const uint64_t max_len = *std::max_element(blen.begin(), blen.end());
    uint32_t bits = 1;
    while (bits < 32 && ((uint64_t)max_item + 1) >> bits) bits++;
    if ((uint64_t)bits * max_len + 32 <= 128) {
        canonical_by_keys<true>(items, off, supp, bits, n_thr);
    } else if ((uint64_t)bits * max_len <= 128) {
        canonical_by_keys<false>(items, off, supp, bits, n_thr);
    } else {
        parallel_for(nblk, n_thr, [&](uint64_t b) {
            for (uint64_t i = b * blk; i < std::min(n, (b + 1) * blk); i++)
                if (o[i + 1] - o[i] > 1) sort_small(it + o[i], o[i + 1] - o[i]);
        });
        canonical_by_compare(items, off, supp, max_item, n_thr);
    }
}

}  // namespace fim
