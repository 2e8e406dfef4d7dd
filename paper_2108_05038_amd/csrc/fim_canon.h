// Host-side helpers for results: a small thread pool loop and the
// canonical (lexicographic) order of itemsets.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <utility>
#include <thread>
#include <vector>

namespace fim {

// Host blocks of at least kHostPoolMin bytes (16 KB) for result arrays: page-locked
// (device copies go straight into them), kept for reuse after release so
// that a later result does not fault its pages in again.  Thread-safe.
constexpr size_t kHostPoolMin = 1u << 14;
// Set while the calling thread runs an entry point that allocates no device
// or page-locked memory: new host blocks then come from the ordinary heap.
extern thread_local bool g_no_pinned;
void *host_pool_alloc(size_t bytes);
void host_pool_free(void *p, size_t bytes);

// std::allocator whose value-less construct leaves the element
// uninitialised, so that resizing large result arrays does not first zero
// them on one thread; large arrays come from the host pool
template <class T>
struct UninitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = UninitAlloc<U>;
    };
    UninitAlloc() = default;
    template <class U>
    UninitAlloc(const UninitAlloc<U> &) {}
    T *allocate(size_t n) {
        if (n * sizeof(T) >= kHostPoolMin) return static_cast<T *>(host_pool_alloc(n * sizeof(T)));
        return std::allocator<T>::allocate(n);
    }
    void deallocate(T *p, size_t n) {
        if (n * sizeof(T) >= kHostPoolMin) host_pool_free(p, n * sizeof(T));
        else std::allocator<T>::deallocate(p, n);
    }
    template <class U>
    void construct(U *p) noexcept {
        ::new ((void *)p) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};

using U32Vec = std::vector<uint32_t, UninitAlloc<uint32_t>>;
using U64Vec = std::vector<uint64_t, UninitAlloc<uint64_t>>;

// run fn(i) for i in [0, count) on up to n_thr threads
template <class Fn>
inline void parallel_for(uint64_t count, uint32_t n_thr, Fn fn) {
    if (n_thr <= 1 || count < 2) {
        for (uint64_t i = 0; i < count; i++) fn(i);
        return;
    }
    std::atomic<uint64_t> next{0};
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < std::min<uint64_t>(n_thr, count); t++)
        th.emplace_back([&] {
            for (uint64_t i; (i = next.fetch_add(1)) < count;) fn(i);
        });
    for (auto &x : th) x.join();
}

// Threads the calling thread may use for host stages (a server lane sets a
// share of the host so that lanes do not oversubscribe it).
extern thread_local uint32_t g_host_thread_cap;

inline uint32_t host_threads(uint64_t work) {
    if (work < 20000) return 1;
    return std::max(1u, std::min({16u, g_host_thread_cap, std::thread::hardware_concurrency()}));
}

// Puts a result into canonical order: items ascending inside every itemset,
// itemsets in lexicographic order (a prefix before its extensions).
void canonicalize(U32Vec &items, U64Vec &off, U32Vec &supp, uint32_t threads = 0);

}  // namespace fim
