// a9 on the GPU: the result of a mining call in canonical order.
//
// The persistent kernel (in key mode) writes every frequent itemset as a
// fixed record of eight words: a 128-bit key holding the itemset's item ids
// ascending, as (id + 1) codes of `bits` bits packed from the most
// significant bit down (zero codes after the last item), then the support
// and the instance.  Comparing two keys of one instance compares the item
// sequences lexicographically, a prefix first (its zero codes sort before
// any item), which is the canonical order.  Sorting the records by
// (instance, key) with two stable radix sorts (the 128-bit key, then the
// instance) and reading the items back out of the keys gives every
// instance's result as CSR, without the host touching a record.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "fim_host.h"

namespace fim {
namespace {

constexpr uint32_t kOrdBlock = 256;

__global__ void k_split(const uint32_t *__restrict__ rec, uint64_t n, rocprim::uint128_t *key,
                        uint32_t *inst, uint32_t *idx) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const uint4 a = reinterpret_cast<const uint4 *>(rec)[2 * q];
        const uint4 b = reinterpret_cast<const uint4 *>(rec)[2 * q + 1];
        const unsigned long long lo = ((unsigned long long)a.y << 32) | a.x;
        const unsigned long long hi = ((unsigned long long)a.w << 32) | a.z;
        key[q] = ((rocprim::uint128_t)hi << 64) | lo;
        inst[q] = b.y;
        idx[q] = (uint32_t)q;
    }
}

template <class T>
__global__ void k_gather(const T *__restrict__ src, const uint32_t *__restrict__ idx, uint64_t n,
                         T *dst) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        dst[q] = src[idx[q]];
}

__device__ __forceinline__ uint32_t code_at(unsigned long long lo, unsigned long long hi,
                                            uint32_t bits, uint32_t k) {
    // code k occupies bits [128 - bits (k + 1), 128 - bits k) of hi:lo
    const uint32_t sh = 128 - bits * (k + 1);
    const unsigned long long mask = (bits == 64) ? ~0ull : ((1ull << bits) - 1);
    unsigned long long v;
    if (sh >= 64) v = hi >> (sh - 64);
    else if (sh == 0) v = lo;
    else v = (lo >> sh) | (hi << (64 - sh));
    return (uint32_t)(v & mask);
}

// items per sorted record (and a trailing zero for the scan)
__global__ void k_lengths(const uint32_t *__restrict__ rec, const uint32_t *__restrict__ idx,
                          uint64_t n, const uint32_t *__restrict__ bits_of, uint32_t *len) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= n; q += stride) {
        if (q == n) {
            len[q] = 0;
            continue;
        }
        const uint32_t *r = rec + 8ull * idx[q];
        const unsigned long long lo = ((unsigned long long)r[1] << 32) | r[0];
        const unsigned long long hi = ((unsigned long long)r[3] << 32) | r[2];
        const uint32_t bits = bits_of[r[5]];
        uint32_t k = 0;
        while (k < 128 / bits && code_at(lo, hi, bits, k)) k++;
        len[q] = k;
    }
}

// items, supports, and the first sorted position of every instance
__global__ void k_decode(const uint32_t *__restrict__ rec, const uint32_t *__restrict__ idx,
                         uint64_t n, const uint32_t *__restrict__ bits_of,
                         const unsigned long long *__restrict__ item_off, uint32_t *items,
                         uint32_t *supp, unsigned long long *first) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const uint32_t *r = rec + 8ull * idx[q];
        const unsigned long long lo = ((unsigned long long)r[1] << 32) | r[0];
        const unsigned long long hi = ((unsigned long long)r[3] << 32) | r[2];
        const uint32_t inst = r[5];
        const uint32_t bits = bits_of[inst];
        const uint64_t a = item_off[q], e = item_off[q + 1];
        for (uint64_t k = 0; k < e - a; k++) items[a + k] = code_at(lo, hi, bits, (uint32_t)k) - 1;
        supp[q] = r[4];
        if (q == 0 || rec[8ull * idx[q - 1] + 5] != inst) first[inst] = q;
    }
}

uint32_t grid_for(uint64_t n) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + kOrdBlock - 1) / kOrdBlock, 65536));
}

#define OCHK(call)                                                                                \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return set_error(FIM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

#define OENSURE(buf, bytes)                                                                       \
    do {                                                                                          \
        if (!(buf).ensure(ctx, (bytes)))                                                          \
            return set_error(FIM_E_OOM_DEVICE, "device allocation for ordering failed");         \
    } while (0)

}  // namespace

fim_status gpu_order(fim_ctx *ctx, hipStream_t s, const uint32_t *d_rec, uint64_t n,
                     const std::vector<uint32_t> &bits_of, std::vector<uint64_t> &first,
                     U64Vec &off, U32Vec &items, U32Vec &supp) {
    const uint32_t n_inst = (uint32_t)bits_of.size();
    first.assign(n_inst, ~0ull);
    off.assign(1, 0);
    items.clear();
    supp.clear();
    if (n == 0) return FIM_OK;
    if (n >= (1ull << 31)) return set_error(FIM_E_OUTPUT_LIMIT, "more than 2^31 itemsets in one call");
    const int ni = (int)n;
    DevBuf key(ctx), key2(ctx), inst(ctx), inst2(ctx), idx(ctx), idx2(ctx), len(ctx),
        ioff(ctx), d_items(ctx), d_supp(ctx), d_first(ctx), d_bits(ctx), tmp(ctx);
    OENSURE(key, n * 16);
    OENSURE(key2, n * 16);
    OENSURE(inst, n * 4);
    OENSURE(inst2, n * 4);
    OENSURE(idx, n * 4);
    OENSURE(idx2, n * 4);
    OENSURE(d_bits, n_inst * 4);
    OCHK(h2d(ctx, d_bits.as<void>(), bits_of.data(), n_inst * 4, s));
    hipLaunchKernelGGL(k_split, dim3(grid_for(n)), dim3(kOrdBlock), 0, s, d_rec, n,
                       key.as<rocprim::uint128_t>(), inst.as<uint32_t>(), idx.as<uint32_t>());
    OCHK(hipGetLastError());
    // temporary storage of the largest pass
    size_t tb = 0, t1 = 0;
    OCHK(rocprim::radix_sort_pairs(nullptr, t1, key.as<rocprim::uint128_t>(),
                                   key2.as<rocprim::uint128_t>(), idx.as<uint32_t>(),
                                   idx2.as<uint32_t>(), ni, 0, 128, s));
    tb = std::max(tb, t1);
    OCHK(rocprim::radix_sort_pairs(nullptr, t1, inst.as<uint32_t>(), inst2.as<uint32_t>(),
                                            idx.as<uint32_t>(), idx2.as<uint32_t>(), ni, 0, 32, s));
    tb = std::max(tb, t1);
    OCHK(rocprim::exclusive_scan(nullptr, t1, len.as<uint32_t>(), ioff.as<unsigned long long>(), 0ull, (size_t)(ni + 1), rocprim::plus<unsigned long long>(), s));
    tb = std::max(tb, t1);
    OENSURE(tmp, std::max<size_t>(tb, 16));
    size_t tbytes = tmp.bytes();
    // pass 1: the whole key
    OCHK(rocprim::radix_sort_pairs(tmp.as<void>(), tbytes, key.as<rocprim::uint128_t>(),
                                   key2.as<rocprim::uint128_t>(), idx.as<uint32_t>(),
                                   idx2.as<uint32_t>(), ni, 0, 128, s));
    std::swap(idx, idx2);
    // pass 2: instance (a batch), in the order of pass 1 (stable)
    if (n_inst > 1) {
        uint32_t ib = 1;
        while (ib < 32 && (n_inst - 1) >> ib) ib++;
        hipLaunchKernelGGL(k_gather<uint32_t>, dim3(grid_for(n)), dim3(kOrdBlock), 0, s,
                           inst.as<uint32_t>(), idx.as<uint32_t>(), n, inst2.as<uint32_t>());
        OCHK(hipGetLastError());
        tbytes = tmp.bytes();
        OCHK(rocprim::radix_sort_pairs(tmp.as<void>(), tbytes, inst2.as<uint32_t>(),
                                                inst.as<uint32_t>(), idx.as<uint32_t>(),
                                                idx2.as<uint32_t>(), ni, 0, (int)ib, s));
        std::swap(idx, idx2);
    }
    // lengths, their scan, then items and supports
    OENSURE(len, (n + 1) * 4);
    OENSURE(ioff, (n + 1) * 8);
    hipLaunchKernelGGL(k_lengths, dim3(grid_for(n + 1)), dim3(kOrdBlock), 0, s, d_rec,
                       idx.as<uint32_t>(), n, d_bits.as<uint32_t>(), len.as<uint32_t>());
    OCHK(hipGetLastError());
    tbytes = tmp.bytes();
    OCHK(rocprim::exclusive_scan(tmp.as<void>(), tbytes, len.as<uint32_t>(), ioff.as<unsigned long long>(), 0ull, (size_t)(ni + 1), rocprim::plus<unsigned long long>(), s));
    // The item count is known on the device only.  A small result is
    // decoded into room for the most items its keys can hold and copied
    // without waiting for the count (the host arrays are cut to it after);
    // a large one waits for the count first, so that no slack is copied.
    uint32_t max_codes = 1;
    for (uint32_t b : bits_of) max_codes = std::max<uint32_t>(max_codes, 128 / std::max<uint32_t>(b, 1));
    const uint64_t bound = (uint64_t)n * max_codes;
    const bool small = bound * 4 <= (8u << 20);
    unsigned long long total = 0;
    if (!small) {
        OCHK(hipMemcpyAsync(&total, ioff.as<unsigned long long>() + n, 8, hipMemcpyDeviceToHost, s));
        OCHK(stream_wait(s));
    }
    const uint64_t room = small ? bound : total;
    OENSURE(d_items, std::max<uint64_t>(room, 1) * 4);
    OENSURE(d_supp, n * 4);
    OENSURE(d_first, n_inst * 8);
    OCHK(launch_fill_u32(d_first.as<uint32_t>(), (uint64_t)n_inst * 2, 0xFFFFFFFFu, s));
    hipLaunchKernelGGL(k_decode, dim3(grid_for(n)), dim3(kOrdBlock), 0, s, d_rec, idx.as<uint32_t>(),
                       n, d_bits.as<uint32_t>(), ioff.as<unsigned long long>(),
                       d_items.as<uint32_t>(), d_supp.as<uint32_t>(),
                       d_first.as<unsigned long long>());
    OCHK(hipGetLastError());
    off.resize(n + 1);
    items.resize(room);
    supp.resize(n);
    OCHK(hipMemcpyAsync(off.data(), ioff.as<void>(), (n + 1) * 8, hipMemcpyDeviceToHost, s));
    if (room)
        OCHK(hipMemcpyAsync(items.data(), d_items.as<void>(), room * 4, hipMemcpyDeviceToHost, s));
    OCHK(hipMemcpyAsync(supp.data(), d_supp.as<void>(), n * 4, hipMemcpyDeviceToHost, s));
    std::vector<unsigned long long> f(n_inst);
    OCHK(hipMemcpyAsync(f.data(), d_first.as<void>(), n_inst * 8, hipMemcpyDeviceToHost, s));
    OCHK(stream_wait(s));
    if (small) {
        total = off[n];
        if (total > room) return set_error(FIM_E_DEVICE, "ordering: more items than keys hold");
        items.resize(total);
    }
    for (uint32_t q = 0; q < n_inst; q++) first[q] = f[q];
    return FIM_OK;
}

}  // namespace fim
