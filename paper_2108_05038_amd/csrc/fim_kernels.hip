// HIP kernels of the frequent-itemset miner, written for gfx950 (CDNA4,
// wave64).  Support counting is integer AND + popcount over vertical
// transaction bitmaps (the bitmap form of the thesis's lemma that the
// support of an itemset is the size of the intersection of the tid-lists of
// two of its covering subsets, appendix "The Eclat algorithm", subsection
// "Support counting").  No MFMA: the work is bitwise, and most of it is
// bound by memory or by the integer vector ALU.
#include <algorithm>
#include <atomic>

#include "fim_internal.h"

namespace fim {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t popc4(uint4 a, uint4 b) {
    return __popc(a.x & b.x) + __popc(a.y & b.y) + __popc(a.z & b.z) + __popc(a.w & b.w);
}

// acc + popcount(x) as one v_bcnt_u32_b32 (the compiler would sum the
// popcounts of a chunk with separate adds: a fifth more VALU operations)
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// acc += popcount(a AND b) over a 128-bit chunk
__device__ __forceinline__ void acc_popc4(uint32_t &acc, uint4 a, uint4 b) {
    acc = bcnt_acc(a.x & b.x, acc);
    acc = bcnt_acc(a.y & b.y, acc);
    acc = bcnt_acc(a.z & b.z, acc);
    acc = bcnt_acc(a.w & b.w, acc);
}

__device__ __forceinline__ uint4 and4(uint4 a, uint4 b) {
    return make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w);
}

// dst = a AND b over C chunks, the wave's lanes striding by 64, four
// chunks in flight per lane
__device__ __forceinline__ void and_rows(uint4 *dst, const uint4 *a, const uint4 *b, uint32_t C,
                                         uint32_t lane) {
    uint32_t c = lane;
    for (; c + 3 * kWave < C; c += 4 * kWave) {
        const uint4 a0 = a[c], b0 = b[c], a1 = a[c + kWave], b1 = b[c + kWave];
        const uint4 a2 = a[c + 2 * kWave], b2 = b[c + 2 * kWave];
        const uint4 a3 = a[c + 3 * kWave], b3 = b[c + 3 * kWave];
        dst[c] = and4(a0, b0);
        dst[c + kWave] = and4(a1, b1);
        dst[c + 2 * kWave] = and4(a2, b2);
        dst[c + 3 * kWave] = and4(a3, b3);
    }
    for (; c < C; c += kWave) dst[c] = and4(a[c], b[c]);
}

// number of set bits of `mask` in lanes below this one
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// a value every lane holds alike, moved to a scalar register
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = __shfl((uint32_t)v, src, kWave);
    uint32_t hi = __shfl((uint32_t)(v >> 32), src, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// lane q's value (q the same in every lane) in scalar registers: a register
// read, not a trip through the LDS crossbar
__device__ __forceinline__ uint32_t lane_val(uint32_t v, uint32_t q) { return __builtin_amdgcn_readlane(v, q); }
__device__ __forceinline__ uint64_t lane_val64(uint64_t v, uint32_t q) {
    return ((uint64_t)lane_val((uint32_t)(v >> 32), q) << 32) | lane_val((uint32_t)v, q);
}
// lane 0's value; for wave-uniform points of the code only
__device__ __forceinline__ uint64_t bcast64(uint64_t v) { return lane_val64(v, 0); }
__device__ __forceinline__ uint32_t bcast32(uint32_t v) { return lane_val(v, 0); }

// Blocks are dispatched round-robin over the 8 XCDs of the chip.  Renumber
// them so that each XCD receives a contiguous range of logical block ids,
// which keeps neighbouring tiles (sharing rows) in the same L2.
__device__ __forceinline__ uint32_t xcd_local_block(uint32_t b, uint32_t nblocks) {
    constexpr uint32_t kXcd = 8;
    uint32_t q = nblocks / kXcd, rmd = nblocks % kXcd;
    uint32_t x = b % kXcd, l = b / kXcd;
    uint32_t start = x < rmd ? x * (q + 1) : rmd * (q + 1) + (x - rmd) * q;
    return start + l;
}

// ------------------------------------------------------------------ a2: item supports

// Up to kHistItems item ids: block b histograms its chunk of the item array
// in LDS and stores the histogram at part[b * n_item_ids ..]; k_item_sum adds
// the block histograms up per item (no contended global atomics).  More item
// ids: global atomics straight into counts.
constexpr uint32_t kHistItems = 12288;

__global__ __launch_bounds__(kBlock) void k_item_hist(const uint32_t *__restrict__ items,
                                                       uint64_t nnz, uint64_t chunk,
                                                       uint32_t n_item_ids, uint32_t *part) {
    extern __shared__ uint32_t hist[];
    for (uint32_t i = threadIdx.x; i < n_item_ids; i += kBlock) hist[i] = 0;
    __syncthreads();
    const uint64_t a = (uint64_t)blockIdx.x * chunk, e = min(nnz, a + chunk);
    for (uint64_t p = a + threadIdx.x; p < e; p += kBlock)
        atomicAdd(&hist[items[p]], 1u);  // transactions are duplicate-free after ingest
    __syncthreads();
    uint32_t *dst = part + (uint64_t)blockIdx.x * n_item_ids;
    for (uint32_t i = threadIdx.x; i < n_item_ids; i += kBlock) dst[i] = hist[i];
}

// 64 items per block; the block's four waves add a quarter of the block
// histograms each (independent loads), then combine in LDS
__global__ __launch_bounds__(kBlock) void k_item_sum(const uint32_t *__restrict__ part, uint32_t nb,
                                                      uint32_t n_item_ids, uint32_t *counts) {
    __shared__ uint32_t acc[kWavesPerBlock][kWave];
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint32_t i = blockIdx.x * kWave + lane;
    uint32_t c = 0;
    if (i < n_item_ids)
        for (uint32_t b = wv; b < nb; b += kWavesPerBlock) c += part[(uint64_t)b * n_item_ids + i];
    acc[wv][lane] = c;
    __syncthreads();
    if (wv == 0 && i < n_item_ids) {
        uint32_t sum = 0;
#pragma unroll
        for (int q = 0; q < kWavesPerBlock; q++) sum += acc[q][lane];
        counts[i] = sum;
    }
}

__global__ __launch_bounds__(kBlock) void k_item_count(const uint32_t *__restrict__ items,
                                                        uint64_t nnz, uint32_t *counts) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < nnz; p += stride)
        atomicAdd(&counts[items[p]], 1u);
}

// Several instances at once: block b belongs to the instance whose block
// range holds it (binary search over first_block) and counts its chunk of
// kCountChunk items in LDS (up to kHistItems item ids; more: global atomics
// per item), then adds its non-zero bins to the instance's supports.
constexpr uint64_t kCountChunk = 1ull << 18;

__global__ __launch_bounds__(kBlock) void k_item_count_many(const CountSrc *__restrict__ src,
                                                             uint32_t n_src, uint32_t *counts) {
    extern __shared__ uint32_t hist[];
    const uint32_t b = blockIdx.x;
    uint32_t lo = 0, hi = n_src;  // src[lo].first_block <= b < src[hi].first_block
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (src[mid].first_block <= b) lo = mid;
        else hi = mid;
    }
    const CountSrc S = src[lo];
    const uint64_t a = (uint64_t)(b - S.first_block) * kCountChunk, e = min(S.nnz, a + kCountChunk);
    uint32_t *dst = counts + S.out;
    if (S.n_item_ids > kHistItems) {
        for (uint64_t p = a + threadIdx.x; p < e; p += kBlock) atomicAdd(&dst[S.items[p]], 1u);
        return;
    }
    for (uint32_t i = threadIdx.x; i < S.n_item_ids; i += kBlock) hist[i] = 0;
    __syncthreads();
    for (uint64_t p = a + threadIdx.x; p < e; p += kBlock) atomicAdd(&hist[S.items[p]], 1u);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < S.n_item_ids; i += kBlock)
        if (hist[i]) atomicAdd(&dst[i], hist[i]);
}

// n words: the 64-bit value v at words [at, at + 2), zero elsewhere
__global__ void k_fill_words(uint32_t *p, uint64_t n, uint64_t at, unsigned long long v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = i == at ? (uint32_t)v : i == at + 1 ? (uint32_t)(v >> 32) : 0u;
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ------------------------------------------------------------------ a3: bitmap build
// A block owns kBuildTx consecutive transactions and walks their item
// positions with consecutive threads (coalesced loads); a thread finds the
// transaction of its position by binary search over the block's offsets in
// LDS and sets bit t % 32 of word t / 32 of the item's row.  kBuildTx is a
// multiple of 32 and blocks start at multiples of it, so every row word is
// written by one block only: its atomic OR needs workgroup scope (done in the
// L2 of the block's XCD) rather than device scope; the rows reach memory at
// the end of the kernel.

constexpr uint32_t kBuildTx = 256;
static_assert(kBuildTx % 32 == 0, "a row word must belong to one block");

__global__ __launch_bounds__(kBlock) void k_bitmap_build(const uint64_t *__restrict__ offsets,
                                                          const uint32_t *__restrict__ items,
                                                          uint64_t n_tx,
                                                          const uint32_t *__restrict__ rank_of_item,
                                                          uint32_t *rows, uint32_t Wp) {
    __shared__ uint64_t s_off[kBuildTx + 1];
    const uint64_t t0 = (uint64_t)blockIdx.x * kBuildTx;
    const uint32_t nt = (uint32_t)min<uint64_t>(kBuildTx, n_tx - t0);
    for (uint32_t e = threadIdx.x; e <= nt; e += kBlock) s_off[e] = offsets[t0 + e];
    __syncthreads();
    const uint64_t p0 = s_off[0], p1 = s_off[nt];
    for (uint64_t pb = p0; pb < p1; pb += 2 * kBlock) {
        // two positions per thread, their loads issued together
        uint32_t r[2];
        uint64_t p[2];
#pragma unroll
        for (int j = 0; j < 2; j++) {
            p[j] = pb + j * kBlock + threadIdx.x;
            r[j] = p[j] < p1 ? items[p[j]] : kNone;
        }
#pragma unroll
        for (int j = 0; j < 2; j++) r[j] = r[j] != kNone ? rank_of_item[r[j]] : kNone;
#pragma unroll
        for (int j = 0; j < 2; j++) {
            if (r[j] == kNone) continue;
            uint32_t lo = 0, hi = nt;  // s_off[lo] <= p < s_off[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (s_off[mid] <= p[j]) lo = mid;
                else hi = mid;
            }
            const uint64_t t = t0 + lo;
            __hip_atomic_fetch_or(&rows[(uint64_t)r[j] * Wp + (t >> 5)], 1u << (t & 31),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

// Column tiles: a block owns words [w K, w K + K) of the rows [r0, r0 + nr)
// of one row group, i.e. those rows' bits of the transactions [32 w K,
// 32 (w + 1) K).  It sets them in an LDS copy of the tile (nr x K words, LDS
// atomics), skipping the items of other row groups, and writes the tile out
// once, K words per row, zeros included: no global atomics, no separate zero
// fill, and the padding words past the last transaction come out zero as
// well.  With K = 32 every row piece is one 128-byte line; row groups keep
// the tile small enough for several blocks per CU, and the blocks of one
// column window run on one XCD, so that its transactions are read from that
// XCD's L2 by all of its row groups.
constexpr uint32_t kTileMaxWords = 32;

__global__ __launch_bounds__(kBlock) void k_bitmap_tile(const uint64_t *__restrict__ offsets,
                                                         const uint32_t *__restrict__ items,
                                                         uint64_t n_tx,
                                                         const uint32_t *__restrict__ rank_of_item,
                                                         uint32_t n, uint32_t *rows, uint32_t Wp,
                                                         uint32_t K, uint32_t nr, uint32_t n_groups) {
    extern __shared__ uint4 tile4[];  // nr * K words, 16-byte aligned
    uint32_t *tile = reinterpret_cast<uint32_t *>(tile4);
    __shared__ uint64_t s_off[32 * kTileMaxWords + 1];
    const uint32_t L = xcd_local_block(blockIdx.x, gridDim.x);
    const uint32_t grp = L % n_groups, win = L / n_groups;
    const uint32_t r0 = grp * nr, nrr = min(nr, n - r0);
    const uint32_t wb = win * K;
    const uint32_t kw = min(K, Wp - wb);  // a multiple of 4 (K and Wp are)
    for (uint32_t e = threadIdx.x; e < nrr * K / 4; e += kBlock) tile4[e] = make_uint4(0u, 0u, 0u, 0u);
    const uint64_t t0 = (uint64_t)wb * 32;
    const uint32_t nt = t0 < n_tx ? (uint32_t)min<uint64_t>((uint64_t)kw * 32, n_tx - t0) : 0u;
    for (uint32_t e = threadIdx.x; nt > 0 && e <= nt; e += kBlock) s_off[e] = offsets[t0 + e];
    __syncthreads();
    if (nt > 0) {
        // kTileUnroll positions per thread at a time: their item and rank
        // loads are unconditional (indices clamped into the block's range)
        // so that they are all in flight together
        constexpr uint32_t kTileUnroll = 8;
        const uint64_t p0 = s_off[0], p1 = s_off[nt];
        for (uint64_t pb = p0; pb < p1; pb += kTileUnroll * kBlock) {
            uint32_t r[kTileUnroll];
#pragma unroll
            for (uint32_t j = 0; j < kTileUnroll; j++) {
                const uint64_t p = pb + j * kBlock + threadIdx.x;
                r[j] = items[p < p1 ? p : p1 - 1];
            }
#pragma unroll
            for (uint32_t j = 0; j < kTileUnroll; j++) r[j] = rank_of_item[r[j]];
#pragma unroll
            for (uint32_t j = 0; j < kTileUnroll; j++) {
                const uint64_t p = pb + j * kBlock + threadIdx.x;
                const uint32_t rr = r[j] - r0;  // kNone and other groups' ranks fall outside
                if (p >= p1 || r[j] == kNone || rr >= nrr) continue;
                uint32_t lo = 0, hi = nt;  // s_off[lo] <= p < s_off[hi]
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_off[mid] <= p) lo = mid;
                    else hi = mid;
                }
                atomicOr(&tile[rr * K + (lo >> 5)], 1u << (lo & 31));
            }
        }
    }
    __syncthreads();
    const uint32_t q4 = kw / 4;  // 16-byte pieces per row
    for (uint32_t e = threadIdx.x; e < nrr * q4; e += kBlock) {
        const uint32_t r = e / q4, q = e % q4;
        const uint4 v = *reinterpret_cast<const uint4 *>(tile + r * K + 4 * q);
        *reinterpret_cast<uint4 *>(rows + (uint64_t)(r0 + r) * Wp + wb + 4 * q) = v;
    }
}

// ------------------------------------------------------------------ a6/a7: root class pairs
// The root class [{} | all frequent items]: the upper triangle of the
// popcount-Gram of the item rows.  A block owns a 64 x 64 tile of pairs;
// word tiles of both row blocks are staged in LDS, so every loaded word is
// reused by 64 pairs; each thread keeps a 4 x 4 block of accumulators.

constexpr int kRootRows = 64;
constexpr int kRootTw = 32;  // words per LDS tile
// Word-range splits: a launch with few tiles over long rows leaves most CUs
// idle, so the words are cut into ranges counted by separate blocks (at
// least kRootSplitMinWords each, at most kRootSplitBlocks blocks in all);
// each block writes its 64 x 64 partial counts and k_root_finish sums them.
constexpr uint32_t kRootSplitMinWords = 256;
constexpr uint32_t kRootSplitBlocks = 512;
constexpr uint32_t kRootTilePairs = kRootRows * kRootRows;

// logical tile index b -> (bi <= bj) in the upper triangle of tiles
__device__ inline void root_tile_of(uint32_t b, uint32_t &bi, uint32_t &bj) {
    bj = (uint32_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((uint64_t)bj * (bj + 1) / 2 > b) bj--;
    while ((uint64_t)(bj + 1) * (bj + 2) / 2 <= b) bj++;
    bi = b - bj * (bj + 1) / 2;
}

// threshold the 4 x 4 supports of a thread, then compact the frequent
// pairs of the wave with one atomic
__device__ inline void root_emit(const uint32_t (&acc)[4][4], uint32_t I0, uint32_t J0, uint32_t n,
                                 uint32_t minsup, uint32_t *pairs, uint64_t cap,
                                 unsigned long long *n_pairs) {
    const uint32_t tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    uint32_t mine = 0;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 4; c++) {
            uint32_t i = I0 + ty + 16 * a, j = J0 + tx + 16 * c;
            bool ok = i < n && j < n && i < j && acc[a][c] >= minsup;
            mine += ok ? 1u : 0u;
        }
    // exclusive scan of `mine` over the wave
    uint32_t incl = mine;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t v = __shfl_up(incl, off, kWave);
        if ((int)lane_id() >= off) incl += v;
    }
    uint32_t total = __shfl(incl, kWave - 1, kWave);
    unsigned long long base = 0;
    if (lane_id() == 0 && total) base = atomicAdd(n_pairs, (unsigned long long)total);
    base = shfl_u64(base, 0);
    uint64_t pos = base + incl - mine;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 4; c++) {
            uint32_t i = I0 + ty + 16 * a, j = J0 + tx + 16 * c;
            if (i < n && j < n && i < j && acc[a][c] >= minsup) {
                if (pos < cap) {
                    pairs[3 * pos + 0] = i;
                    pairs[3 * pos + 1] = j;
                    pairs[3 * pos + 2] = acc[a][c];
                }
                pos++;
            }
        }
}

// blockIdx.x = tile, blockIdx.y = word range [y * chunk, min((y + 1) * chunk, Wp));
// part == nullptr: one range, pairs emitted here; else the partial counts go
// to part[(y * gridDim.x + tile) * kRootTilePairs + (4a + c) * kBlock + thread]
__global__ __launch_bounds__(kBlock) void k_root_pairs(const uint32_t *__restrict__ rows,
                                                        uint32_t n, uint32_t Wp, uint32_t chunk,
                                                        uint32_t minsup, uint32_t *pairs, uint64_t cap,
                                                        unsigned long long *n_pairs,
                                                        uint32_t *__restrict__ part) {
    __shared__ uint32_t sI[kRootRows][kRootTw + 1];
    __shared__ uint32_t sJ[kRootRows][kRootTw + 1];

    const uint32_t b = xcd_local_block(blockIdx.x, gridDim.x);
    uint32_t bi, bj;
    root_tile_of(b, bi, bj);
    const uint32_t I0 = bi * kRootRows, J0 = bj * kRootRows;
    const uint32_t wb = blockIdx.y * chunk;
    const uint32_t we = (uint32_t)min<uint64_t>((uint64_t)wb + chunk, Wp);

    const uint32_t tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    uint32_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 4; c++) acc[a][c] = 0;

    for (uint32_t w0 = wb; w0 < we; w0 += kRootTw) {
        // 64 rows x 32 words per side = 512 uint4; 2 per thread per side
#pragma unroll
        for (int q = 0; q < 2; q++) {
            uint32_t idx = threadIdx.x + q * kBlock;  // 0..511
            uint32_t row = idx >> 3, c4 = (idx & 7) * 4;
            uint4 vi = make_uint4(0, 0, 0, 0), vj = make_uint4(0, 0, 0, 0);
            if (w0 + c4 < we) {
                if (I0 + row < n)
                    vi = *reinterpret_cast<const uint4 *>(rows + (uint64_t)(I0 + row) * Wp + w0 + c4);
                if (J0 + row < n)
                    vj = *reinterpret_cast<const uint4 *>(rows + (uint64_t)(J0 + row) * Wp + w0 + c4);
            }
            sI[row][c4 + 0] = vi.x;
            sI[row][c4 + 1] = vi.y;
            sI[row][c4 + 2] = vi.z;
            sI[row][c4 + 3] = vi.w;
            sJ[row][c4 + 0] = vj.x;
            sJ[row][c4 + 1] = vj.y;
            sJ[row][c4 + 2] = vj.z;
            sJ[row][c4 + 3] = vj.w;
        }
        __syncthreads();
#pragma unroll 4
        for (int w = 0; w < kRootTw; w++) {
            uint32_t x[4], y[4];
#pragma unroll
            for (int a = 0; a < 4; a++) x[a] = sI[ty + 16 * a][w];
#pragma unroll
            for (int c = 0; c < 4; c++) y[c] = sJ[tx + 16 * c][w];
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int c = 0; c < 4; c++) acc[a][c] += __popc(x[a] & y[c]);
        }
        __syncthreads();
    }

    if (part) {
        uint32_t *dst = part + ((uint64_t)blockIdx.y * gridDim.x + b) * kRootTilePairs + threadIdx.x;
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 4; c++) dst[(4 * a + c) * kBlock] = acc[a][c];
        return;
    }
    root_emit(acc, I0, J0, n, minsup, pairs, cap, n_pairs);
}

// sums the `splits` partial counts of each tile written by k_root_pairs,
// then emits its frequent pairs
__global__ __launch_bounds__(kBlock) void k_root_finish(const uint32_t *__restrict__ part,
                                                         uint32_t splits, uint32_t n, uint32_t minsup,
                                                         uint32_t *pairs, uint64_t cap,
                                                         unsigned long long *n_pairs) {
    const uint32_t b = xcd_local_block(blockIdx.x, gridDim.x);
    uint32_t bi, bj;
    root_tile_of(b, bi, bj);
    uint32_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 4; c++) acc[a][c] = 0;
    for (uint32_t y = 0; y < splits; y++) {
        const uint32_t *src = part + ((uint64_t)y * gridDim.x + b) * kRootTilePairs + threadIdx.x;
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 4; c++) acc[a][c] += src[(4 * a + c) * kBlock];
    }
    root_emit(acc, bi * kRootRows, bj * kRootRows, n, minsup, pairs, cap, n_pairs);
}

// ------------------------------------------------------------------ a6/a7: root class over covers
// The pairs (i, j > i) of the root class counted only over the words where
// row i (the sparser one: rows ascend by support) is non-zero, i.e. over
// the cover of the first-level prefix {a_i}.  The other words add nothing
// to popcount(row_i AND row_j), so the supports are the same.  Row i's
// non-zero words and their masks are listed once (k_row_nonzero); the rows
// are transposed word-major (k_transpose), so that for one word of row i the
// lanes of a block read consecutive partner rows j with 128-bit loads.

// one wave per row: the row's non-zero words, compacted with ballot/mbcnt
__global__ __launch_bounds__(kBlock) void k_row_nonzero(const uint32_t *__restrict__ rows,
                                                         uint32_t n, uint32_t Wp,
                                                         const uint64_t *__restrict__ nz_off,
                                                         uint32_t *nz_w, uint32_t *nz_m,
                                                         uint32_t *nz_cnt) {
    const uint32_t r = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (r >= n) return;
    const uint32_t lane = lane_id();
    const uint32_t *row = rows + (uint64_t)r * Wp;
    const uint64_t base = nz_off[r], cap = nz_off[r + 1] - base;
    uint32_t cnt = 0;
    for (uint32_t w0 = 0; w0 < Wp; w0 += kWave) {
        const uint32_t w = w0 + lane;
        const uint32_t x = w < Wp ? row[w] : 0u;
        const uint64_t mask = __ballot(x != 0u);
        if (x) {
            const uint32_t p = cnt + lanes_below(mask);
            if (p < cap) {
                nz_w[base + p] = w;
                nz_m[base + p] = x;
            }
        }
        cnt += (uint32_t)__popcll(mask);
    }
    if (lane == 0) nz_cnt[r] = cnt < cap ? cnt : (uint32_t)cap;
}

// bt[w * np + j] = rows[j * Wp + w] for w < W, j < np (zero for j >= n)
__global__ __launch_bounds__(kBlock) void k_transpose(const uint32_t *__restrict__ rows, uint32_t n,
                                                       uint32_t Wp, uint32_t W, uint32_t *bt,
                                                       uint32_t np) {
    __shared__ uint32_t tile[64][65];
    const uint32_t w0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const uint32_t tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (uint32_t r = ty; r < 64; r += 4) {
        const uint32_t j = j0 + r, w = w0 + tx;
        tile[r][tx] = (j < n && w < W) ? rows[(uint64_t)j * Wp + w] : 0u;
    }
    __syncthreads();
    for (uint32_t r = ty; r < 64; r += 4) {
        const uint32_t w = w0 + r, j = j0 + tx;
        if (w < W && j < np) bt[(uint64_t)w * np + j] = tile[tx][r];
    }
}

constexpr uint32_t kSparseCols = 4 * kBlock;  // partner rows per block

// block (jb, i): row i against partners j in [jb * 1024, jb * 1024 + 1024),
// four per thread
__global__ __launch_bounds__(kBlock) void k_root_sparse(
    const uint32_t *__restrict__ bt, uint32_t np, const uint64_t *__restrict__ nz_off,
    const uint32_t *__restrict__ nz_cnt, const uint32_t *__restrict__ nz_w,
    const uint32_t *__restrict__ nz_m, uint32_t n, uint32_t minsup, uint32_t *pairs, uint64_t cap,
    unsigned long long *n_pairs) {
    const uint32_t i = blockIdx.y;
    const uint32_t jb0 = blockIdx.x * kSparseCols;
    if (jb0 + kSparseCols <= i + 1) return;  // no partner j > i in this block
    const uint32_t j0 = jb0 + threadIdx.x * 4;
    const uint64_t base = nz_off[i];
    const uint32_t cnt = nz_cnt[i];
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    if (j0 < np) {
        const uint32_t *col = bt + j0;
        uint32_t k = 0;
        for (; k + 4 <= cnt; k += 4) {
            const uint32_t w0 = nz_w[base + k], w1 = nz_w[base + k + 1];
            const uint32_t w2 = nz_w[base + k + 2], w3 = nz_w[base + k + 3];
            const uint32_t m0 = nz_m[base + k], m1 = nz_m[base + k + 1];
            const uint32_t m2 = nz_m[base + k + 2], m3 = nz_m[base + k + 3];
            const uint4 x0 = *reinterpret_cast<const uint4 *>(col + (uint64_t)w0 * np);
            const uint4 x1 = *reinterpret_cast<const uint4 *>(col + (uint64_t)w1 * np);
            const uint4 x2 = *reinterpret_cast<const uint4 *>(col + (uint64_t)w2 * np);
            const uint4 x3 = *reinterpret_cast<const uint4 *>(col + (uint64_t)w3 * np);
            a0 += __popc(m0 & x0.x) + __popc(m1 & x1.x) + __popc(m2 & x2.x) + __popc(m3 & x3.x);
            a1 += __popc(m0 & x0.y) + __popc(m1 & x1.y) + __popc(m2 & x2.y) + __popc(m3 & x3.y);
            a2 += __popc(m0 & x0.z) + __popc(m1 & x1.z) + __popc(m2 & x2.z) + __popc(m3 & x3.z);
            a3 += __popc(m0 & x0.w) + __popc(m1 & x1.w) + __popc(m2 & x2.w) + __popc(m3 & x3.w);
        }
        for (; k < cnt; k++) {
            const uint32_t m = nz_m[base + k];
            const uint4 x = *reinterpret_cast<const uint4 *>(col + (uint64_t)nz_w[base + k] * np);
            a0 += __popc(m & x.x);
            a1 += __popc(m & x.y);
            a2 += __popc(m & x.z);
            a3 += __popc(m & x.w);
        }
    }
    const uint32_t acc[4] = {a0, a1, a2, a3};
    uint32_t mine = 0;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const uint32_t j = j0 + c;
        mine += (j > i && j < n && acc[c] >= minsup) ? 1u : 0u;
    }
    uint32_t incl = mine;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, kWave);
        if ((int)lane_id() >= off) incl += v;
    }
    const uint32_t total = __shfl(incl, kWave - 1, kWave);
    unsigned long long b = 0;
    if (lane_id() == 0 && total) b = atomicAdd(n_pairs, (unsigned long long)total);
    b = shfl_u64(b, 0);
    uint64_t pos = b + incl - mine;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const uint32_t j = j0 + c;
        if (j > i && j < n && acc[c] >= minsup) {
            if (pos < cap) {
                pairs[3 * pos + 0] = i;
                pairs[3 * pos + 1] = j;
                pairs[3 * pos + 2] = acc[c];
            }
            pos++;
        }
    }
}

// ------------------------------------------------------------------ a6/a7: root class over projected transactions
// supp({a, b}) is the number of transactions of the cover T(a) that also
// hold b, i.e. the support of b in the database projected on T(a).  The
// transactions are kept as ascending lists of frequent ranks, each closed by
// kRankEnd (larger than any rank), and every entry of the tid list of a
// points at a's own position in its transaction (both built by sorting the
// occurrences).  A block counts the pairs (a, b > a) of a few consecutive
// rows a in LDS: for every transaction of T(a) it reads the ranks after a's
// position up to the end mark.  The work is the number of pairs inside the
// transactions, independent of the bitmap width, which is what makes it the
// choice for long sparse rows.

constexpr uint32_t kRankEnd = 0xFFFFFFFFu;  // equal to kNone: infrequent items sort last
constexpr uint16_t kRankEnd16 = 0xFFFFu;    // the same in the 16-bit ranked transactions

// tl[tl_off[r] ..) = the transactions holding rank r, ascending: the set
// bits of row r, one wave per row, compacted with a wave prefix sum of the
// words' popcounts; tl_rank (or null) receives r for every entry.
__global__ __launch_bounds__(kBlock) void k_tidlist(const uint32_t *__restrict__ rows, uint32_t n,
                                                     uint32_t Wp, const uint64_t *__restrict__ tl_off,
                                                     uint32_t *tl, uint16_t *tl_rank) {
    const uint32_t r = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (r >= n) return;
    const uint32_t lane = lane_id();
    const uint32_t *row = rows + (uint64_t)r * Wp;
    const uint64_t base = tl_off[r], end = tl_off[r + 1];
    uint32_t pos = 0;  // set bits before the current window
    // 4 x 64 words per round: the loads of a window are in flight together
    constexpr int kTlUnroll = 4;
    for (uint32_t w0 = 0; w0 < Wp; w0 += kTlUnroll * kWave) {
        uint32_t x[kTlUnroll];
#pragma unroll
        for (int j = 0; j < kTlUnroll; j++) {
            const uint32_t w = w0 + j * kWave + lane;
            x[j] = w < Wp ? row[w] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kTlUnroll; j++) {
            const uint32_t w = w0 + j * kWave + lane;
            const uint32_t pc = __popc(x[j]);
            uint32_t incl = pc;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const uint32_t v = __shfl_up(incl, o, kWave);
                if ((int)lane >= o) incl += v;
            }
            uint64_t q = base + pos + incl - pc;
            uint32_t y = x[j];
            while (y) {
                const uint32_t b = __ffs(y) - 1;
                if (q < end) {
                    tl[q] = w * 32 + b;
                    if (tl_rank != nullptr) tl_rank[q] = (uint16_t)r;
                }
                q++;
                y &= y - 1;
            }
            pos += __shfl(incl, kWave - 1, kWave);
        }
    }
}

// Ranked transactions: transaction t's ranks ascending at rk[off[t] + t ..),
// its infrequent items' slots and one slot more holding kRankEnd16 (the
// infrequent items' rank kNone is stored as kRankEnd16 as well).  A wave
// takes kRankGroup transactions at a time (their loads overlap): every lane
// holds one item's rank of each and finds its slot by counting the smaller
// ranks (ties, only between infrequent items, by position).  A transaction of
// more than 64 items is done alone, 64 items at a time.  Every store is to
// the transaction's own contiguous slots.
constexpr uint32_t kRankGroup = 4;

__global__ __launch_bounds__(kBlock) void k_rank_tx(const uint64_t *__restrict__ off,
                                                     const uint32_t *__restrict__ items, uint64_t n_tx,
                                                     const uint32_t *__restrict__ rank_of_item,
                                                     uint16_t *rk) {
    const uint32_t lane = lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * kWavesPerBlock;
    const uint64_t n_groups = (n_tx + kRankGroup - 1) / kRankGroup;
    for (uint64_t g = (uint64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; g < n_groups;
         g += waves) {
        const uint64_t tg0 = g * kRankGroup;
        const uint32_t ng = (uint32_t)min<uint64_t>(kRankGroup, n_tx - tg0);
        uint64_t a[kRankGroup];
        uint32_t L[kRankGroup], r[kRankGroup];
        bool small = true;
#pragma unroll
        for (uint32_t j = 0; j < kRankGroup; j++) {
            a[j] = j < ng ? off[tg0 + j] : 0;
            L[j] = j < ng ? (uint32_t)(off[tg0 + j + 1] - a[j]) : 0u;
            // the same for every lane: kept in scalar registers
            a[j] = bcast64(a[j]);
            L[j] = __builtin_amdgcn_readfirstlane(L[j]);
            small = small && L[j] <= (uint32_t)kWave;
        }
        if (small) {
            // loads unconditional (indices clamped in bounds), so that the
            // group's loads are in flight together
#pragma unroll
            for (uint32_t j = 0; j < kRankGroup; j++)
                r[j] = items[L[j] ? a[j] + min(lane, L[j] - 1) : 0];
#pragma unroll
            for (uint32_t j = 0; j < kRankGroup; j++) {
                const uint32_t rr = rank_of_item[r[j]];
                r[j] = lane < L[j] ? rr : kNone;
            }
#pragma unroll
            for (uint32_t j = 0; j < kRankGroup; j++) {
                if (j >= ng) continue;
                uint32_t pos = 0;
                for (uint32_t i = 0; i < L[j]; i++) {
                    const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)r[j], (int)i);
                    pos += (v < r[j] || (v == r[j] && i < lane)) ? 1u : 0u;
                }
                const uint64_t base = a[j] + tg0 + j;
                if (lane < L[j]) rk[base + pos] = (uint16_t)r[j];  // kNone -> kRankEnd16
                if (lane == 0) rk[base + L[j]] = kRankEnd16;
            }
            continue;
        }
        // one transaction at a time, 64 items at a time
        for (uint32_t j = 0; j < ng; j++) {
            const uint64_t t = tg0 + j, base = a[j] + t;
            const uint32_t Lt = L[j];
            for (uint32_t c0 = 0; c0 < Lt; c0 += kWave) {
                const uint32_t c = c0 + lane;
                const uint32_t rc = c < Lt ? rank_of_item[items[a[j] + c]] : kNone;
                uint32_t p = 0;
                for (uint32_t d0 = 0; d0 < Lt; d0 += kWave) {
                    const uint32_t rd = d0 == c0 ? rc
                                                 : (d0 + lane < Lt ? rank_of_item[items[a[j] + d0 + lane]] : kNone);
                    const uint32_t cnt = min(Lt - d0, (uint32_t)kWave);
                    for (uint32_t i = 0; i < cnt; i++) {
                        const uint32_t v = __shfl(rd, (int)i, kWave);
                        p += (v < rc || (v == rc && d0 + i < c)) ? 1u : 0u;
                    }
                }
                if (c < Lt) rk[base + p] = (uint16_t)rc;
            }
            if (lane == 0) rk[base + Lt] = kRankEnd16;
        }
    }
}

// For every tid-list entry q of rank r = suf[q] (written there by
// k_tidlist) and transaction t = tl[q]: tlp[q] = the position of r among t's
// ranked slots, off[t] + t + s with rk[off[t] + t + s] = r, and suf[q] = the
// frequent ranks of t after it.  The L slots of t hold its frequent ranks
// ascending and then kRankEnd16 (infrequent items), so s is the number of
// slots below r and the frequent ranks the number of slots other than
// kRankEnd16: counted over 32 slots (one aligned 64-byte piece) at a time,
// loads issued together, rather than searched load by dependent load.  One
// thread per entry: the loads and stores of the lists are coalesced.  rk is
// padded by kRkPad slots so that a piece never reads past its end.
constexpr uint32_t kRkPad = 40;

__global__ __launch_bounds__(kBlock) void k_tl_slots(const uint64_t *__restrict__ off,
                                                      const uint16_t *__restrict__ rk,
                                                      const uint32_t *__restrict__ tl, uint64_t n_ent,
                                                      uint32_t *tlp, uint16_t *suf) {
    const uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n_ent) return;
    const uint32_t r = suf[q];
    const uint32_t t = tl[q];
    const uint64_t a = off[t];
    const uint64_t s0 = a + t, s1 = s0 + (off[t + 1] - a);  // slots [s0, s1)
    uint32_t below = 0, freq = 0;
    for (uint64_t c = s0 & ~uint64_t(31); c < s1; c += 32) {
        const uint4 *pc = reinterpret_cast<const uint4 *>(rk + c);
        const uint4 v[4] = {pc[0], pc[1], pc[2], pc[3]};
        const uint32_t w[16] = {v[0].x, v[0].y, v[0].z, v[0].w, v[1].x, v[1].y, v[1].z, v[1].w,
                                v[2].x, v[2].y, v[2].z, v[2].w, v[3].x, v[3].y, v[3].z, v[3].w};
#pragma unroll
        for (uint32_t k = 0; k < 32; k++) {
            const uint64_t slot = c + k;
            const uint32_t x = (w[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
            const bool in = slot >= s0 && slot < s1;
            below += (in && x < r) ? 1u : 0u;
            freq += (in && x != kRankEnd16) ? 1u : 0u;
        }
    }
    tlp[q] = (uint32_t)(s0 + below);
    suf[q] = (uint16_t)(freq - 1 - below);
}

constexpr uint32_t kProjectMaxRows = 64;

// block (x, y): rows [i0, i0 + R) (x counted from the last, heaviest rows)
// against partner columns [j0, j0 + J); counters cnt[R][J] in LDS
// One block per R consecutive rows a (and J columns from j0): LDS counters
// of the pairs (a, b), 32-bit, or 16-bit halves of 32-bit words (Packed)
// when no row's support exceeds 65535.  A wave takes 64 tid-list entries at
// a time; each entry (a, t) brings the position of a in t and the number of
// t's ranks after it (suf), and the wave lays those rank reads out flat
// (prefix sum of suf): lane x reads the x-th rank of the lot, found by a
// binary search over the prefix sums in LDS, so that every lane has a read
// in flight however the suffix lengths differ.
template <bool Packed>
__global__ __launch_bounds__(kBlock) void k_root_project(
    const uint16_t *__restrict__ rk, const uint32_t *__restrict__ tlp,
    const uint16_t *__restrict__ suf, const uint64_t *__restrict__ tl_off, uint32_t n, uint32_t R,
    uint32_t J, uint32_t minsup, uint32_t *pairs, uint64_t cap, unsigned long long *n_pairs,
    unsigned long long *work) {
    extern __shared__ uint32_t cnt[];
    __shared__ uint64_t s_off[kProjectMaxRows + 1];
    __shared__ uint32_t s_sc[kWavesPerBlock][kWave], s_q[kWavesPerBlock][kWave],
        s_a[kWavesPerBlock][kWave];
    const uint32_t nrb = (n + R - 1) / R;
    const uint32_t i0 = (nrb - 1 - blockIdx.x) * R, i1 = min(i0 + R, n);
    const uint32_t j0 = blockIdx.y * J, j1 = min(j0 + J, n);
    if (j1 <= i0 + 1) return;  // no pair (a, b > a) in this tile (uniform over the block)
    const uint32_t words = Packed ? (R * J + 1) / 2 : R * J;
    for (uint32_t e = threadIdx.x; e < words; e += kBlock) cnt[e] = 0;
    for (uint32_t e = threadIdx.x; e <= i1 - i0; e += kBlock) s_off[e] = tl_off[i0 + e];
    __syncthreads();
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    uint32_t *sc = s_sc[wv], *sq = s_q[wv], *sa = s_a[wv];
    unsigned long long wk = 0;
    const uint64_t p1 = s_off[i1 - i0];
    uint32_t a_rel = 0;
    // the entries' suffix lengths and positions are loaded one lot ahead, so
    // that their round trip overlaps the rank reads of the lot before
    const uint64_t pfirst = s_off[0] + (uint64_t)wv * kWave;
    uint32_t len_n = pfirst + lane < p1 ? suf[pfirst + lane] : 0u;
    uint32_t q0_n = pfirst + lane < p1 ? tlp[pfirst + lane] + 1 : 0u;
    for (uint64_t pb = pfirst; pb < p1; pb += kBlock) {
        const uint64_t p = pb + lane;
        const bool valid = p < p1;
        while (valid && s_off[a_rel + 1] <= p) a_rel++;  // p only grows: the row only grows
        const uint32_t len = len_n;
        const uint32_t q0 = q0_n;
        {
            const uint64_t pn = p + kBlock;
            len_n = pn < p1 ? suf[pn] : 0u;
            q0_n = pn < p1 ? tlp[pn] + 1 : 0u;
        }
        uint32_t incl = len;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o, kWave);
            if ((int)lane >= o) incl += v;
        }
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        sc[lane] = incl - len;
        sq[lane] = q0;
        sa[lane] = a_rel;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        constexpr uint32_t kReads = 8;  // rank reads per lane in flight
        for (uint32_t k0 = 0; k0 < total; k0 += kReads * kWave) {
            uint32_t b[kReads], row[kReads];
#pragma unroll
            for (uint32_t u = 0; u < kReads; u++) {
                const uint32_t k = k0 + u * kWave + lane;
                b[u] = kRankEnd;
                row[u] = 0;
                if (k < total) {
                    uint32_t lo = 0, hi = kWave;  // sc[lo] <= k < sc[hi] (sc[64] = total)
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (sc[mid] <= k) lo = mid;
                        else hi = mid;
                    }
                    b[u] = rk[sq[lo] + (k - sc[lo])];
                    row[u] = sa[lo];
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < kReads; u++) {
                if (b[u] < j0 || b[u] >= j1) continue;
                const uint32_t e = row[u] * J + (b[u] - j0);
                if (Packed) atomicAdd(&cnt[e >> 1], 1u << ((e & 1) * 16));
                else atomicAdd(&cnt[e], 1u);
                wk++;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    // frequent pairs of the tile, compacted per wave with one atomic
    for (uint32_t e0 = 0; e0 < R * J; e0 += kBlock) {
        const uint32_t e = e0 + threadIdx.x;
        const uint32_t a = i0 + e / J, b = j0 + e % J;
        uint32_t c = 0;
        if (e < R * J) c = Packed ? (cnt[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu : cnt[e];
        const bool ok = e < R * J && a < i1 && b < j1 && b > a && c >= minsup;
        const uint64_t mask = __ballot(ok);
        unsigned long long base = 0;
        if (lane_id() == 0 && mask) base = atomicAdd(n_pairs, (unsigned long long)__popcll(mask));
        base = shfl_u64(base, 0);
        if (ok) {
            const uint64_t pos = base + lanes_below(mask);
            if (pos < cap) {
                pairs[3 * pos + 0] = a;
                pairs[3 * pos + 1] = b;
                pairs[3 * pos + 2] = c;
            }
        }
    }
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) wk += __shfl_xor(wk, o, kWave);
    if (lane_id() == 0 && wk) atomicAdd(work, wk);
}

// ------------------------------------------------------------------ a5-a8: persistent DFS
//
// Every wave is one worker with a private region of `stack_words` words:
// bitmap rows of the classes on its DFS path grow up from the bottom, atom
// lists grow down from the top.  A worker repeatedly claims tasks (rows
// [r0, r1) of a first-level class) from a global counter, materialises the
// class's sibling bitmaps along the prefix path (the thesis's
// Prepare-Tidlists for a prefix of length one), and runs
// Eclat-DFS-Computation below those rows.
//
// A class of at most kGramMax atoms is counted when it is built.  While its
// rows T(P + a_r + a_q) = T(P + a_r) AND T(P + a_q) are formed, word tile by
// word tile, the supports of all of its pairs (the popcount-Gram of the
// class) are accumulated from the same words, so every loaded word serves
// all pairs of the class: up to kRegGram atoms a lane keeps its 128-bit
// chunks of all rows and all pairs in registers; wider classes stage word
// tiles of their rows in LDS, and the (4x4 block, word slice) items of each
// tile are dealt to all lanes (see count_lds).  For every row the frequent later atoms, ordered by
// ascending support (ties by item id), become that row's child class, and
// the frequent pairs are reported.  Expanding row r then counts nothing: it
// builds the child class of row r in the same way.  A class of two atoms
// never writes its rows (its one pair is all there is to count).  Classes
// of more than kGramMax atoms (wide first-level classes) are counted block
// by block instead: when row r is reached, the pairs of the next kWideRows
// rows with all later rows are counted in passes of the same Gram code
// (kWideRows rows against kGramMax - kWideRows later rows at a time) into a
// block of counts on the wave's stack, and each of those rows reads its
// counts when it is expanded, so a later row is loaded once per block of
// rows rather than once per row.

constexpr uint32_t kGramMax = 64;     // widest class counted when it is built
constexpr uint32_t kWideRows = 32;    // rows of a wide class counted per block
constexpr uint32_t kTileMin = 32;     // narrowest LDS row tile (words)
constexpr uint32_t kTileDefault = 256;  // widest LDS row tile unless the autotuner picks another
constexpr uint32_t kGx = 4640;        // LDS words per wave for row tiles and pair supports
constexpr uint32_t kMaxTileRows = 8;  // rows of a tile one lane loads (see count_lds)
constexpr uint32_t kListPad = kWave;  // list entries past a class's lists that a wave may read
static_assert(kGx >= kGramMax * (kGramMax - 1) / 2, "pair supports fit in the tile area");
static_assert(4 * ((kGramMax + 3) / 4) * (kTileMin + 4) +
                      17 * ((kGramMax + 3) / 4) * ((kGramMax + 3) / 4 + 1) / 2 <= kGx,
              "the widest class fits a narrowest tile with its block counts");

struct Frame {
    uint32_t rows_base;    // word offset of the class's row 0 (rows_top when it was pushed)
    uint32_t k;            // atoms (rows) of the class
    uint32_t r;            // next row to expand
    uint32_t r_end;        // rows [0, r_end) are expanded
    uint32_t atoms;        // word offset of ranks[k]; supports at +k, item ids at +2k,
                           // (counted classes) sizes of the rows' child classes at +3k
    uint32_t lists;        // counted classes: word offset of the child-class entries
                           // (rank, support, row, item id); kNone: pairs counted on expansion
    uint32_t lpos;         // counted classes: first entry of row r's child class;
                           // wide classes: rows of the block of counts
    uint32_t meta_restore; // meta pointer to restore when the class is done
    // counted classes: rows whose child class has at least two atoms (bit r
    // of m2) and exactly one (m1); rows outside both are passed over without
    // reading their lists.  Wide classes: m2hi = first row of the block of
    // counts (kNone: none yet), m2lo = its word offset, m1lo = meta before
    // it, m1hi = first later row of the next counting pass.
    uint32_t m2lo, m2hi, m1lo, m1hi;
};

constexpr uint32_t kStageWords = 68;  // words a chunk of 64 projected entries can touch, + slack
static_assert(4 * kStageWords <= kGx, "the projection stage fits in the tile area");

constexpr uint32_t kStageRecs = 64;  // key records a wave gathers in LDS before one reservation

struct alignas(16) WaveShared {
    uint32_t gx[kGx];                // row tiles, then pair supports, of the class being built;
                                     // assembly of projected rows (16-byte aligned)
    uint4 recs[2 * kStageRecs];      // key records not yet in the output arena (two uint4 each)
    uint4 row0[kGramMax];            // the child class of row 0 of the class built last
    uint32_t n_recs;                 // records in `recs`
    uint32_t row0_n, row0_rank, row0_id;  // its size, row 0's rank and item id
    uint32_t xm[4];                  // child-class size masks of the class built last (Frame m2, m1)
    Frame frames[kMaxDepth];
    uint32_t prefix[kMaxDepth + 3];  // ranks of the prefix items
    uint32_t pid[kMaxDepth + 3];     // their item ids
    uint32_t sid[kMaxDepth + 3];     // the prefix's item ids ascending (key records)
    uint32_t cid[kGramMax];          // item ids of the atoms of the class being built
};

struct WaveStats {
    unsigned long long candidates, pair_words, child_rows, given, max_k, max_depth, row_words;
    unsigned long long rec_pending;  // records not yet added to the instance's count
    unsigned long long stack_peak;   // largest stack use of the piece (words)
    unsigned long long out_words;    // words of the records reported (or counted)
};

// per-wave trace record (written when a trace buffer is given)
struct WaveTrace {
    unsigned long long busy, pieces, given, candidates, max_k, max_depth, pad0, pad1;
};

// Where the first class of a piece of work comes from: its prefix itemset,
// its atoms (ranks and supports of prefix + atom) and how many of its rows
// to expand.  A task of the planner is the first-level class of one item;
// donated work is any class a busy worker handed over.
struct FrameSrc {
    const uint32_t *prefix;  // plen ranks
    const uint32_t *ranks;   // k atom ranks
    const uint32_t *supps;   // k supports
    uint32_t plen, k, r_end;
    // second-level class of the piece (index into the instance's l2 atoms):
    // for a one-item prefix the class of row 0 (row r: l2_ref + r), else the
    // class every itemset of the piece belongs to
    uint32_t l2_ref;
    // the itemsets of the piece's first class (prefix + two of its atoms)
    // were already reported (a donated part of a class counted when built)
    uint32_t reported;
};

// the second-level class of the itemsets reported while row r of the
// class at `depth` is expanded
__device__ __forceinline__ uint32_t l2_class(uint32_t plen, uint32_t l2_ref, int depth, uint32_t r,
                                            const WaveShared &ws) {
    if (plen >= 2) return l2_ref;
    return l2_ref + (depth == 0 ? r : ws.frames[0].r - 1);
}

// Work sharing between waves.  An idle wave counts itself in `idle`; a
// busy wave that sees idle > 0 hands over the upper part of the unexpanded
// rows of its shallowest class: it writes a record (instance, prefix,
// remaining atoms) to the donation heap, then publishes the heap offset in
// the next queue slot.  Waves finish when no wave is active and the queue
// is drained; every wait is bounded.
struct Donation {
    unsigned long long *slots;  // per slot: heap offset + 1 once published, 0 before
    uint32_t *heap;
    uint64_t n_slots, heap_words;
    uint64_t wait_ticks;        // longest wait (wall-clock ticks) before giving up
    uint32_t enabled;
    unsigned long long *trace;  // WaveTrace per wave, or null
    uint32_t nap_max;           // longest back-off of an idle wave, in naps of ~8000 cycles
    uint64_t poll_ticks;        // a busy wave looks for idle waves at most this often (wall clock)
};

// Output of one piece of work goes to chunks of the output arena claimed
// with one atomic each: header [size, task, seq, used, inst] then records
// [len, support, len ranks].  Chunks are numbered, so the host can put the
// records of a piece back in its own depth-first order.
struct OutChunk {
    uint64_t base;   // word offset of the chunk, kNoChunk if none
    uint32_t size;   // words allocated
    uint32_t pos;    // words used, header included
    uint32_t seq;    // chunk number within the piece of work
    uint32_t valid;  // 0 once the arena is full (records are then dropped)
};

constexpr uint64_t kNoChunk = ~0ull;

__device__ __forceinline__ void close_chunk(OutChunk &c, uint32_t *out) {
    if (c.base != kNoChunk && c.valid && lane_id() == 0) out[c.base + 3] = c.pos;
}

// make room for `need` words; returns false when the arena is full
__device__ __forceinline__ bool chunk_reserve(OutChunk &c, uint32_t need, uint32_t task, uint32_t inst,
                              uint32_t *out, uint64_t out_cap, DfsCounters *ctr) {
    if (c.base != kNoChunk && c.pos + need <= c.size) return c.valid != 0;
    close_chunk(c, out);
    const uint32_t grow = c.seq < 6 ? (256u << c.seq) : 16384u;
    const uint32_t size = max(grow, need + kChunkHeader);
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(&ctr->out_used.v, (unsigned long long)size);
    base = bcast64(base);
    c.seq += c.base == kNoChunk ? 0u : 1u;
    c.base = base;
    c.size = size;
    c.pos = kChunkHeader;
    c.valid = base + size <= out_cap ? 1u : 0u;
    if (c.valid) {
        if (lane_id() == 0) {
            out[base] = size;
            out[base + 1] = task;
            out[base + 2] = c.seq;
            out[base + 3] = 0;
            out[base + 4] = inst;
        }
    } else if (lane_id() == 0) {
        atomicOr(&ctr->flags, kFlagOutOverflow);
    }
    return c.valid != 0;
}

__device__ __forceinline__ void flag_stack(DfsCounters *ctr, uint64_t need) {
    if (lane_id() == 0) {
        atomicOr(&ctr->flags, kFlagStackOverflow);
        atomicMax(&ctr->stack_need, (unsigned long long)need);
    }
}

// Loads and stores that are coherent across the chip's XCDs (each XCD has
// an L2 of its own).  They avoid agent-scope fences, which would write back
// or invalidate a whole L2 and evict the bitmaps other waves are using.
__device__ __forceinline__ uint64_t load_coherent(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t load_coherent32(const uint32_t *p) {
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_coherent32(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// wait for this wave's own memory operations to complete (no cache maintenance)
__device__ __forceinline__ void wave_mem_wait() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// Sorts nf atoms (ranks, supports, source rows: arrays of stride `si` at
// tmp) ascending by (support, item id), or by item id alone, into dst as
// arrays of stride nf: ranks, supports, item ids, source rows.
__device__ void sort_atoms(const InstDesc &I, const uint32_t *tmp, uint32_t si, uint32_t *dst,
                           uint32_t nf) {
    const uint32_t lane = lane_id();
    for (uint32_t e0 = 0; e0 < nf; e0 += kWave) {
        const uint32_t e = e0 + lane;
        uint64_t key = ~0ull;
        uint32_t rk = 0, sp = 0, src = 0, id = 0;
        if (e < nf) {
            rk = tmp[e];
            sp = tmp[si + e];
            src = tmp[2 * si + e];
            id = I.item_of_rank[rk];
            key = I.order_by_id ? (uint64_t)id : (((uint64_t)sp << 32) | id);
        }
        uint32_t pos = 0;
        for (uint32_t f0 = 0; f0 < nf; f0 += kWave) {
            uint64_t kf = ~0ull;
            if (f0 + lane < nf) {
                const uint32_t idf = I.item_of_rank[tmp[f0 + lane]];
                kf = I.order_by_id ? (uint64_t)idf : (((uint64_t)tmp[si + f0 + lane] << 32) | idf);
            }
            const uint32_t cnt = min(nf - f0, (uint32_t)kWave);
            for (uint32_t t = 0; t < cnt; t++) pos += (lane_val64(kf, t) < key) ? 1u : 0u;
        }
        if (e < nf) {
            dst[pos] = rk;
            dst[nf + pos] = sp;
            dst[2 * nf + pos] = id;
            dst[3 * nf + pos] = src;
        }
    }
}

// Hand the upper part of the unexpanded rows of the shallowest class that
// is worth it to the donation queue.  Rows are split so that both parts
// have about the same number of candidate pairs; a part is worth handing
// over if it holds several candidate pairs per row the receiver has to
// rebuild from the level-1 bitmaps.
__device__ __forceinline__ bool try_donate(const InstDesc &I, uint32_t inst, uint32_t plen, uint32_t l2_ref,
                           int depth, uint32_t *region, WaveShared &ws, Donation &dn,
                           DfsCounters *ctr) {
    const uint32_t lane = lane_id();
    int d0 = -1;
    uint32_t mid = 0;
    for (int d = 0; d <= depth && d0 < 0; d++) {
        const Frame F = ws.frames[d];
        if (F.r_end < F.r + 2) continue;
        // pairs of rows [F.r, F.r_end): row r has F.k - 1 - r partners
        uint64_t total = 0;
        for (uint32_t r = F.r; r < F.r_end; r++) total += F.k - 1 - r;
        uint64_t acc = 0;
        uint32_t m = F.r + 1;
        for (uint32_t r = F.r; r < F.r_end; r++) {
            acc += F.k - 1 - r;
            if (2 * acc >= total) {
                m = max(r + 1, F.r + 1);
                break;
            }
        }
        if (m >= F.r_end) m = F.r_end - 1;
        uint64_t given = 0;
        for (uint32_t r = m; r < F.r_end; r++) given += F.k - 1 - r;
        const uint32_t pl = plen + (uint32_t)d;
        // the rows' subtrees usually hold far more pairs than the rows
        // themselves, so a modest first level already pays for the rebuild
        if (given < 4 || 2 * given < (uint64_t)(F.k - m + pl) || pl + 2 > kMaxDepth) continue;
        d0 = d;
        mid = m;
    }
    if (d0 < 0) return false;
    const Frame F = ws.frames[d0];
    const uint32_t pl = plen + (uint32_t)d0;  // prefix of class d0
    const uint32_t kk = F.k - mid;
    const uint32_t words = 5 + pl + 2 * kk;
    // the donated piece's second-level class reference
    const uint32_t ref = pl == 1 ? l2_ref + mid : (plen >= 2 ? l2_ref : l2_ref + ws.frames[0].r - 1);
    unsigned long long hb = 0, sl = 0;
    if (lane == 0) {
        hb = atomicAdd(&ctr->don_heap_used.v, (unsigned long long)words);
        sl = hb + words <= dn.heap_words ? atomicAdd(&ctr->don_tail.v, 1ull) : ~0ull;
    }
    hb = bcast64(hb);
    sl = bcast64(sl);
    if (sl >= dn.n_slots) return false;  // heap or queue full: keep the work
    uint32_t *rec = dn.heap + hb;
    const uint32_t *ranks = region + F.atoms;
    const uint32_t *supps = ranks + F.k;
    // a class counted when it was built has reported all of its pairs
    const uint32_t reported = F.lists != kNone ? 0x80000000u : 0u;
    if (lane == 0) {
        store_coherent32(rec + 0, inst);
        store_coherent32(rec + 1, pl);
        store_coherent32(rec + 2, kk);
        store_coherent32(rec + 3, (F.r_end - mid) | reported);
        store_coherent32(rec + 4, ref);
    }
    for (uint32_t q = lane; q < pl; q += kWave) store_coherent32(rec + 5 + q, ws.prefix[q]);
    for (uint32_t e = lane; e < kk; e += kWave) {
        store_coherent32(rec + 5 + pl + e, ranks[mid + e]);
        store_coherent32(rec + 5 + pl + kk + e, supps[mid + e]);
    }
    wave_mem_wait();  // the record is complete before it is published
    if (lane == 0) {
        __hip_atomic_store(&dn.slots[sl], (unsigned long long)hb + 1ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(&ctr->donations, 1ull);
    }
    ws.frames[d0].r_end = mid;
    __builtin_amdgcn_wave_barrier();
    return true;
}

// more waves wait than donations are queued for them
__device__ __forceinline__ bool donation_wanted(DfsCounters *ctr) {
    uint32_t want = 0;
    if (lane_id() == 0) {
        const uint64_t idle = load_coherent(&ctr->idle.v);
        if (idle) {
            const uint64_t queued = load_coherent(&ctr->don_tail.v) - load_coherent(&ctr->don_head.v);
            want = idle > queued ? 1u : 0u;
        }
    }
    return bcast32(want) != 0;
}

// CPL > 0: a row spans at most 64 * CPL chunks and the expanded row is held
// in registers (CPL chunks per lane) for all its pairs and child rows, with
// two partner rows loaded per round.  CPL = 0: rows of any width, streamed.
// Key mode: the nf itemsets prefix + child as 8-word records (128-bit key
// of ascending (id + 1) codes, support, instance) at the end of the flat
// arena.  The prefix's item ids are sorted once in LDS; each lane inserts
// its child's id while packing the key.
__device__ void emit_keys(const InstDesc &I, uint32_t inst, uint32_t len, const uint32_t *tmp,
                          uint32_t nj, uint32_t nf, WaveShared &ws, uint32_t *out, uint64_t out_cap,
                          DfsCounters *ctr) {
    const uint32_t lane = lane_id();
    const uint32_t bits = I.key_bits;
    if (len * bits > 128) {
        if (lane == 0) atomicOr(&ctr->flags, kFlagKeyOverflow);
        return;
    }
    // the prefix's item ids ascending in LDS: lane q ranks id q among the
    // distinct ids (len - 1 <= kMaxDepth + 1 < 2 * kWave)
    uint32_t *sp = ws.sid;
    const uint32_t np = len - 1;
    uint32_t v0 = lane < np ? ws.pid[lane] : ~0u;
    uint32_t v1 = lane + kWave < np ? ws.pid[lane + kWave] : ~0u;
    uint32_t p0 = 0, p1 = 0;
    for (uint32_t q = 0; q < np && q < (uint32_t)kWave; q++) {
        const uint32_t u = lane_val(v0, q);
        p0 += u < v0 ? 1u : 0u;
        p1 += u < v1 ? 1u : 0u;
    }
    for (uint32_t q = kWave; q < np; q++) {
        const uint32_t u = lane_val(v1, q - kWave);
        p0 += u < v0 ? 1u : 0u;
        p1 += u < v1 ? 1u : 0u;
    }
    if (lane < np) sp[p0] = v0;
    if (lane + kWave < np) sp[p1] = v1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&ctr->out_used.v, 8ull * nf);
    base = bcast64(base);
    if (base + 8ull * nf > out_cap) {
        if (lane == 0) atomicOr(&ctr->flags, kFlagOutOverflow);
    } else {
        for (uint32_t e = lane; e < nf; e += kWave) {
            const uint32_t c = I.item_of_rank[tmp[e]];
            // The len codes: the prefix items (ascending in sp) merged with c.
            // Code x + 1 goes to bits [sh, sh + bits) of hi:lo through
            // selects on values (a reference to hi or lo would send them
            // through scratch memory).
            unsigned long long hi = 0, lo = 0;
            uint32_t sh = 128, q = 0;
            bool ins = false;
            for (uint32_t k = 0; k < len; k++) {
                const uint32_t v = q + 1 < len ? sp[q] : ~0u;  // next prefix item, if any
                const bool take_c = !ins && c < v;
                const uint32_t x = take_c ? c : v;
                ins = ins || take_c;
                q += take_c ? 0u : 1u;
                const unsigned long long code = (unsigned long long)x + 1;
                sh -= bits;
                hi |= sh >= 64 ? code << (sh - 64) : (sh + bits > 64 ? code >> (64 - sh) : 0ull);
                lo |= sh >= 64 ? 0ull : code << sh;
            }
            uint4 *o = reinterpret_cast<uint4 *>(out + base + 8ull * e);
            o[0] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
            o[1] = make_uint4(tmp[nj + e], inst, 0u, 0u);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// the instance went over its record budget (wave-uniform)
__device__ __forceinline__ bool inst_stopped(const InstDesc &I, InstCounters *ictr, uint32_t inst) {
    if (I.rec_budget == 0) return false;
    uint32_t v = 0;
    if (lane_id() == 0) v = load_coherent32(&ictr[inst].stop);
    return bcast32(v) != 0;
}

// ---------------------------------------------------------------- counting a class when it is built

// Loads and stores of global memory.  The persistent kernel's pointers all
// point to device memory; spelling the address space out keeps the compiler
// from emitting generic (flat) accesses, which wait on both the vector memory
// and the LDS counters.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 *g_cu4;
typedef __attribute__((address_space(1))) u32x4 *g_u4;
typedef __attribute__((address_space(1))) const uint32_t *g_cu32;
typedef __attribute__((address_space(1))) uint32_t *g_u32;
__device__ __forceinline__ uint4 gld4(const uint4 *p) {
    const u32x4 v = *(g_cu4)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gst4(uint4 *p, uint4 v) {
    u32x4 w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    *(g_u4)p = w;
}
__device__ __forceinline__ uint32_t gld(const uint32_t *p) { return *(g_cu32)p; }
__device__ __forceinline__ void gst(uint32_t *p, uint32_t v) { *(g_u32)p = v; }

// index of pair (a, b), a < b < f, in row-major order of the upper triangle
__device__ __forceinline__ uint32_t pair_index(uint32_t a, uint32_t b, uint32_t f) {
    return a * f - a * (a + 1) / 2 + (b - a - 1);
}

// the pair of index p < f (f - 1) / 2 (inverse of pair_index): row a is the
// largest x with pair_index(x, x + 1, f) <= p, the smaller root of
// x^2 - (2f - 1) x + 2p = 0 rounded down; the single-precision estimate is
// corrected by whole rows, so the result is exact
__device__ __forceinline__ void pair_of(uint32_t p, uint32_t f, uint32_t &a, uint32_t &b) {
    const float h = 2.0f * (float)f - 1.0f;
    const float d = h * h - 8.0f * (float)p;
    int x = (int)((h - __builtin_sqrtf(d > 0.0f ? d : 0.0f)) * 0.5f);
    x = max(0, min(x, (int)f - 2));
    auto first = [f](int r) { return (uint32_t)r * f - (uint32_t)r * (uint32_t)(r + 1) / 2; };
    while (x > 0 && first(x) > p) x--;
    while (x + 2 < (int)f && first(x + 1) <= p) x++;
    a = (uint32_t)x;
    b = p - first(x) + (uint32_t)x + 1;
}

// Reduce-scatter of N values (N a power of two, at most 32) over the wave:
// the halving steps exchange half of the values with the lane O apart (lane
// bits 5, 4, ...), so that after log2(N) steps lane l holds one value, the
// one of index (l >> (6 - log2 N)) & (N - 1), summed over the lanes that
// share those bits; the remaining lane bits are then summed as usual.
template <int N, int O = 32>
__device__ __forceinline__ uint32_t reduce_scatter(uint32_t *v, uint32_t lane) {
    if constexpr (N == 1) {
        uint32_t s = v[0];
#pragma unroll
        for (int o = O; o >= 1; o >>= 1) s += __shfl_xor(s, o, kWave);
        return s;
    } else {
        constexpr int H = N / 2;
        const bool up = (lane & O) != 0;
#pragma unroll
        for (int i = 0; i < H; i++) {
            const uint32_t keep = up ? v[i + H] : v[i];
            const uint32_t give = up ? v[i] : v[i + H];
            v[i] = keep + __shfl_xor(give, O, kWave);
        }
        return reduce_scatter<H, O / 2>(v, lane);
    }
}

template <int N>
constexpr int log2i() {
    return N <= 1 ? 0 : 1 + log2i<N / 2>();
}

// Rows of a class of F atoms: row q = xr AND base[src_q] (xr null: base[src_q]
// itself), src_q held by lane q.  Counts the supports of all F (F - 1) / 2
// pairs into gx[pair_index] and writes the rows to dst (if not null), row q
// at dst + q * Wp.  A lane owns 128-bit chunks c = lane, lane + 64, ... of
// every row and all pairs; U chunks of every row are loaded at once.
template <int F, int U>
__device__ __forceinline__ void count_reg(const uint32_t *xr, const uint32_t *base, uint32_t Wp,
                                          uint32_t src, uint32_t *dst, uint32_t *gx) {
    constexpr int NP = F * (F - 1) / 2;
    constexpr int N = NP <= 1 ? 1 : NP <= 2 ? 2 : NP <= 4 ? 4 : NP <= 8 ? 8 : NP <= 16 ? 16 : 32;
    const uint32_t lane = lane_id();
    const uint32_t C = Wp / 4;
    const uint4 *rp[F];
#pragma unroll
    for (int q = 0; q < F; q++)
        rp[q] = reinterpret_cast<const uint4 *>(base + (uint64_t)__builtin_amdgcn_readlane(src, q) * Wp);
    const uint4 *xp = reinterpret_cast<const uint4 *>(xr);
    uint4 *dp = reinterpret_cast<uint4 *>(dst);
    uint32_t acc[N];
#pragma unroll
    for (int p = 0; p < N; p++) acc[p] = 0;
#pragma unroll 1
    for (uint32_t c0 = lane; c0 < C; c0 += U * kWave) {
        uint4 x[U][F];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t c = c0 + u * kWave;
#pragma unroll
            for (int q = 0; q < F; q++) x[u][q] = c < C ? gld4(rp[q] + c) : make_uint4(0, 0, 0, 0);
        }
        if (xp) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint32_t c = c0 + u * kWave;
                const uint4 r = c < C ? gld4(xp + c) : make_uint4(0, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < F; q++) x[u][q] = and4(x[u][q], r);
            }
        }
        if (dp) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint32_t c = c0 + u * kWave;
                if (c < C) {
#pragma unroll
                    for (int q = 0; q < F; q++) gst4(dp + (uint64_t)q * C + c, x[u][q]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            int p = 0;
#pragma unroll
            for (int a = 0; a < F; a++)
#pragma unroll
                for (int b = a + 1; b < F; b++) acc_popc4(acc[p++], x[u][a], x[u][b]);
        }
    }
    const uint32_t s = reduce_scatter<N>(acc, lane);
    const uint32_t idx = (lane >> (6 - log2i<N>())) & (N - 1);
    if ((lane & (kWave / N - 1)) == 0 && idx < (uint32_t)NP) gx[idx] = s;
}

// Blocks (A, B) of four rows each counted for a class of f rows: A over the
// block rows holding rows below r_cnt, B from max(A, bmin) on.
__device__ __forceinline__ uint32_t lds_blocks(uint32_t f, uint32_t r_cnt, uint32_t bmin) {
    const uint32_t nb = (f + 3) / 4, nbr = (r_cnt + 3) / 4;
    uint32_t P = 0;
    for (uint32_t a = 0; a < nbr; a++) P += nb - max(a, bmin);
    return P;
}

// LDS tile width (words) of a class of f atoms with P blocks: the widest
// power of two up to tmax such that the tile (f rows padded to a multiple
// of four, row stride width + 4) and the blocks' counts and table (17 P
// words) fit in kGx words, with at most kMaxTileRows chunks per lane
__device__ __forceinline__ uint32_t lds_tile(uint32_t f, uint32_t P, uint32_t tmax) {
    uint32_t t = tmax;
    while (t > kTileMin && (4 * ((f + 3) / 4) * (t + 4) + 17 * P > kGx || f * t > 256 * kMaxTileRows)) t >>= 1;
    return t;
}

// The same for kRegGram < f <= kGramMax atoms, with the rows staged in LDS
// tile by tile (T words per tile, row stride T + 4 words; lane l loads chunk
// l mod T/4 of its rows).  The next tile is loaded into registers while the
// pairs of the current one are counted.  The pairs are cut into 4x4 blocks
// (lds_blocks), and the words of a tile into G slices; the P G items (block,
// slice) of a tile are dealt to the 64 lanes in rounds, so that all lanes
// count whatever the number of blocks.  A lane reads its slice of the
// block's eight rows 128 bits at a time, accumulates the 16 pairs in
// registers and adds them to the block's counts in LDS.
__device__ __forceinline__ void count_lds(const uint32_t *xr, const uint32_t *base, uint32_t Wp,
                                          uint32_t f, uint32_t r_cnt, uint32_t bmin, uint32_t src,
                                          uint32_t *dst, uint32_t *gx, uint32_t tmax) {
    const uint32_t lane = lane_id();
    const uint32_t nb = (f + 3) / 4, P = lds_blocks(f, r_cnt, bmin);
    const uint32_t T = lds_tile(f, P, tmax), CR = T / 4, stride = T + 4;
    uint32_t *cnt = gx + 4 * nb * stride;  // 16 counts of each block (A row i, B row j at 4 i + j)
    uint32_t *blk = cnt + 16 * P;          // block p: (A << 16) | B
    for (uint32_t p = lane; p < P; p += kWave) {
        uint32_t a = 0, rem = p;
        while (rem >= nb - max(a, bmin)) {
            rem -= nb - max(a, bmin);
            a++;
        }
        blk[p] = (a << 16) | (max(a, bmin) + rem);
    }
    for (uint32_t i = lane; i < 16 * P; i += kWave) cnt[i] = 0u;
    // tile rows from f up to 4 nb pad the last block with zeros
    for (uint32_t i = f * stride + lane; i < 4 * nb * stride; i += kWave) gx[i] = 0u;
    // slices: the G of least cost over the rounds of 64 items, a round
    // costing about 34 operations per word of a slice plus 36 per item
    uint32_t G = 1, best = ~0u;
    for (uint32_t g = 1; g <= CR; g <<= 1) {
        const uint32_t cost = ((P * g + kWave - 1) / kWave) * ((T / g) * 34 + 36);
        if (cost < best) {
            best = cost;
            G = g;
        }
    }
    const uint32_t NI = P * G, SW = T / G;
    // item i = s P + p; a lane's items are lane, lane + 64, ...
    const uint32_t p0 = P ? lane % P : 0u, s0 = P ? lane / P : 0u;
    const uint32_t dp = P ? (uint32_t)kWave % P : 0u, dsl = P ? (uint32_t)kWave / P : 0u;
    // this lane's chunks of a tile: chunk cc of rows q0 + j * (64 / CR)
    const uint32_t cc = lane % CR, q0 = lane / CR, qs = kWave / CR;
    const uint32_t nl = q0 < f ? (f - q0 + qs - 1) / qs : 0u;  // rows of this lane
    uint32_t srcj[kMaxTileRows];
#pragma unroll
    for (int j = 0; j < kMaxTileRows; j++) srcj[j] = __shfl(src, (int)min(q0 + j * qs, f - 1), kWave);
    uint4 buf[kMaxTileRows];
    auto load = [&](uint32_t w0) {
        const uint32_t w = w0 + 4 * cc;
        const bool in = w < Wp;
        const uint4 r = (xr && in) ? gld4(reinterpret_cast<const uint4 *>(xr + w)) : make_uint4(~0u, ~0u, ~0u, ~0u);
#pragma unroll
        for (int j = 0; j < kMaxTileRows; j++) {
            const bool ok = in && (uint32_t)j < nl;
            buf[j] = ok ? and4(gld4(reinterpret_cast<const uint4 *>(base + (uint64_t)srcj[j] * Wp + w)), r)
                        : make_uint4(0, 0, 0, 0);
        }
    };
    load(0);
#pragma unroll 1
    for (uint32_t w0 = 0; w0 < Wp; w0 += T) {
        const uint32_t w = w0 + 4 * cc;
#pragma unroll
        for (int j = 0; j < kMaxTileRows; j++) {
            if ((uint32_t)j < nl) {
                const uint32_t q = q0 + j * qs;
                *reinterpret_cast<uint4 *>(gx + q * stride + 4 * cc) = buf[j];
                if (dst && w < Wp) gst4(reinterpret_cast<uint4 *>(dst + (uint64_t)q * Wp + w), buf[j]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (w0 + T < Wp) load(w0 + T);
        uint32_t p = p0, sl = s0;
#pragma unroll 1
        for (uint32_t i0 = 0; i0 < NI; i0 += kWave) {
            if (i0 + lane < NI) {
                const uint32_t ab = blk[p];
                const uint32_t *ra = gx + 4 * (ab >> 16) * stride + sl * SW;
                const uint32_t *rb = gx + 4 * (ab & 0xffffu) * stride + sl * SW;
                uint32_t acc[16];
#pragma unroll
                for (int e = 0; e < 16; e++) acc[e] = 0;
#pragma unroll 1
                for (uint32_t t = 0; t < SW; t += 4) {
                    uint4 av[4], bv[4];
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        av[i] = *reinterpret_cast<const uint4 *>(ra + i * stride + t);
                        bv[i] = *reinterpret_cast<const uint4 *>(rb + i * stride + t);
                    }
#pragma unroll
                    for (int i = 0; i < 4; i++)
#pragma unroll
                        for (int j = 0; j < 4; j++) acc_popc4(acc[i * 4 + j], av[i], bv[j]);
                }
#pragma unroll
                for (int e = 0; e < 16; e++) atomicAdd(cnt + 16 * p + e, acc[e]);
            }
            p += dp;
            sl += dsl;
            if (p >= P) {
                p -= P;
                sl++;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // the counts of the pairs into gx (below the tile area's end, which
    // holds more than f (f - 1) / 2 words, so no count is overwritten first)
    for (uint32_t e = lane; e < 16 * P; e += kWave) {
        const uint32_t ab = blk[e / 16], q = e % 16;
        const uint32_t a = 4 * (ab >> 16) + q / 4, b = 4 * (ab & 0xffffu) + q % 4;
        if (a < b && b < f && a < r_cnt) gx[pair_index(a, b, f)] = cnt[e];
    }
}

// Pair supports of a class of f atoms (2 <= f <= kGramMax) into ws.gx: the
// pairs (a, b) of rows a < r_cnt at least (up to kRegGram atoms all pairs),
// of the rows b of the four-row blocks from bmin on.
__device__ __forceinline__ void count_class(const uint32_t *xr, const uint32_t *base, uint32_t Wp,
                                            uint32_t f, uint32_t r_cnt, uint32_t bmin, uint32_t src,
                                            uint32_t *dst, uint32_t tmax, WaveShared &ws) {
    switch (f) {
        case 2: count_reg<2, 8>(xr, base, Wp, src, dst, ws.gx); break;
        case 3: count_reg<3, 4>(xr, base, Wp, src, dst, ws.gx); break;
        case 4: count_reg<4, 4>(xr, base, Wp, src, dst, ws.gx); break;
        case 5: count_reg<5, 2>(xr, base, Wp, src, dst, ws.gx); break;
        case 6: count_reg<6, 2>(xr, base, Wp, src, dst, ws.gx); break;
        case 7: count_reg<7, 2>(xr, base, Wp, src, dst, ws.gx); break;
        case 8: count_reg<8, 2>(xr, base, Wp, src, dst, ws.gx); break;
        default: {
            count_lds(xr, base, Wp, f, r_cnt, bmin, src, dst, ws.gx, tmax);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The prefix's item ids (ws.pid[0, np)) ascending into ws.sid.
__device__ __forceinline__ void sort_prefix_ids(uint32_t np, WaveShared &ws) {
    const uint32_t lane = lane_id();
    const uint32_t v0 = lane < np ? ws.pid[lane] : ~0u;
    const uint32_t v1 = lane + kWave < np ? ws.pid[lane + kWave] : ~0u;
    uint32_t p0 = 0, p1 = 0;
    for (uint32_t q = 0; q < np && q < (uint32_t)kWave; q++) {
        const uint32_t u = lane_val(v0, q);
        p0 += u < v0 ? 1u : 0u;
        p1 += u < v1 ? 1u : 0u;
    }
    for (uint32_t q = kWave; q < np; q++) {
        const uint32_t u = lane_val(v1, q - kWave);
        p0 += u < v0 ? 1u : 0u;
        p1 += u < v1 ? 1u : 0u;
    }
    if (lane < np) ws.sid[p0] = v0;
    if (lane + kWave < np) ws.sid[p1] = v1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// 128-bit key of the itemset: the np prefix ids (ascending in ws.sid) and
// the two ids x < y, as (id + 1) codes of `bits` bits from the top bit down.
__device__ __forceinline__ void pair_key(const WaveShared &ws, uint32_t np, uint32_t bits, uint32_t x,
                                         uint32_t y, unsigned long long &hi, unsigned long long &lo) {
    hi = 0;
    lo = 0;
    uint32_t sh = 128, q = 0, t = 0;  // t: 0, 1 or 2 of {x, y} placed
    for (uint32_t k = 0; k < np + 2; k++) {
        const uint32_t v = q < np ? ws.sid[q] : ~0u;
        const uint32_t c = t == 0 ? x : (t == 1 ? y : ~0u);
        const bool take_c = c < v;
        const uint32_t z = take_c ? c : v;
        t += take_c ? 1u : 0u;
        q += take_c ? 0u : 1u;
        const unsigned long long code = (unsigned long long)z + 1;
        sh -= bits;
        hi |= sh >= 64 ? code << (sh - 64) : (sh + bits > 64 ? code >> (64 - sh) : 0ull);
        lo |= sh >= 64 ? 0ull : code << sh;
    }
}

// Where the records of a class go (see finish_class).
struct EmitTo {
    uint32_t np;       // prefix length of the class
    uint32_t r_emit;   // rows whose pairs are reported (0: none)
    uint32_t l2_row0;  // estimate runs: second-level class of row 0 when each row has its own
    uint32_t l2_cls;   //   (kNone), else the class of every pair
};

enum : uint32_t { kBuildOk = 0, kBuildStop = 1, kBuildFull = 2 };

// Moves the key records gathered in LDS to the output arena: one atomic
// reservation for all of them.
__device__ __forceinline__ void flush_recs(WaveShared &ws, uint32_t *out, uint64_t out_cap,
                                           DfsCounters *ctr) {
    const uint32_t lane = lane_id();
    const uint32_t n = uni(ws.n_recs);
    if (n == 0) return;
    unsigned long long b0 = 0;
    if (lane == 0) b0 = atomicAdd(&ctr->out_used.v, 8ull * n);
    const uint64_t base = bcast64(b0);
    if (base + 8ull * n <= out_cap) {
        uint4 *o = reinterpret_cast<uint4 *>(out + base);
        for (uint32_t i = lane; i < 2 * n; i += kWave) gst4(o + i, ws.recs[i]);
    } else if (lane == 0) {
        atomicOr(&ctr->flags, kFlagOutOverflow);
    }
    if (lane == 0) ws.n_recs = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ws.gx holds the supports of the f (f - 1) / 2 pairs of a class (pair_index
// order) whose atom q is held by lane q (rank, support, item id; ws.cid[q] =
// item id).  Below `meta` this writes the class's atom arrays, the size of
// every row's child class and, row after row, those child classes (the
// frequent later atoms as (rank, support, row, item id), ascending by
// (support, item id)); it reports the frequent pairs of rows a < r_emit as
// the itemsets prefix + a + b.  meta moves down to the atom arrays.
__device__ __forceinline__ uint32_t finish_class(const InstDesc &I, uint32_t inst, uint32_t task,
                                                 uint32_t f, uint32_t r_cnt, uint32_t rank, uint32_t supp,
                                                 uint32_t id, const EmitTo &em, uint64_t rows_end, uint64_t &meta,
                                                 uint32_t *region, uint64_t S, WaveShared &ws,
                                                 uint32_t *out, uint64_t out_cap, DfsCounters *ctr,
                                                 InstCounters *ictr, WaveStats &st, OutChunk &oc,
                                                 uint32_t &atoms_off, uint32_t &lists_off, uint4 &xmask) {
    const uint32_t lane = lane_id();
    const uint32_t m = I.minsup;
    // pairs of the rows below r_cnt (the only ones counted), row after row
    const uint32_t NP = r_cnt >= f - 1 ? f * (f - 1) / 2 : pair_index(r_cnt, r_cnt + 1, f);
    // Frequent pairs, 64 at a time in pair_index order (row after row): all
    // of them, and those of the rows that report (the pairs before row
    // r_emit's first pair).
    const uint32_t r_emit = min(em.r_emit, r_cnt);
    const uint32_t emit_end = r_emit == 0 ? 0u : (r_emit >= f - 1 ? NP : pair_index(r_emit, r_emit + 1, f));
    uint32_t nfreq = 0, n_emit = 0;
    for (uint32_t p0 = 0; p0 < NP; p0 += kWave) {
        const uint32_t p = p0 + lane;
        const uint64_t mask = __ballot(p < NP && ws.gx[p] >= m);
        nfreq += (uint32_t)__popcll(mask);
        if (p0 < emit_end) {
            const uint32_t k = min(emit_end - p0, (uint32_t)kWave);
            n_emit += (uint32_t)__popcll(k == 64 ? mask : (mask & ((1ull << k) - 1)));
        }
    }
    nfreq = uni(nfreq);
    n_emit = uni(n_emit);
    const uint32_t len = em.np + 2;
    const bool report = n_emit > 0 && (I.max_len == 0 || len <= I.max_len);
    const bool keys = report && I.key_bits != 0 && I.class_count == nullptr && len * I.key_bits <= 128;
    // Key records are gathered in LDS (one reservation of the arena per
    // kStageRecs records); a class with more records than that reserves its
    // own place now, so that the atomic's round trip overlaps the work below.
    bool staged = false;
    uint32_t at = 0;  // first LDS slot of this class's records
    unsigned long long b0 = 0;
    if (keys) {
        if (n_emit <= kStageRecs) {
            if (uni(ws.n_recs) + n_emit > kStageRecs) flush_recs(ws, out, out_cap, ctr);
            at = uni(ws.n_recs);
            staged = true;
        } else if (lane == 0) {
            b0 = atomicAdd(&ctr->out_used.v, 8ull * n_emit);
        }
    }
    // lists (16-byte aligned entries) and atom arrays below meta
    const uint64_t need = 4ull * (nfreq + kListPad) + 4ull * f + 4;
    if (meta < need || meta - need < rows_end) {
        flag_stack(ctr, rows_end + (S - meta) + need);
        return kBuildFull;
    }
    const uint64_t lists = (meta - 4ull * (nfreq + kListPad)) & ~3ull;
    const uint64_t atoms = lists - 4ull * f;
    uint32_t *A = region + atoms;
    if (lane == 0) {
        ws.row0_n = 0;
        ws.row0_rank = rank;
        ws.row0_id = id;
        ws.xm[0] = ws.xm[1] = ws.xm[2] = ws.xm[3] = 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane < f) {
        gst(A + lane, rank);
        gst(A + f + lane, supp);
        gst(A + 2 * f + lane, id);
        if (lane >= r_cnt) gst(A + 3 * f + lane, 0u);  // rows not counted (and the last row)
    }
    // reporting
    const bool recs = report && I.key_bits == 0 && I.class_count == nullptr;
    uint64_t kbase = 0;
    bool kvalid = false, rvalid = false;
    const uint32_t rec = kRecHeader + len;
    if (report) {
        if (I.rec_budget) st.rec_pending += n_emit;
        st.out_words += (unsigned long long)n_emit * (I.key_bits ? 8u : rec);
    }
    if (report && I.key_bits != 0 && I.class_count == nullptr && len * I.key_bits > 128) {
        if (lane == 0) atomicOr(&ctr->flags, kFlagKeyOverflow);
    } else if (keys) {
        sort_prefix_ids(em.np, ws);
        if (staged) {
            kvalid = true;
            if (lane == 0) ws.n_recs = at + n_emit;
        } else {
            kbase = bcast64(b0);
            kvalid = kbase + 8ull * n_emit <= out_cap;
            if (!kvalid && lane == 0) atomicOr(&ctr->flags, kFlagOutOverflow);
        }
    } else if (recs) {
        rvalid = chunk_reserve(oc, n_emit * rec, task, inst, out, out_cap, ctr);
    } else if (report && I.class_count && em.l2_row0 == kNone && lane == 0) {
        // estimate run: only the number of itemsets per second-level class
        atomicAdd(&I.class_count[em.l2_cls], (unsigned long long)n_emit);
    }
    // the entries, lane-parallel over the pairs: pair (a, b) goes to row a's
    // list at (frequent pairs before row a) + (its rank in row a by (support,
    // item id)); the lane of a row's first pair writes the row's list size
    uint4 *L = reinterpret_cast<uint4 *>(region + lists);
    const bool per_row_count = report && I.class_count && em.l2_row0 != kNone;
    uint32_t before = 0;  // frequent pairs of the earlier chunks
    for (uint32_t p0 = 0; p0 < NP; p0 += kWave) {
        const uint32_t p = p0 + lane;
        uint32_t a = 0, b = 1, s = 0;
        if (p < NP) {
            pair_of(p, f, a, b);
            s = ws.gx[p];
        }
        const bool fr = p < NP && s >= m;
        const uint64_t mask = __ballot(fr);
        const uint32_t rank_b = __shfl(rank, (int)b, kWave);
        const uint32_t rank_a = __shfl(rank, (int)a, kWave);
        if (p < NP) {
            const uint32_t id_b = ws.cid[b];
            const uint64_t key = I.order_by_id ? (uint64_t)id_b : (((uint64_t)s << 32) | id_b);
            // frequent pairs of row a: before b in the row, ahead of b in the
            // list order, and in all
            uint32_t k_before = 0, pos = 0, row_n = 0;
            // pair (a, c) sits at row_p + c: the row's pairs are consecutive
            const uint32_t row_p = pair_index(a, a + 1, f) - (a + 1);
#pragma unroll 4
            for (uint32_t c = a + 1; c < f; c++) {
                const uint32_t sc = ws.gx[row_p + c];
                const uint32_t idc = ws.cid[c];
                const uint64_t kc = I.order_by_id ? (uint64_t)idc : (((uint64_t)sc << 32) | idc);
                const bool fc = sc >= m;
                row_n += fc ? 1u : 0u;
                k_before += (fc && c < b) ? 1u : 0u;
                pos += (fc && c != b && kc < key) ? 1u : 0u;
            }
            if (b == a + 1) {
                gst(A + 3 * f + a, row_n);
                if (row_n >= 2) atomicOr(&ws.xm[a >> 5], 1u << (a & 31));
                else if (row_n == 1) atomicOr(&ws.xm[2 + (a >> 5)], 1u << (a & 31));
                if (a == 0) ws.row0_n = row_n;
                if (per_row_count && a < r_emit && row_n)
                    atomicAdd(&I.class_count[em.l2_row0 + a], (unsigned long long)row_n);
            }
            if (fr) {
                const uint32_t e = before + lanes_below(mask) - k_before + pos;
                const uint4 entry = make_uint4(rank_b, s, b, id_b);
                gst4(L + e, entry);
                if (a == 0) ws.row0[pos] = entry;  // row 0 is expanded next
                if (a < r_emit) {
                    if (kvalid) {
                        const uint32_t id_a = ws.cid[a];
                        unsigned long long hi, lo;
                        pair_key(ws, em.np, I.key_bits, min(id_a, id_b), max(id_a, id_b), hi, lo);
                        const uint4 k0 = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
                        const uint4 k1 = make_uint4(s, inst, 0u, 0u);
                        if (staged) {
                            ws.recs[2 * (at + e)] = k0;
                            ws.recs[2 * (at + e) + 1] = k1;
                        } else {
                            uint4 *o = reinterpret_cast<uint4 *>(out + kbase + 8ull * e);
                            gst4(o, k0);
                            gst4(o + 1, k1);
                        }
                    } else if (rvalid) {
                        uint32_t *o = out + oc.base + oc.pos + (uint64_t)e * rec;
                        o[0] = len;
                        o[1] = s;
                        for (uint32_t q = 0; q < em.np; q++) o[2 + q] = ws.prefix[q];
                        o[2 + em.np] = rank_a;
                        o[3 + em.np] = rank_b;
                    }
                }
            }
        }
        before += (uint32_t)__popcll(mask);
    }
    if (recs) oc.pos += n_emit * rec;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    meta = atoms;
    atoms_off = (uint32_t)atoms;
    lists_off = (uint32_t)lists;
    xmask = make_uint4(uni(ws.xm[0]), uni(ws.xm[1]), uni(ws.xm[2]), uni(ws.xm[3]));
    if (report && I.rec_budget && st.rec_pending >= 4096) {
        // records are added to the instance's count in batches; the count
        // never exceeds the records really found, so the work is abandoned
        // only once the budget is certainly exceeded
        unsigned long long before = 0;
        if (lane == 0) before = atomicAdd(&ictr[inst].records, st.rec_pending);
        before = bcast64(before);
        const unsigned long long now = before + st.rec_pending;
        st.rec_pending = 0;
        if (now > I.rec_budget) {
            if (lane == 0) atomicOr(&ictr[inst].stop, 1u);
            return kBuildStop;
        }
    }
    return kBuildOk;
}

// Depth-first search of a piece of work.  Its first class has k0 atoms,
// their rows at region[0, k0 Wp) and their arrays (ranks, supports, item
// ids) at meta; its rows [0, r_end0) are this piece's.  Classes of at most
// kGramMax atoms are counted when they are built (the first one right away,
// its pairs of rows below r_end0 reported unless `reported0`), and every
// expanded row hands its child class over from their lists; wider classes
// pair row r with every later row when it is expanded (rows streamed from
// memory, g lanes per pair).  All builds go through one block at the end of
// the loop, so that its counting code is present once.
__device__ __forceinline__ void search(const InstDesc &I, const InstDesc &Ig, uint32_t inst, uint32_t task, uint32_t plen,
                       uint32_t l2_ref, uint32_t Wp, uint32_t k0, uint32_t r_end0, uint32_t reported0,
                       uint64_t meta, uint64_t peak, uint32_t tmax, uint32_t *region, uint64_t S,
                       WaveShared &ws, uint32_t *out, uint64_t out_cap, DfsCounters *ctr,
                       InstCounters *ictr, WaveStats &st, OutChunk &oc, Donation &dn) {
    const uint32_t lane = lane_id();
    const uint32_t C = Wp / 4;  // 128-bit chunks per row
    // row-by-row pairing: lanes per pair, about four chunks per lane (their
    // loads in flight at once), at most a wave; narrow rows put several
    // pairs in one pass
    uint32_t g = 1;
    const uint32_t want = (C + 3) / 4;
    while (g < want && g < (uint32_t)kWave) g <<= 1;
    const uint32_t ppp = kWave / g;  // pairs per pass
    const uint32_t grp = lane / g, sub = lane % g;

    uint64_t rows_top = (uint64_t)k0 * Wp;
    // the class to build (lane q holds atom q) and where it goes
    bool build = false;
    uint32_t b_c = 0, b_rank = 0, b_supp = 0, b_id = 0, b_src = 0, b_r_end = 0;
    const uint32_t *b_xr = nullptr, *b_base = nullptr;
    bool b_write = false;
    uint64_t b_rows_base = 0, b_restore = 0;
    EmitTo b_em{0, 0, kNone, 0};
    // a counting pass of a wide class: its pairs go to the frame's block of
    // counts (b_rank = the block's first row, b_restore = the pass's first
    // later row, kNone for the block's own pairs) instead of building a class
    bool b_counts = false;
    int depth;
    if (k0 <= kGramMax) {
        const uint32_t q = lane < k0 ? lane : 0;
        build = true;
        b_c = k0;
        b_rank = region[meta + q];
        b_supp = region[meta + k0 + q];
        b_id = region[meta + 2 * k0 + q];
        b_src = lane;
        b_r_end = r_end0;
        b_base = region;
        b_rows_base = 0;
        b_restore = S;
        b_em = EmitTo{plen, reported0 ? 0u : r_end0, plen == 1 ? l2_ref : kNone, l2_ref};
        depth = -1;
    } else {
        if (lane == 0) ws.frames[0] = Frame{0u, k0, 0u, r_end0, (uint32_t)meta, kNone, 0u, (uint32_t)S, 0u, kNone, 0u, 0u};
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        depth = 0;
    }

    uint32_t cool = 0, iters = 0;
    unsigned long long last_poll = wall_clock64();
    int row0_depth = -1;  // the frame whose row 0 child class is in ws.row0
    for (;;) {
        if (build) {
            // ---- count the class while building it, list its rows' child
            // classes, push it; or (b_counts) count a pass of a wide class's
            // block of counts.  The one call of the counting code serves both.
            build = false;
            const bool counts = b_counts;
            b_counts = false;
            const uint32_t c = b_c;
            const uint64_t rows_need = (b_write && !counts) ? (uint64_t)c * Wp : 0;
            if (!counts) {
                const uint64_t meta_need = 4ull * (c * (c - 1) / 2 + kListPad) + 4ull * c + 4;
                if (meta < meta_need || meta - meta_need < rows_top + rows_need) {
                    flag_stack(ctr, rows_top + rows_need + (S - meta) + meta_need);
                    break;
                }
                if (lane < c) ws.cid[lane] = b_id;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            // a pass against later rows needs no pairs inside the block
            count_class(counts ? nullptr : b_xr, b_base, Wp, c, b_r_end,
                        (counts && (uint32_t)b_restore != kNone) ? uni(ws.frames[depth].lpos) / 4 : 0u, b_src,
                        rows_need ? region + rows_top : nullptr, tmax, ws);
            if (counts) {
                const uint32_t fk = uni(ws.frames[depth].k), nb = uni(ws.frames[depth].lpos);
                const uint32_t jc = (uint32_t)b_restore;
                uint32_t *cb = region + uni(ws.frames[depth].m2lo);
                if (jc == kNone) {
                    // the block's own pairs (a < b < nb); b_rank = its first row
                    const uint32_t np2 = c * (c - 1) / 2;
                    for (uint32_t p = lane; p < np2; p += kWave) {
                        uint32_t a = 0, b = 1;
                        pair_of(p, c, a, b);
                        gst(cb + (uint64_t)a * fk + (b_rank + b), ws.gx[p]);
                    }
                } else {
                    // the block's rows a < nb against the later rows b_jc + q
                    const uint32_t nq = c - nb;
                    for (uint32_t e = lane; e < nb * nq; e += kWave) {
                        const uint32_t a = e / nq, q = e % nq;
                        gst(cb + (uint64_t)a * fk + (jc + q), ws.gx[pair_index(a, nb + q, c)]);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                continue;
            }
            st.pair_words += (unsigned long long)(b_r_end * c - b_r_end * (b_r_end + 1) / 2) * Wp;
            if (depth >= 0) {
                st.row_words += (unsigned long long)c * Wp;
                st.child_rows += b_write ? c : 0u;
            }
            if (c == 2 && depth >= 0 && I.key_bits != 0 && I.class_count == nullptr &&
                I.row_cand == nullptr && I.rec_budget == 0) {
                // A class of two atoms is a leaf: its one pair is reported
                // here (a key record staged as finish_class would), and no
                // frame is pushed, since neither of its rows has a class of
                // two atoms below it.  Its one candidate is counted as the
                // frame's rows would have been.
                const uint32_t s2 = uni(ws.gx[0]);
                const uint32_t len = b_em.np + 2;
                if (b_em.r_emit >= 1 && s2 >= I.minsup && (I.max_len == 0 || len <= I.max_len)) {
                    if (len * I.key_bits > 128) {
                        if (lane == 0) atomicOr(&ctr->flags, kFlagKeyOverflow);
                    } else {
                        if (uni(ws.n_recs) + 1 > kStageRecs) flush_recs(ws, out, out_cap, ctr);
                        sort_prefix_ids(b_em.np, ws);
                        if (lane == 0) {
                            const uint32_t at = ws.n_recs;
                            const uint32_t ia = ws.cid[0], ib = ws.cid[1];
                            unsigned long long hi, lo2;
                            pair_key(ws, b_em.np, I.key_bits, min(ia, ib), max(ia, ib), hi, lo2);
                            ws.recs[2 * at] = make_uint4((uint32_t)lo2, (uint32_t)(lo2 >> 32), (uint32_t)hi,
                                                         (uint32_t)(hi >> 32));
                            ws.recs[2 * at + 1] = make_uint4(s2, inst, 0u, 0u);
                            ws.n_recs = at + 1;
                        }
                        st.out_words += 8;
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                    }
                }
                st.candidates += 1;
                if (2 > st.max_k) st.max_k = 2;
                if ((unsigned long long)(depth + 1) > st.max_depth) st.max_depth = depth + 1;
                continue;
            }
            uint32_t ao = 0, lo = 0;
            uint4 xm;
            if (finish_class(I, inst, task, c, b_r_end, b_rank, b_supp, b_id, b_em, rows_top + rows_need, meta, region,
                             S, ws, out, out_cap, ctr, ictr, st, oc, ao, lo, xm) != kBuildOk)
                break;
            if (lane == 0)
                ws.frames[depth + 1] = Frame{(uint32_t)b_rows_base, c, 0u, b_r_end, ao, lo, 0u, (uint32_t)b_restore,
                                             xm.x, xm.y, xm.z, xm.w};
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            rows_top += rows_need;
            depth++;
            row0_depth = depth;
            const uint64_t use = rows_top + (S - meta);
            if (use > peak) peak = use;
            continue;
        }
        if (depth < 0) break;
        if ((++iters & 63u) == 0 && inst_stopped(I, ictr, inst)) break;
        // idle waves are looked for by wall clock, not by row count: a row
        // of a wide dense class can take far longer than many small rows
        bool poll = false;
        if (dn.enabled && cool == 0) {
            const unsigned long long now = wall_clock64();
            if (now - last_poll >= dn.poll_ticks) {
                poll = true;
                last_poll = now;
            }
        }
        if (poll && donation_wanted(ctr)) {
            const bool gave = try_donate(Ig, inst, plen, l2_ref, depth, region, ws, dn, ctr);
            cool = gave ? 8u : 4u;
            st.given += gave ? 1u : 0u;
        } else if (cool) {
            cool--;
        }
        Frame F = ws.frames[depth];
        __builtin_amdgcn_wave_barrier();
        F.rows_base = uni(F.rows_base);
        F.k = uni(F.k);
        F.r = uni(F.r);
        F.r_end = uni(F.r_end);
        F.atoms = uni(F.atoms);
        F.lists = uni(F.lists);
        F.lpos = uni(F.lpos);
        F.meta_restore = uni(F.meta_restore);
        F.m2lo = uni(F.m2lo);
        F.m2hi = uni(F.m2hi);
        F.m1lo = uni(F.m1lo);
        F.m1hi = uni(F.m1hi);
        if (F.r >= F.r_end) {
            rows_top = F.rows_base;
            meta = F.meta_restore;
            depth--;
            continue;
        }
        uint32_t r = F.r;
        const uint32_t *A = region + F.atoms;
        const uint32_t np = plen + (uint32_t)depth + 1;  // prefix of row r's child class
        if (F.lists != kNone && I.row_cand == nullptr) {
            // Rows whose child class has fewer than two atoms (or would be
            // too long) are passed over from the frame's masks: their
            // candidates are counted and the list position moves past their
            // single entries, with no load.
            const uint64_t m2 = ((uint64_t)F.m2hi << 32) | F.m2lo;
            const uint64_t m1 = ((uint64_t)F.m1hi << 32) | F.m1lo;
            const uint64_t below_end = F.r_end >= 64 ? ~0ull : (1ull << F.r_end) - 1;
            const uint64_t from_r = ~((1ull << r) - 1);  // r < r_end <= k <= kGramMax
            const bool len_ok = I.max_len == 0 || np + 2 <= I.max_len;
            const uint64_t next = len_ok ? (m2 & below_end & from_r) : 0ull;
            const uint32_t r2 = next ? (uint32_t)__builtin_ctzll(next) : F.r_end;
            if (r2 > r) {
                const uint32_t ns = r2 - r;
                // rows r .. r2 - 1 have k - 1 - row candidates each
                st.candidates += (unsigned long long)ns * (F.k - 1) - ((unsigned long long)(r + r2 - 1) * ns) / 2;
                const uint64_t skipped = from_r & (r2 >= 64 ? ~0ull : (1ull << r2) - 1);
                F.lpos += (uint32_t)__popcll(m1 & skipped);
                if (F.k > st.max_k) st.max_k = F.k;
                if ((unsigned long long)depth > st.max_depth) st.max_depth = depth;
                if (r2 >= F.r_end) {
                    if (lane == 0) {
                        ws.frames[depth].r = r2;
                        ws.frames[depth].lpos = F.lpos;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    continue;
                }
                r = r2;
            }
        }
        const uint32_t nj = F.k - r - 1;
        if (F.lists != kNone) {
            // the row's child class, its rank and its item id: from LDS for
            // row 0 of the class built last, else in one round of loads
            uint32_t c, rank_r, id_r;
            uint4 e;
            if (r == 0 && depth == row0_depth) {
                c = uni(ws.row0_n);
                rank_r = uni(ws.row0_rank);
                id_r = uni(ws.row0_id);
                e = ws.row0[lane];
            } else {
                c = uni(gld(A + 3 * F.k + r));
                rank_r = uni(gld(A + r));
                id_r = uni(gld(A + 2 * F.k + r));
                e = gld4(reinterpret_cast<const uint4 *>(region + F.lists) + F.lpos + lane);
            }
            if (lane == 0) {
                ws.frames[depth].r = r + 1;
                ws.frames[depth].lpos = F.lpos + c;
                ws.prefix[plen + depth] = rank_r;
                ws.pid[plen + depth] = id_r;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            st.candidates += nj;
            if (F.k > st.max_k) st.max_k = F.k;
            if ((unsigned long long)depth > st.max_depth) st.max_depth = depth;
            if (I.row_cand && nj && lane == 0)
                atomicAdd(&I.row_cand[l2_class(plen, l2_ref, depth, r, ws)], (unsigned long long)nj);
            if (c < 2 || (I.max_len != 0 && np + 2 > I.max_len)) continue;
            if (depth + 1 >= kMaxDepth || np + 2 > kMaxDepth + 2) {
                if (lane == 0) atomicOr(&ctr->flags, kFlagDepthOverflow);
                continue;
            }
            build = true;
            b_c = c;
            b_rank = e.x;
            b_supp = e.y;
            b_src = e.z;
            b_id = e.w;
            b_r_end = c - 1;
            b_xr = region + F.rows_base + (uint64_t)r * Wp;
            b_base = region + F.rows_base;
            b_write = c >= 3;  // a class of two atoms keeps no rows
            b_rows_base = rows_top;
            b_restore = meta;
            b_em = EmitTo{np, c - 1, kNone, plen >= 2 ? l2_ref : l2_ref + ws.frames[0].r - 1};
            continue;
        }

        // ---- a class too wide to be counted when built: its pairs are
        // counted kWideRows rows at a time (passes through the build block)
        // before those rows are expanded
        if (nj > 0) {
            const uint32_t blk = F.m2hi;
            if (blk == kNone || r >= blk + F.lpos) {
                // a new block of counts for the rows [r, r + nb), below the
                // previous block's place
                const uint64_t m0 = blk == kNone ? meta : (uint64_t)F.m1lo;
                const uint32_t nb = min(min(kWideRows, F.k - 1 - r), F.r_end - r);
                if ((uint64_t)nb * F.k > m0 || m0 - (uint64_t)nb * F.k < rows_top) {
                    flag_stack(ctr, rows_top + (S - m0) + (uint64_t)nb * F.k);
                    break;
                }
                meta = m0 - (uint64_t)nb * F.k;
                if (lane == 0) {
                    ws.frames[depth].m2hi = r;
                    ws.frames[depth].m2lo = (uint32_t)meta;
                    ws.frames[depth].m1lo = (uint32_t)m0;
                    ws.frames[depth].m1hi = r;
                    ws.frames[depth].lpos = nb;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                continue;
            }
            const uint32_t nb = F.lpos;  // rows of the block
            if (F.m1hi < F.k) {
                // one pass: the block's own pairs first, then kGramMax - nb
                // later rows at a time
                const uint32_t jc = F.m1hi;
                const bool own = jc == blk;
                const uint32_t nq = own ? 0u : min(kGramMax - nb, F.k - jc);
                if (lane == 0) ws.frames[depth].m1hi = own ? blk + nb : jc + nq;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                if (own && nb < 2) continue;  // no pair inside a one-row block
                build = true;
                b_counts = true;
                b_c = own ? nb : nb + nq;
                b_r_end = own ? nb - 1 : nb;  // rows whose pairs are counted
                b_src = lane < nb ? blk + lane : jc + (lane - nb);
                b_base = region + F.rows_base;
                b_restore = own ? kNone : jc;
                b_rank = blk;
                continue;
            }
        }
        if (lane == 0) {
            ws.frames[depth].r = r + 1;
            ws.prefix[plen + depth] = A[r];
            ws.pid[plen + depth] = A[2 * F.k + r];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (nj == 0) continue;
        const uint32_t *ranks = A;
        // frequent children of row r, unsorted: ranks, supports, source rows
        if (3ull * nj > meta || meta - 3ull * nj < rows_top) {
            flag_stack(ctr, rows_top + (S - meta) + 3ull * nj);
            break;
        }
        uint32_t *tmp = region + (meta - 3ull * nj);
        const uint4 *row_r = reinterpret_cast<const uint4 *>(region + F.rows_base + (uint64_t)r * Wp);
        // row r's counts: row r - blk of the block
        const uint32_t *cnt_r = region + F.m2lo + (uint64_t)(r - F.m2hi) * F.k;
        uint32_t nf = 0;
        for (uint32_t jb = 0; jb < nj; jb += kWave) {
            const uint32_t jj = jb + lane;
            const uint32_t acc = jj < nj ? gld(cnt_r + r + 1 + jj) : 0u;
            const bool freq = jj < nj && acc >= I.minsup;
            const uint64_t mask = __ballot(freq);
            if (freq) {
                const uint32_t p = nf + lanes_below(mask);
                tmp[p] = ranks[r + 1 + jj];
                tmp[nj + p] = acc;
                tmp[2 * nj + p] = r + 1 + jj;
            }
            nf += (uint32_t)__popcll(mask);
        }
        st.candidates += nj;
        st.pair_words += (unsigned long long)nj * Wp;
        if (I.row_cand && lane == 0)
            atomicAdd(&I.row_cand[l2_class(plen, l2_ref, depth, r, ws)], (unsigned long long)nj);
        if (F.k > st.max_k) st.max_k = F.k;
        if ((unsigned long long)depth > st.max_depth) st.max_depth = depth;
        if (nf == 0) continue;
        __threadfence_block();

        // report the nf itemsets prefix + a_r + child atom
        const uint32_t len = plen + (uint32_t)depth + 2;
        if (I.max_len == 0 || len <= I.max_len) {
            if (I.rec_budget) {
                st.rec_pending += nf;
                if (st.rec_pending >= 4096) {
                    unsigned long long before = 0;
                    if (lane == 0) before = atomicAdd(&ictr[inst].records, st.rec_pending);
                    before = bcast64(before);
                    const unsigned long long now = before + st.rec_pending;
                    st.rec_pending = 0;
                    if (now > I.rec_budget) {
                        if (lane == 0) atomicOr(&ictr[inst].stop, 1u);
                        break;
                    }
                }
            }
            const uint32_t rec = kRecHeader + len;
            st.out_words += (unsigned long long)nf * (I.key_bits ? 8u : rec);
            if (I.class_count) {
                if (lane == 0)
                    atomicAdd(&I.class_count[l2_class(plen, l2_ref, depth, r, ws)], (unsigned long long)nf);
            } else if (I.key_bits) {
                emit_keys(Ig, inst, len, tmp, nj, nf, ws, out, out_cap, ctr);
            } else if (chunk_reserve(oc, nf * rec, task, inst, out, out_cap, ctr)) {
                uint32_t *obase = out + oc.base + oc.pos;
                for (uint32_t e = lane; e < nf; e += kWave) {
                    uint32_t *o = obase + (uint64_t)e * rec;
                    o[0] = len;
                    o[1] = tmp[nj + e];
                    for (uint32_t q = 0; q + 1 < len; q++) o[2 + q] = ws.prefix[q];
                    o[2 + len - 1] = tmp[e];
                }
            }
            if (!I.key_bits) oc.pos += nf * rec;
        }

        // the child class [prefix + a_r | frequent later atoms]
        if (nf < 2 || (I.max_len != 0 && len + 1 > I.max_len)) continue;
        if (depth + 1 >= kMaxDepth || plen + depth + 3 > kMaxDepth + 2) {
            if (lane == 0) atomicOr(&ctr->flags, kFlagDepthOverflow);
            continue;
        }
        const uint64_t restore = meta;
        if (4ull * nf > meta - 3ull * nj || meta - 3ull * nj - 4ull * nf < rows_top) {
            flag_stack(ctr, rows_top + (S - meta) + 3ull * nj + 4ull * nf);
            break;
        }
        const uint64_t new_meta = meta - 3ull * nj - 4ull * nf;
        uint32_t *dst = region + new_meta;
        sort_atoms(Ig, tmp, nj, dst, nf);
        __threadfence_block();
        if (nf <= kGramMax) {
            // the child class is counted as it is built
            const uint32_t q = lane < nf ? lane : 0;
            build = true;
            b_c = nf;
            b_rank = dst[q];
            b_supp = dst[nf + q];
            b_id = dst[2 * nf + q];
            b_src = dst[3 * nf + q];
            b_r_end = nf - 1;
            b_xr = region + F.rows_base + (uint64_t)r * Wp;
            b_base = region + F.rows_base;
            b_write = nf >= 3;
            b_rows_base = rows_top;
            b_restore = restore;
            b_em = EmitTo{np, nf - 1, kNone, plen >= 2 ? l2_ref : l2_ref + ws.frames[0].r - 1};
            meta = new_meta;
            continue;
        }
        if (new_meta < rows_top + (uint64_t)nf * Wp) {
            flag_stack(ctr, rows_top + (uint64_t)nf * Wp + (S - new_meta));
            break;
        }
        // child bitmaps: row_r AND row_src, in the child's atom order
        const uint32_t *srcs = dst + 3 * nf;
        if (g == (uint32_t)kWave) {
            for (uint32_t c = 0; c < nf; c++) {
                const uint4 *row_j = reinterpret_cast<const uint4 *>(region + F.rows_base + (uint64_t)srcs[c] * Wp);
                uint4 *dd = reinterpret_cast<uint4 *>(region + rows_top + (uint64_t)c * Wp);
                and_rows(dd, row_r, row_j, C, lane);
            }
        } else {
            // narrow rows: ppp children at a time, g lanes each
            for (uint32_t c0 = 0; c0 < nf; c0 += ppp) {
                const uint32_t c = c0 + grp;
                if (c < nf) {
                    const uint4 *row_j =
                        reinterpret_cast<const uint4 *>(region + F.rows_base + (uint64_t)srcs[c] * Wp);
                    uint4 *dd = reinterpret_cast<uint4 *>(region + rows_top + (uint64_t)c * Wp);
                    for (uint32_t q = sub; q < C; q += g) dd[q] = and4(row_r[q], row_j[q]);
                }
            }
        }
        __threadfence_block();
        st.child_rows += nf;
        st.row_words += (unsigned long long)nf * Wp;
        if (lane == 0)
            ws.frames[depth + 1] = Frame{(uint32_t)rows_top, nf, 0u, nf - 1, (uint32_t)new_meta, kNone, 0u,
                                         (uint32_t)restore, 0u, kNone, 0u, 0u};
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        rows_top += (uint64_t)nf * Wp;
        meta = new_meta;
        depth++;
        const uint64_t use = rows_top + (S - meta);
        if (use > peak) peak = use;
    }
    st.stack_peak = max(st.stack_peak, (unsigned long long)peak);
}

// the bits of v at the set bits of m, packed from bit 0 up
__device__ __forceinline__ uint32_t pext32(uint32_t v, uint32_t m) {
    uint32_t r = 0, i = 0;
    while (m) {
        const uint32_t b = m & (0u - m);
        if (v & b) r |= 1u << i;
        i++;
        m ^= b;
    }
    return r;
}

// Rows of the first class projected on the cover T(prefix) (see run_frame);
// false when the wave's region is too small.
__device__ bool build_projected(const InstDesc &I, const uint32_t *P, uint32_t s,
                                const uint32_t *ranks, uint32_t k, uint32_t Wq, uint32_t *region,
                                uint64_t S, uint64_t &low, DfsCounters *ctr, uint32_t *stage) {
    const uint32_t lane = lane_id();
    const uint32_t Wf = I.Wp;
    const uint32_t nzc = min(s, Wf);
    if (low < 3ull * nzc + (uint64_t)k * Wq) {
        flag_stack(ctr, (S - low) + 3ull * nzc + (uint64_t)k * Wq);
        return false;
    }
    low -= 3ull * nzc;
    uint32_t *nzw = region + low, *nzm = nzw + nzc, *nzo = nzm + nzc;
    // the non-zero words of T(prefix) and where their bits start in the
    // projected row
    uint32_t cnt = 0, obase = 0;
    for (uint32_t b0 = 0; b0 < Wf; b0 += 8 * kWave) {
        uint32_t xs[8];  // eight words per lane loaded before any is used
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t w = b0 + j * kWave + lane;
            xs[j] = w < Wf ? P[w] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t w = b0 + j * kWave + lane;
            const uint32_t x = xs[j];
            const uint64_t mask = __ballot(x != 0u);
            const uint32_t pc = __popc(x);
            uint32_t incl = pc;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const uint32_t v = __shfl_up(incl, off, kWave);
                if ((int)lane >= off) incl += v;
            }
            if (x) {
                const uint32_t p = cnt + lanes_below(mask);
                nzw[p] = w;
                nzm[p] = x;
                nzo[p] = obase + incl - pc;
            }
            cnt += (uint32_t)__popcll(mask);
            obase += __shfl(incl, kWave - 1, kWave);
        }
    }
    __threadfence_block();
    // words past the projected bits are zero
    const uint32_t used = (s + 31) / 32;
    for (uint32_t e = 0; e < k; e++)
        for (uint32_t q = used + lane; q < Wq; q += kWave) region[(uint64_t)e * Wq + q] = 0u;
    // Lanes take 64 consecutive non-zero words of T(prefix) at a time; the
    // bits of four atoms' rows at those words are packed (pext), ORed into
    // LDS at their offsets in the projected rows (a chunk spans at most 65
    // words), and the touched words are written out.  The first word of a
    // chunk may already hold bits of the previous chunk.
    uint32_t prev_last = ~0u;
    for (uint32_t c0 = 0; c0 < cnt; c0 += kWave) {
        const uint32_t idx = c0 + lane;
        const bool valid = idx < cnt;
        const uint32_t w = valid ? nzw[idx] : 0u, m = valid ? nzm[idx] : 0u;
        const uint32_t o = valid ? nzo[idx] : 0u, nb = __popc(m);
        const uint32_t q0 = uni(o) >> 5;  // lane 0 always holds an entry
        const uint32_t lastl = min(cnt - 1 - c0, (uint32_t)kWave - 1);
        const uint32_t oend = __shfl(o + nb, (int)lastl, kWave);
        const uint32_t nw = ((oend - 1) >> 5) - q0 + 1;
        const uint32_t rel = o - q0 * 32, qq = rel >> 5, sh = rel & 31;
        for (uint32_t e0 = 0; e0 < k; e0 += 4) {
            const uint32_t ne = min(4u, k - e0);
            for (uint32_t i = lane; i < 4 * kStageWords; i += kWave) stage[i] = 0u;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            uint32_t x[4];
#pragma unroll
            for (int j = 0; j < 4; j++)
                x[j] = (valid && (uint32_t)j < ne) ? I.rows[(uint64_t)ranks[e0 + j] * Wf + w] : 0u;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t bits = pext32(x[j] & m, m);
                if (bits) {
                    atomicOr(&stage[j * kStageWords + qq], bits << sh);
                    if (sh && sh + nb > 32) atomicOr(&stage[j * kStageWords + qq + 1], bits >> (32 - sh));
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (uint32_t i = lane; i < nw; i += kWave)
                for (uint32_t j = 0; j < ne; j++) {
                    uint32_t *dst = region + (uint64_t)(e0 + j) * Wq + q0 + i;
                    uint32_t v = stage[j * kStageWords + i];
                    if (i == 0 && q0 == prev_last) v |= *dst;
                    *dst = v;
                }
            wave_mem_wait();  // the next chunk may read its first word back
            __builtin_amdgcn_wave_barrier();
        }
        prev_last = q0 + nw - 1;
    }
    return true;
}

// The first class of a piece of work: its sibling rows T(prefix + atom) for
// every atom (Prepare-Tidlists), at region[0, k Wp) with the atom arrays at
// meta_out; returns the row width used (0: nothing to search).  When the
// cover T(prefix) holds at most a quarter of the row's bits, the rows are
// built projected on that cover: bit i of a projected row is the row's bit
// at the i-th transaction of T(prefix).  Every support below the prefix is
// a popcount of ANDs of such rows, so the results are the same, and the
// whole subtree works on rows of ceil(supp(prefix) / 32) words.
__device__ __forceinline__ uint32_t prepare_frame(const InstDesc &I, const InstDesc &Ig, uint32_t inst,
                                                  const FrameSrc &src,
                                                  uint32_t *region, uint64_t S, WaveShared &ws,
                                                  DfsCounters *ctr, InstCounters *ictr, WaveStats &st,
                                                  uint64_t &meta_out, uint64_t &low_out) {
    if (inst_stopped(I, ictr, inst)) return 0;
    const uint32_t lane = lane_id();
    const uint32_t k = src.k, plen = src.plen;
    if (src.r_end == 0 || src.r_end >= k || plen == 0 || plen + 2 > kMaxDepth) return 0;
    const uint32_t Wf = I.Wp, Cf = Wf / 4;
    if (3ull * k + (uint64_t)k * kRowAlign > S) {
        flag_stack(ctr, 3ull * k + (uint64_t)k * Wf);
        return 0;
    }
    const uint64_t meta = S - 3ull * k;
    for (uint32_t e = lane; e < k; e += kWave) {
        const uint32_t rk = src.ranks[e];
        region[meta + e] = rk;
        region[meta + k + e] = src.supps[e];
        region[meta + 2 * k + e] = I.item_of_rank[rk];
    }
    for (uint32_t q = lane; q < plen; q += kWave) {
        ws.prefix[q] = src.prefix[q];
        ws.pid[q] = I.item_of_rank[src.prefix[q]];
    }
    uint64_t low = meta;  // region[0, low) is free
    // One-item prefix with its transaction list at hand: projected row e
    // holds bit i = [the i-th transaction of T(prefix) holds atom e], 64 bits
    // per ballot
    if (plen == 1 && I.tl != nullptr) {
        const uint64_t t0 = I.tl_off[src.prefix[0]];
        const uint32_t s = uni((uint32_t)(I.tl_off[src.prefix[0] + 1] - t0));
        const uint32_t Wq = max(kRowAlign, ((s + 31) / 32 + kRowAlign - 1) / kRowAlign * kRowAlign);
        if (I.project && 4ull * Wq <= Wf) {
            if (low < (uint64_t)k * Wq) {
                flag_stack(ctr, (S - low) + (uint64_t)k * Wq);
                return 0;
            }
            // Groups of kG ballot rounds (kG * 64 transactions, 2 kG words):
            // the group's transaction ids stay in registers while every atom's
            // words are gathered, kA atoms at a time (kA * kG loads in
            // flight); lane q < 2 kG collects word q of the group and stores
            // it.  The groups cover every word below Wq (zeros past s).
            const uint32_t *tids = I.tl + t0;
            constexpr uint32_t kG = 8, kA = 2;
            for (uint32_t g0 = 0; g0 < s; g0 += kG * kWave) {
                uint32_t tg[kG];
#pragma unroll
                for (uint32_t j = 0; j < kG; j++) {
                    const uint32_t i = g0 + j * kWave + lane;
                    tg[j] = i < s ? tids[i] : kNone;
                }
                const uint32_t wbase = g0 / 32;
                for (uint32_t e0 = 0; e0 < k; e0 += kA) {
                    uint32_t x[kA][kG];
#pragma unroll
                    for (uint32_t a = 0; a < kA; a++) {
                        const uint32_t e = min(e0 + a, k - 1);  // past k: a repeat, not stored
                        const uint32_t *ra = I.rows + (uint64_t)src.ranks[e] * Wf;
#pragma unroll
                        for (uint32_t j = 0; j < kG; j++) {
                            const uint32_t t = tg[j];
                            x[a][j] = t != kNone ? ra[t >> 5] : 0u;
                        }
                    }
#pragma unroll
                    for (uint32_t a = 0; a < kA; a++) {
                        uint32_t w = 0;
#pragma unroll
                        for (uint32_t j = 0; j < kG; j++) {
                            const uint64_t bits = __ballot((x[a][j] >> (tg[j] & 31)) & 1u);
                            if (lane == 2 * j) w = (uint32_t)bits;
                            else if (lane == 2 * j + 1) w = (uint32_t)(bits >> 32);
                        }
                        if (e0 + a < k && lane < 2 * kG && wbase + lane < Wq)
                            region[(uint64_t)(e0 + a) * Wq + wbase + lane] = w;
                    }
                }
            }
            __threadfence_block();
            st.row_words += (unsigned long long)k * Wq;
            meta_out = meta;
            low_out = low;
            return Wq;
        }
    }
    // T(prefix): the item's own row, or the AND of the prefix items' rows
    const uint32_t *P = I.rows + (uint64_t)src.prefix[0] * Wf;
    if (plen > 1) {
        if (low < Wf) {
            flag_stack(ctr, (uint64_t)(k + 1) * Wf + 3ull * k);
            return 0;
        }
        low -= Wf;
        uint4 *pr = reinterpret_cast<uint4 *>(region + low);
        and_rows(pr, reinterpret_cast<const uint4 *>(P),
                 reinterpret_cast<const uint4 *>(I.rows + (uint64_t)src.prefix[1] * Wf), Cf, lane);
        __threadfence_block();
        for (uint32_t q = 2; q < plen; q++) {
            and_rows(pr, pr, reinterpret_cast<const uint4 *>(I.rows + (uint64_t)src.prefix[q] * Wf),
                     Cf, lane);
            __threadfence_block();
        }
        P = region + low;
    }
    // the prefix's support, and the width of rows projected on its cover
    uint32_t s = 0;
    {
        uint32_t w = lane;
        for (; w + 7 * kWave < Wf; w += 8 * kWave) {  // eight loads in flight
            uint32_t x[8];
#pragma unroll
            for (int j = 0; j < 8; j++) x[j] = P[w + j * kWave];
#pragma unroll
            for (int j = 0; j < 8; j++) s += __popc(x[j]);
        }
        for (; w < Wf; w += kWave) s += __popc(P[w]);
    }
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o, kWave);
    s = uni(s);
    const uint32_t Wq = max(kRowAlign, ((s + 31) / 32 + kRowAlign - 1) / kRowAlign * kRowAlign);
    uint32_t Wp = Wf;
    if (I.project && 4ull * Wq <= Wf) {
        if (!build_projected(Ig, P, s, src.ranks, k, Wq, region, S, low, ctr, ws.gx)) return 0;
        Wp = Wq;
    } else {
        if (low < (uint64_t)k * Wf) {
            flag_stack(ctr, (uint64_t)k * Wf + (S - low));
            return 0;
        }
        for (uint32_t e = 0; e < k; e++)
            and_rows(reinterpret_cast<uint4 *>(region + (uint64_t)e * Wf),
                     reinterpret_cast<const uint4 *>(P),
                     reinterpret_cast<const uint4 *>(I.rows + (uint64_t)src.ranks[e] * Wf), Cf, lane);
    }
    __threadfence_block();
    st.row_words += (unsigned long long)k * Wp;
    meta_out = meta;
    low_out = low;
    return Wp;
}

__device__ __forceinline__ void flush_stats(const InstDesc &I, InstCounters *ictr, uint32_t inst,
                                            const WaveStats &st) {
    if (lane_id() == 0) {
        InstCounters &ic = ictr[inst];
        if (st.candidates) atomicAdd(&ic.candidates, st.candidates);
        if (st.pair_words) atomicAdd(&ic.pair_words, st.pair_words);
        if (st.child_rows) atomicAdd(&ic.child_rows, st.child_rows);
        if (st.row_words) atomicAdd(&ic.row_words, st.row_words);
        if (st.out_words) atomicAdd(&ic.out_words, st.out_words);
        if (st.rec_pending &&
            atomicAdd(&ic.records, st.rec_pending) + st.rec_pending > I.rec_budget)
            atomicOr(&ic.stop, 1u);
    }
}

__global__ __launch_bounds__(kBlock) void k_dfs(const InstDesc *insts, const Task *tasks,
                                                uint64_t n_tasks, uint32_t *stack,
                                                uint64_t stack_words, uint32_t tasks_per_claim,
                                                uint32_t tmax,
                                                uint32_t *out, uint64_t out_cap,
                                                DfsCounters *ctr, InstCounters *ictr,
                                                Donation dn, uint32_t waves_per_block) {
    __shared__ WaveShared shared[kWavesPerBlock];
    const uint32_t w = uni(threadIdx.x / kWave);
    // a launch with fewer workers than CUs keeps one wave per block, so that
    // its waves spread over all CUs (the other waves leave at once; there is
    // no block barrier)
    if (w >= waves_per_block) return;
    const uint32_t lane = lane_id();
    WaveShared &ws = shared[w];
    if (lane == 0) ws.n_recs = 0;
    const uint64_t wave_id = (uint64_t)blockIdx.x * waves_per_block + w;
    uint32_t *region = stack + wave_id * stack_words;
    unsigned long long busy = 0;
    WaveTrace wt{0, 0, 0, 0, 0, 0, 0, 0};
    auto note = [&](const WaveStats &st) {
        wt.pieces++;
        wt.given += st.given;
        wt.candidates += st.candidates;
        wt.max_k = max(wt.max_k, st.max_k);
        wt.max_depth = max(wt.max_depth, st.max_depth);
    };
    // Pieces of work: the planned tasks in LPT order, then donated classes
    // until no wave is active and the queue is drained.  Both kinds go
    // through the one call of the search below.
    bool planned = true;
    uint64_t t_next = 0, t_end = 0;
    // statistics of the pieces of instance sum_inst not yet added to its
    // counters (one flush per wave and instance instead of one per piece)
    WaveStats sum{};
    uint32_t sum_inst = kNone;
    unsigned long long stack_peak = 0;  // of all the wave's pieces
    auto flush_sum = [&]() {
        if (sum_inst != kNone) flush_stats(insts[sum_inst], ictr, sum_inst, sum);
        sum = WaveStats{};
        sum_inst = kNone;
    };
    unsigned long long since = 0;
    uint32_t nap = 1;
    for (;;) {
        FrameSrc fs{};
        uint32_t inst = 0, task = 0;
        uint64_t S = stack_words;
        bool have = false;
        if (planned) {
            if (t_next >= t_end) {
                // a wave counts as active from its first claim until no
                // planned task is left, so consecutive claims touch only
                // the task counter (every counter here is one hot line)
                unsigned long long t0 = 0;
                if (lane == 0) {
                    if (!t_end) atomicAdd(&ctr->active.v, 1ull);
                    t0 = atomicAdd(&ctr->task_head.v, (unsigned long long)tasks_per_claim);
                }
                t0 = bcast64(t0);
                if (t0 >= n_tasks) {
                    wave_mem_wait();  // donations of the claimed tasks are published before they count as done
                    if (lane == 0) atomicSub(&ctr->active.v, 1ull);
                    planned = false;
                    if (!dn.enabled) break;
                    if (lane == 0) atomicAdd(&ctr->idle.v, 1ull);
                    since = wall_clock64();
                    continue;
                }
                t_next = t0;
                t_end = min((uint64_t)t0 + tasks_per_claim, n_tasks);
            }
            const uint64_t t = t_next++;
            Task T = tasks[t];
            T.inst = uni(T.inst);
            T.node = uni(T.node);
            T.r0 = uni(T.r0);
            T.r1 = uni(T.r1);
            const InstDesc &I = insts[T.inst];
            const uint32_t a0 = uni(I.l2_off[T.node]), k1 = uni(I.l2_off[T.node + 1]) - a0;
            if (T.r0 >= T.r1 || T.r1 >= k1) continue;  // rows with a later atom only
            fs = FrameSrc{&tasks[t].node, I.l2_atom + a0 + T.r0, I.l2_supp + a0 + T.r0, 1u,
                          k1 - T.r0, T.r1 - T.r0, a0 + T.r0, 0u};
            inst = T.inst;
            task = (uint32_t)t;
            have = true;
        } else {
            unsigned long long got = ~0ull;
            uint32_t done = 0;
            if (lane == 0) {
                const unsigned long long h = load_coherent(&ctr->don_head.v);
                const unsigned long long tl = min(load_coherent(&ctr->don_tail.v), dn.n_slots);
                if (h < tl) {
                    if (atomicCAS(&ctr->don_head.v, h, h + 1) == h) got = h;
                } else if (load_coherent(&ctr->active.v) == 0) {
                    // nobody can donate any more; re-read the queue after
                    // seeing that
                    const unsigned long long h2 = load_coherent(&ctr->don_head.v);
                    const unsigned long long t2 = min(load_coherent(&ctr->don_tail.v), dn.n_slots);
                    done = h2 >= t2 ? 1u : 0u;
                }
            }
            got = bcast64(got);
            done = bcast32(done);
            if (done) break;
            if (got == ~0ull) {
                // A wave that found no donated work for the whole bound
                // leaves quietly: no work is lost, since a donor that runs
                // out of work comes back here and drains the queue itself.
                if (wall_clock64() - since > dn.wait_ticks) break;
                // back off: 1, 2, 4 ... nap_max naps of about 8000 cycles
                for (uint32_t q = 0; q < nap; q++) __builtin_amdgcn_s_sleep(127);
                if (nap < dn.nap_max) nap <<= 1;
                continue;
            }
            nap = 1;
            if (lane == 0) {
                atomicAdd(&ctr->active.v, 1ull);
                atomicSub(&ctr->idle.v, 1ull);
            }
            // wait until the donor has published the slot it reserved
            unsigned long long off = 0;
            const unsigned long long w0 = wall_clock64();
            for (;;) {
                if (lane == 0) off = load_coherent(&dn.slots[got]);
                off = bcast64(off);
                if (off != 0 || wall_clock64() - w0 > dn.wait_ticks) break;
                __builtin_amdgcn_s_sleep(4);
            }
            if (off != 0) {
                // copy the record into this wave's own memory with coherent loads
                const uint32_t *rec = dn.heap + (off - 1);
                const uint32_t di = uni(load_coherent32(rec)), pl = uni(load_coherent32(rec + 1));
                const uint32_t kk = uni(load_coherent32(rec + 2)), rw = uni(load_coherent32(rec + 3));
                const uint32_t ref = uni(load_coherent32(rec + 4));
                const uint32_t re = rw & 0x7FFFFFFFu, reported = rw >> 31;
                const uint32_t words = pl + 2 * kk;
                if ((uint64_t)words <= stack_words / 2) {
                    uint32_t *copy = region + (stack_words - words);
                    for (uint32_t q = lane; q < words; q += kWave) copy[q] = load_coherent32(rec + 5 + q);
                    wave_mem_wait();
                    fs = FrameSrc{copy, copy + pl, copy + pl + kk, pl, kk, re, ref, reported};
                    inst = di;
                    task = (uint32_t)(n_tasks + got);
                    S = stack_words - words;  // the frame's own arrays go below the copy
                    have = true;
                } else if (lane == 0) {
                    atomicOr(&ctr->flags, kFlagStackOverflow);
                    atomicMax(&ctr->stack_need, 2ull * words);
                }
            } else if (lane == 0) {
                atomicOr(&ctr->flags, kFlagSpin);
            }
        }
        if (have) {
            // The descriptor is read once into registers: read through the
            // reference, every use after a store would load it again and
            // wait for all of the wave's outstanding stores (the child rows
            // just written) first.  The out-of-line helpers take the
            // reference.
            const InstDesc &Ig = insts[inst];
            const InstDesc I = Ig;
            WaveStats st{};
            OutChunk oc{kNoChunk, 0u, 0u, 0u, 0u};
            const unsigned long long c0 = wall_clock64();
            uint64_t meta = 0, low = 0;
            const uint32_t Wp = prepare_frame(I, Ig, inst, fs, region, S, ws, ctr, ictr, st, meta, low);
            if (Wp)
                search(I, Ig, inst, task, fs.plen, fs.l2_ref, Wp, fs.k, fs.r_end, fs.reported, meta,
                       (S - low) + (uint64_t)fs.k * Wp, tmax, region, S, ws, out, out_cap, ctr, ictr, st,
                       oc, dn);
            close_chunk(oc, out);
            busy += wall_clock64() - c0;
            if (I.rec_budget) {
                flush_stats(I, ictr, inst, st);  // the budget's stop test needs the records now
            } else {
                if (sum_inst != inst) flush_sum();
                sum_inst = inst;
                sum.candidates += st.candidates;
                sum.pair_words += st.pair_words;
                sum.child_rows += st.child_rows;
                sum.row_words += st.row_words;
                sum.out_words += st.out_words;
            }
            stack_peak = max(stack_peak, st.stack_peak);
            note(st);
        }
        if (!planned) {
            wave_mem_wait();
            if (lane == 0) {
                atomicAdd(&ctr->idle.v, 1ull);
                atomicSub(&ctr->active.v, 1ull);
            }
            since = wall_clock64();
        }
    }
    if (!planned && dn.enabled && lane == 0) atomicSub(&ctr->idle.v, 1ull);
    // key records staged in LDS go out when the stage fills and here
    flush_recs(ws, out, out_cap, ctr);
    flush_sum();
    if (lane == 0 && stack_peak) atomicMax(&ctr->stack_need, stack_peak);
    if (lane == 0 && busy) {
        atomicAdd(&ctr->busy_sum, busy);
        atomicMax(&ctr->busy_max, busy);
    }
    if (lane == 0 && dn.trace) {
        wt.busy = busy;
        WaveTrace *tr = reinterpret_cast<WaveTrace *>(dn.trace) + wave_id;
        *tr = wt;
    }
}

}  // namespace

// ------------------------------------------------------------------ records of the 1- and 2-itemsets
// One thread per record; blockIdx.y is the instance.  Codes (id + 1) of
// `bits` bits from the top of the 128-bit key, items ascending.
__global__ void k_prefix_keys(const PrefixSrc *__restrict__ src, uint32_t *out) {
    const PrefixSrc S = src[blockIdx.y];
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S.n_freq + S.n_pairs) return;
    uint32_t id0, id1 = 0, n, supp;
    if (j < S.n_freq) {
        id0 = S.item_of_rank[j];
        n = 1;
        supp = S.counts[id0];
    } else {
        const uint64_t p = j - S.n_freq;
        const uint32_t a = S.item_of_rank[S.pairs[3 * p]], b = S.item_of_rank[S.pairs[3 * p + 1]];
        id0 = min(a, b);
        id1 = max(a, b);
        n = 2;
        supp = S.pairs[3 * p + 2];
    }
    unsigned long long hi = 0, lo = 0;
    uint32_t sh = 128;
    for (uint32_t x = 0; x < n; x++) {
        const unsigned long long code = (unsigned long long)(x == 0 ? id0 : id1) + 1;
        sh -= S.bits;
        hi |= sh >= 64 ? code << (sh - 64) : (sh + S.bits > 64 ? code >> (64 - sh) : 0ull);
        lo |= sh >= 64 ? 0ull : code << sh;
    }
    uint4 *o = reinterpret_cast<uint4 *>(out + 8ull * (S.out_rec + j));
    o[0] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    o[1] = make_uint4(supp, S.inst, 0u, 0u);
}

// ------------------------------------------------------------------ launch wrappers

// blocks of the per-block histograms and the chunk each one counts
static void item_hist_shape(uint64_t nnz, uint32_t *nb, uint64_t *chunk) {
    const uint64_t c = std::max<uint64_t>(8192, (nnz + 255) / 256);
    *chunk = c;
    *nb = (uint32_t)std::max<uint64_t>(1, (nnz + c - 1) / c);
}

uint64_t item_count_scratch_words(uint64_t nnz, uint32_t n_item_ids) {
    if (nnz == 0 || n_item_ids > kHistItems) return 0;
    uint32_t nb = 0;
    uint64_t chunk = 0;
    item_hist_shape(nnz, &nb, &chunk);
    return (uint64_t)nb * n_item_ids;
}

hipError_t launch_item_count(const uint32_t *items, uint64_t nnz, uint32_t *counts,
                             uint32_t n_item_ids, uint32_t *part, hipStream_t stream) {
    if (n_item_ids == 0) return hipSuccess;
    if (nnz == 0 || n_item_ids > kHistItems) {
        hipError_t e = launch_fill_u32(counts, n_item_ids, 0u, stream);
        if (e != hipSuccess || nnz == 0) return e;
        const uint64_t blocks = std::min<uint64_t>((nnz + kBlock - 1) / kBlock, 4096);
        hipLaunchKernelGGL(k_item_count, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, items,
                           nnz, counts);
        return hipGetLastError();
    }
    uint32_t nb = 0;
    uint64_t chunk = 0;
    item_hist_shape(nnz, &nb, &chunk);
    hipLaunchKernelGGL(k_item_hist, dim3(nb), dim3(kBlock), (size_t)n_item_ids * 4, stream, items,
                       nnz, chunk, n_item_ids, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_item_sum, dim3((n_item_ids + kWave - 1) / kWave), dim3(kBlock), 0, stream,
                       part, nb, n_item_ids, counts);
    return hipGetLastError();
}

uint32_t count_many_blocks(uint64_t nnz) { return (uint32_t)((nnz + kCountChunk - 1) / kCountChunk); }

hipError_t launch_item_count_many(const CountSrc *src, uint32_t n_src, uint32_t blocks, uint32_t max_ids,
                                  uint32_t *counts, hipStream_t stream) {
    if (n_src == 0 || blocks == 0) return hipSuccess;
    const size_t lds = (size_t)std::min<uint32_t>(max_ids, kHistItems) * 4;
    hipLaunchKernelGGL(k_item_count_many, dim3(blocks), dim3(kBlock), lds, stream, src, n_src, counts);
    return hipGetLastError();
}

hipError_t launch_fill_words(uint32_t *p, uint64_t n, uint64_t at, unsigned long long v,
                             hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_fill_words, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, p, n, at, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_bitmap_build(const uint64_t *offsets, const uint32_t *items, uint64_t n_tx,
                               const uint32_t *rank_of_item, uint32_t *rows, uint32_t Wp,
                               hipStream_t stream) {
    if (n_tx == 0) return hipSuccess;
    const uint64_t blocks = (n_tx + kBuildTx - 1) / kBuildTx;
    if (blocks >= (1ull << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bitmap_build, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, offsets,
                       items, n_tx, rank_of_item, rows, Wp);
    return hipGetLastError();
}

hipError_t launch_tidlist(const uint32_t *rows, uint32_t n, uint32_t Wp, const uint64_t *tl_off,
                          uint32_t *tl, uint16_t *tl_rank, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tidlist, dim3((n + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0,
                       stream, rows, n, Wp, tl_off, tl, tl_rank);
    return hipGetLastError();
}

hipError_t launch_rank_only(const uint64_t *off, const uint32_t *items, uint64_t n_tx,
                            const uint32_t *rank_of_item, uint16_t *rk, hipStream_t stream) {
    if (n_tx == 0) return hipSuccess;
    const uint64_t groups = (n_tx + kRankGroup - 1) / kRankGroup;
    const uint64_t blocks = std::min<uint64_t>((groups + kWavesPerBlock - 1) / kWavesPerBlock, 65536);
    hipLaunchKernelGGL(k_rank_tx, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, off, items, n_tx,
                       rank_of_item, rk);
    return hipGetLastError();
}

hipError_t launch_tl_slots(const uint64_t *off, uint64_t n_tx, const uint16_t *rk, const uint32_t *tl,
                           uint64_t n_ent, uint32_t *tlp, uint16_t *suf, hipStream_t stream) {
    if (n_tx == 0 || n_ent == 0) return hipSuccess;
    const uint64_t eb = (n_ent + kBlock - 1) / kBlock;
    if (eb >= (1ull << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tl_slots, dim3((uint32_t)eb), dim3(kBlock), 0, stream, off, rk, tl, n_ent,
                       tlp, suf);
    return hipGetLastError();
}

hipError_t launch_rank_tx(const uint64_t *off, const uint32_t *items, uint64_t n_tx,
                          const uint32_t *rank_of_item, const uint32_t *tl, uint64_t n_ent,
                          uint16_t *rk, uint32_t *tlp, uint16_t *suf, hipStream_t stream) {
    const hipError_t e = launch_rank_only(off, items, n_tx, rank_of_item, rk, stream);
    if (e != hipSuccess) return e;
    return launch_tl_slots(off, n_tx, rk, tl, n_ent, tlp, suf, stream);
}

// words per column tile for n rows within lds_max bytes of LDS, the block's
// transaction offsets included (0: does not fit)
// Tile shape of launch_bitmap_tiles: K words (a power of two, 4 to 32) by
// nr rows.  Every row group scans all items of its column window, so the
// rows are split only when four words of every row do not fit the LDS; K is
// the widest that fits half of it (two blocks per CU; all of it when even
// K = 4 needs more), and shrinks while there are fewer than kTileBlocks
// blocks.  (Measured on 200,000 transactions x 4849 sparse rows: 99 us with
// K = 4 and two blocks per CU, 126 us with K = 8 and one, 314 us with
// 32-word tiles of ten row groups.)
constexpr uint64_t kTileBlocks = 512;

constexpr size_t kTileStaticLds = (32 * kTileMaxWords + 1) * sizeof(uint64_t);  // s_off

static void bitmap_tile_shape(uint32_t n, uint32_t Wp, size_t lds_max, uint32_t *K, uint32_t *nr) {
    const size_t half = lds_max / 2 - kTileStaticLds, all = lds_max - kTileStaticLds;
    const size_t budget = (uint64_t)n * 16 <= half ? half : all;
    const uint32_t rows = (uint32_t)std::max<size_t>(1, std::min<size_t>(n, budget / 16));
    uint32_t k = kTileMaxWords;
    while (k > 4 && (uint64_t)rows * k * 4 > budget) k /= 2;
    while (k > 4 && (uint64_t)((n + rows - 1) / rows) * ((Wp + k - 1) / k) < kTileBlocks) k /= 2;
    *K = k;
    *nr = rows;
}

bool bitmap_tiles_fit(size_t lds_max) { return lds_max >= 2 * kTileStaticLds + 16; }

hipError_t launch_bitmap_tiles(const uint64_t *offsets, const uint32_t *items, uint64_t n_tx,
                               const uint32_t *rank_of_item, uint32_t n, uint32_t *rows,
                               uint32_t Wp, size_t lds_max, hipStream_t stream) {
    if (n == 0 || Wp == 0) return hipSuccess;
    if (Wp % 4 != 0 || !bitmap_tiles_fit(lds_max)) return hipErrorInvalidValue;
    uint32_t K = 0, nr = 0;
    bitmap_tile_shape(n, Wp, lds_max, &K, &nr);
    const uint32_t groups = (n + nr - 1) / nr;
    const uint64_t blocks = (uint64_t)groups * ((Wp + K - 1) / K);
    if (blocks >= (1ull << 31)) return hipErrorInvalidValue;
    const size_t lds = (size_t)nr * K * 4;
    // the kernel's dynamic LDS limit is raised once per device to the
    // largest size asked for (the call costs microseconds per launch)
    constexpr int kDevs = 64;
    static std::atomic<int> lds_set[kDevs];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const bool known = dev >= 0 && dev < kDevs;
    if (!known || lds_set[dev].load() < (int)lds) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bitmap_tile),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        if (known) {
            int cur = lds_set[dev].load();
            while (cur < (int)lds && !lds_set[dev].compare_exchange_weak(cur, (int)lds)) {
            }
        }
    }
    hipLaunchKernelGGL(k_bitmap_tile, dim3((uint32_t)blocks), dim3(kBlock), lds, stream, offsets,
                       items, n_tx, rank_of_item, n, rows, Wp, K, nr, groups);
    return hipGetLastError();
}

hipError_t launch_prefix_keys(const PrefixSrc *src, uint32_t n_src, uint64_t max_rec, uint32_t *out,
                              hipStream_t stream) {
    if (n_src == 0 || max_rec == 0) return hipSuccess;
    const uint64_t bx = (max_rec + kBlock - 1) / kBlock;
    if (bx >= (1ull << 31) || n_src > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_prefix_keys, dim3((uint32_t)bx, n_src), dim3(kBlock), 0, stream, src, out);
    return hipGetLastError();
}

uint64_t root_pairs_scratch_words() { return (uint64_t)kRootSplitBlocks * kRootTilePairs; }

hipError_t launch_root_pairs(const uint32_t *rows, uint32_t n, uint32_t Wp, uint32_t minsup,
                             uint32_t *pairs, uint64_t cap, unsigned long long *n_pairs,
                             uint32_t *part, hipStream_t stream) {
    if (n < 2) return hipSuccess;
    const uint64_t nt = (n + kRootRows - 1) / kRootRows;
    const uint64_t tiles = nt * (nt + 1) / 2;
    if (tiles > 0x7FFFFFFFull) return hipErrorInvalidValue;
    // word ranges: a multiple of the LDS tile width, at least
    // kRootSplitMinWords each, tiles * splits <= kRootSplitBlocks
    uint64_t splits = 1;
    if (part && tiles * 2 <= kRootSplitBlocks)
        splits = std::min<uint64_t>(kRootSplitBlocks / tiles, (Wp + kRootSplitMinWords - 1) / kRootSplitMinWords);
    uint32_t chunk = Wp;
    if (splits > 1) {
        chunk = (uint32_t)(((Wp + splits - 1) / splits + kRootTw - 1) / kRootTw * kRootTw);
        splits = (Wp + chunk - 1) / chunk;
    }
    if (splits <= 1) {
        hipLaunchKernelGGL(k_root_pairs, dim3((uint32_t)tiles, 1), dim3(kBlock), 0, stream, rows, n, Wp,
                           Wp, minsup, pairs, cap, n_pairs, (uint32_t *)nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_root_pairs, dim3((uint32_t)tiles, (uint32_t)splits), dim3(kBlock), 0, stream, rows,
                       n, Wp, chunk, minsup, pairs, cap, n_pairs, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_root_finish, dim3((uint32_t)tiles), dim3(kBlock), 0, stream, part,
                       (uint32_t)splits, n, minsup, pairs, cap, n_pairs);
    return hipGetLastError();
}

hipError_t launch_row_nonzero(const uint32_t *rows, uint32_t n, uint32_t Wp, const uint64_t *nz_off,
                              uint32_t *nz_w, uint32_t *nz_m, uint32_t *nz_cnt,
                              hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_nonzero, dim3((n + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock),
                       0, stream, rows, n, Wp, nz_off, nz_w, nz_m, nz_cnt);
    return hipGetLastError();
}

hipError_t launch_transpose(const uint32_t *rows, uint32_t n, uint32_t Wp, uint32_t W, uint32_t *bt,
                            uint32_t np, hipStream_t stream) {
    if (n == 0 || W == 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose, dim3((W + 63) / 64, (np + 63) / 64), dim3(kBlock), 0, stream,
                       rows, n, Wp, W, bt, np);
    return hipGetLastError();
}

hipError_t launch_root_sparse(const uint32_t *bt, uint32_t np, const uint64_t *nz_off,
                              const uint32_t *nz_cnt, const uint32_t *nz_w, const uint32_t *nz_m,
                              uint32_t n, uint32_t minsup, uint32_t *pairs, uint64_t cap,
                              unsigned long long *n_pairs, hipStream_t stream) {
    if (n < 2) return hipSuccess;
    const uint32_t jblocks = (np + kSparseCols - 1) / kSparseCols;
    hipLaunchKernelGGL(k_root_sparse, dim3(jblocks, n), dim3(kBlock), 0, stream, bt, np, nz_off,
                       nz_cnt, nz_w, nz_m, n, minsup, pairs, cap, n_pairs);
    return hipGetLastError();
}

// counters of a block: R rows x J columns in 60 KB of LDS
void project_tile(uint32_t n, uint32_t *R, uint32_t *J) {
    const uint32_t words = 15360;
    *J = std::max<uint32_t>(1, std::min<uint32_t>(n, words));
    *R = std::max<uint32_t>(1, std::min<uint32_t>(kProjectMaxRows, words / *J));
}

hipError_t launch_root_project(const uint16_t *rk, const uint32_t *tlp, const uint16_t *suf,
                               const uint64_t *tl_off, uint32_t n, uint32_t max_supp,
                               uint32_t minsup, uint32_t *pairs, uint64_t cap,
                               unsigned long long *n_pairs, unsigned long long *work,
                               hipStream_t stream) {
    if (n < 2) return hipSuccess;
    uint32_t R = 0, J = 0;
    project_tile(n, &R, &J);
    const dim3 grid((n + R - 1) / R, (n + J - 1) / J);
    if (max_supp <= 0xFFFFu) {
        hipLaunchKernelGGL(k_root_project<true>, grid, dim3(kBlock), (size_t)(R * J + 1) / 2 * 4,
                           stream, rk, tlp, suf, tl_off, n, R, J, minsup, pairs, cap, n_pairs, work);
    } else {
        hipLaunchKernelGGL(k_root_project<false>, grid, dim3(kBlock), (size_t)R * J * 4, stream, rk,
                           tlp, suf, tl_off, n, R, J, minsup, pairs, cap, n_pairs, work);
    }
    return hipGetLastError();
}

// The persistent kernel has one variant; `variant` is the widest LDS row
// tile (words) of the classes counted from LDS: a power of two from
// kTileMin to kTileDefault (0 = kTileDefault).
uint32_t tile_variant(uint32_t tile_words) {
    uint32_t t = kTileMin;
    while (t < tile_words && t < kTileDefault) t <<= 1;
    return t;
}

uint32_t dfs_variant(uint32_t) { return kTileDefault; }

uint32_t dfs_resident_workers(int n_cu, uint32_t) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_dfs, kBlock, 0) != hipSuccess || blocks <= 0) {
        (void)hipGetLastError();
        blocks = 1;
    }
    return (uint32_t)blocks * kWavesPerBlock * (uint32_t)n_cu;
}

hipError_t launch_dfs(const InstDesc *insts, const Task *tasks, uint64_t n_tasks, uint32_t *stack,
                      uint64_t stack_words, uint32_t n_workers, uint32_t tasks_per_claim,
                      uint32_t *out, uint64_t out_cap, DfsCounters *ctr, InstCounters *ictr,
                      unsigned long long *don_slots, uint64_t n_slots, uint32_t *don_heap,
                      uint64_t heap_words, uint64_t wait_ticks, unsigned long long *trace,
                      uint32_t variant, uint32_t nap_max, uint64_t poll_ticks, uint32_t waves_per_block,
                      hipStream_t stream) {
    if (n_tasks == 0) return hipSuccess;
    const uint32_t wpb = waves_per_block >= 1 && waves_per_block <= (uint32_t)kWavesPerBlock
                             ? waves_per_block : (uint32_t)kWavesPerBlock;
    if (n_workers % wpb != 0) return hipErrorInvalidValue;
    const uint32_t blocks = n_workers / wpb;
    Donation dn{don_slots, don_heap, n_slots, heap_words, wait_ticks,
                (don_slots && don_heap && n_slots && heap_words) ? 1u : 0u, trace,
                nap_max ? nap_max : 64u, poll_ticks ? poll_ticks : 1u};
    const uint32_t tpc = tasks_per_claim ? tasks_per_claim : 1u;
    const uint32_t tmax = variant ? tile_variant(variant) : kTileDefault;
    hipLaunchKernelGGL(k_dfs, dim3(blocks), dim3(kBlock), 0, stream, insts, tasks, n_tasks, stack,
                       stack_words, tpc, tmax, out, out_cap, ctr, ictr, dn, wpb);
    return hipGetLastError();
}

}  // namespace fim
