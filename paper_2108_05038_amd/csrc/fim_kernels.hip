// HIP kernels of the frequent-itemset miner, written for gfx950 (CDNA4,
// wave64).  Support counting is integer AND + popcount over vertical
// transaction bitmaps (the bitmap form of the thesis's lemma that the
// support of an itemset is the size of the intersection of the tid-lists of
// two of its covering subsets, appendix "The Eclat algorithm", subsection
// "Support counting").  No MFMA: the work is bitwise, and most of it is
// bound by memory or by the integer vector ALU.
#include <algorithm>

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

__device__ __forceinline__ uint4 and4(uint4 a, uint4 b) {
    return make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w);
}

// popcount(a AND b) over the 128-bit chunks c = sub, sub + g, ... < C; four
// chunk pairs are loaded before any is used, so a lane keeps eight loads
// in flight
__device__ __forceinline__ uint32_t popc_rows(const uint4 *a, const uint4 *b, uint32_t C,
                                              uint32_t sub, uint32_t g) {
    uint32_t acc = 0, c = sub;
    for (; c + 3 * g < C; c += 4 * g) {
        const uint4 a0 = a[c], b0 = b[c], a1 = a[c + g], b1 = b[c + g];
        const uint4 a2 = a[c + 2 * g], b2 = b[c + 2 * g], a3 = a[c + 3 * g], b3 = b[c + 3 * g];
        acc += popc4(a0, b0) + popc4(a1, b1) + popc4(a2, b2) + popc4(a3, b3);
    }
    for (; c < C; c += g) acc += popc4(a[c], b[c]);
    return acc;
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

// Column tiles: a block owns words [b K, b K + K) of every row, i.e. the
// transactions [32 b K, 32 (b + 1) K).  It sets their bits in an LDS copy of
// the tile (n x K words, LDS atomics) and writes the tile out once, K words
// per row, zeros included: no global atomics, no separate zero fill, and
// the padding words past the last transaction come out zero as well.
constexpr uint32_t kTileMaxWords = 8;

__global__ __launch_bounds__(kBlock) void k_bitmap_tile(const uint64_t *__restrict__ offsets,
                                                         const uint32_t *__restrict__ items,
                                                         uint64_t n_tx,
                                                         const uint32_t *__restrict__ rank_of_item,
                                                         uint32_t n, uint32_t *rows, uint32_t Wp,
                                                         uint32_t K) {
    extern __shared__ uint4 tile4[];  // n * K words, 16-byte aligned
    uint32_t *tile = reinterpret_cast<uint32_t *>(tile4);
    __shared__ uint64_t s_off[32 * kTileMaxWords + 1];
    const uint32_t wb = blockIdx.x * K;
    const uint32_t kw = min(K, Wp - wb);  // a multiple of 4 (K and Wp are)
    for (uint32_t e = threadIdx.x; e < n * K; e += kBlock) tile[e] = 0;
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
                if (p >= p1 || r[j] == kNone) continue;
                uint32_t lo = 0, hi = nt;  // s_off[lo] <= p < s_off[hi]
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_off[mid] <= p) lo = mid;
                    else hi = mid;
                }
                atomicOr(&tile[r[j] * K + (lo >> 5)], 1u << (lo & 31));
            }
        }
    }
    __syncthreads();
    const uint32_t q4 = kw / 4;  // 16-byte pieces per row
    for (uint32_t e = threadIdx.x; e < n * q4; e += kBlock) {
        const uint32_t r = e / q4, q = e % q4;
        const uint4 v = *reinterpret_cast<const uint4 *>(tile + r * K + 4 * q);
        *reinterpret_cast<uint4 *>(rows + (uint64_t)r * Wp + wb + 4 * q) = v;
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
// words' popcounts.  rowpre[r * Wb + j] = set bits of row r before word 8 j,
// the coarse rank index k_rank_tx uses to place a transaction in the list.
__global__ __launch_bounds__(kBlock) void k_tidlist(const uint32_t *__restrict__ rows, uint32_t n,
                                                     uint32_t Wp, const uint64_t *__restrict__ tl_off,
                                                     uint32_t *tl, uint32_t *rowpre, uint32_t Wb) {
    const uint32_t r = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (r >= n) return;
    const uint32_t lane = lane_id();
    const uint32_t *row = rows + (uint64_t)r * Wp;
    uint32_t *pre = rowpre + (uint64_t)r * Wb;
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
            const uint32_t before = pos + incl - pc;
            if (rowpre != nullptr && w < Wp && (w & 7) == 0) pre[w >> 3] = before;
            uint64_t q = base + before;
            uint32_t y = x[j];
            while (y) {
                const uint32_t b = __ffs(y) - 1;
                if (q < end) tl[q] = w * 32 + b;
                q++;
                y &= y - 1;
            }
            pos += __shfl(incl, kWave - 1, kWave);
        }
    }
}

// Ranked transactions: transaction t's ranks ascending at rk[off[t] + t ..),
// its infrequent items' slots and one slot more holding kRankEnd.  A wave
// takes kRankGroup transactions at a time (their loads overlap): every lane
// holds one item's rank of each and finds its slot by counting the smaller
// ranks (ties, only between infrequent items, by position).  A transaction of
// more than 64 items is done alone, 64 items at a time.  For a frequent rank
// r the lane also finds t's index in the tid list of r, the set bits of row r
// before t (rowpre plus at most eight words), and stores the slot's address
// there: tlp[tl_off[r] + index] = off[t] + t + slot.

constexpr uint32_t kRankGroup = 4;

__device__ __forceinline__ uint32_t tid_index(const uint32_t *__restrict__ rows, uint32_t Wp,
                                              const uint32_t *__restrict__ rowpre, uint32_t Wb,
                                              uint32_t r, uint64_t t) {
    // words w8 .. w of row r: w8 + 3 < Wp always (Wp is a multiple of 4), the
    // second half only when w reaches into it
    const uint32_t w = (uint32_t)(t >> 5), tb = (uint32_t)(t & 31), w8 = w & ~7u;
    const uint32_t *row = rows + (uint64_t)r * Wp;
    const uint4 x0 = *reinterpret_cast<const uint4 *>(row + w8);
    const uint4 x1 = w >= w8 + 4 ? *reinterpret_cast<const uint4 *>(row + w8 + 4)
                                 : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    uint32_t idx = rowpre[(uint64_t)r * Wb + (w >> 3)];
#pragma unroll
    for (uint32_t q = 0; q < 8; q++) {
        if (w8 + q < w) idx += __popc(xs[q]);
        else if (w8 + q == w) idx += __popc(xs[q] & ((1u << tb) - 1u));
    }
    return idx;
}

__global__ __launch_bounds__(kBlock) void k_rank_tx(
    const uint64_t *__restrict__ off, const uint32_t *__restrict__ items, uint64_t n_tx,
    const uint32_t *__restrict__ rank_of_item, const uint32_t *__restrict__ rows, uint32_t Wp,
    const uint32_t *__restrict__ rowpre, uint32_t Wb, const uint64_t *__restrict__ tl_off,
    uint16_t *rk, uint32_t *tlp, uint16_t *suf) {
    const uint32_t lane = lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * kWavesPerBlock;
    const uint64_t n_groups = (n_tx + kRankGroup - 1) / kRankGroup;
    // each XCD takes a contiguous range of transactions, so that the row
    // pieces and prefix counts nearby transactions share stay in its L2
    const uint32_t blk = xcd_local_block(blockIdx.x, gridDim.x);
    for (uint64_t g = (uint64_t)blk * kWavesPerBlock + threadIdx.x / kWave; g < n_groups;
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
            uint32_t pos[kRankGroup];
#pragma unroll
            for (uint32_t j = 0; j < kRankGroup; j++) {
                pos[j] = 0;
                for (uint32_t i = 0; i < L[j]; i++) {
                    const uint32_t v = __shfl(r[j], (int)i, kWave);
                    pos[j] += (v < r[j] || (v == r[j] && i < lane)) ? 1u : 0u;
                }
            }
            uint32_t idx[kRankGroup];
            uint64_t lo[kRankGroup];
#pragma unroll
            for (uint32_t j = 0; j < kRankGroup; j++) {
                // lanes without a frequent rank look up row 0 (in bounds) and
                // drop the result
                const uint32_t rq = r[j] != kNone ? r[j] : 0u;
                idx[j] = tid_index(rows, Wp, rowpre, Wb, rq, j < ng ? tg0 + j : tg0);
                lo[j] = tl_off[rq];
            }
#pragma unroll
            for (uint32_t j = 0; j < kRankGroup; j++) {
                if (j >= ng) continue;
                const uint64_t base = a[j] + tg0 + j;
                const uint32_t lf = (uint32_t)__popcll(__ballot(r[j] != kNone));  // frequent items
                if (lane < L[j]) {
                    rk[base + pos[j]] = (uint16_t)r[j];  // kNone -> kRankEnd16
                    if (r[j] != kNone) {
                        tlp[lo[j] + idx[j]] = (uint32_t)(base + pos[j]);
                        suf[lo[j] + idx[j]] = (uint16_t)(lf - 1 - pos[j]);
                    }
                }
                if (lane == 0) rk[base + L[j]] = kRankEnd16;
            }
            continue;
        }
        // one transaction at a time, 64 items at a time
        for (uint32_t j = 0; j < ng; j++) {
            const uint64_t t = tg0 + j, base = a[j] + t;
            const uint32_t Lt = L[j];
            uint32_t lf = 0;  // frequent items of t
            for (uint32_t c0 = 0; c0 < Lt; c0 += kWave) {
                const uint32_t c = c0 + lane;
                const bool f = c < Lt && rank_of_item[items[a[j] + c]] != kNone;
                lf += (uint32_t)__popcll(__ballot(f));
            }
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
                if (c >= Lt) continue;
                rk[base + p] = (uint16_t)rc;
                if (rc != kNone) {
                    const uint64_t i = tl_off[rc] + tid_index(rows, Wp, rowpre, Wb, rc, t);
                    tlp[i] = (uint32_t)(base + p);
                    suf[i] = (uint16_t)(lf - 1 - p);
                }
            }
            if (lane == 0) rk[base + Lt] = kRankEnd16;
        }
    }
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
    for (uint64_t pb = s_off[0] + (uint64_t)wv * kWave; pb < p1; pb += kBlock) {
        const uint64_t p = pb + lane;
        const bool valid = p < p1;
        while (valid && s_off[a_rel + 1] <= p) a_rel++;  // p only grows: the row only grows
        const uint32_t len = valid ? suf[p] : 0u;
        const uint32_t q0 = valid ? tlp[p] + 1 : 0u;
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
        constexpr uint32_t kReads = 4;  // rank reads per lane in flight
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
// lists (ranks, supports, source rows) grow down from the top.  A worker
// repeatedly claims tasks (rows [r0, r1) of a first-level class) from a
// global counter, materialises the class's sibling bitmaps along the prefix
// path (the thesis's Prepare-Tidlists for a prefix of length one), and runs
// Eclat-DFS-Computation below those rows: for a row r of a class with k
// atoms, the supports of (r, j) for all later atoms j are AND-popcounts of
// the two rows; the frequent ones are reported, ordered by ascending
// support (ties by item id), their bitmaps are written, and that child
// class is searched before row r + 1.

struct Frame {
    uint32_t rows_base;    // word offset of the class's row 0
    uint32_t k;            // atoms (rows) of the class
    uint32_t r;            // next row to expand
    uint32_t r_end;        // rows [0, r_end) are expanded
    uint32_t atoms;        // word offset of ranks[k]; supports at +stride, source rows at +2*stride
    uint32_t stride;       // capacity of each of the three atom arrays
    uint32_t meta_restore; // meta pointer to restore when the class is done
    uint32_t pad_;
};

constexpr uint32_t kStageWords = 68;  // words a chunk of 64 projected entries can touch, + slack

struct WaveShared {
    Frame frames[kMaxDepth];
    uint32_t prefix[kMaxDepth + 3];
    uint32_t stage[4 * kStageWords];  // assembly of projected rows, four at a time
};

struct WaveStats {
    unsigned long long candidates, pair_words, child_rows, given, max_k, max_depth, row_words;
    unsigned long long rec_pending;  // records not yet added to the instance's count
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
__device__ bool chunk_reserve(OutChunk &c, uint32_t need, uint32_t task, uint32_t inst,
                              uint32_t *out, uint64_t out_cap, DfsCounters *ctr) {
    if (c.base != kNoChunk && c.pos + need <= c.size) return c.valid != 0;
    close_chunk(c, out);
    const uint32_t grow = c.seq < 6 ? (256u << c.seq) : 16384u;
    const uint32_t size = max(grow, need + kChunkHeader);
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(&ctr->out_used.v, (unsigned long long)size);
    base = shfl_u64(base, 0);
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

// Rank of every key of `tmp` among all nf keys; writes the sorted atoms.
// Sorts nf atoms (arrays of stride `si` at tmp) ascending by (support, item
// id) into dst (arrays of stride nf).
__device__ void sort_atoms(const InstDesc &I, const uint32_t *tmp, uint32_t si, uint32_t *dst,
                           uint32_t nf) {
    const uint32_t lane = lane_id();
    for (uint32_t e0 = 0; e0 < nf; e0 += kWave) {
        const uint32_t e = e0 + lane;
        uint64_t key = ~0ull;
        uint32_t rk = 0, sp = 0, src = 0;
        if (e < nf) {
            rk = tmp[e];
            sp = tmp[si + e];
            src = tmp[2 * si + e];
            key = ((uint64_t)sp << 32) | I.item_of_rank[rk];
        }
        uint32_t pos = 0;
        for (uint32_t f0 = 0; f0 < nf; f0 += kWave) {
            uint64_t kf = ~0ull;
            if (f0 + lane < nf)
                kf = ((uint64_t)tmp[si + f0 + lane] << 32) | I.item_of_rank[tmp[f0 + lane]];
            const uint32_t cnt = min(nf - f0, (uint32_t)kWave);
            for (uint32_t t = 0; t < cnt; t++) pos += (shfl_u64(kf, t) < key) ? 1u : 0u;
        }
        if (e < nf) {
            dst[pos] = rk;
            dst[nf + pos] = sp;
            dst[2 * nf + pos] = src;
        }
    }
}

// Hand the upper part of the unexpanded rows of the shallowest class that
// is worth it to the donation queue.  Rows are split so that both parts
// have about the same number of candidate pairs; a part is worth handing
// over if it holds several candidate pairs per row the receiver has to
// rebuild from the level-1 bitmaps.
__device__ bool try_donate(const InstDesc &I, uint32_t inst, uint32_t plen, uint32_t l2_ref,
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
    hb = shfl_u64(hb, 0);
    sl = shfl_u64(sl, 0);
    if (sl >= dn.n_slots) return false;  // heap or queue full: keep the work
    uint32_t *rec = dn.heap + hb;
    const uint32_t *ranks = region + F.atoms;
    const uint32_t *supps = ranks + F.stride;
    if (lane == 0) {
        store_coherent32(rec + 0, inst);
        store_coherent32(rec + 1, pl);
        store_coherent32(rec + 2, kk);
        store_coherent32(rec + 3, F.r_end - mid);
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
    return __shfl(want, 0, kWave) != 0;
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
    uint32_t *sp = ws.stage;  // 4 * kStageWords >= kMaxDepth + 2 words
    const uint32_t np = len - 1;
    uint32_t v0 = lane < np ? I.item_of_rank[ws.prefix[lane]] : ~0u;
    uint32_t v1 = lane + kWave < np ? I.item_of_rank[ws.prefix[lane + kWave]] : ~0u;
    uint32_t p0 = 0, p1 = 0;
    for (uint32_t q = 0; q < np && q < (uint32_t)kWave; q++) {
        const uint32_t u = __shfl(v0, (int)q, kWave);
        p0 += u < v0 ? 1u : 0u;
        p1 += u < v1 ? 1u : 0u;
    }
    for (uint32_t q = kWave; q < np; q++) {
        const uint32_t u = __shfl(v1, (int)(q - kWave), kWave);
        p0 += u < v0 ? 1u : 0u;
        p1 += u < v1 ? 1u : 0u;
    }
    if (lane < np) sp[p0] = v0;
    if (lane + kWave < np) sp[p1] = v1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&ctr->out_used.v, 8ull * nf);
    base = shfl_u64(base, 0);
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
    return __shfl(v, 0, kWave) != 0;
}

template <int CPL>
__device__ void process_frame(const InstDesc &I, uint32_t inst, uint32_t task, uint32_t plen,
                              uint32_t l2_ref, uint32_t k, uint32_t r_end, uint32_t Wp, uint64_t meta,
                              uint64_t peak0,
                              uint32_t *region, uint64_t S, WaveShared &ws, uint32_t *out,
                              uint64_t out_cap, DfsCounters *ctr, InstCounters *ictr, WaveStats &st,
                              OutChunk &oc, Donation &dn) {
    const uint32_t lane = lane_id();
    const uint32_t C = Wp / 4;  // 128-bit chunks per row

    // lanes per pair: about four chunks per lane (their loads in flight at
    // once), at most a wave; narrow rows put several pairs in one pass
    uint32_t g = 1;
    const uint32_t want = (C + 3) / 4;
    while (g < want && g < (uint32_t)kWave) g <<= 1;
    const uint32_t ppp = kWave / g;  // pairs per pass
    const uint32_t grp = lane / g, sub = lane % g;

    // the first class's rows are region[0, k * Wp), its atom arrays at meta
    int depth = 0;
    ws.frames[0] = Frame{0u, k, 0u, r_end, (uint32_t)meta, k, (uint32_t)S, 0u};
    __builtin_amdgcn_wave_barrier();
    uint64_t rows_top = (uint64_t)k * Wp;
    uint64_t peak = peak0;
    uint32_t polls = 0, cool = 0, iters = 0;

    while (depth >= 0) {
        if ((++iters & 15u) == 0 && inst_stopped(I, ictr, inst)) return;
        if (dn.enabled && cool == 0 && ((++polls & 3u) == 0) && donation_wanted(ctr)) {
            const bool gave = try_donate(I, inst, plen, l2_ref, depth, region, ws, dn, ctr);
            cool = gave ? 8u : 4u;
            st.given += gave ? 1u : 0u;
        }
        else if (cool)
            cool--;
        Frame F = ws.frames[depth];
        __builtin_amdgcn_wave_barrier();
        F.rows_base = uni(F.rows_base);
        F.k = uni(F.k);
        F.r = uni(F.r);
        F.r_end = uni(F.r_end);
        F.atoms = uni(F.atoms);
        F.stride = uni(F.stride);
        F.meta_restore = uni(F.meta_restore);
        if (F.r >= F.r_end) {
            rows_top = F.rows_base;
            meta = F.meta_restore;
            depth--;
            continue;
        }
        const uint32_t r = F.r;
        ws.frames[depth].r = r + 1;
        const uint32_t nj = F.k - r - 1;
        if (nj == 0) continue;
        const uint32_t *ranks = region + F.atoms;
        ws.prefix[plen + depth] = ranks[r];
        __builtin_amdgcn_wave_barrier();

        // frequent children of row r, unsorted: ranks, supports, source rows
        if (3ull * nj > meta || meta - 3ull * nj < rows_top) {
            flag_stack(ctr, rows_top + (S - meta) + 3ull * nj);
            return;
        }
        uint32_t *tmp = region + (meta - 3ull * nj);
        const uint4 *row_r =
            reinterpret_cast<const uint4 *>(region + F.rows_base + (uint64_t)r * Wp);
        uint32_t nf = 0;
        uint4 rr[CPL > 0 ? CPL : 1];
        if constexpr (CPL > 0) {
            // row r in registers; partners two at a time, all their loads in flight
#pragma unroll
            for (int m = 0; m < CPL; m++) {
                const uint32_t c = lane + m * kWave;
                rr[m] = c < C ? row_r[c] : make_uint4(0, 0, 0, 0);
            }
            for (uint32_t jj = 0; jj < nj; jj += 2) {
                const bool two = jj + 1 < nj;
                const uint4 *r0 = reinterpret_cast<const uint4 *>(
                    region + F.rows_base + (uint64_t)(r + 1 + jj) * Wp);
                const uint4 *r1 = two ? r0 + Wp / 4 : r0;
                uint4 x0[CPL], x1[CPL];
#pragma unroll
                for (int m = 0; m < CPL; m++) {
                    const uint32_t c = lane + m * kWave;
                    x0[m] = c < C ? r0[c] : make_uint4(0, 0, 0, 0);
                    x1[m] = c < C ? r1[c] : make_uint4(0, 0, 0, 0);
                }
                uint32_t a0 = 0, a1 = 0;
#pragma unroll
                for (int m = 0; m < CPL; m++) {
                    a0 += popc4(rr[m], x0[m]);
                    a1 += popc4(rr[m], x1[m]);
                }
#pragma unroll
                for (int off = kWave / 2; off >= 1; off >>= 1) {
                    a0 += __shfl_xor(a0, off, kWave);
                    a1 += __shfl_xor(a1, off, kWave);
                }
                const bool f0 = a0 >= I.minsup, f1 = two && a1 >= I.minsup;
                if (lane == 0) {
                    if (f0) {
                        tmp[nf] = ranks[r + 1 + jj];
                        tmp[nj + nf] = a0;
                        tmp[2 * nj + nf] = r + 1 + jj;
                    }
                    if (f1) {
                        const uint32_t p = nf + (f0 ? 1u : 0u);
                        tmp[p] = ranks[r + 2 + jj];
                        tmp[nj + p] = a1;
                        tmp[2 * nj + p] = r + 2 + jj;
                    }
                }
                nf += (f0 ? 1u : 0u) + (f1 ? 1u : 0u);
            }
        } else {
            for (uint32_t jb = 0; jb < nj; jb += ppp) {
                const uint32_t jj = jb + grp;
                uint32_t acc = 0;
                if (jj < nj) {
                    const uint4 *row_j = reinterpret_cast<const uint4 *>(
                        region + F.rows_base + (uint64_t)(r + 1 + jj) * Wp);
                    acc = popc_rows(row_r, row_j, C, sub, g);
                }
                for (uint32_t off = g >> 1; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, kWave);
                const bool freq = sub == 0 && jj < nj && acc >= I.minsup;
                const uint64_t mask = __ballot(freq);
                if (freq) {
                    const uint32_t p = nf + lanes_below(mask);
                    tmp[p] = ranks[r + 1 + jj];
                    tmp[nj + p] = acc;
                    tmp[2 * nj + p] = r + 1 + jj;
                }
                nf += (uint32_t)__popcll(mask);
            }
        }
        st.candidates += nj;
        st.pair_words += (unsigned long long)nj * Wp;
        if (F.k > st.max_k) st.max_k = F.k;
        if ((unsigned long long)depth > st.max_depth) st.max_depth = depth;
        if (nf == 0) continue;
        __threadfence_block();

        // report the nf itemsets prefix + a_r + child atom
        const uint32_t len = plen + (uint32_t)depth + 2;
        if (I.max_len == 0 || len <= I.max_len) {
            if (I.rec_budget) {
                // records are added to the instance's count in batches; the
                // count never exceeds the records really found, so the work
                // is abandoned only once the budget is certainly exceeded
                st.rec_pending += nf;
                if (st.rec_pending >= 4096) {
                    unsigned long long before = 0;
                    if (lane == 0) before = atomicAdd(&ictr[inst].records, st.rec_pending);
                    before = shfl_u64(before, 0);
                    const unsigned long long now = before + st.rec_pending;
                    st.rec_pending = 0;
                    if (now > I.rec_budget) {
                        if (lane == 0) atomicOr(&ictr[inst].stop, 1u);
                        return;
                    }
                }
            }
            const uint32_t rec = kRecHeader + len;
            st.out_words += (unsigned long long)nf * (I.key_bits ? 8u : rec);
            if (I.class_count) {
                // estimate run: only the number of itemsets per second-level class
                if (lane == 0) atomicAdd(&I.class_count[l2_class(plen, l2_ref, depth, r, ws)],
                                         (unsigned long long)nf);
            } else if (I.key_bits) {
                emit_keys(I, inst, len, tmp, nj, nf, ws, out, out_cap, ctr);
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
        if (nf >= 2 && (I.max_len == 0 || len + 1 <= I.max_len)) {
            if (depth + 1 >= kMaxDepth || plen + depth + 3 > kMaxDepth + 2) {
                if (lane == 0) atomicOr(&ctr->flags, kFlagDepthOverflow);
                continue;
            }
            const uint64_t restore = meta;
            uint64_t new_meta = meta - 3ull * nj;
            const uint32_t *sorted = tmp;
            uint32_t sstride = nj;
            if (!I.order_by_id) {
                if (3ull * nf > new_meta || new_meta - 3ull * nf < rows_top + (uint64_t)nf * Wp) {
                    flag_stack(ctr, rows_top + (uint64_t)nf * Wp + (S - new_meta) + 3ull * nf);
                    return;
                }
                new_meta -= 3ull * nf;
                uint32_t *dst = region + new_meta;
                sort_atoms(I, tmp, nj, dst, nf);
                __threadfence_block();
                sorted = dst;
                sstride = nf;
            } else if (new_meta < rows_top + (uint64_t)nf * Wp) {
                flag_stack(ctr, rows_top + (uint64_t)nf * Wp + (S - new_meta));
                return;
            }
            // child bitmaps: row_r AND row_src, in the child's atom order
            if constexpr (CPL > 0) {
                for (uint32_t c = 0; c < nf; c += 2) {
                    const bool two = c + 1 < nf;
                    const uint4 *s0 = reinterpret_cast<const uint4 *>(
                        region + F.rows_base + (uint64_t)sorted[2 * sstride + c] * Wp);
                    const uint4 *s1 = two ? reinterpret_cast<const uint4 *>(
                                                region + F.rows_base +
                                                (uint64_t)sorted[2 * sstride + c + 1] * Wp)
                                          : s0;
                    uint4 *d0 = reinterpret_cast<uint4 *>(region + rows_top + (uint64_t)c * Wp);
                    uint4 *d1 = d0 + Wp / 4;
                    uint4 x0[CPL], x1[CPL];
#pragma unroll
                    for (int m = 0; m < CPL; m++) {
                        const uint32_t q = lane + m * kWave;
                        x0[m] = q < C ? s0[q] : make_uint4(0, 0, 0, 0);
                        x1[m] = q < C ? s1[q] : make_uint4(0, 0, 0, 0);
                    }
#pragma unroll
                    for (int m = 0; m < CPL; m++) {
                        const uint32_t q = lane + m * kWave;
                        if (q < C) {
                            d0[q] = and4(rr[m], x0[m]);
                            if (two) d1[q] = and4(rr[m], x1[m]);
                        }
                    }
                }
            } else if (g == (uint32_t)kWave) {
                for (uint32_t c = 0; c < nf; c++) {
                    const uint32_t sr = sorted[2 * sstride + c];
                    const uint4 *row_j =
                        reinterpret_cast<const uint4 *>(region + F.rows_base + (uint64_t)sr * Wp);
                    uint4 *dst = reinterpret_cast<uint4 *>(region + rows_top + (uint64_t)c * Wp);
                    and_rows(dst, row_r, row_j, C, lane);
                }
            } else {
                // narrow rows: ppp children at a time, g lanes each
                for (uint32_t c0 = 0; c0 < nf; c0 += ppp) {
                    const uint32_t c = c0 + grp;
                    if (c < nf) {
                        const uint32_t sr = sorted[2 * sstride + c];
                        const uint4 *row_j = reinterpret_cast<const uint4 *>(
                            region + F.rows_base + (uint64_t)sr * Wp);
                        uint4 *dst = reinterpret_cast<uint4 *>(region + rows_top + (uint64_t)c * Wp);
                        for (uint32_t q = sub; q < C; q += g) dst[q] = and4(row_r[q], row_j[q]);
                    }
                }
            }
            __threadfence_block();
            st.child_rows += nf;
            st.row_words += (unsigned long long)nf * Wp;
            ws.frames[depth + 1] = Frame{(uint32_t)rows_top, nf, 0u, nf - 1,
                                         (uint32_t)(sorted - region), sstride, (uint32_t)restore, 0u};
            __builtin_amdgcn_wave_barrier();
            rows_top += (uint64_t)nf * Wp;
            meta = new_meta;
            depth++;
            const uint64_t use = rows_top + (S - meta);
            if (use > peak) peak = use;
        }
    }
    if (lane == 0) atomicMax(&ctr->stack_need, (unsigned long long)peak);
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
// every atom (Prepare-Tidlists), then its depth-first search.  When the
// cover T(prefix) holds at most a quarter of the row's bits, the rows are
// built projected on that cover: bit i of a projected row is the row's bit
// at the i-th transaction of T(prefix).  Every support below the prefix is
// a popcount of ANDs of such rows, so the results are the same, and the
// whole subtree works on rows of ceil(supp(prefix) / 32) words.  The
// process_frame variant is then picked for the width actually used: rows
// of more than 64 and at most 64 * CPL chunks are held in registers.
template <int CPL>
__device__ void run_frame(const InstDesc &I, uint32_t inst, uint32_t task, const FrameSrc &src,
                          uint32_t *region, uint64_t S, WaveShared &ws, uint32_t *out,
                          uint64_t out_cap, DfsCounters *ctr, InstCounters *ictr, WaveStats &st,
                          OutChunk &oc, Donation &dn) {
    if (inst_stopped(I, ictr, inst)) return;
    const uint32_t lane = lane_id();
    const uint32_t k = src.k, plen = src.plen;
    if (src.r_end == 0 || src.r_end >= k || plen == 0 || plen + 2 > kMaxDepth) return;
    const uint32_t Wf = I.Wp, Cf = Wf / 4;
    if (3ull * k + (uint64_t)k * kRowAlign > S) {
        flag_stack(ctr, 3ull * k + (uint64_t)k * Wf);
        return;
    }
    const uint64_t meta = S - 3ull * k;
    for (uint32_t e = lane; e < k; e += kWave) {
        region[meta + e] = src.ranks[e];
        region[meta + k + e] = src.supps[e];
        region[meta + 2 * k + e] = e;
    }
    for (uint32_t q = lane; q < plen; q += kWave) ws.prefix[q] = src.prefix[q];
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
                return;
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
            const uint64_t peak0 = (S - low) + (uint64_t)k * Wq;
            const uint32_t C = Wq / 4;
            if (CPL > 0 && C > (uint32_t)kWave && C <= (uint32_t)(CPL * kWave))
                process_frame<CPL>(I, inst, task, plen, src.l2_ref, k, src.r_end, Wq, meta, peak0, region, S, ws,
                                   out, out_cap, ctr, ictr, st, oc, dn);
            else
                process_frame<0>(I, inst, task, plen, src.l2_ref, k, src.r_end, Wq, meta, peak0, region, S, ws,
                                 out, out_cap, ctr, ictr, st, oc, dn);
            return;
        }
    }
    // T(prefix): the item's own row, or the AND of the prefix items' rows
    const uint32_t *P = I.rows + (uint64_t)src.prefix[0] * Wf;
    if (plen > 1) {
        if (low < Wf) {
            flag_stack(ctr, (uint64_t)(k + 1) * Wf + 3ull * k);
            return;
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
        if (!build_projected(I, P, s, src.ranks, k, Wq, region, S, low, ctr, ws.stage)) return;
        Wp = Wq;
    } else {
        if (low < (uint64_t)k * Wf) {
            flag_stack(ctr, (uint64_t)k * Wf + (S - low));
            return;
        }
        for (uint32_t e = 0; e < k; e++)
            and_rows(reinterpret_cast<uint4 *>(region + (uint64_t)e * Wf),
                     reinterpret_cast<const uint4 *>(P),
                     reinterpret_cast<const uint4 *>(I.rows + (uint64_t)src.ranks[e] * Wf), Cf, lane);
    }
    __threadfence_block();
    st.row_words += (unsigned long long)k * Wp;
    const uint64_t peak0 = (S - low) + (uint64_t)k * Wp;
    const uint32_t C = Wp / 4;
    if (CPL > 0 && C > (uint32_t)kWave && C <= (uint32_t)(CPL * kWave))
        process_frame<CPL>(I, inst, task, plen, src.l2_ref, k, src.r_end, Wp, meta, peak0, region, S, ws, out,
                           out_cap, ctr, ictr, st, oc, dn);
    else
        process_frame<0>(I, inst, task, plen, src.l2_ref, k, src.r_end, Wp, meta, peak0, region, S, ws, out,
                         out_cap, ctr, ictr, st, oc, dn);
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

template <int CPL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(CPL == 4 ? 2 : 1))) void k_dfs(const InstDesc *insts, const Task *tasks,
                                                uint64_t n_tasks, uint32_t *stack,
                                                uint64_t stack_words, uint32_t tasks_per_claim,
                                                uint32_t *out, uint64_t out_cap,
                                                DfsCounters *ctr, InstCounters *ictr,
                                                Donation dn) {
    __shared__ WaveShared shared[kWavesPerBlock];
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    WaveShared &ws = shared[w];
    const uint64_t wave_id = (uint64_t)blockIdx.x * kWavesPerBlock + w;
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
    // planned tasks, in LPT order
    for (;;) {
        unsigned long long t0 = 0;
        if (lane == 0) {
            atomicAdd(&ctr->active.v, 1ull);
            t0 = atomicAdd(&ctr->task_head.v, (unsigned long long)tasks_per_claim);
        }
        t0 = shfl_u64(t0, 0);
        if (t0 >= n_tasks) {
            wave_mem_wait();
            if (lane == 0) atomicSub(&ctr->active.v, 1ull);
            break;
        }
        const uint64_t t1 = min((uint64_t)t0 + tasks_per_claim, n_tasks);
        for (uint64_t t = t0; t < t1; t++) {
            const Task T = tasks[t];
            const InstDesc &I = insts[T.inst];
            const uint32_t a0 = I.l2_off[T.node], k1 = I.l2_off[T.node + 1] - a0;
            if (T.r0 >= T.r1 || T.r1 >= k1) continue;  // rows with a later atom only
            WaveStats st{};
            OutChunk oc{kNoChunk, 0u, 0u, 0u, 0u};
            const FrameSrc fs{&tasks[t].node, I.l2_atom + a0 + T.r0, I.l2_supp + a0 + T.r0, 1u,
                              k1 - T.r0, T.r1 - T.r0, a0 + T.r0};
            const unsigned long long c0 = wall_clock64();
            run_frame<CPL>(I, T.inst, (uint32_t)t, fs, region, stack_words, ws, out, out_cap, ctr,
                           ictr, st, oc, dn);
            close_chunk(oc, out);
            busy += wall_clock64() - c0;
            flush_stats(I, ictr, T.inst, st);
            note(st);
        }
        wave_mem_wait();  // donations of this task are published before it counts as done
        if (lane == 0) atomicSub(&ctr->active.v, 1ull);
    }
    // donated work until no wave is active and the queue is drained
    if (dn.enabled) {
        if (lane == 0) atomicAdd(&ctr->idle.v, 1ull);
        unsigned long long since = wall_clock64();
        uint32_t nap = 1;
        for (;;) {
            unsigned long long got = ~0ull;
            uint32_t done = 0;
            if (lane == 0) {
                const unsigned long long h = load_coherent(&ctr->don_head.v);
                const unsigned long long t = min(load_coherent(&ctr->don_tail.v), dn.n_slots);
                if (h < t) {
                    if (atomicCAS(&ctr->don_head.v, h, h + 1) == h) got = h;
                } else if (load_coherent(&ctr->active.v) == 0) {
                    // nobody can donate any more; re-read the queue after
                    // seeing that
                    const unsigned long long h2 = load_coherent(&ctr->don_head.v);
                    const unsigned long long t2 = min(load_coherent(&ctr->don_tail.v), dn.n_slots);
                    done = h2 >= t2 ? 1u : 0u;
                }
            }
            got = shfl_u64(got, 0);
            done = __shfl(done, 0, kWave);
            if (done) break;
            if (got == ~0ull) {
                if (wall_clock64() - since > dn.wait_ticks) {
                    if (lane == 0) atomicOr(&ctr->flags, kFlagSpin);
                    break;
                }
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
                off = shfl_u64(off, 0);
                if (off != 0 || wall_clock64() - w0 > dn.wait_ticks) break;
                __builtin_amdgcn_s_sleep(4);
            }
            if (off != 0) {
                // copy the record into this wave's own memory with coherent loads
                const uint32_t *rec = dn.heap + (off - 1);
                const uint32_t inst = load_coherent32(rec), pl = load_coherent32(rec + 1);
                const uint32_t kk = load_coherent32(rec + 2), re = load_coherent32(rec + 3);
                const uint32_t ref = load_coherent32(rec + 4);
                const uint32_t words = pl + 2 * kk;
                if ((uint64_t)words <= stack_words / 2) {
                    uint32_t *copy = region + (stack_words - words);
                    for (uint32_t q = lane; q < words; q += kWave)
                        copy[q] = load_coherent32(rec + 5 + q);
                    wave_mem_wait();
                    const InstDesc &I = insts[inst];
                    const FrameSrc fs{copy, copy + pl, copy + pl + kk, pl, kk, re, ref};
                    WaveStats st{};
                    OutChunk oc{kNoChunk, 0u, 0u, 0u, 0u};
                    const unsigned long long c0 = wall_clock64();
                    // the frame's own atom arrays go below the copy
                    run_frame<CPL>(I, inst, (uint32_t)(n_tasks + got), fs, region,
                                   stack_words - words, ws, out, out_cap, ctr, ictr, st, oc, dn);
                    close_chunk(oc, out);
                    busy += wall_clock64() - c0;
                    flush_stats(I, ictr, inst, st);
                    note(st);
                } else if (lane == 0) {
                    atomicOr(&ctr->flags, kFlagStackOverflow);
                    atomicMax(&ctr->stack_need, 2ull * words);
                }
            } else if (lane == 0) {
                atomicOr(&ctr->flags, kFlagSpin);
            }
            wave_mem_wait();
            if (lane == 0) {
                atomicAdd(&ctr->idle.v, 1ull);
                atomicSub(&ctr->active.v, 1ull);
            }
            since = wall_clock64();
        }
        if (lane == 0) atomicSub(&ctr->idle.v, 1ull);
    }
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
                          uint32_t *tl, uint32_t *rowpre, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tidlist, dim3((n + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0,
                       stream, rows, n, Wp, tl_off, tl, rowpre, rowpre_words(Wp));
    return hipGetLastError();
}

hipError_t launch_rank_tx(const uint64_t *off, const uint32_t *items, uint64_t n_tx,
                          const uint32_t *rank_of_item, const uint32_t *rows, uint32_t Wp,
                          const uint32_t *rowpre, const uint64_t *tl_off, uint16_t *rk,
                          uint32_t *tlp, uint16_t *suf, hipStream_t stream) {
    if (n_tx == 0) return hipSuccess;
    const uint64_t groups = (n_tx + kRankGroup - 1) / kRankGroup;
    const uint64_t blocks = std::min<uint64_t>((groups + kWavesPerBlock - 1) / kWavesPerBlock, 65536);
    hipLaunchKernelGGL(k_rank_tx, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, off, items, n_tx,
                       rank_of_item, rows, Wp, rowpre, rowpre_words(Wp), tl_off, rk, tlp, suf);
    return hipGetLastError();
}

// words per column tile for n rows within lds_max bytes of LDS, the block's
// transaction offsets included (0: does not fit)
uint32_t bitmap_tile_words(uint32_t n, size_t lds_max) {
    const size_t fixed = (32 * kTileMaxWords + 1) * sizeof(uint64_t);
    if (lds_max <= fixed) return 0;
    for (uint32_t K = kTileMaxWords; K >= 4; K /= 2)
        if ((uint64_t)n * K * 4 <= lds_max - fixed) return K;
    return 0;
}

hipError_t launch_bitmap_tiles(const uint64_t *offsets, const uint32_t *items, uint64_t n_tx,
                               const uint32_t *rank_of_item, uint32_t n, uint32_t *rows,
                               uint32_t Wp, uint32_t K, hipStream_t stream) {
    if (n == 0 || Wp == 0) return hipSuccess;
    if (K < 4 || K > kTileMaxWords || K % 4 != 0 || Wp % 4 != 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)n * K * 4;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bitmap_tile),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bitmap_tile, dim3((Wp + K - 1) / K), dim3(kBlock), lds, stream, offsets,
                       items, n_tx, rank_of_item, n, rows, Wp, K);
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

// row tile in words -> register-resident variant (256 words and wider than
// 2048 words: streamed)
uint32_t tile_variant(uint32_t tile_words) {
    if (tile_words <= 256) return 0;
    if (tile_words <= 512) return 2;
    if (tile_words <= 1024) return 4;
    if (tile_words <= 2048) return 8;
    return 0;
}

uint32_t dfs_variant(uint32_t max_chunks) {
    if (max_chunks <= (uint32_t)kWave) return 0;
    if (max_chunks <= 2u * kWave) return 2;
    if (max_chunks <= 4u * kWave) return 4;
    if (max_chunks <= 8u * kWave) return 8;
    return 0;
}

template <int CPL>
static uint32_t resident(int n_cu) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_dfs<CPL>, kBlock, 0) != hipSuccess ||
        blocks <= 0) {
        (void)hipGetLastError();
        blocks = 1;
    }
    return (uint32_t)blocks * kWavesPerBlock * (uint32_t)n_cu;
}

uint32_t dfs_resident_workers(int n_cu, uint32_t variant) {
    switch (variant) {
        case 2: return resident<2>(n_cu);
        case 4: return resident<4>(n_cu);
        case 8: return resident<8>(n_cu);
        default: return resident<0>(n_cu);
    }
}

hipError_t launch_dfs(const InstDesc *insts, const Task *tasks, uint64_t n_tasks, uint32_t *stack,
                      uint64_t stack_words, uint32_t n_workers, uint32_t tasks_per_claim,
                      uint32_t *out, uint64_t out_cap, DfsCounters *ctr, InstCounters *ictr,
                      unsigned long long *don_slots, uint64_t n_slots, uint32_t *don_heap,
                      uint64_t heap_words, uint64_t wait_ticks, unsigned long long *trace,
                      uint32_t variant, uint32_t nap_max, hipStream_t stream) {
    if (n_tasks == 0) return hipSuccess;
    const uint32_t blocks = (n_workers + kWavesPerBlock - 1) / kWavesPerBlock;
    Donation dn{don_slots, don_heap, n_slots, heap_words, wait_ticks,
                (don_slots && don_heap && n_slots && heap_words) ? 1u : 0u, trace,
                nap_max ? nap_max : 64u};
    const uint32_t tpc = tasks_per_claim ? tasks_per_claim : 1u;
    switch (variant) {
        case 2:
            hipLaunchKernelGGL(k_dfs<2>, dim3(blocks), dim3(kBlock), 0, stream, insts, tasks,
                               n_tasks, stack, stack_words, tpc, out, out_cap, ctr, ictr, dn);
            break;
        case 4:
            hipLaunchKernelGGL(k_dfs<4>, dim3(blocks), dim3(kBlock), 0, stream, insts, tasks,
                               n_tasks, stack, stack_words, tpc, out, out_cap, ctr, ictr, dn);
            break;
        case 8:
            hipLaunchKernelGGL(k_dfs<8>, dim3(blocks), dim3(kBlock), 0, stream, insts, tasks,
                               n_tasks, stack, stack_words, tpc, out, out_cap, ctr, ictr, dn);
            break;
        default:
            hipLaunchKernelGGL(k_dfs<0>, dim3(blocks), dim3(kBlock), 0, stream, insts, tasks,
                               n_tasks, stack, stack_words, tpc, out, out_cap, ctr, ictr, dn);
    }
    return hipGetLastError();
}

}  // namespace fim
