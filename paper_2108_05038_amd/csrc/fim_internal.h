// Internal declarations shared by the host runtime and the HIP kernels of
// libfim.so.  Nothing here is part of the public ABI (include/fim.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fim {

// Bitmap layout: item row r holds bit (t % 32) of word (t / 32) for every
// transaction t that contains the item (LSB first).  Rows are padded to a
// multiple of kRowAlign words with zero words, so that 128-bit loads never
// cross a row and the padding never adds to a popcount.
constexpr uint32_t kRowAlign = 4;

constexpr uint32_t kNone = 0xFFFFFFFFu;

// Largest class depth below a first-level class that one worker can hold.
constexpr int kMaxDepth = 96;

// Device-side description of one mining instance.
struct InstDesc {
    const uint32_t *rows;        // level-1 arena, n_freq rows of Wp words, rank order
    const uint32_t *item_of_rank;// original item id of each rank (order tie-break)
    const uint32_t *l2_off;      // [n_freq + 1] CSR of the atoms of each first-level class
    const uint32_t *l2_atom;     // ranks of the atoms, ascending (support, item id)
    const uint32_t *l2_supp;     // supports of {rank, atom}
    uint32_t Wp;                 // words per row (multiple of kRowAlign)
    uint32_t n_freq;             // frequent items
    uint32_t minsup;             // absolute minimum support
    uint32_t max_len;            // longest itemset to report (0 = unlimited)
    uint32_t order_by_id;        // 1: extensions in item-id order instead of support
    uint32_t project;            // 1: rows of a piece of work may be projected on its prefix's cover
    // itemsets below the first level the instance may report before its
    // remaining work is abandoned (0 = unlimited)
    unsigned long long rec_budget;
    // ascending transaction ids of every rank (tl[tl_off[r] ..)), or null
    const uint32_t *tl;
    const uint64_t *tl_off;
    // estimate run: itemsets counted per second-level class (l2 atom index)
    // instead of reported; null in a mining run
    unsigned long long *class_count;
    // candidate pairs per second-level class (a class profile is asked
    // for), else null
    unsigned long long *row_cand;
    // key mode (> 0): every itemset is written as an 8-word record holding
    // its item ids ascending as (id + 1) codes of key_bits bits in a 128-bit
    // key, its support and the instance (the arena is then a flat array of
    // records); 0: variable-length records in per-piece chunks
    uint32_t key_bits;
    uint32_t pad2_;
};

// One unit of work of the persistent kernel: rows [r0, r1) of the
// first-level class of rank `node` of instance `inst`, i.e. the classes
// [{node, a_r} | later atoms] for those rows and everything below them.
struct Task {
    uint32_t inst;
    uint32_t node;
    uint32_t r0;
    uint32_t r1;
};

// Global counters of a persistent launch (device memory, zeroed before it).
// Counters that many waves touch concurrently sit on cache lines of their
// own, so that polling one does not slow the others.
struct alignas(128) CtrLine {
    unsigned long long v;
    unsigned long long pad_[15];
};

struct DfsCounters {
    CtrLine task_head;      // next task to hand out
    CtrLine out_used;       // output words reserved (may pass capacity)
    CtrLine don_head;       // next donation slot to take
    CtrLine don_tail;       // donation slots reserved
    CtrLine idle;           // waves waiting for donated work
    CtrLine active;         // waves working on a task or donation
    CtrLine don_heap_used;  // words of the donation heap used
    unsigned long long candidates;  // pair supports computed
    unsigned long long pair_words;  // words AND-popcounted
    unsigned long long child_rows;  // child bitmaps written
    unsigned long long stack_need;  // largest per-worker stack use seen (words)
    unsigned long long busy_sum;    // wall-clock ticks workers spent on tasks, summed
    unsigned long long busy_max;    // ... and of the busiest worker
    unsigned long long donations;   // donations published
    unsigned int flags;             // kFlag* bits
    unsigned int pad_;
};

// Per-instance counters of a persistent launch (device memory, zeroed).
struct InstCounters {
    unsigned long long candidates;  // pair supports computed
    unsigned long long pair_words;  // words AND-popcounted
    unsigned long long child_rows;  // child bitmaps written
    unsigned long long records;     // itemsets reported (counted when rec_budget > 0)
    unsigned long long row_words;   // words of sibling rows written (first frames and children)
    unsigned long long out_words;   // words of the records reported (or counted)
    uint32_t stop;                  // 1 once records exceeded rec_budget
    uint32_t pad_;
};

constexpr unsigned kFlagStackOverflow = 1u;
constexpr unsigned kFlagDepthOverflow = 2u;
constexpr unsigned kFlagOutOverflow = 4u;
constexpr unsigned kFlagSpin = 8u;  // a bounded wait of the work sharing ran out
constexpr unsigned kFlagKeyOverflow = 16u;  // an itemset too long for a 128-bit key

// Output arena: chunks with a header of kChunkHeader words (size, task,
// seq, used, inst) followed by records of kRecHeader + len words (len, support,
// len ranks in the instance's item order).
constexpr uint32_t kChunkHeader = 5;
constexpr uint32_t kRecHeader = 2;

// ---------------------------------------------------------------- launches
// All launches are asynchronous on `stream`; they return hipSuccess or the
// launch error.

// Item supports: counts[i] = occurrences of item i.  part is scratch of
// item_count_scratch_words(nnz, n_item_ids) words (may be 0, then part is
// unused).
uint64_t item_count_scratch_words(uint64_t nnz, uint32_t n_item_ids);
hipError_t launch_item_count(const uint32_t *items, uint64_t nnz, uint32_t *counts,
                             uint32_t n_item_ids, uint32_t *part, hipStream_t stream);

// Item supports of many instances in one launch: instance q's items
// counted into counts[out, out + n_item_ids) (zero-filled before; the
// launch adds to them); first_block = the instance's first block, blocks in
// all = the sum of count_many_blocks(nnz) over the instances in order.
struct CountSrc {
    const uint32_t *items;
    uint64_t nnz;
    uint64_t out;
    uint32_t n_item_ids;
    uint32_t first_block;
};
uint32_t count_many_blocks(uint64_t nnz);
hipError_t launch_item_count_many(const CountSrc *src, uint32_t n_src, uint32_t blocks, uint32_t max_ids,
                                  uint32_t *counts, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t stream);
// n words set to zero, except the 64-bit value v at words [at, at + 2)
hipError_t launch_fill_words(uint32_t *p, uint64_t n, uint64_t at, unsigned long long v,
                             hipStream_t stream);

// Bitmap rows (n x Wp words) of the frequent ranks.  launch_bitmap_build
// sets bits with global atomics into zero-filled rows; launch_bitmap_tiles
// writes every word of the rows from LDS tiles of up to 32 words by a group
// of rows (bitmap_tiles_fit(lds_max) tells whether the device's LDS allows
// it).
hipError_t launch_bitmap_build(const uint64_t *offsets, const uint32_t *items, uint64_t n_tx,
                               const uint32_t *rank_of_item, uint32_t *rows, uint32_t Wp,
                               hipStream_t stream);
bool bitmap_tiles_fit(size_t lds_max);
hipError_t launch_bitmap_tiles(const uint64_t *offsets, const uint32_t *items, uint64_t n_tx,
                               const uint32_t *rank_of_item, uint32_t n, uint32_t *rows,
                               uint32_t Wp, size_t lds_max, hipStream_t stream);

// Upper-triangle pair supports of the n rows (the root class): every pair
// (i < j) with popcount(row_i & row_j) >= minsup is appended as
// (i, j, support) to pairs (capacity cap triples); *n_pairs counts all
// frequent pairs (it may exceed cap, then nothing past cap is written).
// part (root_pairs_scratch_words() words, or nullptr) lets a launch with few
// tiles over long rows split the words over more blocks: partial counts go
// there and a second kernel sums them; it is used in stream order.
uint64_t root_pairs_scratch_words();
hipError_t launch_root_pairs(const uint32_t *rows, uint32_t n, uint32_t Wp, uint32_t minsup,
                             uint32_t *pairs, uint64_t cap, unsigned long long *n_pairs,
                             uint32_t *part, hipStream_t stream);

// Preparation of the projected root kernel.  launch_tidlist: the tid lists
// tl (at offsets tl_off[n + 1]) from the rows, and (tl_rank not null) the
// rank of every entry.  launch_rank_tx: rk (nnz + n_tx + 48 halfwords; fewer
// than 65535 frequent items) = every transaction's frequent ranks ascending
// at off[t] + t, closed by 0xFFFF (also in the slots of infrequent items),
// and for the n_ent tid-list entries tl (their ranks in suf, as tl_rank
// wrote them): tlp = for entry p the position in rk of its own rank, and suf
// = the number of frequent ranks after it in its transaction (transactions
// shorter than 65536 items).
hipError_t launch_tidlist(const uint32_t *rows, uint32_t n, uint32_t Wp, const uint64_t *tl_off,
                          uint32_t *tl, uint16_t *tl_rank, hipStream_t stream);
hipError_t launch_rank_tx(const uint64_t *off, const uint32_t *items, uint64_t n_tx,
                          const uint32_t *rank_of_item, const uint32_t *tl, uint64_t n_ent,
                          uint16_t *rk, uint32_t *tlp, uint16_t *suf, hipStream_t stream);
// The two halves of launch_rank_tx: rk alone (it needs no tid list, so it
// can run beside the bitmap and list kernels), then tlp and suf.
hipError_t launch_rank_only(const uint64_t *off, const uint32_t *items, uint64_t n_tx,
                            const uint32_t *rank_of_item, uint16_t *rk, hipStream_t stream);
hipError_t launch_tl_slots(const uint64_t *off, uint64_t n_tx, const uint16_t *rk, const uint32_t *tl,
                           uint64_t n_ent, uint32_t *tlp, uint16_t *suf, hipStream_t stream);
// Root class over projected transactions: rk, tlp and suf as above (tid
// lists at offsets tl_off[n + 1]); 16-bit counters when max_supp (the
// largest row support) is at most 65535.  Pairs as for launch_root_pairs;
// *work receives the pair increments.
void project_tile(uint32_t n, uint32_t *R, uint32_t *J);
hipError_t launch_root_project(const uint16_t *rk, const uint32_t *tlp, const uint16_t *suf,
                               const uint64_t *tl_off, uint32_t n, uint32_t max_supp,
                               uint32_t minsup, uint32_t *pairs, uint64_t cap,
                               unsigned long long *n_pairs, unsigned long long *work,
                               hipStream_t stream);
// Variant of the persistent kernel for rows of at most max_chunks 128-bit
// chunks (0 = rows are streamed, 2/4/8 = chunks per lane held in registers).
uint32_t tile_variant(uint32_t tile_words);
uint32_t dfs_variant(uint32_t max_chunks);

// Root class over the covers of its first-level prefixes (sparse rows):
// non-zero words of every row (capacity offsets nz_off[n+1], counts
// nz_cnt[n]), the word-major transpose bt[W][np] (np = n rounded up to 4),
// and the pair supports counted over row i's non-zero words only.
hipError_t launch_row_nonzero(const uint32_t *rows, uint32_t n, uint32_t Wp, const uint64_t *nz_off,
                              uint32_t *nz_w, uint32_t *nz_m, uint32_t *nz_cnt,
                              hipStream_t stream);
hipError_t launch_transpose(const uint32_t *rows, uint32_t n, uint32_t Wp, uint32_t W, uint32_t *bt,
                            uint32_t np, hipStream_t stream);
hipError_t launch_root_sparse(const uint32_t *bt, uint32_t np, const uint64_t *nz_off,
                              const uint32_t *nz_cnt, const uint32_t *nz_w, const uint32_t *nz_m,
                              uint32_t n, uint32_t minsup, uint32_t *pairs, uint64_t cap,
                              unsigned long long *n_pairs, hipStream_t stream);

// The key records (see the persistent kernel's key mode) of every frequent
// item and frequent pair of an instance, written on the device: records
// [out_rec, out_rec + n_freq + n_pairs) of the output arena, the items
// first (support counts[id]), then the pairs of the root kernel's triples
// (rank a, rank b, support).
struct PrefixSrc {
    const uint32_t *item_of_rank;
    const uint32_t *counts;
    const uint32_t *pairs;
    uint32_t n_freq, bits, inst, pad_;
    uint64_t n_pairs, out_rec;
};
hipError_t launch_prefix_keys(const PrefixSrc *src, uint32_t n_src, uint64_t max_rec, uint32_t *out,
                              hipStream_t stream);

// Waves of that persistent kernel variant that fit on the device at once.
uint32_t dfs_resident_workers(int n_cu, uint32_t variant);

// Persistent depth-first search over the tasks: n_workers waves, in blocks
// of waves_per_block active waves (1 to 4; n_workers a multiple of it).
hipError_t launch_dfs(const InstDesc *insts, const Task *tasks, uint64_t n_tasks,
                      uint32_t *stack, uint64_t stack_words, uint32_t n_workers,
                      uint32_t tasks_per_claim, uint32_t *out, uint64_t out_cap,
                      DfsCounters *ctr, InstCounters *ictr, unsigned long long *don_slots,
                      uint64_t n_slots, uint32_t *don_heap, uint64_t heap_words,
                      uint64_t wait_ticks, unsigned long long *trace, uint32_t variant,
                      uint32_t nap_max, uint64_t poll_ticks, uint32_t waves_per_block,
                      hipStream_t stream);

}  // namespace fim
