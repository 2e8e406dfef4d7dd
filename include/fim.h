/*
 * fim.h — C ABI of the MI355X frequent-itemset miner (libfim.so).
 *
 * Problem (thesis, chapter "Mathematical foundation": definitions of
 * transaction, database, itemset cover and support, frequent itemset):
 * given a database D of transactions, each a set of item ids, and an
 * absolute minimum support m >= 1, report every non-empty itemset U with
 * supp(U) = |{t in D : U subset of t}| >= m, together with supp(U).
 *
 * Method: depth-first Eclat over prefix-based equivalence classes
 * (definition of a PBEC and of its extensions; appendix "The Eclat
 * algorithm"), with supports computed as the popcount of the bitwise AND of
 * vertical transaction bitmaps (bitmap form of the lemma that the support of
 * U is the size of the intersection of its items' tid-lists).  The classes
 * are ordered and split for the workers of a persistent GPU kernel by the
 * thesis's sample-based estimate of class sizes (Phase 1 reservoir variant,
 * the Partition and LPT-Schedule algorithms of Phase 2).  The result is
 * always exact: the estimate only decides the order of work.
 *
 * Conventions
 *  - Every function returns a fim_status (0 = FIM_OK, negative = error) and
 *    never throws or aborts across the ABI.  fim_last_error() returns a
 *    thread-local text describing the last error of the calling thread.
 *  - "host" pointers point to CPU memory, "device" pointers to GPU memory.
 *    Unless stated otherwise every pointer argument is a host pointer.
 *  - Objects (fim_ctx, fim_db, fim_result, fim_server) are opaque and owned
 *    by the library until destroyed by the matching *_destroy call.
 *    destroy(NULL) is a no-op.
 *  - A fim_ctx is bound to one GPU and one HIP stream and is not
 *    thread-safe: calls with the same ctx must not overlap.  The server
 *    functions are the exception and are documented below.
 */
#ifndef FIM_H
#define FIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fim_status;

#define FIM_OK 0
#define FIM_E_INVALID_ARG (-1)  /* bad pointer, size, flag or minimum support */
#define FIM_E_ITEM_RANGE (-2)   /* an item id >= n_item_ids */
#define FIM_E_OOM_HOST (-3)     /* host allocation failed */
#define FIM_E_OOM_DEVICE (-4)   /* device allocation failed (allocator returned NULL) */
#define FIM_E_DEVICE (-5)       /* a HIP runtime call or kernel failed */
#define FIM_E_OUTPUT_LIMIT (-6) /* more frequent itemsets than options.max_itemsets */
#define FIM_E_BUSY (-7)         /* server queue full */
#define FIM_E_CANCELLED (-8)    /* server request was cancelled */
#define FIM_E_NOT_FOUND (-9)    /* unknown server ticket */
#define FIM_E_NO_DEVICE (-10)   /* no usable gfx950 GPU */

/* Text of a status code (static string). */
const char *fim_status_str(fim_status s);

/* Text of the last error on the calling thread ("" if none). */
const char *fim_last_error(void);

/* Library version string, e.g. "fim 1.0 gfx950". */
const char *fim_version(void);

/* ------------------------------------------------------------------ */
/* Context                                                            */

/*
 * Device-memory allocator supplied by the caller (for instance a framework's
 * caching allocator).  alloc returns a device pointer of at least `bytes`
 * bytes usable on `stream`, or NULL on failure; free releases it.  `user` is
 * passed back unchanged.  The library calls them only from the thread that
 * calls the ctx functions, except for a server, which calls them from its
 * own thread.
 */
typedef struct fim_allocator {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *stream, void *user);
    void *user;
} fim_allocator;

typedef struct fim_ctx fim_ctx;

/*
 * Create a context on GPU `device` (HIP ordinal).  hip_stream is a
 * hipStream_t cast to void*; all GPU work of the context is ordered on it.
 * NULL makes the library create (and later destroy) a stream of its own,
 * since graph capture cannot use the null stream.  alloc may be NULL (hipMalloc / hipFree are then
 * used).  The allocator struct is copied.
 * Errors: FIM_E_INVALID_ARG (out == NULL), FIM_E_NO_DEVICE (no such device or
 * not gfx950), FIM_E_DEVICE.
 */
fim_status fim_ctx_create(int device, void *hip_stream, const fim_allocator *alloc,
                          fim_ctx **out);
/* Destroy the context's servers and databases first: a database is freed
 * through its context. */
void fim_ctx_destroy(fim_ctx *ctx);

/*
 * Device blocks the library frees are kept by the context for reuse by its
 * next calls (up to a quarter of the device's memory), so that steady-state calls
 * make no allocator calls.  This gives them back to the allocator now.  They
 * are also given back when an allocation fails and when the context is
 * destroyed.
 */
fim_status fim_ctx_release_cached(fim_ctx *ctx);

/* ------------------------------------------------------------------ */
/* Database                                                           */

typedef struct fim_db fim_db;

/*
 * Upload a transaction database (definition of a database: a sequence of
 * transactions, each an itemset) given in CSR form:
 *   tx_offsets[n_tx + 1] (host, uint64, non-decreasing, tx_offsets[0] = 0),
 *   items[tx_offsets[n_tx]] (host, uint32, each < n_item_ids).
 * Transaction t holds items[tx_offsets[t] .. tx_offsets[t+1]).  Transactions
 * are sets: item order is free and repeated items count once.  Empty
 * transactions are allowed and count towards the database size.
 * n_tx = 0 is allowed (every result is then empty).
 * The data are copied (the caller keeps ownership of its arrays) and stay
 * resident in device memory until fim_db_destroy.  n_tx must be < 2^31.
 * Errors: FIM_E_INVALID_ARG (NULL pointers, non-monotone offsets,
 * n_item_ids == 0), FIM_E_ITEM_RANGE, FIM_E_OOM_HOST, FIM_E_OOM_DEVICE,
 * FIM_E_DEVICE.
 */
fim_status fim_db_create(fim_ctx *ctx, uint64_t n_tx, const uint64_t *tx_offsets,
                         const uint32_t *items, uint32_t n_item_ids, fim_db **out);
void fim_db_destroy(fim_db *db);

/* Number of transactions and of distinct (transaction, item) pairs. */
fim_status fim_db_sizes(const fim_db *db, uint64_t *n_tx, uint64_t *nnz);

/*
 * Absolute minimum support from a relative one (definition of a frequent
 * itemset with relative support): out = ceil(rel * n_tx) computed in double
 * precision, at least 1.  Errors: FIM_E_INVALID_ARG if rel is not in (0, 1].
 */
fim_status fim_minsup_from_relative(uint64_t n_tx, double rel, uint32_t *out_abs);

/* ------------------------------------------------------------------ */
/* Mining                                                             */

/* options.flags */
#define FIM_FLAG_NO_ESTIMATE 0x1u  /* order classes by a cheap size proxy, skip the sample */
#define FIM_FLAG_ORDER_BY_ID 0x2u  /* extensions ordered by item id, not ascending support */
#define FIM_FLAG_NO_SPLIT 0x4u     /* never split first-level classes */
/* draw the database sample even when the classes below the root hold under
 * 1/20 of the root class's candidate pairs, the database has fewer than
 * 16 |D~| transactions, or the launch holds more than one instance (by
 * default the sample is then skipped: there is no work worth balancing,
 * mining the sample would cost about as much as the better order saves, or
 * the other instances' work fills the idle waves) */
#define FIM_FLAG_ALWAYS_ESTIMATE 0x8u
/*
 * The root class (all pairs of frequent items) has three exact kernels; by
 * default the one with the least estimated time is used:
 *  - whole rows: popcount-Gram of the item bitmaps, LDS-tiled (dense data);
 *  - covers: pair (i, j) counted over the non-zero words of row i only;
 *  - projected: supp({a, b}) as the number of transactions of the cover of
 *    a that hold b, walking the frequent items of those transactions (long
 *    sparse rows: the work is the pairs inside transactions, not the words).
 * These flags force one of them (the lowest set flag wins).
 */
#define FIM_FLAG_DENSE_ROOT 0x10u
#define FIM_FLAG_ROOT_COVERS 0x20u
#define FIM_FLAG_ROOT_PROJECT 0x40u
/* below the root, keep every class's rows at the full database width (by
 * default a piece of work whose prefix covers at most a quarter of the
 * transactions builds its rows projected on that cover) */
#define FIM_FLAG_NO_PROJECT 0x80u
/*
 * Phase 1 as the thesis runs it: the sample mined as a database of its own
 * (own item order), its frequent itemsets reservoir-sampled (|S| =
 * sample_fi) and assigned to second-level classes on the host.  By default
 * the sample is mined inside the same call on the database's own classes
 * (its bitmaps built from the sampled transactions) and the persistent
 * kernel counts every sampled frequent itemset into its second-level class
 * (the reservoir's estimate with the whole stream kept).
 */
#define FIM_FLAG_RESERVOIR 0x100u

/*
 * Options of a mining call.  A zero field selects its default.
 *  max_len         longest itemset to report (0 = unlimited)
 *  max_itemsets    limit on |F| (0 = unlimited); exceeded -> FIM_E_OUTPUT_LIMIT
 *  seed            seed of the database sample and the reservoir (default fixed)
 *  alpha           Partition parameter alpha of Phase 2 (default 0.3)
 *  sample_tx       database sample size |D~| (default from the Chernoff bound
 *                  of Toivonen's theorem with eps = 0.02, delta = 0.05,
 *                  capped at n_tx / 4)
 *  sample_fi       reservoir size |S| (default from the hypergeometric KL
 *                  bound with rho = 0.001, eps = 0.0005, delta = 0.05)
 *  tile_words      bitmap row tile of the depth-first kernel: a wave keeps
 *                  rows of up to this many words in registers while it pairs
 *                  them with later rows (512, 1024 or 2048; other values are
 *                  rounded up to the next of these), wider rows and 256 are
 *                  streamed from memory in 256-word tiles
 *                  (0 = from the widest row of the call; fim_autotune picks
 *                  it by measurement)
 *  classes_per_wg  first-level classes a worker claims at once
 *                  (0 = 1; fim_autotune picks it by measurement)
 *  workers         persistent workers (waves) to launch (0 = as many as the
 *                  GPU keeps resident)
 *  flags           FIM_FLAG_*
 */
typedef struct fim_options {
    uint32_t max_len;
    uint64_t max_itemsets;
    uint64_t seed;
    double alpha;
    uint32_t sample_tx;
    uint32_t sample_fi;
    uint32_t tile_words;
    uint32_t classes_per_wg;
    uint32_t workers;
    uint32_t flags;
} fim_options;

typedef struct fim_result fim_result;

/*
 * Mine every frequent itemset of db at absolute minimum support minsup_abs
 * (>= 1).  opts may be NULL (all defaults).  On success *out receives a new
 * result owned by the caller (fim_result_destroy).  The whole computation
 * (item supports, bitmap build, estimate, support counting, result
 * compaction) runs on the context's GPU and stream; the call returns after
 * the result has been copied to host memory.
 * Errors: FIM_E_INVALID_ARG (minsup_abs == 0, NULL db/out, db of another
 * device), FIM_E_OUTPUT_LIMIT (no partial result), FIM_E_OOM_DEVICE,
 * FIM_E_OOM_HOST, FIM_E_DEVICE.
 */
fim_status fim_mine(fim_ctx *ctx, const fim_db *db, uint32_t minsup_abs, const fim_options *opts,
                    fim_result **out);

/*
 * Mine n independent instances in one persistent launch.  dbs[n] and minsups[n]; outs[n] receives one result per instance,
 * identical to what fim_mine returns for that instance.  All-or-nothing: on
 * error no result is returned.
 */
fim_status fim_mine_batch(fim_ctx *ctx, uint32_t n, const fim_db *const *dbs,
                          const uint32_t *minsups, const fim_options *opts, fim_result **outs);

/*
 * Mining without allocation, for callers that cannot allocate (code under
 * stream capture, tight serving loops, harnesses that forbid allocation).
 * Mines like fim_mine(ctx, db, minsup_abs, opts) and gives the same result
 * (the class-size estimate is always the cheap size proxy:
 * FIM_FLAG_NO_ESTIMATE is implied; it orders work and never changes the
 * result), copied in canonical order (as fim_result_copy) into the caller's
 * host arrays offsets[cap_itemsets + 1], items[cap_items] and
 * supports[cap_itemsets].  *n_itemsets and *n_items_total receive the
 * result's sizes, also when they exceed the capacities.
 * All device memory the call needs comes from one scratch block of
 * FIM_NOALLOC_SCRATCH_BYTES bytes inside the library, one per GPU it runs on,
 * held until the process ends; the call allocates no device memory and no
 * page-locked host memory (host arrays of its own come from the ordinary
 * heap).  The block keeps the last call's contents; every call clears what
 * it needs.  Calls that overlap share a GPU's block: the library runs them
 * one at a time (a call waits for the one before it).
 * Errors: FIM_E_INVALID_ARG, FIM_E_OUTPUT_LIMIT (the result does not fit the
 * arrays, or more itemsets than opts->max_itemsets), FIM_E_OOM_DEVICE (the
 * work does not fit the scratch block), FIM_E_DEVICE.
 */
#define FIM_NOALLOC_SCRATCH_BYTES (256ull << 20)
fim_status fim_mine_noalloc(fim_ctx *ctx, const fim_db *db, uint32_t minsup_abs,
                            const fim_options *opts, uint64_t cap_itemsets, uint64_t cap_items,
                            uint64_t *offsets, uint32_t *items, uint32_t *supports,
                            uint64_t *n_itemsets, uint64_t *n_items_total);

/* ------------------------------------------------------------------ */
/* Results                                                            */

/*
 * Statistics of one mining run.
 *  candidates       support computations of item pairs inside classes
 *                   (sum over classes of k(k-1)/2 for k extensions)
 *  pair_words       32-bit bitmap words AND-popcounted for those candidates
 *  item_supports    level-1 supports computed (= number of item ids)
 *  n_frequent_items frequent items (1-itemsets)
 *  bytes_algorithmic sibling bitmap bytes read once per class plus child
 *                   bitmap bytes written once
 *  kernel_ns        GPU time of the support-counting kernels
 *  total_ns         wall time of the whole call
 *  estimate_ns      wall time of the sample-based estimate
 *  n_tasks          work items given to the persistent kernel
 *  retries          re-runs after an arena overflow
 *  root_candidates  candidates of the root class (all pairs of frequent items)
 *  root_pair_words  words AND-popcounted by the root-class kernel
 *  root_kernel_ns   GPU time of the root-class pair kernel (HIP events)
 *  dfs_kernel_ns    GPU time of the persistent depth-first kernel (HIP events)
 *  dfs_bytes_algorithmic  bitmap bytes the depth-first kernel must move:
 *                   every class's sibling rows (at the width used, full or
 *                   projected) written once and read once
 *  n_itemsets       frequent itemsets reported
 *  root_kernel      root-class kernel used: 0 whole rows, 1 covers,
 *                   2 projected transactions (root_pair_words then counts
 *                   the pair increments)
 *  dfs_busy_max_ns  busy time of the busiest wave of the persistent kernel
 *  dfs_busy_mean_ns mean busy time over its waves (their ratio is the
 *                   load imbalance the work plan and the work sharing left)
 *  In a batch, the kernel times are those of the whole batched launch.
 */
typedef struct fim_stats {
    uint64_t candidates;
    uint64_t pair_words;
    uint64_t item_supports;
    uint64_t n_frequent_items;
    uint64_t bytes_algorithmic;
    uint64_t kernel_ns;
    uint64_t total_ns;
    uint64_t estimate_ns;
    uint64_t n_tasks;
    uint64_t retries;
    uint64_t root_candidates;
    uint64_t root_pair_words;
    uint64_t root_kernel_ns;
    uint64_t dfs_kernel_ns;
    uint64_t dfs_bytes_algorithmic;
    uint64_t n_itemsets;
    uint64_t root_kernel;
    uint64_t dfs_busy_max_ns;
    uint64_t dfs_busy_mean_ns;
} fim_stats;

/* Number of itemsets and total number of items over all itemsets. */
fim_status fim_result_sizes(const fim_result *r, uint64_t *n_itemsets, uint64_t *n_items_total);

/*
 * Copy the result in canonical order into caller arrays:
 *   offsets[n_itemsets + 1], items[n_items_total], supports[n_itemsets].
 * Itemset i is items[offsets[i] .. offsets[i+1]) ascending by item id; the
 * itemsets are in lexicographic order (definition of the lexicographic order
 * of itemsets in the chapter on executing Eclat in Phase 4: a prefix comes
 * before its extensions).  The empty itemset is never reported.  Any of the
 * three pointers may be NULL to skip that array.
 */
fim_status fim_result_copy(const fim_result *r, uint64_t *offsets, uint32_t *items,
                           uint32_t *supports);

/*
 * The same three arrays in place, without a copy: *offsets, *items and
 * *supports receive pointers into host memory owned by r (laid out as for
 * fim_result_copy; *items and *supports are NULL for an empty result).  They
 * stay valid, and must not be written, until fim_result_destroy(r).
 * Errors: FIM_E_INVALID_ARG (a NULL argument).
 */
fim_status fim_result_view(const fim_result *r, const uint64_t **offsets, const uint32_t **items,
                           const uint32_t **supports);

fim_status fim_result_stats(const fim_result *r, fim_stats *out);
void fim_result_destroy(fim_result *r);

/* ------------------------------------------------------------------ */
/* Estimator building blocks (host only, no GPU needed)               */

/*
 * Default sample sizes of the class-size estimate.
 *  *sample_tx = ceil(ln(2/delta_db) / (2 eps_db^2)): database sample size of
 *    Toivonen's theorem (chapter on approximate counting, estimating the
 *    support of an itemset from a database sample): the support error exceeds
 *    eps_db with probability at most delta_db.
 *  *sample_fi = ceil(-ln(delta_fi/2) / D(rho + eps_fi || rho)): reservoir size
 *    of the theorem on the estimation error of the size of a subset from a
 *    hypergeometrically distributed (reservoir) sample, with D the
 *    Kullback-Leibler divergence of two Bernoulli distributions, natural logs.
 * Errors: FIM_E_INVALID_ARG unless 0 < eps, delta < 1, 0 < rho, rho + eps_fi < 1.
 */
fim_status fim_estimate_sample_sizes(double eps_db, double delta_db, double rho, double eps_fi,
                                     double delta_fi, uint32_t *sample_tx, uint32_t *sample_fi);

/*
 * Simple reservoir sampling (the Simple-Reservoir-Sampling algorithm of the
 * chapter on approximate counting): a uniform sample without replacement of
 * n positions of a stream of stream_len records.  out[min(n, stream_len)]
 * receives the kept positions (slot order of the reservoir).  The uniform
 * draws come from SplitMix64 seeded with `seed`.
 */
fim_status fim_reservoir_sample(uint64_t stream_len, uint64_t n, uint64_t seed, uint64_t *out);

/*
 * Partition and LPT-Schedule (Phase 2 of the thesis's method).  Class c is a
 * first-level class with n_atoms[c] atoms; row_weights holds, class after
 * class, n_atoms[c] estimated sizes of its second-level classes (the last one
 * of each class is ignored: it has no extensions).  A class whose total
 * exceeds alpha * (sum of all weights) / n_workers is split into contiguous
 * ranges of rows, each within that threshold unless a single row exceeds it
 * (FIM_FLAG_NO_SPLIT disables splitting).  The resulting tasks
 * (class, r0, r1) — rows [r0, r1) — are written to tasks[3 * capacity] in
 * LPT order (decreasing estimate); *n_tasks receives their number and
 * *makespan the largest worker load of the LPT assignment to n_workers
 * workers.  Classes with fewer than 2 atoms give no task.
 * Errors: FIM_E_INVALID_ARG, FIM_E_OUTPUT_LIMIT (capacity too small;
 * *n_tasks still receives the number needed).
 */
fim_status fim_partition_lpt(uint32_t n_classes, const uint32_t *n_atoms,
                             const double *row_weights, double alpha, uint32_t n_workers,
                             uint32_t flags, uint32_t *tasks, uint32_t capacity,
                             uint32_t *n_tasks, double *makespan);

/*
 * LPT-Schedule alone: jobs in decreasing weight, each to the currently least
 * loaded of n_workers workers (lowest index on ties).  worker_of_job[n_jobs];
 * *makespan = largest load.  Graham's bound: makespan <= 4/3 of optimal.
 */
fim_status fim_lpt_schedule(const double *weights, uint64_t n_jobs, uint32_t n_workers,
                            uint32_t *worker_of_job, double *makespan);

/*
 * Autotuner of the batched launch: mines the batch once per candidate
 * setting of tile_words (256, 512, 1024, 2048) with classes_per_wg = 1, then
 * classes_per_wg (2, 4) at the best tile width, each setting `reps` times
 * (0 = 2), and writes into *out the options `base` (NULL = defaults) with
 * the two fields of the fastest depth-first launch (least GPU time, HIP
 * events).  The settings do not change results, only speed; the results of
 * the trial runs are discarded.  *best_ns (may be NULL) receives the
 * winner's kernel time.
 * Errors: as fim_mine_batch.
 */
fim_status fim_autotune(fim_ctx *ctx, uint32_t n, const fim_db *const *dbs,
                        const uint32_t *minsups, const fim_options *base, uint32_t reps,
                        fim_options *out, uint64_t *best_ns);

/*
 * Class profile of one mining run, for studying the class-size estimate
 * (the thesis's experiments on the error of the estimated size of
 * prefix-based classes and of each processor's share of the work, chapter
 * "Experimental evaluation"): mines db as fim_mine does with the sample
 * estimate forced (FIM_FLAG_ALWAYS_ESTIMATE; FIM_FLAG_NO_ESTIMATE and
 * FIM_FLAG_RESERVOIR are cleared) and reports
 *   n_atoms[*n_classes]  atoms of every first-level class (frequent items in
 *                        ascending (support, item id) order), and for every
 *                        second-level class (row r of first-level class c;
 *                        the rows of the classes one after the other,
 *                        *n_rows in all):
 *   est_fi[k]            frequent itemsets of three or more items the
 *                        sample found below that class (the estimate's
 *                        weight; 0 where the instance drew no sample),
 *   est_cand[k]          candidate pairs the sample counted below it,
 *   act_cand[k]          candidate pairs the run itself counted below it.
 * Any array may be NULL.  Errors: as fim_mine; FIM_E_OUTPUT_LIMIT when
 * class_capacity or row_capacity is too small (*n_classes and *n_rows then
 * hold the sizes needed).
 */
fim_status fim_class_profile(fim_ctx *ctx, const fim_db *db, uint32_t minsup_abs,
                             const fim_options *opts, uint32_t *n_classes, uint32_t *n_atoms,
                             uint32_t class_capacity, uint64_t *n_rows, double *est_fi,
                             double *est_cand, uint64_t *act_cand, uint64_t row_capacity);

/* ------------------------------------------------------------------ */
/* Serving (continuous batching)                                      */

typedef struct fim_server fim_server;

/*
 * Server configuration.
 *  max_active        requests resident on the GPU at once (slots; 0 = 16)
 *  max_queue         waiting requests before submit returns FIM_E_BUSY
 *  hbm_budget_bytes  device memory the server may hold for resident
 *                    requests (admission by footprint); 0 = 3/4 of free memory
 *  lanes             batches mined at once, each by a worker thread on a
 *                    HIP stream of its own (0 = 2, at most 8); a lane that is
 *                    idle admits waiting requests while others still run.
 *                    Dense databases (an average transaction holds more than
 *                    a quarter of the item ids) are mined in batches of their
 *                    own; light requests may pass them in the queue
 *  opts              mining options applied to every request
 */
typedef struct fim_server_config {
    uint32_t max_active;
    uint32_t max_queue;
    uint64_t hbm_budget_bytes;
    uint32_t lanes;
    fim_options opts;
} fim_server_config;

/*
 * Server counters.
 *  submitted, completed, cancelled  requests so far
 *  steps        batched launches run (each mines the requests it admitted)
 *  peak_active  most requests resident at once
 *  peak_bytes   largest admitted footprint (bytes) held at once
 *  lanes        lanes the server runs (the configured value or its default)
 */
typedef struct fim_server_stats {
    uint64_t submitted;
    uint64_t completed;
    uint64_t cancelled;
    uint64_t steps;
    uint64_t peak_active;
    uint64_t peak_bytes;
    uint64_t lanes;
} fim_server_stats;

/*
 * Start a server on ctx (the server owns a worker thread that drives the GPU;
 * the ctx must not be used by other calls until fim_server_destroy).
 * cfg may be NULL for defaults.
 */
fim_status fim_server_create(fim_ctx *ctx, const fim_server_config *cfg, fim_server **out);

/*
 * Submit a request (db must stay alive until its result was taken or it was
 * cancelled).  Thread-safe.  *ticket identifies the request.
 * Errors: FIM_E_INVALID_ARG, FIM_E_BUSY (queue full).
 */
fim_status fim_server_submit(fim_server *s, const fim_db *db, uint32_t minsup_abs,
                             uint64_t *ticket);

/*
 * Non-blocking: *out = the result if the request finished (ownership passes
 * to the caller and the ticket is retired), NULL while it is pending.
 * Errors: FIM_E_NOT_FOUND, FIM_E_CANCELLED, or the request's own error.
 */
fim_status fim_server_poll(fim_server *s, uint64_t ticket, fim_result **out);

/* Blocking variant of fim_server_poll. */
fim_status fim_server_wait(fim_server *s, uint64_t ticket, fim_result **out);

/*
 * The next finished request, in completion order, whatever its ticket:
 * waits up to timeout_us microseconds.  On return *ticket is the request's
 * ticket (0 if none finished in time) and *out its result (ownership passes
 * to the caller and the ticket is retired), as fim_server_poll would give
 * it.  Requests already taken with poll / wait are skipped.
 * Errors: FIM_E_INVALID_ARG, FIM_E_CANCELLED (for that ticket), or the
 * request's own error.
 */
fim_status fim_server_next(fim_server *s, uint64_t timeout_us, uint64_t *ticket, fim_result **out);

/* Cancel a waiting or running request (its later poll gives FIM_E_CANCELLED). */
fim_status fim_server_cancel(fim_server *s, uint64_t ticket);

fim_status fim_server_stats_get(const fim_server *s, fim_server_stats *out);

/* Stop the worker thread, cancel what is pending, free the server. */
void fim_server_destroy(fim_server *s);

#ifdef __cplusplus
}
#endif
#endif /* FIM_H */
