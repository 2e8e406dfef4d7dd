/*
 * CPU oracle for frequent-itemset mining.  TEST INFRASTRUCTURE ONLY: this
 * file is used by the test-suite, by the benchmark's CPU-baseline leg and by
 * the smoke check, never by the GPU library, and shares no code with it.
 *
 * What it computes (thesis, "Mathematical foundation", definitions of
 * itemset cover/support and of a frequent itemset):
 *     F = { (U, s) : U non-empty, s = |{t in D : U subset of t}| >= minsupp }.
 * Transactions are sets (definition of a transaction), so duplicate items in
 * an input transaction count once.  The empty itemset is never reported.
 *
 * Three independent ways to get F:
 *   orc_bruteforce  every subset of the items present, support by scanning
 *                   all transactions (tiny inputs only);
 *   orc_eclat       Eclat depth-first search over sorted tid-lists,
 *                   following the Eclat-DFS / Eclat-DFS-Computation
 *                   algorithms of the appendix on sequential algorithms,
 *                   with support counting by tid-list intersection (the
 *                   "support counting" subsection of the Eclat section) and
 *                   optional ascending-support ordering of every class's
 *                   extensions ("Ordering of items in DFS algorithms");
 *   orc_apriori     level-wise Apriori (appendix, the Apriori algorithm):
 *                   join of itemsets sharing all but the last item, pruning
 *                   of candidates with an infrequent subset (monotonicity of
 *                   support), supports counted per transaction.
 * plus orc_support: the support of one itemset by a scan of the database.
 *
 * Results are returned as a CSR (offsets, items, supports) in canonical
 * order: the items of an itemset ascending by id, itemsets in the
 * lexicographic order of the thesis's Phase-4 chapter (a prefix before its
 * extensions).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_ORDER_ID = 0, ORC_ORDER_ASCENDING_SUPPORT = 1 };

typedef struct {
    uint64_t n_sets;       /* number of itemsets */
    uint64_t n_items;      /* total items over all itemsets */
    uint64_t *offsets;     /* [n_sets + 1] */
    uint32_t *items;       /* [n_items] */
    uint32_t *supports;    /* [n_sets] */
    uint64_t candidates;   /* support computations of pairs inside classes */
    int overflow;          /* 1 if max_sets was exceeded (result incomplete) */
} orc_result;

/* ------------------------------------------------------------------ */
/* growable itemset list                                               */

typedef struct {
    uint64_t n_sets, cap_sets, n_items, cap_items;
    uint64_t *offsets;
    uint32_t *items, *supports;
    uint64_t max_sets;
    int overflow, oom;
} setlist;

static void sl_init(setlist *s, uint64_t max_sets) {
    memset(s, 0, sizeof(*s));
    s->max_sets = max_sets;
    s->cap_sets = 1024;
    s->cap_items = 4096;
    s->offsets = (uint64_t *)malloc((s->cap_sets + 1) * sizeof(uint64_t));
    s->supports = (uint32_t *)malloc(s->cap_sets * sizeof(uint32_t));
    s->items = (uint32_t *)malloc(s->cap_items * sizeof(uint32_t));
    if (!s->offsets || !s->supports || !s->items) s->oom = 1;
    else s->offsets[0] = 0;
}

static void sl_free(setlist *s) {
    free(s->offsets);
    free(s->items);
    free(s->supports);
    memset(s, 0, sizeof(*s));
}

/* append itemset head[0..nh) + {tail} (tail ignored when has_tail == 0) */
static void sl_add(setlist *s, const uint32_t *head, uint32_t nh, int has_tail, uint32_t tail,
                   uint32_t supp) {
    if (s->oom) return;
    if (s->max_sets && s->n_sets >= s->max_sets) {
        s->overflow = 1;
        return;
    }
    uint32_t len = nh + (has_tail ? 1 : 0);
    if (s->n_sets == s->cap_sets) {
        uint64_t nc = s->cap_sets * 2;
        uint64_t *no = (uint64_t *)realloc(s->offsets, (nc + 1) * sizeof(uint64_t));
        if (!no) { s->oom = 1; return; }
        s->offsets = no;
        uint32_t *ns = (uint32_t *)realloc(s->supports, nc * sizeof(uint32_t));
        if (!ns) { s->oom = 1; return; }
        s->supports = ns;
        s->cap_sets = nc;
    }
    while (s->n_items + len > s->cap_items) {
        uint64_t nc = s->cap_items * 2;
        uint32_t *ni = (uint32_t *)realloc(s->items, nc * sizeof(uint32_t));
        if (!ni) { s->oom = 1; return; }
        s->items = ni;
        s->cap_items = nc;
    }
    memcpy(s->items + s->n_items, head, nh * sizeof(uint32_t));
    if (has_tail) s->items[s->n_items + nh] = tail;
    s->n_items += len;
    s->supports[s->n_sets] = supp;
    s->n_sets++;
    s->offsets[s->n_sets] = s->n_items;
}

/* ------------------------------------------------------------------ */
/* canonical order                                                     */

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

typedef struct {
    const uint32_t *items;
    uint32_t len;
    uint32_t supp;
} setref;

/* lexicographic order of two ascending itemsets: first differing item
 * decides; if one is a prefix of the other, the shorter comes first */
static int cmp_setref(const void *a, const void *b) {
    const setref *x = (const setref *)a, *y = (const setref *)b;
    uint32_t n = x->len < y->len ? x->len : y->len;
    for (uint32_t i = 0; i < n; i++)
        if (x->items[i] != y->items[i]) return x->items[i] < y->items[i] ? -1 : 1;
    return (x->len > y->len) - (x->len < y->len);
}

/* sort items inside every itemset, then sort the itemsets, into *out */
static int sl_canonical(setlist *s, orc_result *out) {
    memset(out, 0, sizeof(*out));
    out->overflow = s->overflow;
    for (uint64_t i = 0; i < s->n_sets; i++)
        qsort(s->items + s->offsets[i], s->offsets[i + 1] - s->offsets[i], sizeof(uint32_t),
              cmp_u32);
    setref *refs = (setref *)malloc((s->n_sets + 1) * sizeof(setref));
    out->offsets = (uint64_t *)malloc((s->n_sets + 1) * sizeof(uint64_t));
    out->items = (uint32_t *)malloc((s->n_items + 1) * sizeof(uint32_t));
    out->supports = (uint32_t *)malloc((s->n_sets + 1) * sizeof(uint32_t));
    if (!refs || !out->offsets || !out->items || !out->supports) {
        free(refs);
        free(out->offsets);
        free(out->items);
        free(out->supports);
        memset(out, 0, sizeof(*out));
        return -1;
    }
    for (uint64_t i = 0; i < s->n_sets; i++) {
        refs[i].items = s->items + s->offsets[i];
        refs[i].len = (uint32_t)(s->offsets[i + 1] - s->offsets[i]);
        refs[i].supp = s->supports[i];
    }
    qsort(refs, s->n_sets, sizeof(setref), cmp_setref);
    uint64_t pos = 0;
    out->offsets[0] = 0;
    for (uint64_t i = 0; i < s->n_sets; i++) {
        memcpy(out->items + pos, refs[i].items, refs[i].len * sizeof(uint32_t));
        pos += refs[i].len;
        out->offsets[i + 1] = pos;
        out->supports[i] = refs[i].supp;
    }
    out->n_sets = s->n_sets;
    out->n_items = pos;
    free(refs);
    return 0;
}

void orc_result_free(orc_result *r) {
    if (!r) return;
    free(r->offsets);
    free(r->items);
    free(r->supports);
    memset(r, 0, sizeof(*r));
}

/* ------------------------------------------------------------------ */
/* input: transactions as sorted duplicate-free item arrays            */

typedef struct {
    uint64_t n_tx;
    uint64_t *off;
    uint32_t *items;
    uint32_t n_item_ids;
} txdb;

/* copy the CSR, sort every transaction and drop repeated items */
static int txdb_make(uint64_t n_tx, const uint64_t *offsets, const uint32_t *items,
                     uint32_t n_item_ids, txdb *db) {
    db->n_tx = n_tx;
    db->n_item_ids = n_item_ids;
    uint64_t nnz = offsets[n_tx];
    db->off = (uint64_t *)malloc((n_tx + 1) * sizeof(uint64_t));
    db->items = (uint32_t *)malloc((nnz + 1) * sizeof(uint32_t));
    if (!db->off || !db->items) return -1;
    uint64_t pos = 0;
    db->off[0] = 0;
    for (uint64_t t = 0; t < n_tx; t++) {
        uint64_t a = offsets[t], b = offsets[t + 1];
        uint32_t *dst = db->items + pos;
        uint64_t n = b - a;
        memcpy(dst, items + a, n * sizeof(uint32_t));
        qsort(dst, n, sizeof(uint32_t), cmp_u32);
        uint64_t w = 0;
        for (uint64_t i = 0; i < n; i++)
            if (w == 0 || dst[w - 1] != dst[i]) dst[w++] = dst[i];
        pos += w;
        db->off[t + 1] = pos;
    }
    return 0;
}

static void txdb_free(txdb *db) {
    free(db->off);
    free(db->items);
}

/* is the ascending itemset u[0..n) a subset of transaction t? */
static int tx_contains(const txdb *db, uint64_t t, const uint32_t *u, uint32_t n) {
    const uint32_t *x = db->items + db->off[t];
    uint64_t m = db->off[t + 1] - db->off[t], i = 0;
    for (uint32_t k = 0; k < n; k++) {
        while (i < m && x[i] < u[k]) i++;
        if (i == m || x[i] != u[k]) return 0;
        i++;
    }
    return 1;
}

/* support of one itemset (any order, no duplicates required) by a full scan */
uint64_t orc_support(uint64_t n_tx, const uint64_t *offsets, const uint32_t *items,
                     const uint32_t *itemset, uint32_t len) {
    uint32_t *u = (uint32_t *)malloc((len + 1) * sizeof(uint32_t));
    memcpy(u, itemset, len * sizeof(uint32_t));
    qsort(u, len, sizeof(uint32_t), cmp_u32);
    uint64_t cnt = 0;
    for (uint64_t t = 0; t < n_tx; t++) {
        /* transactions may hold duplicates: test membership of each item */
        const uint32_t *x = items + offsets[t];
        uint64_t m = offsets[t + 1] - offsets[t];
        int all = 1;
        for (uint32_t k = 0; k < len && all; k++) {
            int found = 0;
            for (uint64_t i = 0; i < m; i++)
                if (x[i] == u[k]) { found = 1; break; }
            all = found;
        }
        cnt += (uint64_t)all;
    }
    free(u);
    return cnt;
}

/* ------------------------------------------------------------------ */
/* brute force: all subsets of the items present                       */

int orc_bruteforce(uint64_t n_tx, const uint64_t *offsets, const uint32_t *items,
                   uint32_t n_item_ids, uint32_t minsup, orc_result *out) {
    memset(out, 0, sizeof(*out));
    if (minsup == 0) return -1;
    txdb db;
    if (txdb_make(n_tx, offsets, items, n_item_ids, &db)) return -2;
    /* distinct items present, ascending */
    uint8_t *seen = (uint8_t *)calloc(n_item_ids + 1, 1);
    uint32_t present[24], np = 0;
    for (uint64_t i = 0; i < db.off[n_tx]; i++) {
        uint32_t it = db.items[i];
        if (!seen[it]) {
            seen[it] = 1;
            if (np == 24) { free(seen); txdb_free(&db); return -3; }
            present[np++] = it;
        }
    }
    free(seen);
    qsort(present, np, sizeof(uint32_t), cmp_u32);
    setlist s;
    sl_init(&s, 0);
    uint32_t sub[24];
    for (uint64_t mask = 1; mask < (1ull << np); mask++) {
        uint32_t n = 0;
        for (uint32_t b = 0; b < np; b++)
            if (mask & (1ull << b)) sub[n++] = present[b];
        uint64_t cnt = 0;
        for (uint64_t t = 0; t < n_tx; t++) cnt += (uint64_t)tx_contains(&db, t, sub, n);
        if (cnt >= minsup) sl_add(&s, sub, n, 0, 0, (uint32_t)cnt);
    }
    txdb_free(&db);
    int rc = s.oom ? -2 : sl_canonical(&s, out);
    sl_free(&s);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Eclat over sorted tid-lists                                         */

typedef struct {
    uint32_t item;  /* last item of the itemset this tid-list belongs to */
    uint32_t n;     /* support = length of the tid-list */
    uint32_t *tids; /* ascending transaction ids */
} atom;

typedef struct {
    uint32_t minsup;
    int order;
    setlist out;
    uint64_t candidates;
} eclat_ctx;

static int cmp_atom_supp(const void *a, const void *b) {
    const atom *x = (const atom *)a, *y = (const atom *)b;
    if (x->n != y->n) return x->n < y->n ? -1 : 1;
    return (x->item > y->item) - (x->item < y->item);
}

static int cmp_atom_item(const void *a, const void *b) {
    const atom *x = (const atom *)a, *y = (const atom *)b;
    return (x->item > y->item) - (x->item < y->item);
}

/* |A ∩ B| with the intersection written to dst (both inputs ascending) */
static uint32_t intersect(const uint32_t *a, uint32_t na, const uint32_t *b, uint32_t nb,
                          uint32_t *dst) {
    uint32_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) i++;
        else if (a[i] > b[j]) j++;
        else {
            dst[k++] = a[i];
            i++;
            j++;
        }
    }
    return k;
}

/*
 * One class: prefix P = prefix[0..plen) and its atoms (the frequent
 * extensions, each with the tid-list of P with that item added).  For every
 * atom a_i, the atoms a_j after it are tried; T(P+a_i+a_j) is the
 * intersection of the two tid-lists; the frequent ones form the atoms of
 * the class of P+a_i, are reported, and that class is searched next.
 */
static void eclat_class(eclat_ctx *c, atom *atoms, uint32_t k, uint32_t *prefix, uint32_t plen) {
    for (uint32_t i = 0; i + 1 < k && !c->out.overflow && !c->out.oom; i++) {
        prefix[plen] = atoms[i].item;
        atom *child = (atom *)malloc((k - i - 1) * sizeof(atom));
        uint32_t nc = 0;
        for (uint32_t j = i + 1; j < k; j++) {
            uint32_t cap = atoms[i].n < atoms[j].n ? atoms[i].n : atoms[j].n;
            uint32_t *t = (uint32_t *)malloc((cap + 1) * sizeof(uint32_t));
            uint32_t s = intersect(atoms[i].tids, atoms[i].n, atoms[j].tids, atoms[j].n, t);
            c->candidates++;
            if (s >= c->minsup) {
                child[nc].item = atoms[j].item;
                child[nc].n = s;
                child[nc].tids = t;
                nc++;
                sl_add(&c->out, prefix, plen + 1, 1, atoms[j].item, s);
            } else {
                free(t);
            }
        }
        if (c->order == ORC_ORDER_ASCENDING_SUPPORT) qsort(child, nc, sizeof(atom), cmp_atom_supp);
        eclat_class(c, child, nc, prefix, plen + 1);
        for (uint32_t j = 0; j < nc; j++) free(child[j].tids);
        free(child);
    }
}

/* vertical representation: tid-list of every item (ascending tids) */
static atom *build_vertical(const txdb *db, uint32_t *n_atoms, uint32_t minsup) {
    uint32_t ni = db->n_item_ids;
    uint32_t *cnt = (uint32_t *)calloc(ni + 1, sizeof(uint32_t));
    for (uint64_t i = 0; i < db->off[db->n_tx]; i++) cnt[db->items[i]]++;
    uint32_t k = 0;
    for (uint32_t it = 0; it < ni; it++) k += cnt[it] >= minsup;
    atom *atoms = (atom *)calloc(k + 1, sizeof(atom));
    uint32_t *slot = (uint32_t *)malloc((ni + 1) * sizeof(uint32_t));
    k = 0;
    for (uint32_t it = 0; it < ni; it++) {
        slot[it] = UINT32_MAX;
        if (cnt[it] >= minsup) {
            slot[it] = k;
            atoms[k].item = it;
            atoms[k].tids = (uint32_t *)malloc((cnt[it] + 1) * sizeof(uint32_t));
            atoms[k].n = 0;
            k++;
        }
    }
    for (uint64_t t = 0; t < db->n_tx; t++)
        for (uint64_t i = db->off[t]; i < db->off[t + 1]; i++) {
            uint32_t s = slot[db->items[i]];
            if (s != UINT32_MAX) atoms[s].tids[atoms[s].n++] = (uint32_t)t;
        }
    free(cnt);
    free(slot);
    *n_atoms = k;
    return atoms;
}

typedef struct {
    eclat_ctx ctx;
    atom *atoms;
    uint32_t k;
    uint32_t *next; /* shared counter of first-level classes */
    pthread_mutex_t *mu;
} worker_arg;

/* a worker takes first-level classes [a_i | a_{i+1}..] one at a time */
static void *eclat_worker(void *p) {
    worker_arg *w = (worker_arg *)p;
    uint32_t *prefix = (uint32_t *)malloc((w->k + 2) * sizeof(uint32_t));
    for (;;) {
        pthread_mutex_lock(w->mu);
        uint32_t i = (*w->next)++;
        pthread_mutex_unlock(w->mu);
        if (i + 1 >= w->k || w->ctx.out.overflow || w->ctx.out.oom) break;
        /* the class of a_i alone: run the loop body for atom i only */
        atom *a = w->atoms;
        prefix[0] = a[i].item;
        atom *child = (atom *)malloc((w->k - i - 1) * sizeof(atom));
        uint32_t nc = 0;
        for (uint32_t j = i + 1; j < w->k; j++) {
            uint32_t cap = a[i].n < a[j].n ? a[i].n : a[j].n;
            uint32_t *t = (uint32_t *)malloc((cap + 1) * sizeof(uint32_t));
            uint32_t s = intersect(a[i].tids, a[i].n, a[j].tids, a[j].n, t);
            w->ctx.candidates++;
            if (s >= w->ctx.minsup) {
                child[nc].item = a[j].item;
                child[nc].n = s;
                child[nc].tids = t;
                nc++;
                sl_add(&w->ctx.out, prefix, 1, 1, a[j].item, s);
            } else {
                free(t);
            }
        }
        if (w->ctx.order == ORC_ORDER_ASCENDING_SUPPORT)
            qsort(child, nc, sizeof(atom), cmp_atom_supp);
        eclat_class(&w->ctx, child, nc, prefix, 1);
        for (uint32_t j = 0; j < nc; j++) free(child[j].tids);
        free(child);
    }
    free(prefix);
    return NULL;
}

/*
 * Eclat-DFS: vertical representation, atoms = frequent items (reported as
 * 1-itemsets), then the DFS over classes.  order selects the order of the
 * atoms of every class: by item id, or by ascending support with ties by
 * item id.  n_threads > 1 hands first-level classes to threads one at a
 * time; the result is the same set.  max_sets > 0 stops early with
 * overflow = 1 once that many itemsets were found.
 */
int orc_eclat(uint64_t n_tx, const uint64_t *offsets, const uint32_t *items, uint32_t n_item_ids,
              uint32_t minsup, int order, int n_threads, uint64_t max_sets, orc_result *out) {
    memset(out, 0, sizeof(*out));
    if (minsup == 0) return -1;
    txdb db;
    if (txdb_make(n_tx, offsets, items, n_item_ids, &db)) return -2;
    uint32_t k;
    atom *atoms = build_vertical(&db, &k, minsup);
    txdb_free(&db);
    if (order == ORC_ORDER_ASCENDING_SUPPORT) qsort(atoms, k, sizeof(atom), cmp_atom_supp);
    else qsort(atoms, k, sizeof(atom), cmp_atom_item);

    if (n_threads < 1) n_threads = 1;
    worker_arg *w = (worker_arg *)calloc(n_threads, sizeof(worker_arg));
    pthread_t *th = (pthread_t *)calloc(n_threads, sizeof(pthread_t));
    pthread_mutex_t mu = PTHREAD_MUTEX_INITIALIZER;
    uint32_t next = 0;
    uint64_t per_thread_cap = max_sets;
    for (int t = 0; t < n_threads; t++) {
        w[t].ctx.minsup = minsup;
        w[t].ctx.order = order;
        sl_init(&w[t].ctx.out, per_thread_cap);
        w[t].atoms = atoms;
        w[t].k = k;
        w[t].next = &next;
        w[t].mu = &mu;
    }
    /* the 1-itemsets */
    for (uint32_t i = 0; i < k; i++) sl_add(&w[0].ctx.out, &atoms[i].item, 1, 0, 0, atoms[i].n);
    if (n_threads == 1) {
        eclat_worker(&w[0]);
    } else {
        for (int t = 0; t < n_threads; t++) pthread_create(&th[t], NULL, eclat_worker, &w[t]);
        for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
    }
    /* merge the per-thread lists */
    setlist all;
    sl_init(&all, 0);
    uint64_t cands = 0;
    int overflow = 0, oom = 0;
    for (int t = 0; t < n_threads; t++) {
        setlist *s = &w[t].ctx.out;
        cands += w[t].ctx.candidates;
        overflow |= s->overflow;
        oom |= s->oom;
        for (uint64_t i = 0; i < s->n_sets && !oom; i++)
            sl_add(&all, s->items + s->offsets[i], (uint32_t)(s->offsets[i + 1] - s->offsets[i]),
                   0, 0, s->supports[i]);
        sl_free(s);
    }
    oom |= all.oom;
    if (max_sets && all.n_sets > max_sets) overflow = 1;
    all.overflow = overflow;
    for (uint32_t i = 0; i < k; i++) free(atoms[i].tids);
    free(atoms);
    free(w);
    free(th);
    int rc = oom ? -2 : sl_canonical(&all, out);
    out->candidates = cands;
    out->overflow = overflow;
    sl_free(&all);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Apriori, level-wise                                                 */

/* position of the ascending itemset u (length len) in the sorted level
 * array lv (n sets of length len, row-major), or -1 */
static int64_t level_find(const uint32_t *lv, uint64_t n, uint32_t len, const uint32_t *u) {
    int64_t lo = 0, hi = (int64_t)n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        const uint32_t *x = lv + (uint64_t)mid * len;
        int c = 0;
        for (uint32_t i = 0; i < len && !c; i++)
            if (x[i] != u[i]) c = x[i] < u[i] ? -1 : 1;
        if (!c) return mid;
        if (c < 0) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

int orc_apriori(uint64_t n_tx, const uint64_t *offsets, const uint32_t *items,
                uint32_t n_item_ids, uint32_t minsup, orc_result *out) {
    memset(out, 0, sizeof(*out));
    if (minsup == 0) return -1;
    txdb db;
    if (txdb_make(n_tx, offsets, items, n_item_ids, &db)) return -2;
    setlist s;
    sl_init(&s, 0);
    /* L1 */
    uint32_t *cnt = (uint32_t *)calloc(n_item_ids + 1, sizeof(uint32_t));
    for (uint64_t i = 0; i < db.off[n_tx]; i++) cnt[db.items[i]]++;
    uint64_t nl = 0;
    uint32_t *lv = (uint32_t *)malloc((n_item_ids + 1) * sizeof(uint32_t));
    for (uint32_t it = 0; it < n_item_ids; it++)
        if (cnt[it] >= minsup) {
            lv[nl++] = it;
            sl_add(&s, &it, 1, 0, 0, cnt[it]);
        }
    free(cnt);
    uint32_t len = 1;
    uint32_t *sub = (uint32_t *)malloc((n_item_ids + 2) * sizeof(uint32_t));
    while (nl > 1) {
        /* candidates of length len+1: join sets that agree on the first len-1 items */
        uint64_t cap = 1024, nc = 0;
        uint32_t *cand = (uint32_t *)malloc(cap * (len + 1) * sizeof(uint32_t));
        for (uint64_t a = 0; a < nl; a++) {
            const uint32_t *x = lv + a * len;
            for (uint64_t b = a + 1; b < nl; b++) {
                const uint32_t *y = lv + b * len;
                if (memcmp(x, y, (len - 1) * sizeof(uint32_t)) != 0) break;
                /* x[len-1] < y[len-1] since the level is sorted */
                uint32_t *c = sub;
                memcpy(c, x, len * sizeof(uint32_t));
                c[len] = y[len - 1];
                /* prune: every len-subset must be frequent */
                int ok = 1;
                uint32_t tmp[64];
                uint32_t *t = len + 1 <= 64 ? tmp : (uint32_t *)malloc((len + 1) * sizeof(uint32_t));
                for (uint32_t drop = 0; drop + 2 < len + 1 && ok; drop++) {
                    uint32_t w = 0;
                    for (uint32_t q = 0; q <= len; q++)
                        if (q != drop) t[w++] = c[q];
                    ok = level_find(lv, nl, len, t) >= 0;
                }
                if (t != tmp) free(t);
                if (!ok) continue;
                if (nc == cap) {
                    cap *= 2;
                    cand = (uint32_t *)realloc(cand, cap * (len + 1) * sizeof(uint32_t));
                }
                memcpy(cand + nc * (len + 1), c, (len + 1) * sizeof(uint32_t));
                nc++;
            }
        }
        /* count: test every candidate against every transaction */
        uint32_t *sc = (uint32_t *)calloc(nc + 1, sizeof(uint32_t));
        for (uint64_t t = 0; t < n_tx; t++) {
            if (db.off[t + 1] - db.off[t] < len + 1) continue;
            for (uint64_t q = 0; q < nc; q++)
                sc[q] += (uint32_t)tx_contains(&db, t, cand + q * (len + 1), len + 1);
        }
        uint64_t nn = 0;
        for (uint64_t q = 0; q < nc; q++)
            if (sc[q] >= minsup) {
                memmove(cand + nn * (len + 1), cand + q * (len + 1), (len + 1) * sizeof(uint32_t));
                sl_add(&s, cand + nn * (len + 1), len + 1, 0, 0, sc[q]);
                nn++;
            }
        free(sc);
        free(lv);
        lv = cand; /* already in lexicographic order */
        nl = nn;
        len++;
    }
    free(lv);
    free(sub);
    txdb_free(&db);
    int rc = s.oom ? -2 : sl_canonical(&s, out);
    sl_free(&s);
    return rc;
}
