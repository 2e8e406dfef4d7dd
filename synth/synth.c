/*
 * Seeded synthetic transaction databases for frequent-itemset mining.
 *
 * This module only draws random inputs. It holds none of the mining
 * arithmetic and is shared by the CPU oracle and the GPU library's tests and
 * benchmarks, which both consume the CSR it produces.
 *
 * Random numbers: xoshiro256** (Blackman & Vigna, 2018) seeded through
 * SplitMix64 (Steele, Lea & Flood, 2014). Distributions are written out here
 * (not std::*_distribution, whose algorithms are implementation-defined):
 *   - Poisson(l):      Knuth's product-of-uniforms method (TAOCP vol. 2, 3.4.1).
 *   - Exponential(mu): inversion, -mu * ln(1 - U).
 *   - Normal(mu, s):   Box-Muller, first of the pair.
 *   - Gamma(k), k int: sum of k unit exponentials, -ln(U1 * ... * Uk).
 *   - Beta(a, b), a,b int: Ga / (Ga + Gb).
 *
 * Two generators:
 *   synth_basket : market-basket data in the style of the IBM Quest generator
 *                  that produced the thesis's T..I..P..PL..TL.. databases
 *                  (Experimental evaluation, dataset description): latent
 *                  patterns with exponential weights, correlation with the
 *                  previous pattern, and per-pattern corruption.
 *   synth_dense  : dense data, each item present independently with a
 *                  Beta-distributed probability, plus planted correlated groups.
 *
 * Output: CSR with offsets[n_tx + 1] (uint64) and items[nnz] (uint32). Every
 * transaction is sorted ascending and free of duplicates.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t s[4];
} rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl64(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

/* uniform double in [0, 1) with 53 random bits */
static double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0, n), n < 2^32, by the multiply-high method */
static uint32_t rng_below(rng_t *r, uint32_t n) {
    return (uint32_t)(((rng_next(r) >> 32) * (uint64_t)n) >> 32);
}

static uint32_t rng_poisson(rng_t *r, double lambda) {
    if (lambda <= 0.0) return 0;
    double L = exp(-lambda), p = 1.0;
    uint32_t k = 0;
    do {
        k++;
        p *= rng_u01(r);
    } while (p > L);
    return k - 1;
}

static double rng_exponential(rng_t *r, double mean) { return -mean * log(1.0 - rng_u01(r)); }

static double rng_normal(rng_t *r, double mu, double sd) {
    double u1 = 1.0 - rng_u01(r); /* (0, 1] */
    double u2 = rng_u01(r);
    return mu + sd * sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

static double rng_gamma_int(rng_t *r, int k) {
    double prod = 1.0;
    for (int i = 0; i < k; i++) prod *= 1.0 - rng_u01(r);
    return -log(prod);
}

static double rng_beta_int(rng_t *r, int a, int b) {
    double x = rng_gamma_int(r, a), y = rng_gamma_int(r, b);
    return x / (x + y);
}

/* ------------------------------------------------------------------ */

typedef struct {
    uint64_t n_tx;
    uint64_t nnz;
    uint32_t n_items;
    uint64_t *offsets;
    uint32_t *items;
} synth_db;

void synth_free(synth_db *db) {
    if (!db) return;
    free(db->offsets);
    free(db->items);
    free(db);
}

/* growable item buffer */
typedef struct {
    uint32_t *v;
    uint64_t n, cap;
} ubuf;

static int ubuf_push(ubuf *b, uint32_t x) {
    if (b->n == b->cap) {
        uint64_t nc = b->cap ? b->cap * 2 : 1 << 16;
        uint32_t *nv = (uint32_t *)realloc(b->v, nc * sizeof(uint32_t));
        if (!nv) return -1;
        b->v = nv;
        b->cap = nc;
    }
    b->v[b->n++] = x;
    return 0;
}

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Basket generator.
 * Patterns p = 0..n_patterns-1:
 *   length      = max(1, Poisson(mean_pat_len)), at most n_items;
 *   a fraction min(1, Exponential(corr_mean)) of its items (rounded down)
 *   is copied from the previous pattern, chosen uniformly without replacement;
 *   the remaining items are distinct uniform items;
 *   weight      = Exponential(1) (normalised by the cumulative table);
 *   corruption  = Normal(corrupt_mean, corrupt_sd) clamped to [0, 1].
 * Transaction:
 *   target length L = Poisson(mean_len);
 *   while |t| < L: pick a pattern by weight, drop each of its items with
 *   probability equal to its corruption, add the rest (the last pattern is
 *   added whole, so |t| may exceed L). L = 0 gives an empty transaction.
 *   A guard of 64 * (L + 1) pattern draws bounds the loop when corruption
 *   drops nearly everything.
 */
int synth_basket(uint64_t seed, uint64_t n_tx, uint32_t n_items, double mean_len,
                 uint32_t n_patterns, double mean_pat_len, double corr_mean,
                 double corrupt_mean, double corrupt_sd, synth_db **out) {
    if (!out || n_items == 0 || n_patterns == 0) return -1;
    *out = NULL;
    rng_t r;
    rng_seed(&r, seed);

    uint64_t *pat_off = (uint64_t *)malloc((n_patterns + 1) * sizeof(uint64_t));
    double *cum = (double *)malloc(n_patterns * sizeof(double));
    double *corrupt = (double *)malloc(n_patterns * sizeof(double));
    uint32_t *mark = (uint32_t *)calloc(n_items, sizeof(uint32_t));
    ubuf pit = {0}, tit = {0};
    uint64_t *offsets = (uint64_t *)malloc((n_tx + 1) * sizeof(uint64_t));
    uint32_t *tmp = NULL;
    int rc = -2;
    if (!pat_off || !cum || !corrupt || !mark || !offsets) goto done;

    /* latent patterns */
    uint32_t stamp = 0;
    double wsum = 0.0;
    pat_off[0] = 0;
    for (uint32_t p = 0; p < n_patterns; p++) {
        uint32_t len = rng_poisson(&r, mean_pat_len);
        if (len < 1) len = 1;
        if (len > n_items) len = n_items;
        stamp++;
        uint32_t have = 0;
        if (p > 0) {
            double frac = rng_exponential(&r, corr_mean);
            if (frac > 1.0) frac = 1.0;
            uint64_t prev0 = pat_off[p - 1], prevn = pat_off[p] - pat_off[p - 1];
            uint32_t ncopy = (uint32_t)floor(frac * (double)len);
            if (ncopy > prevn) ncopy = (uint32_t)prevn;
            /* copy ncopy distinct items of the previous pattern */
            uint32_t tries = 0;
            while (have < ncopy && tries < 64 * (ncopy + 1)) {
                uint32_t it = pit.v[prev0 + rng_below(&r, (uint32_t)prevn)];
                tries++;
                if (mark[it] == stamp) continue;
                mark[it] = stamp;
                if (ubuf_push(&pit, it)) goto done;
                have++;
            }
        }
        while (have < len) {
            uint32_t it = rng_below(&r, n_items);
            if (mark[it] == stamp) continue;
            mark[it] = stamp;
            if (ubuf_push(&pit, it)) goto done;
            have++;
        }
        pat_off[p + 1] = pit.n;
        wsum += rng_exponential(&r, 1.0);
        cum[p] = wsum;
        double c = rng_normal(&r, corrupt_mean, corrupt_sd);
        corrupt[p] = c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c);
    }

    /* transactions */
    tmp = (uint32_t *)malloc((size_t)n_items * sizeof(uint32_t));
    if (!tmp) goto done;
    offsets[0] = 0;
    for (uint64_t t = 0; t < n_tx; t++) {
        uint32_t L = rng_poisson(&r, mean_len);
        uint32_t cnt = 0;
        uint64_t guard = 64ull * ((uint64_t)L + 1);
        stamp++;
        if (stamp == 0) { /* wrapped: reset marks */
            memset(mark, 0, n_items * sizeof(uint32_t));
            stamp = 1;
        }
        while (cnt < L && guard--) {
            double u = rng_u01(&r) * wsum;
            /* first p with cum[p] > u */
            uint32_t lo = 0, hi = n_patterns - 1;
            while (lo < hi) {
                uint32_t mid = (lo + hi) / 2;
                if (cum[mid] > u) hi = mid;
                else lo = mid + 1;
            }
            double c = corrupt[lo];
            for (uint64_t q = pat_off[lo]; q < pat_off[lo + 1]; q++) {
                if (rng_u01(&r) < c) continue;
                uint32_t it = pit.v[q];
                if (mark[it] == stamp) continue;
                mark[it] = stamp;
                tmp[cnt++] = it;
            }
        }
        qsort(tmp, cnt, sizeof(uint32_t), cmp_u32);
        for (uint32_t q = 0; q < cnt; q++)
            if (ubuf_push(&tit, tmp[q])) goto done;
        offsets[t + 1] = tit.n;
    }

    synth_db *db = (synth_db *)calloc(1, sizeof(synth_db));
    if (!db) goto done;
    db->n_tx = n_tx;
    db->nnz = tit.n;
    db->n_items = n_items;
    db->offsets = offsets;
    db->items = tit.v;
    offsets = NULL;
    tit.v = NULL;
    *out = db;
    rc = 0;
done:
    free(pat_off);
    free(cum);
    free(corrupt);
    free(mark);
    free(pit.v);
    free(tit.v);
    free(offsets);
    free(tmp);
    return rc;
}

/*
 * Dense generator.
 * Item i is present in a transaction independently with probability
 * p_i ~ Beta(beta_a, beta_b). n_groups planted groups of size uniform in
 * [gmin, gmax] (distinct items inside a group; groups may overlap) each have
 * an activation probability uniform in [act_lo, act_hi); in a transaction
 * where a group is active, each of its items is set with probability keep.
 */
int synth_dense(uint64_t seed, uint64_t n_tx, uint32_t n_items, int beta_a, int beta_b,
                uint32_t n_groups, uint32_t gmin, uint32_t gmax, double act_lo, double act_hi,
                double keep, synth_db **out) {
    if (!out || n_items == 0 || gmin > gmax || gmax > n_items || beta_a < 1 || beta_b < 1)
        return -1;
    *out = NULL;
    rng_t r;
    rng_seed(&r, seed);
    double *p = (double *)malloc(n_items * sizeof(double));
    uint32_t *gsz = (uint32_t *)malloc((n_groups + 1) * sizeof(uint32_t));
    uint32_t *gitems = (uint32_t *)malloc(((size_t)n_groups * gmax + 1) * sizeof(uint32_t));
    double *gact = (double *)malloc((n_groups + 1) * sizeof(double));
    uint8_t *present = (uint8_t *)malloc(n_items);
    uint64_t *offsets = (uint64_t *)malloc((n_tx + 1) * sizeof(uint64_t));
    ubuf tit = {0};
    int rc = -2;
    if (!p || !gsz || !gitems || !gact || !present || !offsets) goto done;

    for (uint32_t i = 0; i < n_items; i++) p[i] = rng_beta_int(&r, beta_a, beta_b);
    for (uint32_t g = 0; g < n_groups; g++) {
        uint32_t sz = gmin + rng_below(&r, gmax - gmin + 1);
        gsz[g] = sz;
        uint32_t have = 0;
        while (have < sz) {
            uint32_t it = rng_below(&r, n_items);
            int dup = 0;
            for (uint32_t q = 0; q < have; q++)
                if (gitems[(size_t)g * gmax + q] == it) dup = 1;
            if (dup) continue;
            gitems[(size_t)g * gmax + have++] = it;
        }
        gact[g] = act_lo + (act_hi - act_lo) * rng_u01(&r);
    }
    offsets[0] = 0;
    for (uint64_t t = 0; t < n_tx; t++) {
        for (uint32_t i = 0; i < n_items; i++) present[i] = rng_u01(&r) < p[i];
        for (uint32_t g = 0; g < n_groups; g++) {
            if (!(rng_u01(&r) < gact[g])) continue;
            for (uint32_t q = 0; q < gsz[g]; q++)
                if (rng_u01(&r) < keep) present[gitems[(size_t)g * gmax + q]] = 1;
        }
        for (uint32_t i = 0; i < n_items; i++)
            if (present[i] && ubuf_push(&tit, i)) goto done;
        offsets[t + 1] = tit.n;
    }
    synth_db *db = (synth_db *)calloc(1, sizeof(synth_db));
    if (!db) goto done;
    db->n_tx = n_tx;
    db->nnz = tit.n;
    db->n_items = n_items;
    db->offsets = offsets;
    db->items = tit.v;
    offsets = NULL;
    tit.v = NULL;
    *out = db;
    rc = 0;
done:
    free(p);
    free(gsz);
    free(gitems);
    free(gact);
    free(present);
    free(offsets);
    free(tit.v);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Draws used to pick workload parameters (batch instances, request
 * streams). Exposed so that every parameter comes from the same seeded
 * generator. */

typedef struct {
    uint64_t seed;
    uint64_t n_tx;
    uint32_t n_items;
    double mean_len;
    double rel_minsup;
    uint32_t n_patterns;
    double mean_pat_len;
} synth_basket_params;

/* 64-bit seed of substream `index` of `base` */
uint64_t synth_substream(uint64_t base, uint64_t index) {
    uint64_t x = base ^ (0xD1B54A32D192ED03ULL * (index + 1));
    return splitmix64(&x);
}

/*
 * Parameters of one batch instance (log-uniform sizes and minimum supports):
 *   n_tx      = round(exp U(ln lo_tx, ln hi_tx))
 *   n_items   = round(exp U(ln lo_items, ln hi_items))
 *   mean_len  = U(lo_len, hi_len)
 *   rel_minsup= exp U(ln lo_rel, ln hi_rel)
 *   patterns  = 2 * n_items, pattern mean length = max(2, round(0.3 * mean_len))
 */
void synth_draw_basket_params(uint64_t seed, uint64_t lo_tx, uint64_t hi_tx, uint32_t lo_items,
                              uint32_t hi_items, double lo_len, double hi_len, double lo_rel,
                              double hi_rel, synth_basket_params *out) {
    rng_t r;
    rng_seed(&r, seed);
    double a = log((double)lo_tx), b = log((double)hi_tx);
    out->n_tx = (uint64_t)llround(exp(a + (b - a) * rng_u01(&r)));
    a = log((double)lo_items);
    b = log((double)hi_items);
    out->n_items = (uint32_t)llround(exp(a + (b - a) * rng_u01(&r)));
    out->mean_len = lo_len + (hi_len - lo_len) * rng_u01(&r);
    a = log(lo_rel);
    b = log(hi_rel);
    out->rel_minsup = exp(a + (b - a) * rng_u01(&r));
    out->n_patterns = 2 * out->n_items;
    double pm = floor(0.3 * out->mean_len + 0.5);
    out->mean_pat_len = pm < 2.0 ? 2.0 : pm;
    out->seed = splitmix64(&seed);
}

/* n uniform doubles in [0, 1) and n exponential draws, for request streams */
void synth_uniforms(uint64_t seed, uint64_t n, double *out) {
    rng_t r;
    rng_seed(&r, seed);
    for (uint64_t i = 0; i < n; i++) out[i] = rng_u01(&r);
}

void synth_exponentials(uint64_t seed, uint64_t n, double mean, double *out) {
    rng_t r;
    rng_seed(&r, seed);
    for (uint64_t i = 0; i < n; i++) out[i] = rng_exponential(&r, mean);
}

/* first n raw 64-bit outputs, for reproducibility checks of the generator */
void synth_raw(uint64_t seed, uint64_t n, uint64_t *out) {
    rng_t r;
    rng_seed(&r, seed);
    for (uint64_t i = 0; i < n; i++) out[i] = rng_next(&r);
}
