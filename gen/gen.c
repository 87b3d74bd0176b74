/*
 * Seeded synthetic graph inputs.
 *
 * This module only makes inputs: edge samples, the CSR built from them (rows sorted,
 * self-loops and duplicate edges removed), the symmetrized CSR, per-edge weights and
 * source vertices.  It holds none of the traversal or cost-model arithmetic; both the
 * CPU oracle and the GPU library consume what it writes.
 *
 *  - R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each sample descends `scale`
 *    levels of the adjacency matrix, choosing quadrant (0,0),(0,1),(1,0),(1,1) with
 *    probabilities a, b, c, 1-a-b-c.  No per-level noise and no label permutation, so
 *    vertex 0 is the largest hub.
 *  - Erdos-Renyi G(n, m): m uniform directed (u, v) pairs.
 *
 * Randomness is SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) used as a counter-based generator: draw i of the stream
 * keyed by s is mix(s + (i + 1) * GOLDEN).  Any sample can therefore be regenerated
 * from its index alone, which lets the CSR be built in two passes (count, then
 * scatter) without ever storing the edge list.
 *
 * Weights are w(u, v) = 1 + (mix(wkey ^ (u << 32 | v)) mod maxw): a function of the
 * edge, not of its position, so any relabelling or reordering keeps them.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* draw i (0-based) of the SplitMix64 stream keyed by s */
static inline uint64_t draw(uint64_t s, uint64_t i) { return mix64(s + (i + 1) * GOLDEN); }

typedef struct gen_graph {
    uint64_t n, m;
    uint64_t *off; /* n + 1 */
    uint32_t *col; /* m */
} gen_graph;

/* ------------------------------------------------------------------ threads */
typedef void (*range_fn)(void *ctx, uint64_t lo, uint64_t hi, int tid);
typedef struct {
    range_fn fn;
    void *ctx;
    uint64_t total, chunk;
    uint64_t next; /* atomic */
    int tid;
} par_job;

static void *par_worker(void *p) {
    par_job *j = (par_job *)p;
    int tid = __atomic_fetch_add(&j->tid, 1, __ATOMIC_RELAXED);
    for (;;) {
        uint64_t lo = __atomic_fetch_add(&j->next, j->chunk, __ATOMIC_RELAXED);
        if (lo >= j->total) break;
        uint64_t hi = lo + j->chunk < j->total ? lo + j->chunk : j->total;
        j->fn(j->ctx, lo, hi, tid);
    }
    return NULL;
}

static int g_threads = 0;
static int nthreads_default(void) {
    if (g_threads > 0) return g_threads;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    const char *e = getenv("OMP_NUM_THREADS");
    if (e && atoi(e) > 0 && atoi(e) < c) c = atoi(e);
    if (c < 1) c = 1;
    if (c > 64) c = 64;
    return (int)c;
}
void gen_set_threads(int t) { g_threads = t; }

static void parallel_for(uint64_t total, uint64_t chunk, range_fn fn, void *ctx) {
    if (total == 0) return;
    par_job j = {fn, ctx, total, chunk ? chunk : 1, 0, 0};
    int nt = nthreads_default();
    if ((uint64_t)nt > (total + j.chunk - 1) / j.chunk) nt = (int)((total + j.chunk - 1) / j.chunk);
    if (nt <= 1) {
        par_worker(&j);
        return;
    }
    pthread_t th[64];
    int started = 0;
    for (int i = 0; i < nt; i++) {
        if (pthread_create(&th[started], NULL, par_worker, &j) != 0) break; /* e.g. a thread limit */
        started++;
    }
    par_worker(&j); /* the caller takes work too, so the job finishes with any number started */
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------ edge sources */
typedef struct {
    int kind; /* 0 rmat, 1 er, 2 explicit pairs, 3 symmetrize csr */
    uint64_t n, nsamples, seed;
    int scale;
    uint32_t ta, tab, tabc; /* R-MAT quadrant thresholds on a 32-bit draw */
    const uint32_t *ps, *pd; /* explicit pairs */
    const gen_graph *g;      /* symmetrize */
} edge_src;

static inline void rmat_sample(const edge_src *s, uint64_t k, uint32_t *pu, uint32_t *pv) {
    uint32_t u = 0, v = 0;
    uint64_t r = 0;
    for (int l = 0; l < s->scale; l++) {
        if ((l & 1) == 0) r = draw(s->seed, k * 16 + (uint64_t)(l >> 1));
        uint32_t x = (l & 1) ? (uint32_t)(r >> 32) : (uint32_t)r;
        /* quadrants by x: [0,ta) -> (0,0), [ta,tab) -> (0,1), [tab,tabc) -> (1,0), rest -> (1,1) */
        const uint32_t ge_a = x >= s->ta, ge_ab = x >= s->tab, ge_abc = x >= s->tabc;
        const uint32_t sh = (uint32_t)(s->scale - 1 - l);
        u |= ge_ab << sh;
        v |= ((ge_a ^ ge_ab) | ge_abc) << sh;
    }
    *pu = u;
    *pv = v;
}
static inline void er_sample(const edge_src *s, uint64_t k, uint32_t *pu, uint32_t *pv) {
    uint64_t r0 = draw(s->seed, 2 * k), r1 = draw(s->seed, 2 * k + 1);
    *pu = (uint32_t)(((unsigned __int128)r0 * s->n) >> 64);
    *pv = (uint32_t)(((unsigned __int128)r1 * s->n) >> 64);
}

/* ------------------------------------------------------------- CSR build */
/* Edges are routed to 2^bbits buckets by the top bits of u.  Pass A counts edges per
   (item block, bucket) over a fixed split of the items into blocks; pass B regenerates
   the same items and scatters (u << 32 | v) keys into their (bucket, block) slots;
   pass C sorts every bucket (LSD radix over the bits that vary inside it), drops
   duplicates and self-loops and counts each row; pass D copies the kept keys into the
   final CSR.  No atomics: every slot and every row has exactly one writer. */
typedef struct {
    const edge_src *s;
    uint64_t nitems;
    uint32_t nblk;     /* item blocks of the fixed split */
    uint32_t nb;       /* buckets */
    uint32_t shift;    /* bucket = u >> shift */
    uint32_t vbits;    /* bits of a vertex id */
    uint64_t *slot;    /* nblk x nb: counts, then write cursors */
    uint64_t *keys;
    uint64_t *bstart;  /* nb + 1 */
    uint64_t *bkept;   /* nb */
    uint32_t *deg;     /* n */
    uint64_t *off;
    uint32_t *col;
    int pass;
    int oom;
} bctx;

static inline void route(bctx *c, uint64_t blk, uint32_t u, uint32_t v) {
    uint64_t *sl = &c->slot[blk * c->nb + (u >> c->shift)];
    if (c->pass == 0)
        (*sl)++;
    else
        c->keys[(*sl)++] = ((uint64_t)u << 32) | v;
}

static void items_fn(void *ctx, uint64_t lo, uint64_t hi, int tid) {
    (void)tid;
    bctx *c = (bctx *)ctx;
    const edge_src *s = c->s;
    for (uint64_t blk = lo; blk < hi; blk++) {
        const uint64_t k0 = c->nitems * blk / c->nblk, k1 = c->nitems * (blk + 1) / c->nblk;
        for (uint64_t k = k0; k < k1; k++) {
            uint32_t u, v;
            switch (s->kind) {
            case 0: rmat_sample(s, k, &u, &v); route(c, blk, u, v); break;
            case 1: er_sample(s, k, &u, &v); route(c, blk, u, v); break;
            case 2: route(c, blk, s->ps[k], s->pd[k]); break;
            default: {
                /* k indexes source vertices of the CSR being symmetrized */
                const gen_graph *g = s->g;
                for (uint64_t e = g->off[k]; e < g->off[k + 1]; e++) {
                    route(c, blk, (uint32_t)k, g->col[e]);
                    route(c, blk, g->col[e], (uint32_t)k);
                }
            }
            }
        }
    }
}

#define RADIX_BITS 11
static void sort_bucket_fn(void *ctx, uint64_t lo, uint64_t hi, int tid) {
    (void)tid;
    bctx *c = (bctx *)ctx;
    const uint64_t vmask = (c->vbits >= 32) ? 0xFFFFFFFFull : ((1ull << c->vbits) - 1);
    const uint64_t umask = (1ull << c->shift) - 1;
    const uint32_t nbits = c->shift + c->vbits;
    for (uint64_t b = lo; b < hi; b++) {
        uint64_t *k = c->keys + c->bstart[b];
        const uint64_t len = c->bstart[b + 1] - c->bstart[b];
        if (len <= 32) {
            for (uint64_t i = 1; i < len; i++) {
                uint64_t x = k[i], j = i;
                while (j > 0 && k[j - 1] > x) { k[j] = k[j - 1]; j--; }
                k[j] = x;
            }
        } else {
            uint64_t *tmp = (uint64_t *)malloc(len * sizeof(uint64_t));
            if (!tmp) { c->oom = 1; return; }
            uint64_t *src = k, *dst = tmp;
            static __thread uint64_t hist[1u << RADIX_BITS];
            for (uint32_t sh = 0; sh < nbits; sh += RADIX_BITS) {
                memset(hist, 0, sizeof(hist));
                for (uint64_t i = 0; i < len; i++) {
                    uint64_t ck = (((src[i] >> 32) & umask) << c->vbits) | (src[i] & vmask);
                    hist[(ck >> sh) & ((1u << RADIX_BITS) - 1)]++;
                }
                uint64_t run = 0;
                for (uint32_t d = 0; d < (1u << RADIX_BITS); d++) { uint64_t h = hist[d]; hist[d] = run; run += h; }
                for (uint64_t i = 0; i < len; i++) {
                    uint64_t ck = (((src[i] >> 32) & umask) << c->vbits) | (src[i] & vmask);
                    dst[hist[(ck >> sh) & ((1u << RADIX_BITS) - 1)]++] = src[i];
                }
                uint64_t *t = src; src = dst; dst = t;
            }
            if (src != k) memcpy(k, src, len * sizeof(uint64_t));
            free(tmp);
        }
        uint64_t w = 0;
        for (uint64_t i = 0; i < len; i++) {
            const uint32_t u = (uint32_t)(k[i] >> 32), v = (uint32_t)k[i];
            if (u == v) continue;
            if (w > 0 && k[w - 1] == k[i]) continue;
            k[w++] = k[i];
            c->deg[u]++;
        }
        c->bkept[b] = w;
    }
}

static void write_rows_fn(void *ctx, uint64_t lo, uint64_t hi, int tid) {
    (void)tid;
    bctx *c = (bctx *)ctx;
    for (uint64_t b = lo; b < hi; b++) {
        /* buckets cover 2^vbits >= n ids: those starting at or past n hold no keys, and
           their first id would index past off[n] */
        if (!c->bkept[b]) continue;
        const uint64_t *k = c->keys + c->bstart[b];
        uint32_t *out = c->col + c->off[b << c->shift];
        for (uint64_t i = 0; i < c->bkept[b]; i++) out[i] = (uint32_t)k[i];
    }
}

static gen_graph *build_csr(const edge_src *s, uint64_t n, uint64_t nitems) {
    gen_graph *g = (gen_graph *)calloc(1, sizeof(gen_graph));
    if (!g) return NULL;
    g->n = n;
    bctx c;
    memset(&c, 0, sizeof(c));
    c.s = s;
    c.nitems = nitems;
    c.vbits = 1;
    while (c.vbits < 32 && (1ull << c.vbits) < n) c.vbits++;
    const uint32_t bbits = c.vbits < 12 ? c.vbits : 12;
    c.shift = c.vbits - bbits;
    c.nb = 1u << bbits;
    c.nblk = (uint32_t)(nitems < 4096 ? (nitems ? nitems : 1) : 4096);
    c.slot = (uint64_t *)calloc((uint64_t)c.nblk * c.nb, sizeof(uint64_t));
    c.bstart = (uint64_t *)malloc((c.nb + 1) * sizeof(uint64_t));
    c.bkept = (uint64_t *)calloc(c.nb, sizeof(uint64_t));
    c.deg = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    g->off = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    if (!c.slot || !c.bstart || !c.bkept || !c.deg || !g->off) goto fail;
    c.pass = 0;
    parallel_for(c.nblk, 1, items_fn, &c);
    /* bucket-major, block-minor prefix: slot becomes each (block, bucket) cursor */
    uint64_t run = 0;
    for (uint32_t b = 0; b < c.nb; b++) {
        c.bstart[b] = run;
        for (uint32_t blk = 0; blk < c.nblk; blk++) {
            uint64_t *sl = &c.slot[(uint64_t)blk * c.nb + b];
            uint64_t h = *sl;
            *sl = run;
            run += h;
        }
    }
    c.bstart[c.nb] = run;
    c.keys = (uint64_t *)malloc((run ? run : 1) * sizeof(uint64_t));
    if (!c.keys) goto fail;
    c.pass = 1;
    parallel_for(c.nblk, 1, items_fn, &c);
    parallel_for(c.nb, 1, sort_bucket_fn, &c);
    if (c.oom) goto fail;
    g->off[0] = 0;
    for (uint64_t u = 0; u < n; u++) g->off[u + 1] = g->off[u] + c.deg[u];
    g->m = g->off[n];
    g->col = (uint32_t *)malloc((g->m ? g->m : 1) * sizeof(uint32_t));
    if (!g->col) goto fail;
    c.off = g->off;
    c.col = g->col;
    parallel_for(c.nb, 1, write_rows_fn, &c);
    free(c.slot); free(c.bstart); free(c.bkept); free(c.deg); free(c.keys);
    return g;
fail:
    free(c.slot); free(c.bstart); free(c.bkept); free(c.deg); free(c.keys);
    free(g->off);
    free(g->col);
    free(g);
    return NULL;
}

/* ------------------------------------------------------------------ public */
gen_graph *gen_rmat(int scale, uint64_t nsamples, double a, double b, double c, uint64_t seed) {
    if (scale < 1 || scale > 31 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return NULL;
    edge_src s;
    memset(&s, 0, sizeof(s));
    s.kind = 0;
    s.scale = scale;
    s.n = 1ull << scale;
    s.nsamples = nsamples;
    s.seed = mix64(seed ^ 0x524D4154ULL); /* stream key for "RMAT" */
    double two32 = 4294967296.0;
    double ta = a * two32, tab = (a + b) * two32, tabc = (a + b + c) * two32;
    s.ta = ta >= two32 ? 0xFFFFFFFFu : (uint32_t)ta;
    s.tab = tab >= two32 ? 0xFFFFFFFFu : (uint32_t)tab;
    s.tabc = tabc >= two32 ? 0xFFFFFFFFu : (uint32_t)tabc;
    return build_csr(&s, s.n, nsamples);
}

gen_graph *gen_er(uint64_t n, uint64_t nsamples, uint64_t seed) {
    if (n == 0 || n > 0xFFFFFFFEull) return NULL;
    edge_src s;
    memset(&s, 0, sizeof(s));
    s.kind = 1;
    s.n = n;
    s.nsamples = nsamples;
    s.seed = mix64(seed ^ 0x4552ULL); /* "ER" */
    return build_csr(&s, n, nsamples);
}

/* explicit (src[i], dst[i]) pairs; every id must be < n */
gen_graph *gen_from_pairs(uint64_t n, uint64_t npairs, const uint32_t *src, const uint32_t *dst) {
    for (uint64_t i = 0; i < npairs; i++)
        if (src[i] >= n || dst[i] >= n) return NULL;
    edge_src s;
    memset(&s, 0, sizeof(s));
    s.kind = 2;
    s.n = n;
    s.ps = src;
    s.pd = dst;
    return build_csr(&s, n, npairs);
}

/* CSR of E union E^T */
gen_graph *gen_symmetrize(const gen_graph *g) {
    edge_src s;
    memset(&s, 0, sizeof(s));
    s.kind = 3;
    s.n = g->n;
    s.g = g;
    return build_csr(&s, g->n, g->n);
}

/* symmetrize a caller-held CSR */
gen_graph *gen_symmetrize_csr(uint64_t n, const uint64_t *off, const uint32_t *col) {
    gen_graph tmp = {n, off[n], (uint64_t *)off, (uint32_t *)col};
    return gen_symmetrize(&tmp);
}

uint64_t gen_num_vertices(const gen_graph *g) { return g->n; }
uint64_t gen_num_edges(const gen_graph *g) { return g->m; }
void gen_copy_out(const gen_graph *g, uint64_t *off, uint32_t *col) {
    memcpy(off, g->off, (g->n + 1) * sizeof(uint64_t));
    memcpy(col, g->col, g->m * sizeof(uint32_t));
}
void gen_free(gen_graph *g) {
    if (!g) return;
    free(g->off);
    free(g->col);
    free(g);
}

typedef struct {
    const uint64_t *off;
    const uint32_t *col;
    uint32_t *w;
    uint64_t key;
    uint32_t maxw;
} wctx;
static void weights_fn(void *ctx, uint64_t lo, uint64_t hi, int tid) {
    (void)tid;
    wctx *c = (wctx *)ctx;
    for (uint64_t u = lo; u < hi; u++)
        for (uint64_t e = c->off[u]; e < c->off[u + 1]; e++)
            c->w[e] = 1u + (uint32_t)(mix64(c->key ^ ((u << 32) | c->col[e])) % c->maxw);
}
/* w[e] = 1 + hash(u, v) mod maxw, in [1, maxw] */
void gen_weights(uint64_t n, const uint64_t *off, const uint32_t *col, uint64_t seed, uint32_t maxw, uint32_t *w) {
    wctx c = {off, col, w, mix64(seed ^ 0x57454947ULL), maxw ? maxw : 1};
    parallel_for(n, 4096, weights_fn, &c);
}

/* k distinct sources, uniform over vertices with out-degree >= 1 (rejection on a
   counter stream); returns the number written (fewer if not enough such vertices) */
uint64_t gen_sources(uint64_t n, const uint64_t *off, uint64_t k, uint64_t seed, uint32_t *out) {
    uint64_t have = 0, eligible = 0;
    for (uint64_t u = 0; u < n; u++) eligible += off[u + 1] > off[u];
    if (k > eligible) k = eligible;
    uint64_t key = mix64(seed ^ 0x53524353ULL);
    for (uint64_t i = 0; have < k; i++) {
        uint32_t v = (uint32_t)(((unsigned __int128)draw(key, i) * n) >> 64);
        if (off[v + 1] == off[v]) continue;
        int dup = 0;
        for (uint64_t j = 0; j < have; j++) dup |= out[j] == v;
        if (!dup) out[have++] = v;
    }
    return have;
}
