/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, single-threaded, obviously-correct C for what the hybrid-transfer traversal
 * computes.  Only the tests, the smoke check and the benchmark's CPU-baseline leg call
 * it; the GPU library never links, loads or calls it, and it shares no code with it.
 *
 * Paper: "HyTGraph: GPU-Accelerated Graph Processing with Hybrid Transfer Management"
 * (Wang, Ai, Zhang, Chen, Yu; arXiv 2208.14935).
 *
 * Graph: CSR with uint64 offsets off[0..n], uint32 neighbour ids col[0..m), optional
 * uint32 weights w[0..m).  Unreached vertices hold UINT32_MAX.
 *
 * Parts:
 *  - orc_bfs      : hop levels by a FIFO queue (Sec. 2.1 vertex-centric push model;
 *                   BFS listed among the algorithms of Sec. 7.1).
 *  - orc_sssp     : Dijkstra with a binary heap and 64-bit sums (Sec. 2.1, Fig. 1's
 *                   SSSP example; Sec. 7.1).
 *  - orc_sssp_check : the complete shortest-path certificate of a proposed answer, for
 *                   graphs too large to run Dijkstra on in a test.
 *  - orc_sync_rounds : synchronous Bellman-Ford / label-propagation round count, used
 *                   only as the upper bound of an asynchronous run's iteration count.
 *  - orc_cc       : union-find (union by size, path halving), label = min vertex id
 *                   in the component (Sec. 7.1 "connected component").
 *  - orc_pagerank : FP64 power iteration, T synchronous steps (Sec. 3, Sec. 7.1).
 *  - orc_ppr      : personalized PageRank: the same iteration with the restart mass
 *                   on one source vertex instead of spread over all of them, x_0 = e_s
 *                   (the query served alongside BFS and SSSP).  FP64.
 *  - orc_hub_order: hub sorting (Sec. 6.1): the top 8% of vertices by
 *                   H(v) = D_o(v) D_i(v) / (D_omax D_imax), highest first, ahead of the
 *                   other vertices in their natural order.
 *  - orc_partition: chunk-based edge-balanced partitioning into consecutive vertex
 *                   ranges (Sec. 4).
 *  - orc_partition_stats / orc_select : the per-partition cost model, Eq. 1-3 with the
 *                   zero-copy round-trip damping and the alpha/beta selection rule
 *                   (Sec. 5.1, Algorithm 1 "cost analysis and engine selection"),
 *                   evaluated in exact rational arithmetic.
 *  - orc_combine  : task combination of consecutive filter partitions (Sec. 5.2,
 *                   Algorithm 1 "task combination").
 *  - orc_gather   : the compaction engine's output: active neighbour lists packed in
 *                   order plus the new index array (Sec. 2.2, Sec. 6.3).
 *
 * Readings of the paper that the code below takes are listed where they apply.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define UNREACHED 0xFFFFFFFFu

/* engine codes written by orc_select */
enum { ORC_NONE = 0, ORC_RESIDENT = 1, ORC_FILTER = 2, ORC_ZEROCOPY = 3, ORC_COMPACT = 4 };

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ BFS */
/* level[v] = fewest edges on a directed path source -> v.  Returns the number of
   non-empty frontiers, i.e. 1 + the largest finite level. */
uint32_t orc_bfs(uint64_t n, const uint64_t *off, const uint32_t *col, uint32_t source, uint32_t *level) {
    for (uint64_t v = 0; v < n; v++) level[v] = UNREACHED;
    uint32_t *queue = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint64_t head = 0, tail = 0;
    level[source] = 0;
    queue[tail++] = source;
    uint32_t maxlevel = 0;
    while (head < tail) {
        uint32_t u = queue[head++];
        if (level[u] > maxlevel) maxlevel = level[u];
        for (uint64_t e = off[u]; e < off[u + 1]; e++) {
            uint32_t v = col[e];
            if (level[v] == UNREACHED) {
                level[v] = level[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return maxlevel + 1;
}

/* ----------------------------------------------------------------- SSSP */
typedef struct {
    uint64_t d;
    uint32_t v;
} heap_item;

static void heap_push(heap_item *h, uint64_t *size, heap_item x) {
    uint64_t i = (*size)++;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (h[p].d <= x.d) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = x;
}
static heap_item heap_pop(heap_item *h, uint64_t *size) {
    heap_item top = h[0];
    heap_item last = h[--(*size)];
    uint64_t i = 0;
    for (;;) {
        uint64_t c = 2 * i + 1;
        if (c >= *size) break;
        if (c + 1 < *size && h[c + 1].d < h[c].d) c++;
        if (last.d <= h[c].d) break;
        h[i] = h[c];
        i = c;
    }
    if (*size > 0) h[i] = last;
    return top;
}

/* dist[v] = min over directed paths source -> v of the summed weights.  Returns 0 on
   success, 1 if some finite distance does not fit below UINT32_MAX (the value that
   marks an unreached vertex). */
int orc_sssp(uint64_t n, const uint64_t *off, const uint32_t *col, const uint32_t *w, uint32_t source,
             uint32_t *dist) {
    uint64_t *d = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    unsigned char *done = (unsigned char *)calloc(n ? n : 1, 1);
    uint64_t cap = off[n] + 1, size = 0;
    heap_item *h = (heap_item *)malloc(cap * sizeof(heap_item));
    const uint64_t INF = ~0ull;
    for (uint64_t v = 0; v < n; v++) d[v] = INF;
    d[source] = 0;
    heap_push(h, &size, (heap_item){0, source});
    while (size > 0) {
        heap_item it = heap_pop(h, &size);
        if (done[it.v]) continue; /* lazy deletion */
        done[it.v] = 1;
        uint32_t u = it.v;
        for (uint64_t e = off[u]; e < off[u + 1]; e++) {
            uint64_t nd = d[u] + w[e];
            if (nd < d[col[e]]) {
                d[col[e]] = nd;
                heap_push(h, &size, (heap_item){nd, col[e]});
            }
        }
    }
    int overflow = 0;
    for (uint64_t v = 0; v < n; v++) {
        if (d[v] == INF)
            dist[v] = UNREACHED;
        else if (d[v] >= UNREACHED) {
            overflow = 1;
            dist[v] = UNREACHED;
        } else
            dist[v] = (uint32_t)d[v];
    }
    free(d);
    free(done);
    free(h);
    return overflow;
}

/* Shortest-path certificate for weights >= 1, one pass over the edges (Sec. 2.1, Fig. 1:
   the distances SSSP converges to).  dist is a proposed answer: UNREACHED or a value below
   it per vertex.  It holds exactly when
     (a) dist[source] = 0;
     (b) no edge (u, v) with u reached offers v less: dist[u] + w >= dist[v], where an
         unreached v counts as 2^32-1 (a sum that fits must have reached it);
     (c) every reached v other than the source has a tight in-edge, dist[u] + w = dist[v]
         with u reached.
   (b) bounds every distance from below by the true one along any path; (c) with positive
   weights gives each reached vertex a path of exactly its distance.  Returns 0 when all
   hold, else the violated condition (1, 2, 3) with *bad set to the vertex concerned. */
int orc_sssp_check(uint64_t n, const uint64_t *off, const uint32_t *col, const uint32_t *w, uint32_t source,
                   const uint32_t *dist, uint64_t *bad) {
    if (dist[source] != 0) {
        *bad = source;
        return 1;
    }
    unsigned char *tight = (unsigned char *)calloc(n ? n : 1, 1);
    for (uint64_t u = 0; u < n; u++) {
        if (dist[u] == UNREACHED) continue;
        for (uint64_t e = off[u]; e < off[u + 1]; e++) {
            uint32_t v = col[e];
            uint64_t sum = (uint64_t)dist[u] + w[e];
            if (sum < dist[v]) {
                *bad = v;
                free(tight);
                return 2;
            }
            if (sum == dist[v]) tight[v] = 1;
        }
    }
    for (uint64_t v = 0; v < n; v++) {
        if (v != source && dist[v] != UNREACHED && !tight[v]) {
            *bad = v;
            free(tight);
            return 3;
        }
    }
    free(tight);
    return 0;
}

/* Rounds of a fully synchronous push iteration until nothing changes, counting the
   non-empty frontiers processed.  kind 0: SSSP (min of value + w; w may be NULL for
   unit weights); kind 1: min-label propagation with every vertex initially active
   (value[v] = v).  Values in round t+1 are computed only from round-t values. */
uint32_t orc_sync_rounds(uint64_t n, const uint64_t *off, const uint32_t *col, const uint32_t *w, int kind,
                         uint32_t source) {
    uint64_t *cur = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t *nxt = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    unsigned char *act = (unsigned char *)calloc(n ? n : 1, 1);
    unsigned char *nact = (unsigned char *)calloc(n ? n : 1, 1);
    uint64_t nactive = 0;
    for (uint64_t v = 0; v < n; v++) {
        cur[v] = kind == 0 ? ~0ull : v;
        act[v] = kind == 1;
    }
    if (kind == 0) {
        cur[source] = 0;
        act[source] = 1;
    }
    for (uint64_t v = 0; v < n; v++) nactive += act[v];
    uint32_t rounds = 0;
    while (nactive > 0) {
        rounds++;
        memcpy(nxt, cur, n * sizeof(uint64_t));
        memset(nact, 0, n);
        for (uint64_t u = 0; u < n; u++) {
            if (!act[u]) continue;
            for (uint64_t e = off[u]; e < off[u + 1]; e++) {
                uint64_t cand = cur[u] + (kind == 0 && w ? w[e] : (kind == 0 ? 1 : 0));
                uint32_t v = col[e];
                if (cand < nxt[v]) {
                    nxt[v] = cand;
                    nact[v] = 1;
                }
            }
        }
        nactive = 0;
        for (uint64_t v = 0; v < n; v++) nactive += nact[v];
        uint64_t *t = cur; cur = nxt; nxt = t;
        unsigned char *ta = act; act = nact; nact = ta;
    }
    free(cur); free(nxt); free(act); free(nact);
    return rounds;
}

/* ------------------------------------------------------------------- CC */
static uint32_t uf_find(uint32_t *parent, uint32_t x) {
    while (parent[x] != x) {
        parent[x] = parent[parent[x]]; /* path halving */
        x = parent[x];
    }
    return x;
}

/* label[v] = smallest vertex id in v's weakly connected component (edges taken as
   undirected).  Returns the number of components. */
uint64_t orc_cc(uint64_t n, const uint64_t *off, const uint32_t *col, uint32_t *label) {
    uint32_t *parent = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *size = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *minid = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    for (uint64_t v = 0; v < n; v++) {
        parent[v] = (uint32_t)v;
        size[v] = 1;
    }
    for (uint64_t u = 0; u < n; u++)
        for (uint64_t e = off[u]; e < off[u + 1]; e++) {
            uint32_t a = uf_find(parent, (uint32_t)u), b = uf_find(parent, col[e]);
            if (a == b) continue;
            if (size[a] < size[b]) { uint32_t t = a; a = b; b = t; }
            parent[b] = a;
            size[a] += size[b];
        }
    for (uint64_t v = 0; v < n; v++) minid[v] = UNREACHED;
    uint64_t comps = 0;
    for (uint64_t v = 0; v < n; v++) {
        uint32_t r = uf_find(parent, (uint32_t)v);
        if (minid[r] == UNREACHED) { minid[r] = (uint32_t)v; comps++; } /* v ascending: first seen is min */
    }
    for (uint64_t v = 0; v < n; v++) label[v] = minid[uf_find(parent, (uint32_t)v)];
    free(parent); free(size); free(minid);
    return comps;
}

/* ------------------------------------------------------------- PageRank */
/* x_0(v) = 1/n; x_{t+1}(v) = (1-d)/n + d * sum over edges (u,v) of x_t(u)/D_o(u);
   T steps, FP64.  A vertex with no out-edges passes nothing on (its mass leaks). */
void orc_pagerank(uint64_t n, const uint64_t *off, const uint32_t *col, double d, uint32_t T, double *x) {
    double *acc = (double *)malloc((n ? n : 1) * sizeof(double));
    for (uint64_t v = 0; v < n; v++) x[v] = 1.0 / (double)n;
    for (uint32_t t = 0; t < T; t++) {
        for (uint64_t v = 0; v < n; v++) acc[v] = 0.0;
        for (uint64_t u = 0; u < n; u++) {
            uint64_t deg = off[u + 1] - off[u];
            if (deg == 0) continue;
            double share = x[u] / (double)deg;
            for (uint64_t e = off[u]; e < off[u + 1]; e++) acc[col[e]] += share;
        }
        for (uint64_t v = 0; v < n; v++) x[v] = (1.0 - d) / (double)n + d * acc[v];
    }
    free(acc);
}

/* Personalized PageRank from `source`: x_0 = e_s and
       x_{t+1}(v) = (1 - d) [v == s] + d * sum over edges (u, v) of x_t(u) / D_o(u),
   T steps; a vertex without out-edges passes nothing on (its mass leaks), as in
   orc_pagerank. */
void orc_ppr(uint64_t n, const uint64_t *off, const uint32_t *col, uint32_t source, double d, uint32_t T,
             double *x) {
    double *acc = (double *)malloc((n ? n : 1) * sizeof(double));
    for (uint64_t v = 0; v < n; v++) x[v] = v == source ? 1.0 : 0.0;
    for (uint32_t t = 0; t < T; t++) {
        for (uint64_t v = 0; v < n; v++) acc[v] = 0.0;
        for (uint64_t u = 0; u < n; u++) {
            uint64_t deg = off[u + 1] - off[u];
            if (deg == 0 || x[u] == 0.0) continue;
            double share = x[u] / (double)deg;
            for (uint64_t e = off[u]; e < off[u + 1]; e++) acc[col[e]] += share;
        }
        for (uint64_t v = 0; v < n; v++) x[v] = (v == source ? 1.0 - d : 0.0) + d * acc[v];
    }
    free(acc);
}

/* ----------------------------------------------------------- hub sorting */
/* New vertex order of hub sorting (Sec. 6.1).  H(v) is proportional to D_o(v) * D_i(v)
   (the maxima in its denominator are the same for every v), so ranking by the integer
   product ranks by H.  Readings: the hubs are the floor(n * num / den) highest-ranked
   vertices among those with H > 0 (num/den = 8/100), ties to the smaller id; hubs come
   first in decreasing H, then every other vertex in increasing id.  order[i] = the
   original id of new vertex i.  Returns the number of hubs. */
typedef struct {
    unsigned __int128 score;
    uint32_t v;
} orc_scored;

static int orc_by_score(const void *a, const void *b) {
    const orc_scored *x = (const orc_scored *)a, *y = (const orc_scored *)b;
    if (x->score != y->score) return x->score > y->score ? -1 : 1;
    return x->v < y->v ? -1 : (x->v > y->v ? 1 : 0);
}

uint64_t orc_hub_order(uint64_t n, const uint64_t *off, const uint32_t *col, uint32_t num, uint32_t den,
                       uint32_t *order) {
    uint64_t *din = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    for (uint64_t e = 0; e < off[n]; e++) din[col[e]]++;
    orc_scored *sc = (orc_scored *)malloc((n ? n : 1) * sizeof(orc_scored));
    uint64_t pos = 0;
    for (uint64_t v = 0; v < n; v++) {
        unsigned __int128 h = (unsigned __int128)(off[v + 1] - off[v]) * din[v];
        if (h) {
            sc[pos].score = h;
            sc[pos].v = (uint32_t)v;
            pos++;
        }
    }
    qsort(sc, pos, sizeof(orc_scored), orc_by_score);
    uint64_t k = (uint64_t)(((unsigned __int128)n * num) / den);
    if (k > pos) k = pos;
    uint8_t *hub = (uint8_t *)calloc(n ? n : 1, 1);
    for (uint64_t i = 0; i < k; i++) {
        order[i] = sc[i].v;
        hub[sc[i].v] = 1;
    }
    uint64_t i = k;
    for (uint64_t v = 0; v < n; v++)
        if (!hub[v]) order[i++] = (uint32_t)v;
    free(hub);
    free(sc);
    free(din);
    return k;
}

/* ----------------------------------------------------------- partitions */
/* Chunk-based, edge-balanced partitioning into consecutive vertex ranges (Sec. 4).
   Reading: walk vertices in id order; close the current partition before vertex v when
   it already holds at least one edge and adding D_o(v) would take it past `target`
   edges.  A vertex with more than `target` edges therefore ends up alone; zero-degree
   vertices join the partition that is open when they are reached.  Writes the start vertex of each partition
   plus a final n into bounds[0..count]; returns count. */
uint64_t orc_partition(uint64_t n, const uint64_t *off, uint64_t target, uint64_t *bounds) {
    uint64_t count = 0, edges = 0;
    bounds[count++] = 0;
    for (uint64_t v = 0; v < n; v++) {
        uint64_t deg = off[v + 1] - off[v];
        if (edges > 0 && edges + deg > target) {
            bounds[count++] = v;
            edges = 0;
        }
        edges += deg;
    }
    if (n == 0) return 0;
    bounds[count] = n;
    return count;
}

/* Transactions of an m-byte-line engine for a list of len bytes at byte offset start of
   its array (the arrays start on a line boundary): ceil(len/m), plus one when the list's
   misaligned start makes it cross one more line boundary (the footnote to Eq. 3 computes
   it from the list's length and physical start). */
static uint64_t list_tx(uint64_t start, uint64_t len, uint64_t m) {
    uint64_t base = (len + m - 1) / m;
    return base + ((start % m) + len > base * m ? 1 : 0);
}

/* Per-partition activity statistics for one frontier (Sec. 5.1).
   active[v] != 0 marks v active.  A_i is read as the active vertices of P_i that have
   at least one out-edge: an active vertex with no out-edges has nothing to push and
   needs neither an index entry nor a transfer.
     nA[i] = |A_i|
     Ea[i] = sum over A_i of D_o(v)                 (active edges)
     Rq[i] = sum over A_i, over each edge array read, of the list's transactions
   where the neighbour array has 4-byte entries and, with wbytes > 0, a weight array of
   wbytes-byte entries is read beside it (wbytes = 4: the same count twice; wbytes = 1: a
   weight list of D_o(v) bytes at byte offset off(v)).  Eq. 3 counts the requests the
   zero-copy engine issues for the data it reads; each array is read with its own
   requests. */
void orc_partition_stats(uint64_t npart, const uint64_t *bounds, const uint64_t *off, const unsigned char *active,
                         uint32_t wbytes, uint32_t line_bytes, uint64_t *nA, uint64_t *Ea, uint64_t *Rq) {
    for (uint64_t i = 0; i < npart; i++) {
        nA[i] = Ea[i] = Rq[i] = 0;
        for (uint64_t v = bounds[i]; v < bounds[i + 1]; v++) {
            uint64_t deg = off[v + 1] - off[v];
            if (!active[v] || deg == 0) continue;
            nA[i] += 1;
            Ea[i] += deg;
            Rq[i] += list_tx(off[v] * 4, deg * 4, line_bytes);
            if (wbytes) Rq[i] += list_tx(off[v] * wbytes, deg * wbytes, line_bytes);
        }
    }
}

/* The m-byte lines of an array of b-byte entries that the lists of A_i touch, each
   counted once.  The lists lie in vertex order, so a line repeats only as the previous
   list's last line. */
static uint64_t lines_distinct(uint64_t lo, uint64_t hi, const uint64_t *off, const unsigned char *active,
                               uint64_t b, uint64_t m) {
    uint64_t count = 0, last = UINT64_MAX;
    for (uint64_t v = lo; v < hi; v++) {
        if (!active[v] || off[v + 1] == off[v]) continue;
        for (uint64_t line = off[v] * b / m; line <= (off[v + 1] * b - 1) / m; line++)
            if (line != last) {
                count++;
                last = line;
            }
    }
    return count;
}

/* Zero-copy requests counted as distinct lines (a reading for kernels that read a line
   shared by two consecutive active lists once): Rq[i] = the different m-byte lines the
   lists of A_i touch in the neighbour array, plus, with wbytes > 0, those they touch in
   the weight array of wbytes-byte entries. */
void orc_partition_lines_distinct(uint64_t npart, const uint64_t *bounds, const uint64_t *off,
                                  const unsigned char *active, uint32_t wbytes, uint32_t line_bytes, uint64_t *Rq) {
    for (uint64_t i = 0; i < npart; i++) {
        Rq[i] = lines_distinct(bounds[i], bounds[i + 1], off, active, 4, line_bytes);
        if (wbytes) Rq[i] += lines_distinct(bounds[i], bounds[i + 1], off, active, wbytes, line_bytes);
    }
}

/* Exact non-negative rational p/q (q > 0). */
typedef struct {
    u128 p, q;
} rat;
static rat rat_make(u128 p, u128 q) { return (rat){p, q}; }
static rat rat_mul(rat a, rat b) { return (rat){a.p * b.p, a.q * b.q}; }
static rat rat_add(rat a, rat b) { return (rat){a.p * b.q + b.p * a.q, a.q * b.q}; }
static int rat_lt(rat a, rat b) { return a.p * b.q < b.p * a.q; }
static u128 ceil_div(u128 a, u128 b) { return (a + b - 1) / b; }

typedef struct {
    uint32_t line_bytes;            /* m: bytes per outstanding request (128) */
    uint32_t max_outstanding;       /* MR: outstanding requests per TLP window (256) */
    uint32_t d1;                    /* bytes per edge over the edge arrays read */
    uint32_t d2;                    /* bytes per index entry */
    uint32_t alpha_num, alpha_den;  /* 4/5 */
    uint32_t beta_num, beta_den;    /* 2/5 */
    uint32_t gamma_num, gamma_den;  /* 5/8 */
    uint32_t gather_num, gather_den; /* 0/1: link rate / host gather rate (extension, see below) */
    uint32_t zc_tie;                /* 0: a Tiz = Tef tie goes to filter (the prose); 1: to zero-copy */
} orc_cost_params;

/* Engine selection for every partition (Sec. 5.1, Algorithm 1 cost analysis), with
   RTT = 1 (it cancels in every comparison):
     Tef = ceil(E_i * d1 / m / MR)                                        (Eq. 1)
     Tec = ceil((Ea_i * d1 + |A_i| * d2) / m / MR)   -- transfer term only  (Eq. 2)
     Tiz = ceil(Rq_i / MR) * RTTzc,
       RTTzc = gamma + (1 - gamma) * Ea_i / E_i                            (Eq. 3)
   Compaction if Tec < alpha*Tef and Tec < beta*Tiz; otherwise zero-copy if Tiz < Tef;
   otherwise filter.  Readings: a tie between Tiz and Tef goes to filter, as the prose
   states (the listing's branch order would give zero-copy); a partition with no active
   edge is not scheduled (NONE); the first nres partitions are device-resident and
   need no transfer (RESIDENT).  force: 0 = cost model, else every scheduled partition
   gets that engine code.
   Extension beyond the paper (its Eq. 2 compute term, which it leaves to future work):
   with gather = link rate / host gather rate > 0, the host gather of the active edges is
   priced in the same units, Tgc = ceil(Ea_i * d1 * gather / m / MR), and since gathering
   and copying run as a pipeline, compaction costs max(Tec, Tgc).  gather = 0 is the
   paper's rule.
   zc_tie = 1 hands a Tiz = Tef tie to zero-copy, for hosts whose full-line zero-copy reads
   are as fast as explicit copies (the tie then means equal bytes at an equal rate). */
void orc_select(uint64_t npart, const uint64_t *E, const uint64_t *nA, const uint64_t *Ea, const uint64_t *Rq,
                uint64_t nres, const orc_cost_params *cp, int force, unsigned char *p) {
    const u128 L = (u128)cp->line_bytes * cp->max_outstanding;
    const rat alpha = rat_make(cp->alpha_num, cp->alpha_den);
    const rat beta = rat_make(cp->beta_num, cp->beta_den);
    const rat gamma = rat_make(cp->gamma_num, cp->gamma_den);
    const rat one_minus_gamma = rat_make(cp->gamma_den - cp->gamma_num, cp->gamma_den);
    for (uint64_t i = 0; i < npart; i++) {
        if (Ea[i] == 0) { p[i] = ORC_NONE; continue; }
        if (i < nres) { p[i] = ORC_RESIDENT; continue; }
        if (force) { p[i] = (unsigned char)force; continue; }
        rat Tef = rat_make(ceil_div((u128)E[i] * cp->d1, L), 1);
        rat Tec = rat_make(ceil_div((u128)Ea[i] * cp->d1 + (u128)nA[i] * cp->d2, L), 1);
        if (cp->gather_num) {
            rat Tgc = rat_make(ceil_div((u128)Ea[i] * cp->d1 * cp->gather_num, L * cp->gather_den), 1);
            if (rat_lt(Tec, Tgc)) Tec = Tgc;
        }
        rat RTTzc = rat_add(gamma, rat_mul(one_minus_gamma, rat_make(Ea[i], E[i])));
        rat Tiz = rat_mul(rat_make(ceil_div(Rq[i], cp->max_outstanding), 1), RTTzc);
        if (rat_lt(Tec, rat_mul(alpha, Tef)) && rat_lt(Tec, rat_mul(beta, Tiz)))
            p[i] = ORC_COMPACT;
        else if (rat_lt(Tiz, Tef) || (cp->zc_tie && !rat_lt(Tef, Tiz)))
            p[i] = ORC_ZEROCOPY;
        else
            p[i] = ORC_FILTER;
    }
}

/* Task combination (Sec. 5.2, Algorithm 1): runs of adjacent filter partitions form
   tasks of at most k partitions.  Reading: the partition that meets a full task starts
   the next task (the listing as printed would drop it), and runs are broken by any
   partition that is not filter, without creating empty tasks.  A task is also closed
   before a partition that would take its edge count past max_edges (0 = no limit):
   that keeps every task within one staging slot.  Writes task t as partitions
   [first[t], last[t]) and returns the number of tasks. */
uint64_t orc_combine(uint64_t npart, const unsigned char *p, const uint64_t *E, uint32_t k, uint64_t max_edges,
                     uint64_t *first, uint64_t *last) {
    uint64_t ntask = 0, len = 0, edges = 0;
    for (uint64_t i = 0; i < npart; i++) {
        if (p[i] != ORC_FILTER) {
            len = 0;
            continue;
        }
        int fits = len > 0 && len < k && (max_edges == 0 || edges + E[i] <= max_edges);
        if (fits) {
            last[ntask - 1] = i + 1;
            len++;
            edges += E[i];
        } else {
            first[ntask] = i;
            last[ntask] = i + 1;
            ntask++;
            len = 1;
            edges = E[i];
        }
    }
    return ntask;
}

/* The compaction engine's output for the active list vc[0..count): neighbour lists
   packed in list order (Sec. 2.2) and the new index array (Sec. 6.3) as offsets into
   the packed buffer, newoff[0..count]. */
void orc_gather(uint64_t count, const uint32_t *vc, const uint64_t *off, const uint32_t *col, uint32_t *packed,
                uint64_t *newoff) {
    uint64_t pos = 0;
    for (uint64_t j = 0; j < count; j++) {
        newoff[j] = pos;
        for (uint64_t e = off[vc[j]]; e < off[vc[j] + 1]; e++) packed[pos++] = col[e];
    }
    newoff[count] = pos;
}
