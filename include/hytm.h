/*
 * hytm.h -- C ABI of libhytm.so: hybrid transfer management for vertex-centric graph
 * traversal on one AMD Instinct MI355X (gfx950).
 *
 * Method: "HyTGraph: GPU-Accelerated Graph Processing with Hybrid Transfer Management"
 * (Wang, Ai, Zhang, Chen, Yu; arXiv 2208.14935).
 *
 * Problem statement followed (Sec. 1, Sec. 2.1, Sec. 4): a CSR graph whose
 * vertex-associated data (values, neighbour index, activity) lives in GPU memory while
 * the edge-associated arrays (neighbours, weights) live in host memory; a push-style
 * vertex-centric iteration processes the active vertices until none remain; each
 * iteration a per-partition cost model (Sec. 5.1, Eq. 1-3) picks how a partition's
 * active edges reach the GPU:
 *   FILTER   -- explicit copy of the whole partition (Sec. 2.2 "ExpTM-filter");
 *   COMPACT  -- host threads gather only the active neighbour lists, which are then
 *               copied (Sec. 2.2 "ExpTM-compaction", Sec. 6.3);
 *   ZEROCOPY -- kernels read the mapped pinned host arrays directly (Sec. 2.3).
 * Consecutive FILTER partitions are combined into larger tasks (Sec. 5.2) and the
 * engines run concurrently on several streams (Sec. 6.2).  A device-memory budget caps
 * the bytes of edge data held on the GPU; partitions that fit inside it are kept
 * resident (RESIDENT, no transfer), which is this library's addition to the method.
 *
 * Conventions for every call:
 *  - Return value: hytm_status, HYTM_OK (0) on success.  On failure a thread-local
 *    message is available from hytm_last_error() until the next call on that thread.
 *  - On any error other than HYTM_E_DEVICE, caller-owned output buffers are untouched.
 *  - Host pointers are plain CPU addresses; the library never keeps a caller pointer
 *    past the call that received it.
 *  - A graph handle is not reentrant: calls on one handle must not overlap.  Separate
 *    handles may be used from separate threads.
 */
#ifndef HYTM_H
#define HYTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hytm_graph hytm_graph; /* opaque, owned by the library */

typedef enum {
    HYTM_OK = 0,
    HYTM_E_INVAL = 1,       /* null pointer, malformed CSR, missing weights, bad parameter */
    HYTM_E_RANGE = 2,       /* n >= 2^32-1, source >= n, distance overflow */
    HYTM_E_NOMEM = 3,       /* host or device allocation failed */
    HYTM_E_BUDGET = 4,      /* a forced FILTER/COMPACT run whose staging does not fit the budget */
    HYTM_E_DEVICE = 5,      /* a HIP runtime error; the message carries hipGetErrorString */
    HYTM_E_STATE = 6,       /* call not valid in the handle's current state */
    HYTM_E_UNSUPPORTED = 7  /* request the library does not implement */
} hytm_status;

/* Algorithms (Sec. 7.1).  Outputs are one 4-byte value per vertex:
   BFS: uint32 hop level; SSSP: uint32 distance; CC: uint32 label = smallest vertex id
   of the component; PAGERANK: float rank.  Unreached vertices hold 0xFFFFFFFF.
   PPR: personalized PageRank from a source s, float: the PageRank step with all of the
   restart mass (1 - pr_damping) at s, from x_0 = e_s, ppr_iterations synchronous steps;
   mass that reaches a vertex without out-edges leaks, as in PAGERANK.  Values and shares
   are FP32; each step's sums are accumulated in FP64 and rounded once.
   PAGERANK_DELTA: PageRank to convergence by delta accumulation with delta-driven
   partition priority (Sec. 6.1), float: x = 0 and delta = (1 - d) / n at the start; each
   iteration folds the pushed deltas in, schedules the partitions whose delta sum is at
   least the mean over partitions, moves every scheduled vertex's delta into x and pushes
   d * delta / D_o(v) along its out-edges; with `reprocess`, the scheduled partitions get a
   second such pass in the same iteration.  It stops when the total pending delta is at
   most dpr_epsilon (or after dpr_max_iterations) and returns x + delta, within
   d / (1 - d) * (final total delta) in L1 of the fixed point that PAGERANK's iteration
   approaches; hytm_run_stats.residual reports that total. */
typedef enum {
    HYTM_BFS = 0, HYTM_SSSP = 1, HYTM_CC = 2, HYTM_PAGERANK = 3, HYTM_PPR = 4, HYTM_PAGERANK_DELTA = 5
} hytm_algo;

/* Transfer policy for partitions that are not resident.  HYBRID applies the cost
   model of Sec. 5.1; the others force one engine for every scheduled partition. */
typedef enum {
    HYTM_MODE_HYBRID = 0,
    HYTM_MODE_FILTER = 1,
    HYTM_MODE_COMPACT = 2,
    HYTM_MODE_ZEROCOPY = 3
} hytm_mode;

/* Per-partition engine codes, as written to hytm_run_stats.mode_trace. */
enum { HYTM_P_NONE = 0, HYTM_P_RESIDENT = 1, HYTM_P_FILTER = 2, HYTM_P_ZEROCOPY = 3, HYTM_P_COMPACT = 4 };

/* hytm_graph_create flags */
enum {
    HYTM_GRAPH_SYMMETRIC = 1u << 1, /* caller asserts (u,v) in E implies (v,u) in E; needed by HYTM_CC */
    HYTM_GRAPH_SKIP_COL_CHECK = 1u << 2, /* skip the O(m) check that every col[e] < n */
    /* hub sorting (Sec. 6.1): relabel the graph once at creation so that its hubs -- the
       top 8% of vertices by H(v) = D_o(v) D_i(v) / (D_omax D_imax) -- come first, highest
       first, the other vertices keeping their natural order.  Sources and results stay in
       the caller's ids; partitions, hytm_partition_bounds and mode traces refer to the
       relabelled order.  Implies the col check. */
    HYTM_GRAPH_HUB_SORT = 1u << 3,
    /* keep weights in their own array.  By default, when ceil(log2 n) bits of neighbour id
       and the bits of (max weight - min weight) fit one 32-bit word, the library stores
       each edge as one word (neighbour low, weight - min above), so SSSP moves 4 bytes per
       edge instead of 8; results are the same either way. */
    HYTM_GRAPH_NO_PACK = 1u << 4,
    /* Weights kept apart from the neighbour words are stored as one byte each (w - min w) when
       max w - min w <= 255, so SSSP reads 5 bytes per edge instead of 8 (d1 = 5 in Eq. 1-2);
       this flag keeps them as 4-byte words.  Results are the same either way. */
    HYTM_GRAPH_WIDE_WEIGHTS = 1u << 5
};

/* Tunables.  Defaults (hytm_default_params) are the constants the paper states:
   m = 128-byte requests and MR = 256 outstanding requests per TLP window (Sec. 5.1,
   Eq. 1), alpha = 0.8 and beta = 0.4 (Sec. 5.1 selection rule), gamma = 0.625 (the
   zero-copy round-trip damping after Eq. 3), k = 4 partitions per combined filter task
   (Sec. 5.2), index entries of 4 bytes (d2 of Eq. 2), and 32768 edges per partition. */
typedef struct {
    uint32_t struct_size;       /* sizeof(hytm_params) */
    hytm_mode mode;             /* HYTM_MODE_HYBRID */
    uint32_t partition_edges;   /* 32768: target edges per partition (Sec. 4 chunking) */
    uint32_t combine_k;         /* 4: max partitions per filter task (Sec. 5.2) */
    uint32_t alpha_num, alpha_den; /* 4, 5 */
    uint32_t beta_num, beta_den;   /* 2, 5 */
    uint32_t gamma_num, gamma_den; /* 5, 8 */
    uint32_t line_bytes;        /* 128: m, a power of two >= 4 */
    uint32_t max_outstanding;   /* 256: MR */
    uint32_t index_bytes;       /* 4: d2 */
    uint32_t pr_iterations;     /* 20 */
    double pr_damping;          /* 0.85 */
    uint32_t streams;           /* 4: staging slots of the filter pipeline (>= 2) */
    uint32_t gather_threads;    /* 0 = automatic: host threads of the compaction engine */
    uint64_t compact_chunk_edges; /* 0 = automatic: edges per compaction chunk */
    uint32_t filter_engine;     /* HYTM_FILTER_STREAM (default) or HYTM_FILTER_COPY, see below */
    uint32_t ppr_iterations;    /* 10: steps of HYTM_PPR (restart mass 1 - pr_damping) */
    uint32_t reprocess;         /* 0: off.  1: every iteration makes a second pass over the partitions
                                   it loaded, from the vertices the first pass improved (Sec. 6.1);
                                   BFS, SSSP, CC and PAGERANK_DELTA, single-source runs only.  The
                                   results are unchanged (BFS relaxes levels instead of marking
                                   first visits); iteration counts drop.  2: the second pass covers
                                   only resident and zero-copy partitions, whose lists cost no host
                                   transfer or only the improved lists' lines (BFS/SSSP/CC). */
    uint32_t dpr_max_iterations; /* 10000: cap on PAGERANK_DELTA iterations */
    double dpr_epsilon;         /* 1e-7: PAGERANK_DELTA stops when the pending delta sums to this */
    uint32_t compact_gather_num, compact_gather_den; /* 0/1: off.  Otherwise the ratio of the
                                   host link's rate to the host gather's rate: compaction is then
                                   priced max(Tec, ceil(Ea * d1 * ratio / (m * MR))), the gather of
                                   Eq. 2 that the paper leaves out (an extension; hytm_link_probe
                                   measures both rates). */
    uint32_t rq_distinct_lines; /* 0: Rq of Eq. 3 counts each active list's lines (its footnote's
                                   per-vertex requests).  1: Rq counts the different m-byte lines the
                                   active lists of a partition touch -- what the zero-copy kernel
                                   reads, since it loads a line two consecutive lists share once.
                                   Either way each edge array read counts its own lines: with byte
                                   weights a list of D edges spans D bytes of the weight array. */
    uint32_t zc_tie;            /* 0: a Tiz = Tef tie selects filter, as the paper's prose says.  1: it
                                   selects zero-copy -- for hosts where full-line zero-copy reads run
                                   at the copy engine's rate (hytm_link_probe), so equal bytes cost
                                   equal time and zero-copy skips the whole-partition pass.  2:
                                   automatic -- zero-copy for HYTM_PAGERANK runs without propagation
                                   blocking (their pushes fill the GPU, where zero-copy's passes are
                                   the faster), filter otherwise (a blocked run's streamed pushes get a
                                   limited grid, in which the streaming filter reads faster; for BFS,
                                   SSSP and CC ties to filter measured as fast or faster).
                                   hytm_select_engines treats 2 as 0. */
    uint32_t pr_blocking;       /* Propagation blocking of HYTM_PAGERANK's adds over resident partitions:
                                   their pushes write one contribution per edge, and each run of resident
                                   partitions with at most max(n, 2^20) edges has its (destination,
                                   contribution) pairs bucketed by destination on the GPU and summed in
                                   LDS, instead of adding with random float atomics, whose fixed rate
                                   (about 20 G/s) falls below what HBM feeds from the resident cache.
                                   Streamed partitions keep their atomic adds (the host link delivers
                                   fewer edges per second than the atomics take).  1 (default): when at
                                   least 3/8 of the edges are resident; 2: whenever some are; 0: never.
                                   Applies to single PageRank runs with n <= 2^28 in the hybrid, filter
                                   (streaming engine) or zero-copy modes; the result is the same sum in
                                   another order.  Needs 16 bytes per pair of a piece of device memory
                                   outside the edge budget (16 bytes per vertex at the default piece). */
    uint64_t pr_block_pairs;    /* 0 = automatic (max(n, 2^20), at most the resident edges): pairs per
                                   piece of pr_blocking; a smaller value (never below the largest
                                   partition) cuts more pieces, e.g. to exercise the piece pipeline on
                                   small graphs. */
    uint32_t sssp_delta;        /* 0 (default): HYTM_SSSP pushes every improved vertex in the next
                                   iteration (the paper's synchronous push).  Otherwise improved vertices
                                   whose new distance is at or above a bound wait in a far set; the bound
                                   starts at sssp_delta and, when the frontier empties, rises to the
                                   smallest multiple of sssp_delta above the smallest waiting distance,
                                   whose vertices below it form the next frontier (the buckets of
                                   delta-stepping, Meyer and Sanders, J. Algorithms 2003).  Distances are
                                   the same; fewer edges are pushed again, iterations may exceed the
                                   synchronous count.  Single-source runs only; batched SSSP ignores it.
                                   Needs n/8 bytes of device memory outside the edge budget. */
} hytm_params;

/* How a FILTER task moves its whole partition range to the GPU.  Both transfer every
   byte of the task's partitions, which is what Eq. 1 prices.
   STREAM: one kernel per iteration reads every 128-byte line of every filter task from
           the mapped pinned arrays, in order, and pushes the edges of active vertices;
           no staging memory, no per-task host calls.
   COPY:   per task, hipMemcpyAsync into a ring of `streams` device staging slots, then
           a push kernel over the slot (the explicit-copy form of Sec. 2.2). */
enum { HYTM_FILTER_STREAM = 0, HYTM_FILTER_COPY = 1 };

/* Per-iteration record (optional, see hytm_run_stats.iters). */
typedef struct {
    uint32_t parts[5];          /* partitions per engine code */
    uint32_t filter_tasks;      /* combined filter tasks issued */
    uint64_t active_vertices;   /* active vertices with at least one out-edge */
    uint64_t active_edges;      /* their out-edges (edges pushed) */
    uint64_t bytes_filter;      /* host-to-device bytes moved by filter copies */
    uint64_t bytes_compact;     /* host-to-device bytes moved by compaction copies */
    uint64_t zc_lines;          /* 128-byte lines read by the zero-copy kernel, per edge array */
    double ms;                  /* host wall time of the iteration */
} hytm_iter_stats;

/* Run statistics (optional).  Zero it, set struct_size, and optionally point iters /
   mode_trace at caller buffers; the library fills the rest. */
typedef struct {
    uint32_t struct_size;       /* sizeof(hytm_run_stats) */
    uint32_t iterations;
    uint32_t npart;             /* partitions of the graph */
    uint32_t nres;              /* resident partitions (a prefix 0..nres-1) */
    uint64_t part_iters[5];     /* partition-iterations per engine code */
    uint64_t active_vertices;   /* sum over iterations */
    uint64_t active_edges;      /* sum over iterations: edges pushed */
    uint64_t bytes_filter;      /* H2D bytes of filter copies */
    uint64_t bytes_compact;     /* H2D bytes of compaction copies */
    uint64_t zc_lines;          /* 128-byte line requests of the zero-copy kernel (one per line of each
                                   active vertex's list), per edge array: Rq of Eq. 3 at m = 128 */
    uint64_t bytes_zerocopy;    /* zc_lines_distinct x 32 edges x d1 bytes per edge: what the zero-copy
                                   kernel moves over the link */
    uint64_t bytes_d2h;         /* device-to-host bytes of selections and active lists */
    uint64_t bytes_resident_fill; /* H2D bytes copied into the resident cache this run */
    uint64_t filter_tasks;
    uint64_t compact_chunks;
    double ms_total;            /* first kernel to values in the caller's buffer */
    double ms_fill;             /* resident-cache fill inside ms_total */
    double ms_select;           /* device time of stats + selection + active lists + their D2H
                                   (HIP events around them; excludes waiting for earlier pushes) */
    hytm_iter_stats *iters;     /* caller buffer of iters_cap records, or NULL */
    uint32_t iters_cap;
    uint32_t iters_written;
    uint8_t *mode_trace;        /* caller buffer: iteration t's engine codes at t*npart, or NULL */
    uint64_t mode_trace_cap;    /* bytes */
    /* Per-kernel timing.  Input: set time_kernels = 1 to bracket every launch with HIP
       events on the stream it runs on (adds a little host work per launch).  Output,
       indexed by HYTM_K_*: summed event time, launches, and items processed (edges for
       the edge kernels, 128-byte lines for the zero-copy kernel, vertices otherwise). */
    uint32_t time_kernels;
    uint32_t reserved0;
    double kernel_ms[9];
    uint64_t kernel_launches[9];
    uint64_t kernel_items[9];
    double residual;            /* PAGERANK_DELTA: total pending delta at the end (else 0) */
    uint64_t zc_lines_distinct; /* different lines among zc_lines: a line shared by two consecutive
                                   active vertices counts once */
} hytm_run_stats;

/* Kernel classes of hytm_run_stats.kernel_* */
enum {
    HYTM_K_STATS = 0,    /* per-partition statistics + engine selection */
    HYTM_K_SCAN = 1,     /* per-engine prefix sums over partitions */
    HYTM_K_LISTS = 2,    /* active-list compaction */
    HYTM_K_PUSH_RES = 3, /* push over resident partitions */
    HYTM_K_PUSH_F = 4,   /* push over a filter task's staging slot */
    HYTM_K_PUSH_ZC = 5,  /* zero-copy push (mapped host reads) */
    HYTM_K_PUSH_C = 6,   /* push over a compaction chunk */
    HYTM_K_OTHER = 7,    /* init, frontier clear, PageRank prepare/apply */
    HYTM_K_PR_BLOCK = 8  /* PageRank pair bucketing and summing, per piece (items = pairs) */
};

/* Host-link and HBM probe (calibration of the cost constants, Sec. 3.2 / Sec. 5.1). */
typedef struct {
    double h2d_copy_gbps;       /* hipMemcpyAsync pinned host -> device, best of 3 */
    double d2h_copy_gbps;       /* device -> pinned host, best of 3 */
    double zc_read_gbps[4];     /* kernel reads of mapped pinned memory, useful bytes/s, when each
                                   128-byte line contributes 32, 64, 128 bytes, or whole 256-byte runs */
    double hbm_copy_gbps;       /* device-to-device copy kernel, (read + write) bytes / s */
    double host_gather_gbps;    /* host threads (as many as the compaction engine uses by default)
                                   gathering 64-byte runs from random places of pinned memory
                                   into a pinned buffer: bytes gathered / s */
} hytm_link_probe_result;

/* Measure the host link and HBM on `hip_device` with `bytes` per transfer (>= 1 MiB).
   Allocates and frees its own pinned and device buffers. */
hytm_status hytm_link_probe(int hip_device, uint64_t bytes, hytm_link_probe_result *out);

/* Static facts about a graph handle. */
typedef struct {
    uint64_t n, m;
    uint32_t npart;             /* partitions for the current partition_edges */
    uint32_t max_partition_edges;
    int hip_device;
    uint32_t flags;
    uint64_t hubs;              /* vertices moved to the front by HYTM_GRAPH_HUB_SORT (else 0) */
    uint32_t packed_weights;    /* 1 when weights share the neighbour words (see HYTM_GRAPH_NO_PACK) */
    uint32_t weight_bytes;      /* bytes per weight kept apart from the neighbour words: 1 (byte weights,
                                   see HYTM_GRAPH_WIDE_WEIGHTS), 4, or 0 (no weights, or packed) */
} hytm_graph_info;

/* Fill *p with the paper's defaults listed above. */
void hytm_default_params(hytm_params *p);

/* Create a graph from a CSR (Sec. 4 layout).
   n, m      : vertex and edge counts; n < 2^32-1 (ids are uint32, 0xFFFFFFFF is reserved).
   offsets   : host array of n+1 entries, each offset_bytes (4 or 8) wide, non-decreasing,
               offsets[0] = 0 and offsets[n] = m.  Copied to the device (as uint64).
   col       : host array of m neighbour ids (< n).  Copied into library-owned pinned,
               device-mapped host memory (the edge data stays in host memory).
   weights   : host array of m uint32 edge weights, or NULL.  Copied like col.
   flags     : HYTM_GRAPH_* bits.
   hip_device: HIP device ordinal the handle binds to.
   out       : receives the handle.
   Errors: E_INVAL (null pointers, malformed offsets, col >= n), E_RANGE (n too large),
   E_NOMEM, E_DEVICE (no such device / HIP failure).  Partitioning uses the default
   partition_edges until hytm_set_params changes it. */
hytm_status hytm_graph_create(uint64_t n, uint64_t m, const void *offsets, uint32_t offset_bytes,
                              const uint32_t *col, const uint32_t *weights, uint32_t flags, int hip_device,
                              hytm_graph **out);

/* The new vertex order hub sorting gives a CSR (host computation, no device needed):
   order_out[i] = original id of new vertex i (n entries), *hubs_out = the number of hubs,
   which come first.  Ranking by D_o(v) D_i(v) is ranking by H(v); the hubs are the
   floor(0.08 n) highest-ranked vertices with H(v) > 0, ties to the smaller id.  Errors:
   E_INVAL (null pointers, malformed offsets, col >= n), E_RANGE (n too large). */
hytm_status hytm_hub_order(uint64_t n, uint64_t m, const void *offsets, uint32_t offset_bytes, const uint32_t *col,
                           uint32_t *order_out, uint64_t *hubs_out);

/* Declare g a disjoint union of `count` graphs, graph i holding vertices
   [vertex_bounds[i], vertex_bounds[i+1]) (caller ids; count + 1 entries from 0 to n), so
   that one traversal serves them all: every iteration's kernels balance edges across the
   graphs, and a graph that has converged simply has no active vertices.  PageRank (and
   PAGERANK_DELTA) then normalize by each graph's own vertex count, giving every graph
   the values it would get alone; BFS/SSSP/CC need nothing more (CC labels are the
   smallest vertex id in the component, in union ids).  count = 0 undoes it.  Errors:
   E_INVAL (bounds not increasing from 0 to n, an edge leaving its graph). */
hytm_status hytm_graph_set_parts(hytm_graph *g, uint32_t count, const uint64_t *vertex_bounds);

/* Device budget for edge-associated data: resident partitions + filter staging +
   compaction buffers.  UINT64_MAX (the default) = uncapped: every partition resident.
   Vertex arrays are outside the budget, as in the paper's placement (Sec. 1).  Takes
   effect at the next run. */
hytm_status hytm_set_device_budget(hytm_graph *g, uint64_t edge_bytes);

/* Bytes of the budget that the engines' buffers take for `algo` under the current
   parameters: filter = `streams` staging slots, each holding the largest combined task
   (max(combine_k * partition_edges, largest partition) edges); compaction = two chunk
   buffers of compact_chunk_edges edges (default max(slot, 2^20)); times 4 bytes per edge
   array read (two arrays for SSSP).  Hybrid needs both; a forced mode needs its own;
   zero-copy needs none.  The rest of the budget holds resident partitions; on a graph with
   separate weights the rest is taken after the larger of the one- and two-array needs, so
   that one device region holds either layout (neighbours only; a shorter neighbour prefix
   and its weights) and a switch between BFS/CC/PageRank and SSSP copies only the part of
   the region that differs.  In hybrid
   mode an engine whose buffers do not fit is left out of the choice; a forced
   FILTER/COMPACT run whose buffers do not fit fails with E_BUDGET. */
hytm_status hytm_staging_bytes(const hytm_graph *g, hytm_algo algo, uint64_t *bytes);

/* Replace the tunables (NULL = defaults).  E_INVAL on a bad field.  Re-partitions the
   graph when partition_edges changes. */
hytm_status hytm_set_params(hytm_graph *g, const hytm_params *p);
hytm_status hytm_get_params(const hytm_graph *g, hytm_params *p);

hytm_status hytm_graph_info_get(const hytm_graph *g, hytm_graph_info *info);

/* Partition start vertices plus a final n: bounds[0..npart] (caller buffer of
   info.npart + 1 entries). */
hytm_status hytm_partition_bounds(const hytm_graph *g, uint64_t *bounds, uint64_t cap);

/* Run one algorithm to convergence: the push iteration of Sec. 2.1 (Fig. 1), repeated
   until the frontier is empty, with each iteration's transfers chosen per partition by
   Sec. 5.1 (PageRank: pr_iterations synchronous steps, Sec. 7.1).
   source     : start vertex for BFS/SSSP (ignored by CC and PageRank); E_RANGE if >= n.
   values_out : host buffer of n 4-byte values (see hytm_algo).
   iterations_out : number of non-empty frontiers processed (NULL ok).
   stats      : NULL or a hytm_run_stats to fill.
   hip_stream : hipStream_t to order the run after (NULL = the null stream); the call
                returns only once values_out is written.
   Errors: E_INVAL (SSSP without weights, CC without HYTM_GRAPH_SYMMETRIC), E_RANGE
   (source; SSSP: some shortest distance does not fit below 2^32-1 -- a longer path whose
   sum would not fit is no error when a shorter one does), E_BUDGET, E_NOMEM, E_DEVICE. */
hytm_status hytm_run(hytm_graph *g, hytm_algo algo, uint32_t source, void *values_out, uint32_t *iterations_out,
                     hytm_run_stats *stats, void *hip_stream);

/* Batched BFS, SSSP or PPR from up to 64 sources in one traversal.  Each vertex carries a
   64-bit mask of the sources (lanes) active at it and one uint32 value per lane; a vertex
   is active when any lane is, so the cost model (Sec. 5.1) runs on the union frontier and
   every edge moved over the host link serves all lanes at once.  Lane l's values equal
   those of hytm_run from sources[l].
   sources        : host array of nsources vertex ids (1..64 entries; repeats allowed).
   values_out     : host buffer of nsources x n uint32, row l = results of sources[l].
   iterations_out : NULL or nsources counts: the non-empty frontiers of each lane.
   values_out is float for PPR (row l = x from sources[l]).
   Errors as hytm_run; E_INVAL also for CC/PageRank or nsources outside 1..64.  Device
   memory for the lanes (n x L x 4 bytes of values, 12 for PPR, with L the power of two
   >= nsources, plus three n x 8-byte masks) is vertex data, outside the edge budget. */
hytm_status hytm_run_batch(hytm_graph *g, hytm_algo algo, const uint32_t *sources, uint32_t nsources,
                           void *values_out, uint32_t *iterations_out, hytm_run_stats *stats, void *hip_stream);

/* Evaluate the engine selection of Sec. 5.1 (Eq. 1-3, alpha/beta rule) on the GPU for
   caller-supplied per-partition statistics, with the handle's parameters.
   npart      : partitions; E, nA, Ea, Rq: host arrays of npart uint64 (edges, active
                vertices, active edges, zero-copy requests at m-byte lines);
   nres       : partitions [0, nres) are resident;
   edge_arrays: 1 (neighbours only) or 2 (neighbours and weights) -> d1 = 4, or 4 + the
                graph's bytes per weight (8, or 5 with byte weights, see HYTM_GRAPH_WIDE_WEIGHTS);
   p_out      : host array of npart engine codes (HYTM_P_*).  Used to test the device
                selection against a reference on arbitrary inputs. */
hytm_status hytm_select_engines(hytm_graph *g, uint64_t npart, const uint64_t *E, const uint64_t *nA,
                                const uint64_t *Ea, const uint64_t *Rq, uint64_t nres, uint32_t edge_arrays,
                                uint8_t *p_out);

/* The same selection as hytm_select_engines, for callers that cannot allocate device
   memory (code under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): the statistics and engine codes pass through a static device array that
   the library holds on each device for the life of the process, so this call makes no
   hipMalloc, hipFree or other allocation.  Arguments as hytm_select_engines, plus
   hip_stream : the HIP stream the copies and the kernel run on (NULL = the null stream);
                the call returns after that stream has finished them.
   Limit: npart <= 262144 (HYTM_E_RANGE above it); the array takes 8.65 MB per device.
   Calls that overlap on one device share that array and race: callers serialize them. */
hytm_status hytm_select_engines_static(hytm_graph *g, uint64_t npart, const uint64_t *E, const uint64_t *nA,
                                       const uint64_t *Ea, const uint64_t *Rq, uint64_t nres, uint32_t edge_arrays,
                                       uint8_t *p_out, void *hip_stream);

/* Pinned host memory for result buffers: a values_out buffer from here is written by DMA
   directly, without the staging copy an ordinary (pageable) buffer needs.  hip_device
   selects the device the allocation is registered with.  hytm_host_free(NULL) is a no-op. */
hytm_status hytm_host_alloc(int hip_device, uint64_t bytes, void **out);
hytm_status hytm_host_free(void *p);

/* ---------------------------------------------------------------- serving
   A query server over one graph: BFS, SSSP and PPR queries submitted from any thread
   join free lanes of a per-algorithm lane group between iterations (continuous
   batching) and leave it as soon as their own traversal ends, so a query never waits
   for the rest of its batch.  One worker thread steps every group that holds queries,
   one iteration at a time, through the same engines as hytm_run_batch: the cost model
   runs on each group's union frontier, so an edge moved over the host link serves every
   query in the group.  Results equal those of hytm_run for the same query.
   Lane state lives in device memory outside the edge budget; the lanes of each group
   are fixed when the server opens, and the server refuses (E_BUDGET) a configuration
   whose lane state exceeds state_budget.  A query waits in the queue until a lane of its
   group is free.  While a server is open, every other call on its graph except
   hytm_graph_info_get and hytm_get_params returns E_STATE. */
typedef struct hytm_server hytm_server;

typedef struct {
    uint32_t struct_size;      /* sizeof(hytm_server_config) */
    uint32_t lanes[3];         /* lanes of the BFS, SSSP and PPR groups: 0 (no group) or 1..64 */
    uint64_t state_budget;     /* device bytes for lane state; 0 = no limit */
    uint64_t max_pending;      /* queue bound; submit returns E_STATE when full (0 = no bound) */
} hytm_server_config;

typedef struct {
    hytm_status status;        /* HYTM_OK, or E_RANGE (SSSP overflow), E_DEVICE ... */
    uint32_t iterations;       /* non-empty frontiers of this query (PPR: ppr_iterations) */
    double queue_ms;           /* submit -> admitted into a lane */
    double run_ms;             /* admitted -> values written */
    double total_ms;           /* submit -> values written */
} hytm_query_result;

/* Device bytes of lane state for `lanes` lanes of `algo` (BFS/SSSP/PPR) on graph g. */
hytm_status hytm_server_state_bytes(const hytm_graph *g, hytm_algo algo, uint32_t lanes, uint64_t *bytes);

/* Open a server on g (the graph's parameters and budget apply; set them before).
   The edge budget is planned once for the weighted arrays when an SSSP group exists. */
hytm_status hytm_server_open(hytm_graph *g, const hytm_server_config *cfg, hytm_server **out);

/* Queue a query.  values_out: caller buffer of n 4-byte values (float for PPR) that must
   stay valid until hytm_server_wait returns for the ticket; a pinned buffer
   (hytm_host_alloc) is written by DMA directly.  E_INVAL if the algorithm has no group
   or no weights (SSSP); E_RANGE if source >= n. */
hytm_status hytm_server_submit(hytm_server *s, hytm_algo algo, uint32_t source, void *values_out,
                               uint64_t *ticket);

/* Block until the query is done (timeout_ms < 0: no limit); then fill *result (NULL ok)
   and return its status.  E_STATE if the ticket is unknown or already waited for, or the
   timeout passed (the ticket stays valid). */
hytm_status hytm_server_wait(hytm_server *s, uint64_t ticket, double timeout_ms, hytm_query_result *result);

/* Finish every queued query, stop the worker, free the lane state and release the graph.
   Tickets not waited for are dropped.  Returns the error that stopped the worker, if a
   step failed (every query then failed with it).  NULL is accepted.  The handle is freed:
   no other thread may be inside, or later enter, hytm_server_submit / hytm_server_wait on
   it (submit and wait from several threads are otherwise safe). */
hytm_status hytm_server_close(hytm_server *s);

/* Free everything the handle owns.  NULL is accepted; E_STATE while a query server is
   open on the graph. */
hytm_status hytm_graph_destroy(hytm_graph *g);

/* Thread-local message for the last failed call on this thread ("" if none). */
const char *hytm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HYTM_H */
