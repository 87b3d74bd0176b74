// Device kernels of the hybrid-transfer traversal and their host-side launchers.
// Every launcher is asynchronous on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace hytm {

// Engine codes per partition (same values as HYTM_P_* in hytm.h).
enum : uint8_t { P_NONE = 0, P_RES = 1, P_FILTER = 2, P_ZC = 3, P_COMPACT = 4 };
// Active lists are laid out in segments ordered RESIDENT, FILTER, ZEROCOPY, COMPACT
// (segment index = engine code - 1); COMPACT is last so that the work prefix of its
// final entry is the grand total.
constexpr int NSEG = 4;
constexpr int SEG_R = 0, SEG_F = 1, SEG_Z = 2, SEG_C = 3;

// ALGO_MBFS / ALGO_MSSSP: up to 64 sources at once, one bit / value lane per source.
// ALGO_MPPR: personalized PageRank, one value lane per source.
// ALGO_BFS_RELAX: BFS by level relaxation (lvl[v] = min(lvl[v], lvl[u] + 1)), exact under
// the asynchronous reprocessing that first-visit marking would get wrong.
enum Algo : int {
    ALGO_BFS = 0, ALGO_SSSP = 1, ALGO_CC = 2, ALGO_PR = 3, ALGO_MBFS = 4, ALGO_MSSSP = 5, ALGO_MPPR = 6,
    ALGO_BFS_RELAX = 7
};
constexpr uint32_t MAX_LANES = 64;

// Sources of a batched run, passed by value to the init kernel.
struct LaneSources {
    uint32_t src[MAX_LANES];
    uint32_t count;
};
// A set of lanes with one source and one level base each (lane admission / extraction).
struct LaneSet {
    uint64_t mask;              // lanes taking part
    uint32_t src[MAX_LANES];    // source vertex of each lane in mask
    uint32_t base[MAX_LANES];   // BFS: iteration at which the lane joined (level offset)
};

// Zero-copy kernel line: 32 four-byte elements = 128 bytes.
constexpr uint32_t ZC_LINE_SHIFT = 5;

// Inputs of the engine selection (Sec. 5.1), all integers.
struct SelParams {
    uint64_t L;           // m * MR: bytes carried by one saturated TLP window
    uint32_t MR;          // outstanding requests per window
    uint32_t d1, d2;      // bytes per edge (over the arrays read), bytes per index entry
    uint32_t an, ad;      // alpha = an / ad
    uint32_t bn, bd;      // beta  = bn / bd
    uint32_t gn, gd;      // gamma = gn / gd
    uint32_t cost_shift;  // log2(m / 4): elements per m-byte request line
    uint32_t wbytes;      // bytes per entry of the weight array read beside the neighbours (0: none, 1 or 4)
    uint32_t force;       // 0: cost model; else the engine code for every scheduled partition
    uint32_t nres;        // partitions [0, nres) are resident
    uint32_t allow_filter, allow_compact; // engines whose staging fits the budget
    uint32_t gn_c, gd_c;  // host gather cost: link rate / gather rate = gn_c / gd_c (0 = off)
    uint32_t rq_distinct; // zero-copy requests: 0 = per vertex (Eq. 3), 1 = distinct lines touched
    uint32_t zc_tie;      // 1: a Tiz = Tef tie selects zero-copy instead of filter
};

// Written by the scan kernel, copied to the host every iteration.
struct Header {
    uint32_t seg_parts[NSEG];
    uint32_t seg_list_start[NSEG];
    uint32_t seg_list_count[NSEG];
    uint64_t seg_work_start[NSEG];
    uint64_t seg_work_total[NSEG];
    uint64_t seg_edges[NSEG];
    uint64_t seg_cost_lines[NSEG];
    uint64_t total_active;   // list entries (active vertices with out-edges)
    uint64_t frontier;       // all active vertices, including those without out-edges
};

// Edge word layout.  shift < 32: neighbour and weight share one word, neighbour in the low
// `shift` bits, weight - wmin above them (the weight array is not read); shift = 32: the
// word is the neighbour and weights, if any, come from their own array.
struct Pack {
    uint32_t mask;    // neighbour bits
    uint32_t shift;   // weight position, 32 = not packed
    uint32_t wmin;    // smallest weight, added back
    uint32_t wbytes;  // weights kept apart: 4 = one uint32 each, 1 = one byte each holding w - wmin
};
// Vertex state an algorithm's push operator touches.
struct AlgoState {
    int algo;
    uint32_t* val;        // BFS level / SSSP distance / CC label
    uint32_t* visited;    // BFS: discovered-vertex bitmap
    uint32_t* next;       // next-frontier bitmap
    uint32_t* overflow;   // SSSP: lane bits raised when a candidate distance reaches 2^32-1 (it is skipped)
    float* acc;           // PageRank accumulators: acc_copies (+ 1 with blocking) x acc_slots(n) floats
    uint32_t acc_copies;  // PageRank: copies the atomic adds spread over (a power of two, <= ACC_COPIES)
    const float* contrib; // PageRank x[u] / D_o(u)
    uint32_t level_next;  // BFS: level given to vertices discovered this iteration
    uint64_t n;           // vertices
    // batched runs: per-vertex lane masks and per (vertex, lane) values in rows of
    // 2^lshift lanes (lshift <= 6)
    const uint64_t* mcur; // lanes active at each vertex this iteration
    uint64_t* mnext;      // lanes improved this iteration
    uint64_t* mvisited;   // BFS: lanes that have reached each vertex
    uint32_t* lval;       // BFS: level (plus the lane's join iteration); SSSP: distance
    float* lx;            // PPR: x of each lane; scaled to x / D_o in place before a push
    double* lacc;         // PPR: per-lane accumulators (FP64), zero between iterations
    uint32_t lshift;
    const float* inv_n;   // PageRank over a union of graphs: 1 / (vertices of v's graph), else null
    Pack pk;              // how edge words are laid out
    uint32_t link_grid;   // 0, or at most this many workgroups for the host-reading pushes
    uint32_t* far;        // SSSP with a bound: improved vertices at or above it wait here (bitmap)
    uint32_t bound;       // SSSP: distances below it join the next frontier; 0xFFFFFFFF = no bound
};

// PageRank spreads its atomic adds over up to one accumulator copy per XCD (the die id,
// masked to the copies in use), plus one copy after them for the sums of propagation
// blocking; the apply step sums them.  Copies relieve contention on hub slots, which only
// adds at HBM speed create: a run with blocking (whose atomic adds come from the host link)
// uses one, other runs four.  Measured on MI355X: R-MAT 28 at 8 GB with blocking, 20 steps:
// 3.72 s with one copy, 3.77-3.79 s with eight; R-MAT 24 at 25% without blocking: 410 ms with
// one, 311 ms with two, four or eight.
constexpr uint32_t ACC_COPIES = 8;
inline uint32_t pr_acc_copies(bool blocked) { return blocked ? 1u : 4u; }

// Propagation blocking of PageRank's adds over resident edges.  Random float atomics run
// at a fixed rate (about 20 G/s on MI355X whatever the footprint): above what the host
// link delivers (at most ~14 G edges/s), so streamed edges keep their atomic adds, but
// below what HBM feeds from the resident cache.  The resident pushes instead write one
// contribution per edge into a piece buffer, a piece being a run of resident partitions
// with at most a buffer's worth of edges; the (destination, contribution) pairs of a
// piece (destinations from the resident edge words) are bucketed by destination in one
// counting-sort pass when the fine bins fit one LDS sort, else two (coarse bins of
// PB_FINE_PER_COARSE fine bins, then fine bins of PB_FINE accumulator slots), and each
// fine bin is summed in LDS and added to the blocking accumulator copy with coalesced
// read-modify-writes.  Bucket sizes of a piece are the same in every PageRank iteration
// (every vertex is active), so they are counted once.
constexpr uint32_t PB_FINE_SHIFT = 14;
constexpr uint32_t PB_FINE = 1u << PB_FINE_SHIFT;   // accumulator slots per fine bin (64 KB of LDS)
constexpr uint32_t PB_MAX_FINE = 16384;             // fine bins (LDS histogram): n <= 2^28
constexpr uint32_t PB_FINE_PER_COARSE = 32;
// Fine bins of n vertices; the accumulation segment length for pieces of `pairs` (twice a
// bin's average, at least 16384: only bins well above the average -- the hubs' -- are
// split over several workgroups); the bound on a piece's segments.
__host__ __device__ inline uint32_t pb_fine_bins(uint64_t n) { return (uint32_t)((n + PB_FINE - 1) >> PB_FINE_SHIFT); }
__host__ __device__ inline uint32_t pb_coarse_bins(uint32_t nfine) {
    return (nfine + PB_FINE_PER_COARSE - 1) / PB_FINE_PER_COARSE;
}
__host__ __device__ inline uint32_t pb_seg_len(uint32_t nfine, uint64_t pairs) {
    const uint64_t avg = (pairs + nfine - 1) / nfine;
    return (uint32_t)(2 * avg > 16384 ? 2 * avg : 16384);
}
__host__ __device__ inline uint32_t pb_max_segs(uint32_t nfine, uint64_t pairs, uint32_t seg) {
    return nfine + (uint32_t)((pairs + seg - 1) / seg);
}
// hist[f] += pairs of pv[0, cnt) whose destination (pv[i] & vmask) lies in fine bin f
// (hist zeroed by the caller).  A destination outside [0, nfine * PB_FINE) sets *err.
hipError_t launch_pb_hist(const uint32_t* pv, uint32_t vmask, uint64_t cnt, uint32_t nfine, uint32_t* hist,
                          uint32_t* err, hipStream_t st);
// From a piece's fine histogram: foff[0..nfine] = its exclusive prefix sum (bin starts in
// the bucketed buffer), segs = the accumulation segments of `seg` pairs, two words each
// (fine bin, segment index within the bin), *nsegs = their count (<= pb_max_segs).
hipError_t launch_pb_plan(const uint32_t* hist, uint32_t nfine, uint32_t seg, uint32_t* foff, uint32_t* segs,
                          uint32_t* nsegs, hipStream_t st);
// A counting-sort pass with atomic cursors (the second, fine pass): pair i of
// (in_v, in_c)[0, cnt) goes to the bin of key in_v[i] >> kshift, at the position its
// cursor hands out.  Bins are fine bins (kshift = PB_FINE_SHIFT, stride 1) or coarse bins
// (kshift = PB_FINE_SHIFT + 5, stride PB_FINE_PER_COARSE); bin k ends at
// foff[min((k + 1) * stride, nfine)], and a pair that would pass its bin's end is dropped
// and sets *err (counts that do not match the pairs).
hipError_t launch_pb_scatter(const uint32_t* in_v, const float* in_c, uint64_t cnt, uint32_t kshift, uint32_t stride,
                             uint32_t nfine, const uint32_t* foff, uint32_t* cursor, uint32_t* out_v, float* out_c,
                             uint32_t* err, hipStream_t st);
// Resident push of a piece with every vertex active: pc[t] = contrib of the source of the
// piece's edge t, t in [0, cnt), for the resident list entries [ja, jb) whose work (edge)
// ranges wpre[j] - wa tile [0, cnt).  tiles writes tj[k] = the entry holding slot
// k * 4096, for the ceil(cnt / 4096) tiles (once per piece); expand uses it.
hipError_t launch_pb_tiles(const uint64_t* wpre, uint32_t ja, uint32_t jb, uint64_t wa, uint64_t cnt, uint32_t* tj,
                           hipStream_t st);
hipError_t launch_pb_expand(const uint32_t* list, const uint64_t* wpre, uint32_t jb, uint64_t wa, uint64_t cnt,
                            const uint32_t* tj, const float* contrib, float* pc, hipStream_t st);
inline uint64_t pb_tiles(uint64_t cnt) { return (cnt + 4095) / 4096; }
// First sort pass with places fixed per workgroup slice (the slices' pairs recur every
// PageRank iteration): plan_a counts each of at most PB_A_WG slices' pairs per bin (key =
// v >> kshift, bins of `stride` fine bins, at most 1024 of them) and turns the counts into
// output starts offA[slice][bin] (pb_max_offa entries); scatter_a moves the pairs there
// with no global atomics and, with fcur != null, sets the second pass's cursors to foff.
constexpr uint32_t PB_A_WG = 1024;
constexpr uint32_t PB_LOCAL_BINS = 1024;  // bins one LDS counting sort handles
inline uint64_t pb_max_offa(uint32_t nkeys) { return (uint64_t)PB_A_WG * nkeys; }
// The first pass reads destinations as in_v[i] & vmask (resident edge words may carry
// packed weights above the neighbour bits).
hipError_t launch_pb_plan_a(const uint32_t* pv, uint32_t vmask, uint64_t cnt, uint32_t kshift, uint32_t stride,
                            uint32_t nfine, const uint32_t* foff, uint32_t* offA, uint32_t* err, hipStream_t st);
hipError_t launch_pb_scatter_a(const uint32_t* in_v, uint32_t vmask, const float* in_c, uint64_t cnt,
                               uint32_t kshift, uint32_t stride, uint32_t nfine, const uint32_t* foff,
                               const uint32_t* offA, uint32_t* out_v, float* out_c, uint32_t* fcur, uint32_t* err,
                               hipStream_t st);
// Sum each segment's pairs (bucketed by fine bin) in LDS and add the bin's slots into
// acc (slot order, acc_slot): plain read-modify-write when the bin is one segment,
// atomic adds of the non-zero slots when it spans several.  Launched with max_segs
// workgroups; those past *nsegs exit.
hipError_t launch_pb_accum(const uint32_t* pv, const float* pc, const uint32_t* foff, const uint32_t* segs,
                           const uint32_t* nsegs, uint32_t max_segs, uint32_t seg, uint64_t n, float* acc,
                           uint32_t* err, hipStream_t st);

hipError_t launch_init(const AlgoState& s, uint64_t n, uint32_t source, float pr_x0, float* pr_x, uint32_t* cur,
                       uint32_t nwords, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t st);

hipError_t launch_stats_select(uint32_t npart, const uint32_t* pv, const uint64_t* off, const uint32_t* cur,
                               const SelParams& sp, uint8_t* mode, uint32_t* nA, uint32_t* nF, uint64_t* Ea,
                               uint64_t* Rq, uint64_t* K, hipStream_t st);

// Batched runs: initialise lane masks, lane values and the union frontier.
hipError_t launch_init_lanes(const AlgoState& s, const LaneSources& src, uint32_t* cur_union, uint32_t nwords,
                             hipStream_t st);
// OR of the lane masks of all vertices into *lanes (one uint64, zeroed by the caller).
hipError_t launch_lane_union(const uint64_t* mask, uint64_t n, unsigned long long* lanes, hipStream_t st);
// Rows k = 0.. of out (n values each) <- the lanes of `set` in increasing lane order,
// from n rows of 2^lshift 32-bit values; with sub_base, a value other than UNREACHED has
// the lane's base subtracted (BFS levels of lanes that joined late).  order (or null):
// vertex v's value goes to position order[v] of its row (back to the caller's ids).
hipError_t launch_extract_lanes(const uint32_t* vals, uint64_t n, uint32_t lshift, const LaneSet& set, bool sub_base,
                                const uint32_t* order, uint32_t* out, hipStream_t st);
// Back to the caller's ids after hub sorting: dst[v] = src[rank[v]] for v < n.
hipError_t launch_gather_u32(const uint32_t* src, const uint32_t* rank, uint64_t n, uint32_t* dst, hipStream_t st);
// CC labels back to the caller's ids: every component's label becomes its smallest
// original id.  lab: labels in the relabelled order; order / rank: new -> original and
// original -> new ids; minold: n words of scratch.
hipError_t launch_cc_relabel(const uint32_t* lab, const uint32_t* order, const uint32_t* rank, uint64_t n,
                             uint32_t* minold, uint32_t* dst, hipStream_t st);
// SSSP's far set: *out = min(*out, smallest distance of a far vertex) (the caller sets *out
// to 0xFFFFFFFF first); then the far vertices with distance below `bound` move into `cur`.
hipError_t launch_far_min(const uint32_t* far, const uint32_t* dist, uint32_t nwords, uint32_t* out, hipStream_t st);
hipError_t launch_far_move(uint32_t* far, const uint32_t* dist, uint32_t* cur, uint32_t nwords, uint32_t bound,
                           hipStream_t st);
// SSSP overflow after convergence: *out |= the lanes of `mask` for which some edge of the
// mapped host array col leads from a vertex they reached to one they did not (dist: n rows
// of 2^lshift lanes; *out zeroed by the caller).  Such a lane's distances do not all fit
// below 2^32-1.
hipError_t launch_sssp_ovf_check(const uint64_t* off, const uint32_t* col, const Pack& pk, const uint32_t* dist,
                                 uint32_t lshift, uint64_t mask, uint64_t n, unsigned long long* out, hipStream_t st);
// Start the lanes of `set` at their sources (their columns must hold the reset values):
// BFS level = base, SSSP distance = 0, PPR x = 1; lane bits at the source in mcur (and
// mvisited), source bits in the union frontier `cur`.
hipError_t launch_admit_lanes(const AlgoState& s, const LaneSet& set, uint32_t* cur, hipStream_t st);
// Return the lanes in `mask` to the reset state: values UNREACHED (BFS/SSSP) or 0 (PPR x
// and accumulators), their bits cleared from mcur, mnext, mvisited and the two
// overflow words.
hipError_t launch_reset_lanes(const AlgoState& s, uint64_t mask, hipStream_t st);
// PPR step around the push: prepare scales each active (vertex, lane) x by 1 / D_o;
// apply sets x = damping * acc for every lane in mcur | mnext and clears acc; restart
// adds 1 - damping at each lane's source and marks it active for the next step.
hipError_t launch_ppr_prepare(const AlgoState& s, const uint64_t* off, hipStream_t st);
hipError_t launch_ppr_apply(const AlgoState& s, float damping, hipStream_t st);
hipError_t launch_ppr_restart(const AlgoState& s, const LaneSet& set, float restart, hipStream_t st);

// Scan of the selection: scratch holds scan_scratch_words(npart) uint64 (tile totals and bases).
constexpr int SCAN_THREADS = 512;
constexpr int SCAN_PER = 8;                                        // partitions per thread
constexpr uint32_t SCAN_TILE = (uint32_t)SCAN_THREADS * SCAN_PER;  // partitions per workgroup
inline uint32_t scan_tiles(uint32_t npart) { return (npart + SCAN_TILE - 1) / SCAN_TILE; }
inline uint64_t scan_scratch_words(uint32_t npart) { return (uint64_t)std::max(scan_tiles(npart), 1u) * (7 * NSEG + 1); }
hipError_t launch_scan(uint32_t npart, const uint8_t* mode, const uint32_t* nA, const uint32_t* nF,
                       const uint64_t* Ea, const uint64_t* Rq, const uint64_t* K, uint32_t* lbase, uint64_t* wbase,
                       Header* hdr, uint64_t* wpre, uint64_t* scratch, hipStream_t st);

hipError_t launch_build_lists(uint32_t npart, const uint32_t* pv, const uint64_t* off, const uint32_t* cur,
                              const uint8_t* mode, const uint32_t* lbase, const uint64_t* wbase, uint32_t* list,
                              uint64_t* wpre, hipStream_t st);

// Push over edge items [item_lo, item_hi) of list entries [ja, jb).  Edge e of vertex
// list[j] is read at col[off[v] - shift + (item - wpre[j])]; with compacted = true it
// is read at col[item - shift] (the compaction buffer starts at item `shift`).
hipError_t launch_push_edges(const AlgoState& s, const uint32_t* list, const uint64_t* wpre, uint32_t ja,
                             uint32_t jb, uint64_t item_lo, uint64_t item_hi, const uint64_t* off,
                             const uint32_t* col, const uint32_t* w, uint64_t shift, bool compacted,
                             hipStream_t st);

// Push over 128-byte line items [item_lo, item_hi) of list entries [ja, jb), reading
// the mapped host arrays col / w at absolute edge indices.  distinct (or null) gains the
// number of different lines read: an item that is its vertex's first line and the
// previous list entry's last line counts once.
hipError_t launch_push_lines(const AlgoState& s, const uint32_t* list, const uint64_t* wpre, uint32_t ja,
                             uint32_t jb, uint64_t item_lo, uint64_t item_hi, const uint64_t* off,
                             const uint32_t* col, const uint32_t* w, unsigned long long* distinct, hipStream_t st);

// A filter task streamed from the mapped host arrays: edges [e0, e1) of a run of
// consecutive filter partitions whose active vertices are list entries [ja, jb).
// chunk0 = chunks of all earlier tasks (a chunk is FSTREAM_LINES 128-byte lines).
struct FTask {
    uint64_t e0, e1;
    uint32_t ja, jb;
    uint64_t chunk0;
};
// 48 lines keep a chunk's staging at ~15 KB of LDS, so LDS does not cap the kernel below
// 8 workgroups of 256 threads per CU (64 lines needed 20 KB: 7 workgroups)
constexpr uint32_t FSTREAM_LINES = 48;
inline uint64_t fstream_chunks(uint64_t e0, uint64_t e1) {
    const uint64_t lines = ((e1 - 1) >> ZC_LINE_SHIFT) - (e0 >> ZC_LINE_SHIFT) + 1;
    return (lines + FSTREAM_LINES - 1) / FSTREAM_LINES;
}

// Filter engine, streaming form: every line of every task is read once from host
// memory (the whole partition is transferred); edges of active vertices are pushed.
hipError_t launch_push_fstream(const AlgoState& s, const FTask* tasks, uint32_t ntasks, uint64_t total_chunks,
                               const uint32_t* list, const uint64_t* off, const uint32_t* col, const uint32_t* w,
                               hipStream_t st);

// PageRank accumulator slot of vertex v: the low 12 bits are XORed with a hash of the
// high bits (a bijection on each 4096-aligned block) so that the R-MAT hubs, whose ids
// share many zero bits, spread over the L2 channels instead of piling onto one.
__host__ __device__ inline uint32_t acc_slot(uint32_t v) {
    return v ^ (((v >> 12) * 0x9E3779B1u) >> 20);
}
__host__ __device__ inline uint64_t acc_slots(uint64_t n) { return (n + 4095) & ~uint64_t(4095); }

// contrib = x / D_o and the first `copies` accumulator copies zeroed (acc_copies, or
// acc_copies + 1 with propagation blocking).
hipError_t launch_pr_prepare(uint64_t n, const uint64_t* off, const float* x, float* contrib, float* acc,
                             uint32_t copies, hipStream_t st);
// x = base + damping * (sum of the first `copies` accumulator copies); with inv_n, the
// base of v is restart * inv_n[v] (graph-wise normalization of a union of graphs).
hipError_t launch_pr_apply(uint64_t n, float* x, const float* acc, uint32_t copies, float base, float damping,
                           const float* inv_n, float restart, hipStream_t st);
// delta[v] = restart * (inv_n ? inv_n[v] : 1 / n): the initial pending mass of delta PageRank.
hipError_t launch_dpr_init(uint64_t n, float* delta, const float* inv_n, float restart, hipStream_t st);

// Reprocessing (Sec. 6.1): cur2 <- the vertices of next that lie in partitions whose mode
// m has bit m set in mode_mask (engine codes of the pass that just ran).  Clears cur2 first.
hipError_t launch_loaded_frontier(uint32_t npart, const uint32_t* pv, const uint8_t* mode, uint32_t mode_mask,
                                  const uint32_t* next, uint32_t* cur2, uint32_t nwords, hipStream_t st);
// Delta-based PageRank.  fold: delta[v] += the accumulator copies of v (then zeroed) and
// psum[p] = the partition's delta sum (FP64).  activate: in every partition with
// sched[p] != 0, each vertex with delta > 0 moves delta into x, shares damping * delta /
// D_o(v) as its contribution and joins the frontier cur (cleared first).
hipError_t launch_dpr_fold(uint32_t npart, const uint32_t* pv, uint64_t n, float* acc, uint32_t copies, float* delta,
                           double* psum, hipStream_t st);
hipError_t launch_dpr_activate(uint32_t npart, const uint32_t* pv, const uint64_t* off, const uint8_t* sched,
                               float* delta, float* x, float* contrib, uint32_t* cur, uint32_t nwords, float damping,
                               hipStream_t st);
// x[v] += delta[v] for every v (the pending mass, after a final fold).
hipError_t launch_dpr_finish(uint64_t n, float* x, const float* delta, hipStream_t st);

// Probes of the host link and HBM.  words_per_line in {8, 16, 32}: each 128-byte line
// of the mapped buffer contributes that many leading 4-byte words; 0 = stream the whole
// buffer with 16-byte loads.
hipError_t launch_zc_probe(const uint32_t* src, uint64_t bytes, uint32_t words_per_line, uint32_t* sink,
                           hipStream_t st);
hipError_t launch_copy_probe(void* dst, const void* src, uint64_t bytes, hipStream_t st);

hipError_t launch_select_only(uint64_t npart, const uint64_t* E, const uint64_t* nA, const uint64_t* Ea,
                              const uint64_t* Rq, const SelParams& sp, uint8_t* p, hipStream_t st);

// Allocation-free selection: a static device array of STATIC_SEL_WORDS words per device
// holds the statistics (4 x npart uint64) and then the engine codes (npart bytes) for at
// most STATIC_SEL_MAX_PARTS partitions.  static_select_scratch gives its address on
// `device`, which must be the current device (resolved on the first call per device).
constexpr uint64_t STATIC_SEL_MAX_PARTS = 1ull << 18;
constexpr uint64_t STATIC_SEL_WORDS = 4 * STATIC_SEL_MAX_PARTS + STATIC_SEL_MAX_PARTS / 8;
constexpr int STATIC_SCRATCH_DEVICES = 64;
hipError_t static_select_scratch(int device, uint64_t** out);

}  // namespace hytm
