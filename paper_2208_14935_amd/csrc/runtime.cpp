// Host runtime of libhytm.so: the C ABI declared in include/hytm.h.
//
// One handle = one CSR graph bound to one GPU.  Placement follows Sec. 1 / Sec. 4 of
// the paper: offsets (the neighbour index), vertex values and frontiers live in device
// memory; neighbour and weight arrays live in pinned host memory mapped into the GPU
// address space.  Each iteration of hytm_run:
//   1. the GPU computes per-partition statistics, selects an engine per partition
//      (Sec. 5.1) and lays the active vertices out by engine (Algorithm 1);
//   2. the host copies back the selection, combines consecutive filter partitions into
//      tasks (Sec. 5.2) and issues, concurrently (Sec. 6.2):
//        - resident partitions: push kernel on the main stream;
//        - zero-copy: one push kernel over all zero-copy vertices (mapped host reads);
//        - filter tasks: H2D copy into a ring of staging slots, then a push kernel;
//        - compaction: a host thread pool gathers the active neighbour lists into
//          pinned buffers in chunks, each copied and pushed while the next is
//          gathered (Sec. 6.3);
//   3. the main stream waits for every engine; the next frontier becomes current.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hytm.h"
#include "hubsort.h"
#include "hytm_kernels.h"
#include "pool.h"

using namespace hytm;

namespace {

thread_local std::string g_err;

hytm_status fail(hytm_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

struct HipError {
    hytm_status status;
};

#define HIP_CHECK(expr)                                                                                   \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) {                                                                           \
            (void)hipGetLastError(); /* clear it, or the next launch check would report it again */        \
            fail(e_ == hipErrorOutOfMemory ? HYTM_E_NOMEM : HYTM_E_DEVICE, "%s failed: %s (%s:%d)", #expr, \
                 hipGetErrorString(e_), __FILE__, __LINE__);                                              \
            throw HipError{e_ == hipErrorOutOfMemory ? HYTM_E_NOMEM : HYTM_E_DEVICE};                    \
        }                                                                                                 \
    } while (0)

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ device buffer
// Owns its allocation, or (view) points into another buffer's.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    bool owns = true;
    void ensure(size_t count) {
        if (count <= n && p && owns) return;
        release();
        HIP_CHECK(hipMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T)));
        n = count;
        owns = true;
    }
    void view(void* at, size_t count) {
        release();
        p = (T*)at;
        n = count;
        owns = false;
    }
    void release() {
        if (p && owns) (void)hipFree(p);
        p = nullptr;
        n = 0;
        owns = true;
    }
};

template <class T>
struct HostBuf {  // pinned host memory
    T* p = nullptr;
    size_t n = 0;
    bool owns = true;
    void ensure(size_t count) {
        if (count <= n && p && owns) return;
        release();
        HIP_CHECK(hipHostMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault));
        n = count;
        owns = true;
    }
    void view(void* at, size_t count) {
        release();
        p = (T*)at;
        n = count;
        owns = false;
    }
    void release() {
        if (p && owns) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        owns = true;
    }
};

constexpr uint32_t kMaxSlots = 16;
constexpr int kClasses = 9;

// Optional per-launch HIP-event timing, by kernel class (HYTM_K_*).  Launches may come
// from the main thread and the compaction thread, hence the lock.
struct KTimer {
    bool on = false;
    std::mutex mu;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec {
        int cls;
        hipEvent_t a, b;
        uint64_t items;
    };
    std::vector<Rec> recs;

    template <class F>
    hipError_t run(int cls, uint64_t items, hipStream_t st, F&& launch) {
        if (!on) return launch();
        std::lock_guard<std::mutex> lk(mu);
        hipEvent_t a = take(), b = take();
        hipError_t e = hipEventRecord(a, st);
        if (e != hipSuccess) return e;
        e = launch();
        if (e != hipSuccess) return e;
        e = hipEventRecord(b, st);
        if (e == hipSuccess) recs.push_back({cls, a, b, items});
        return e;
    }
    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e;
            HIP_CHECK(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    // after every recorded launch has completed
    void collect(double* ms, uint64_t* launches, uint64_t* items) {
        for (const Rec& r : recs) {
            float t = 0;
            HIP_CHECK(hipEventElapsedTime(&t, r.a, r.b));
            ms[r.cls] += t;
            launches[r.cls] += 1;
            items[r.cls] += r.items;
        }
        recs.clear();
        used = 0;
    }
    void destroy() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
        recs.clear();
        used = 0;
    }
};

}  // namespace

struct hytm_graph {
    int device = 0;
    uint64_t n = 0, m = 0;
    uint32_t flags = 0;
    hytm_params params{};
    uint64_t budget = UINT64_MAX;

    // host side
    std::vector<uint64_t> h_off;      // n + 1
    uint32_t* h_col = nullptr;        // pinned, device-mapped
    uint32_t* h_w = nullptr;          // pinned, device-mapped, or null (also when packed)
    bool weighted = false;            // the graph has edge weights
    Pack pk{0xFFFFFFFFu, 32, 0, 4};      // edge word layout: weights packed into h_col when shift < 32
    uint32_t* d_col_map = nullptr;    // device addresses of the mapped arrays
    uint32_t* d_w_map = nullptr;

    // partitions
    std::vector<uint32_t> pv;         // npart + 1 vertex bounds
    std::vector<uint64_t> pE;         // edges per partition
    uint32_t npart = 0;
    uint64_t max_part_edges = 0;
    DevBuf<uint32_t> d_pv;
    DevBuf<uint64_t> d_off;

    // per-vertex / per-partition device state
    DevBuf<uint32_t> d_val, d_cur, d_next, d_visited, d_list, d_overflow;
    DevBuf<float> d_x, d_contrib, d_acc;
    DevBuf<uint64_t> d_wpre, d_Ea, d_Rq, d_K, d_wbase;
    DevBuf<uint32_t> d_nA, d_nF, d_lbase;
    DevBuf<uint8_t> d_mode;
    DevBuf<Header> d_hdr;
    DevBuf<uint64_t> d_sel_in;  // hytm_select_engines scratch
    DevBuf<uint8_t> d_sel_out;
    DevBuf<FTask> d_tasks;        // streaming filter tasks of the current iteration
    HostBuf<FTask> h_tasks;
    // batched runs (up to 64 lanes): lane masks, lane values, lanes active this iteration
    DevBuf<uint64_t> d_mcur, d_mnext, d_mvis, d_lanes;
    DevBuf<uint32_t> d_lval;
    DevBuf<float> d_lx;           // batched PPR: x rows (FP32)
    DevBuf<double> d_lacc;        // ... and accumulator rows (FP64)
    DevBuf<uint32_t> d_xout;      // lanes extracted for the copy back
    DevBuf<uint32_t> d_cur2;      // frontier of the reprocessing pass
    DevBuf<uint64_t> d_scan;      // selection scan: per-tile totals and bases
    DevBuf<uint32_t> d_far;       // SSSP with sssp_delta: improved vertices waiting for a higher bound
    DevBuf<uint32_t> d_farmin;    // smallest waiting distance
    HostBuf<uint32_t> h_farmin;
    DevBuf<uint64_t> d_zcl;       // distinct 128-byte lines read by the zero-copy kernel this run
    DevBuf<uint64_t> d_ovf;       // SSSP: lanes whose distances overflow (checked after convergence)
    DevBuf<float> d_delta;        // delta-based PageRank: pending delta per vertex
    DevBuf<double> d_psum;        // ... and per partition
    HostBuf<double> h_psum;
    DevBuf<uint8_t> d_sched;      // ... partitions scheduled this iteration
    HostBuf<uint8_t> h_sched;
    HostBuf<uint64_t> h_lanes;
    // PageRank propagation blocking: contribution buffers [0], [1] of alternate pieces
    // (destination words [0], [1] only for the second sort pass, which writes them), [2] =
    // the first sort pass's target; bucket plans per piece
    DevBuf<uint32_t> d_pb_v[3];
    DevBuf<float> d_pb_c[3];
    DevBuf<uint32_t> d_pb_hist, d_pb_foff, d_pb_segs, d_pb_nsegs, d_pb_offa, d_pb_fcur, d_pb_err, d_pb_tj;

    // host mirrors of the per-iteration selection (views into h_sel, as the device arrays
    // d_hdr, d_wbase, d_lbase, d_mode are views into d_sel)
    DevBuf<uint8_t> d_sel;
    HostBuf<uint8_t> h_sel;
    uint32_t sel_npart = UINT32_MAX;  // partitions the views were laid out for
    HostBuf<Header> h_hdr;
    HostBuf<uint8_t> h_mode;
    HostBuf<uint32_t> h_lbase;
    HostBuf<uint64_t> h_wbase;
    HostBuf<uint32_t> h_clist;
    HostBuf<uint64_t> h_cwpre;

    // edge-budget buffers
    uint32_t res_parts = 0, res_arrays = 0;
    uint64_t res_edges = 0;
    bool res_valid = false;            // false: nothing in d_res is known to hold edge data
    // One region holds the resident cache: the neighbour prefix col[0, res_col) from word 0,
    // and the weight prefix w[0, res_w) from word res_w_at.  A one-array run keeps col[0, E1)
    // there; a two-array run col[0, E2) followed by w[0, E2) at word E2, so a switch between
    // the two copies only the part that differs.  d_res_col / d_res_w are views into it.
    DevBuf<uint32_t> d_res;
    uint64_t res_col = 0, res_w = 0, res_w_at = 0;
    DevBuf<uint32_t> d_res_col, d_res_w;
    DevBuf<uint32_t> d_slot_col[kMaxSlots], d_slot_w[kMaxSlots];
    DevBuf<uint32_t> d_cbuf_col[2], d_cbuf_w[2];
    HostBuf<uint32_t> h_cbuf_col[2], h_cbuf_w[2];

    // streams / events
    hipStream_t s_main = nullptr, s_copy = nullptr, s_fk = nullptr, s_zc = nullptr, s_c = nullptr, s_pb = nullptr;
    hipEvent_t ev_copied[kMaxSlots] = {}, ev_free[kMaxSlots] = {};
    hipEvent_t ev_pbpush = nullptr, ev_pbfree[2] = {};
    hipEvent_t ev_cdone[2] = {}, ev_join[4] = {}, ev_start = nullptr, ev_clist = nullptr, ev_go = nullptr;
    hipEvent_t ev_sel[2] = {};    // timing events around each pass's selection (statistics to D2H)

    Pool* pool = nullptr;
    KTimer timer;
    hytm_server* server = nullptr;  // open query server (owns the graph while set)

    // hub sorting: the graph is held relabelled; callers' ids map through these
    uint64_t hubs = 0;
    std::vector<uint32_t> h_rank;        // caller id -> internal id
    DevBuf<uint32_t> d_rank, d_order;    // caller -> internal, internal -> caller
    DevBuf<uint32_t> d_minold;           // CC label canonicalization scratch

    // a disjoint union of graphs (hytm_graph_set_parts): PageRank per graph
    std::vector<uint64_t> parts;         // vertex bounds in caller ids, or empty
    DevBuf<float> d_inv_n;               // per internal vertex: 1 / (vertices of its graph)
    bool hub_sorted() const { return !h_rank.empty(); }
    uint32_t inner(uint32_t v) const { return h_rank.empty() ? v : h_rank[v]; }
};

namespace {

bool params_valid(const hytm_params& p, std::string* why) {
    auto bad = [&](const char* s) {
        *why = s;
        return false;
    };
    if (p.mode < HYTM_MODE_HYBRID || p.mode > HYTM_MODE_ZEROCOPY) return bad("mode out of range");
    if (p.partition_edges == 0) return bad("partition_edges must be > 0");
    if (p.combine_k == 0) return bad("combine_k must be > 0");
    auto frac_ok = [](uint32_t a, uint32_t b, bool le1) { return b > 0 && b <= 65536 && a <= 65536 && (!le1 || a <= b); };
    if (!frac_ok(p.alpha_num, p.alpha_den, false)) return bad("alpha must be num/den with den in 1..65536");
    if (!frac_ok(p.beta_num, p.beta_den, false)) return bad("beta must be num/den with den in 1..65536");
    if (!frac_ok(p.gamma_num, p.gamma_den, true)) return bad("gamma must be in [0, 1] with den in 1..65536");
    if (p.line_bytes < 4 || (p.line_bytes & (p.line_bytes - 1))) return bad("line_bytes must be a power of two >= 4");
    if (p.max_outstanding == 0) return bad("max_outstanding must be > 0");
    if (p.index_bytes > 64) return bad("index_bytes must be <= 64");
    if (!(p.pr_damping >= 0.0 && p.pr_damping <= 1.0)) return bad("pr_damping must be in [0, 1]");
    if (p.reprocess > 2) return bad("reprocess must be 0, 1 or 2");
    if (p.rq_distinct_lines > 1) return bad("rq_distinct_lines must be 0 or 1");
    if (p.zc_tie > 2) return bad("zc_tie must be 0, 1 or 2");
    if (p.pr_blocking > 2) return bad("pr_blocking must be 0, 1 or 2");
    if (p.pr_block_pairs >= (1ull << 31)) return bad("pr_block_pairs must be below 2^31");
    if (!frac_ok(p.compact_gather_num, p.compact_gather_den, false))
        return bad("compact_gather must be num/den with den in 1..65536");
    if (!(p.dpr_epsilon >= 0.0)) return bad("dpr_epsilon must be >= 0");
    if (p.streams < 2 || p.streams > kMaxSlots) return bad("streams must be in 2..16");
    if (p.gather_threads > 256) return bad("gather_threads must be <= 256");
    if (p.filter_engine != HYTM_FILTER_STREAM && p.filter_engine != HYTM_FILTER_COPY)
        return bad("filter_engine must be HYTM_FILTER_STREAM or HYTM_FILTER_COPY");
    return true;
}

// Greedy chunk partitioning (Sec. 4): walk vertices in order and close the current
// partition before v when it already holds an edge and D_o(v) would take it past the
// target; an oversize vertex therefore forms a partition of its own.
void partition_graph(hytm_graph* g) {
    const uint64_t target = g->params.partition_edges;
    g->pv.clear();
    g->pE.clear();
    g->pv.push_back(0);
    uint64_t edges = 0;
    for (uint64_t v = 0; v < g->n; v++) {
        const uint64_t d = g->h_off[v + 1] - g->h_off[v];
        if (edges > 0 && edges + d > target) {
            g->pv.push_back((uint32_t)v);
            g->pE.push_back(edges);
            edges = 0;
        }
        edges += d;
    }
    g->pv.push_back((uint32_t)g->n);
    g->pE.push_back(edges);
    g->npart = (uint32_t)g->pE.size();
    g->max_part_edges = 0;
    for (uint64_t e : g->pE) g->max_part_edges = std::max(g->max_part_edges, e);
    g->d_pv.ensure(g->pv.size());
    HIP_CHECK(hipMemcpy(g->d_pv.p, g->pv.data(), g->pv.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    g->res_valid = false;
}

// Edge arrays an algorithm reads per edge: SSSP reads neighbours and weights, unless the
// weights are packed into the neighbour words.
uint32_t edge_arrays(const hytm_graph* g, int algo) { return algo == HYTM_SSSP && g->pk.shift == 32 ? 2 : 1; }

// Bytes per edge a run reads with `arrays` edge arrays: the neighbour word, plus the weight
// (4 bytes, or 1 when the weights are kept as bytes).  This is d1 of Eq. 1-2.
uint32_t edge_bytes(const hytm_graph* g, uint32_t arrays) { return arrays == 2 ? 4 + g->pk.wbytes : 4; }

// 32-bit words that `count` weights take in device buffers.
uint64_t weight_words(const hytm_graph* g, uint64_t count) { return (count * g->pk.wbytes + 3) / 4; }

SelParams make_sel(const hytm_graph* g, uint32_t arrays) {
    const hytm_params& p = g->params;
    SelParams sp{};
    sp.L = (uint64_t)p.line_bytes * p.max_outstanding;
    sp.MR = p.max_outstanding;
    sp.d1 = edge_bytes(g, arrays);
    sp.d2 = p.index_bytes;
    sp.an = p.alpha_num;
    sp.ad = p.alpha_den;
    sp.bn = p.beta_num;
    sp.bd = p.beta_den;
    sp.gn = p.gamma_num;
    sp.gd = p.gamma_den;
    uint32_t sh = 0;
    while ((4u << sh) < p.line_bytes) sh++;
    sp.cost_shift = sh;
    sp.wbytes = arrays == 2 ? g->pk.wbytes : 0u;
    sp.force = p.mode == HYTM_MODE_FILTER ? P_FILTER
               : p.mode == HYTM_MODE_COMPACT ? P_COMPACT
               : p.mode == HYTM_MODE_ZEROCOPY ? P_ZC
                                              : 0;
    sp.allow_filter = 1;
    sp.allow_compact = 1;
    sp.gn_c = p.compact_gather_num;
    sp.gd_c = p.compact_gather_den;
    sp.rq_distinct = p.rq_distinct_lines;
    sp.zc_tie = p.zc_tie == 1 ? 1u : 0u;  // 2 (automatic) is resolved per run, see resolve_tie
    return sp;
}

// Split of the edge budget (reading of the paper's placement: the budget covers only
// edge-associated device memory).
// Byte layout of the selection block: header, work bases (8 B), list bases (4 B), engine
// codes (1 B) per partition.
struct SelLayout {
    size_t wbase, lbase, mode, bytes;
};
SelLayout sel_layout(uint32_t npart) {
    SelLayout L;
    L.wbase = (sizeof(Header) + 15) & ~size_t(15);
    L.lbase = L.wbase + 8 * (size_t)npart;
    L.mode = L.lbase + 4 * (size_t)npart;
    L.bytes = L.mode + npart;
    return L;
}
size_t sel_block_bytes(uint32_t npart) { return sel_layout(npart).bytes; }

struct Plan {
    uint32_t nres = 0;
    uint64_t res_edges = 0;
    uint64_t res_words = 0;  // words of the resident region under this budget
    uint64_t slot_edges = 0;
    uint32_t nslots = 0;
    uint64_t cchunk = 0;
    bool allow_filter = false, allow_compact = false;
};

// Edge-budget bytes the engines' buffers take: filter = `streams` staging slots, each
// holding the largest combined task; compaction = two chunk buffers.
struct Staging {
    uint64_t slot_edges, cchunk, f_bytes, c_bytes;
};
Staging staging_of(const hytm_graph* g, uint32_t arrays) {
    const hytm_params& p = g->params;
    const uint64_t d1 = edge_bytes(g, arrays);
    Staging s;
    s.slot_edges = std::max<uint64_t>((uint64_t)p.combine_k * p.partition_edges, g->max_part_edges);
    // two chunk buffers of 2^20 edges: 8 MB per edge array, which a 263 MB budget (R-MAT 24 at
    // 25%) would otherwise hold as resident edges (4x that cost 2% of the budget's edges)
    s.cchunk = p.compact_chunk_edges ? p.compact_chunk_edges : std::max<uint64_t>(s.slot_edges, 1ull << 20);
    // the streaming filter engine reads host memory directly and stages nothing
    s.f_bytes = p.filter_engine == HYTM_FILTER_COPY ? s.slot_edges * p.streams * d1 : 0;
    s.c_bytes = 2 * s.cchunk * d1;
    return s;
}

// Edge-budget bytes the engines' buffers take under the handle's mode for staging `sg`
// (hybrid leaves out an engine whose staging does not fit, as make_plan does).
uint64_t engine_bytes(const hytm_graph* g, const Staging& sg, uint64_t B) {
    switch (g->params.mode) {
    case HYTM_MODE_FILTER:
        return sg.f_bytes;
    case HYTM_MODE_COMPACT:
        return sg.c_bytes;
    case HYTM_MODE_ZEROCOPY:
        return 0;
    default:
        if (sg.f_bytes + sg.c_bytes <= B) return sg.f_bytes + sg.c_bytes;
        if (sg.f_bytes <= B) return sg.f_bytes;
        if (sg.c_bytes <= B) return sg.c_bytes;
        return 0;
    }
}

hytm_status make_plan(const hytm_graph* g, uint32_t arrays, Plan* out) {
    const hytm_params& p = g->params;
    const uint64_t d1 = edge_bytes(g, arrays);
    Plan pl;
    if (g->budget == UINT64_MAX) {
        pl.nres = g->npart;
        pl.res_edges = g->m;
        pl.res_words = arrays * g->m;
        *out = pl;
        return HYTM_OK;
    }
    const uint64_t B = g->budget;
    const Staging sg = staging_of(g, arrays);
    pl.slot_edges = sg.slot_edges;
    pl.nslots = p.streams;
    pl.cchunk = sg.cchunk;
    uint64_t used = 0;
    switch (p.mode) {
    case HYTM_MODE_FILTER:
        if (sg.f_bytes > B)
            return fail(HYTM_E_BUDGET, "filter staging needs %llu bytes (%u slots x %llu edges), budget is %llu",
                        (unsigned long long)sg.f_bytes, pl.nslots, (unsigned long long)pl.slot_edges,
                        (unsigned long long)B);
        pl.allow_filter = true;
        used = sg.f_bytes;
        break;
    case HYTM_MODE_COMPACT:
        if (sg.c_bytes > B)
            return fail(HYTM_E_BUDGET, "compaction buffers need %llu bytes (2 x %llu edges), budget is %llu",
                        (unsigned long long)sg.c_bytes, (unsigned long long)pl.cchunk, (unsigned long long)B);
        pl.allow_compact = true;
        used = sg.c_bytes;
        break;
    case HYTM_MODE_ZEROCOPY:
        break;
    default:  // hybrid: an engine whose staging does not fit is left out of the choice
        if (sg.f_bytes + sg.c_bytes <= B) {
            pl.allow_filter = pl.allow_compact = true;
            used = sg.f_bytes + sg.c_bytes;
        } else if (sg.f_bytes <= B) {
            pl.allow_filter = true;
            used = sg.f_bytes;
        } else if (sg.c_bytes <= B) {
            pl.allow_compact = true;
            used = sg.c_bytes;
        }
    }
    // The resident share is the same for both edge-array counts a graph with separate
    // weights runs with (the budget less the larger of their staging needs), so that one
    // region holds either layout and the budget covers both.
    uint64_t used_res = used;
    if (g->h_w && g->pk.shift == 32) {
        const uint64_t u = engine_bytes(g, staging_of(g, 3 - arrays), B);
        if (u <= B) used_res = std::max(used_res, u);
    }
    const uint64_t res_bytes = B - used_res;
    uint32_t nres = 0;
    uint64_t edges = 0;
    while (nres < g->npart && (edges + g->pE[nres]) * d1 <= res_bytes) edges += g->pE[nres++];
    pl.nres = nres;
    pl.res_edges = edges;
    pl.res_words = res_bytes / 4;
    *out = pl;
    return HYTM_OK;
}

void ensure_streams(hytm_graph* g) {
    if (g->s_copy) return;
    HIP_CHECK(hipStreamCreateWithFlags(&g->s_main, hipStreamNonBlocking));
    HIP_CHECK(hipStreamCreateWithFlags(&g->s_copy, hipStreamNonBlocking));
    HIP_CHECK(hipStreamCreateWithFlags(&g->s_fk, hipStreamNonBlocking));
    HIP_CHECK(hipStreamCreateWithFlags(&g->s_zc, hipStreamNonBlocking));
    HIP_CHECK(hipStreamCreateWithFlags(&g->s_c, hipStreamNonBlocking));
    HIP_CHECK(hipStreamCreateWithFlags(&g->s_pb, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&g->ev_pbpush, hipEventDisableTiming));
    for (auto& e : g->ev_pbfree) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (uint32_t i = 0; i < kMaxSlots; i++) {
        HIP_CHECK(hipEventCreateWithFlags(&g->ev_copied[i], hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&g->ev_free[i], hipEventDisableTiming));
    }
    for (auto& e : g->ev_cdone) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : g->ev_join) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&g->ev_start, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&g->ev_clist, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&g->ev_go, hipEventDisableTiming));
    for (auto& e : g->ev_sel) HIP_CHECK(hipEventCreate(&e));
}

void release_all(hytm_graph* g) {
    if (g->s_copy) (void)hipDeviceSynchronize();
    for (auto* b : {&g->d_val, &g->d_cur, &g->d_next, &g->d_visited, &g->d_list, &g->d_overflow, &g->d_nA, &g->d_nF,
                    &g->d_lbase, &g->d_pv, &g->d_res_col, &g->d_res_w, &g->d_res})
        b->release();
    for (auto* b : {&g->d_x, &g->d_contrib, &g->d_acc}) b->release();
    for (auto* b : {&g->d_wpre, &g->d_Ea, &g->d_Rq, &g->d_K, &g->d_wbase, &g->d_off, &g->d_sel_in}) b->release();
    g->d_mode.release();
    g->d_sel_out.release();
    g->d_tasks.release();
    g->h_tasks.release();
    for (auto* b : {&g->d_mcur, &g->d_mnext, &g->d_mvis, &g->d_lanes}) b->release();
    g->d_lval.release();
    g->d_lx.release();
    g->d_lacc.release();
    g->d_xout.release();
    g->d_cur2.release();
    g->d_far.release();
    g->d_scan.release();
    g->d_farmin.release();
    g->h_farmin.release();
    g->d_zcl.release();
    g->d_ovf.release();
    g->d_delta.release();
    g->d_psum.release();
    g->h_psum.release();
    g->d_sched.release();
    g->h_sched.release();
    g->d_rank.release();
    g->d_order.release();
    g->d_minold.release();
    g->d_inv_n.release();
    g->h_lanes.release();
    g->d_hdr.release();
    for (int i = 0; i < 3; i++) {
        g->d_pb_v[i].release();
        g->d_pb_c[i].release();
    }
    for (auto* b : {&g->d_pb_hist, &g->d_pb_foff, &g->d_pb_segs, &g->d_pb_nsegs, &g->d_pb_offa, &g->d_pb_fcur,
                    &g->d_pb_err, &g->d_pb_tj})
        b->release();
    for (uint32_t i = 0; i < kMaxSlots; i++) {
        g->d_slot_col[i].release();
        g->d_slot_w[i].release();
    }
    for (int i = 0; i < 2; i++) {
        g->d_cbuf_col[i].release();
        g->d_cbuf_w[i].release();
        g->h_cbuf_col[i].release();
        g->h_cbuf_w[i].release();
    }
    g->h_hdr.release();
    g->h_mode.release();
    g->d_sel.release();  // after its views
    g->h_sel.release();
    g->sel_npart = UINT32_MAX;
    g->h_lbase.release();
    g->h_wbase.release();
    g->h_clist.release();
    g->h_cwpre.release();
    if (g->h_col) (void)hipHostFree(g->h_col);
    if (g->h_w) (void)hipHostFree(g->h_w);
    g->h_col = g->h_w = nullptr;
    for (hipStream_t s : {g->s_main, g->s_copy, g->s_fk, g->s_zc, g->s_c, g->s_pb})
        if (s) (void)hipStreamDestroy(s);
    if (g->ev_pbpush) (void)hipEventDestroy(g->ev_pbpush);
    for (auto e : g->ev_pbfree)
        if (e) (void)hipEventDestroy(e);
    for (uint32_t i = 0; i < kMaxSlots; i++) {
        if (g->ev_copied[i]) (void)hipEventDestroy(g->ev_copied[i]);
        if (g->ev_free[i]) (void)hipEventDestroy(g->ev_free[i]);
    }
    for (auto e : g->ev_cdone)
        if (e) (void)hipEventDestroy(e);
    for (auto e : g->ev_join)
        if (e) (void)hipEventDestroy(e);
    if (g->ev_start) (void)hipEventDestroy(g->ev_start);
    if (g->ev_clist) (void)hipEventDestroy(g->ev_clist);
    if (g->ev_go) (void)hipEventDestroy(g->ev_go);
    for (auto e : g->ev_sel)
        if (e) (void)hipEventDestroy(e);
    delete g->pool;
    g->pool = nullptr;
    g->timer.destroy();
}

void parallel_copy(void* dst, const void* src, size_t bytes) {
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (bytes < (64u << 20) || nt == 1) {
        memcpy(dst, src, bytes);
        return;
    }
    std::vector<std::thread> th;
    const size_t chunk = (bytes / nt + 4095) & ~size_t(4095);
    for (unsigned i = 0; i < nt; i++) {
        const size_t a = i * chunk;
        if (a >= bytes) break;
        const size_t b = std::min(bytes, a + chunk);
        th.emplace_back([=] { memcpy((char*)dst + a, (const char*)src + a, b - a); });
    }
    for (auto& t : th) t.join();
}

// ------------------------------------------------------------------- run
// Totals of one traversal, summed over its iterations.
struct Totals {
    uint32_t iters = 0;
    double select_ms = 0, fill_ms = 0;
    uint64_t fill_bytes = 0;
    uint64_t part_iters[5] = {0, 0, 0, 0, 0};
    uint64_t av = 0, ae = 0, bf = 0, bc = 0, zcl = 0, d2h = 0, ftasks = 0, cchunks = 0;
};

// A run of consecutive resident partitions whose edges fit one piece buffer (PageRank
// with propagation blocking), with the part of the selection's resident list covering it.
struct PbPiece {
    uint64_t e0 = 0, cnt = 0;        // CSR edge range [e0, e0 + cnt): slot = edge - e0
    uint32_t ja = 0, jb = 0;         // resident list range
    uint64_t wa = 0, wb = 0;         // ... and its work range
    uint64_t tj = 0;                 // first entry of its expand-tile table
};

// One traversal: a single-source or whole-graph run, or one group of lanes (a batched
// run or a lane group of the query server).  The per-graph scratch it steps through
// (lists, selection, staging) is shared; the frontier and value state is its own.
struct RunCtx {
    hytm_graph* g = nullptr;
    int algo = 0;         // hytm_algo
    uint32_t arrays = 1;  // edge arrays read per edge (SSSP: neighbours and weights)
    bool batched = false;
    Plan plan;
    SelParams sp{};
    AlgoState as{};
    hytm_run_stats* stats = nullptr;
    uint32_t nwords = 0;
    uint32_t *cur = nullptr, *nxt = nullptr;   // frontier bitmaps (union over lanes)
    uint64_t *mcur = nullptr, *mnxt = nullptr; // lane masks
    LaneSet ppr{};                             // PPR lanes stepping, restarted at their sources
    bool reprocess = false;                    // second pass over loaded partitions (Sec. 6.1)
    // PageRank's frontier is every vertex in every iteration, so the first iteration's
    // selection, lists and filter tasks hold for all of them: later iterations replay them
    struct {
        bool ok = false;
        Header h{};
        uint32_t ftasks = 0;
        uint64_t fchunks = 0, fbytes = 0;
    } replay;
    uint32_t last_ftasks = 0;                  // streaming filter tasks of the last pass
    uint64_t last_fchunks = 0;
    // PageRank with propagation blocking: the first iteration's selection cut into pieces
    bool pb_on = false;
    struct {
        bool ok = false;
        Header h{};
        std::vector<PbPiece> pieces;    // over the resident partitions, in order
        uint64_t cap = 0;               // pairs per piece buffer
        uint32_t nfine = 0, seg = 0, max_segs = 0;
        uint32_t keys_a = 0;            // bins of the first sort pass (coarse, or fine if only one pass)
        uint32_t ftasks = 0;            // streaming filter tasks of the streamed partitions
        uint64_t fchunks = 0, fedges = 0;
    } pb;
    uint32_t t = 0;                            // iterations taken
    Totals tot;
};

// Gather list entries' edges for items [x0, x1) of the compaction segment into
// the pinned chunk buffer (Sec. 6.3 compaction engine).
void gather_chunk(hytm_graph* g, uint32_t arrays, const uint32_t* clist, const uint64_t* cwpre, uint32_t count,
                  uint64_t x0, uint64_t x1, uint32_t* out_col, uint32_t* out_w) {
    const unsigned parts = std::max(1u, g->pool->size() * 2);
    const uint64_t total = x1 - x0;
    const uint64_t step = (total + parts - 1) / parts;
    g->pool->run(parts, [&](unsigned t) {
        const uint64_t y0 = x0 + std::min<uint64_t>(total, t * step);
        const uint64_t y1 = x0 + std::min<uint64_t>(total, (uint64_t)(t + 1) * step);
        if (y0 >= y1) return;
        // last entry j with cwpre[j] <= y0
        uint32_t j = (uint32_t)(std::upper_bound(cwpre, cwpre + count, y0) - cwpre) - 1;
        uint64_t y = y0;
        while (y < y1) {
            const uint32_t v = clist[j];
            const uint64_t pre = cwpre[j], end = cwpre[j + 1];
            const uint64_t a = y, b = std::min(end, y1);
            const uint64_t src = g->h_off[v] + (a - pre);
            memcpy(out_col + (a - x0), g->h_col + src, (b - a) * sizeof(uint32_t));
            if (arrays == 2) {
                const uint32_t wb = g->pk.wbytes;
                memcpy((uint8_t*)out_w + (a - x0) * wb, (const uint8_t*)g->h_w + src * wb, (b - a) * wb);
            }
            y = b;
            j++;
        }
    });
}

// The compaction engine for one iteration, run on its own host thread.
void run_compaction(RunCtx* rc, uint32_t cs, uint32_t cc, uint64_t w0, uint64_t w1, uint64_t* chunks,
                    uint64_t* bytes, uint64_t* d2h, hytm_status* st_out, std::string* msg) {
    hytm_graph* g = rc->g;
    try {
        // active list and work prefix of the compaction segment (Vc and its offsets)
        HIP_CHECK(hipMemcpyAsync(g->h_clist.p, g->d_list.p + cs, cc * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                 g->s_c));
        HIP_CHECK(hipMemcpyAsync(g->h_cwpre.p, g->d_wpre.p + cs, (cc + 1) * sizeof(uint64_t),
                                 hipMemcpyDeviceToHost, g->s_c));
        HIP_CHECK(hipEventRecord(g->ev_clist, g->s_c));
        HIP_CHECK(hipEventSynchronize(g->ev_clist));
        *d2h += cc * (sizeof(uint32_t) + sizeof(uint64_t));
        const uint64_t chunk = rc->plan.cchunk;
        uint64_t x0 = w0;
        uint32_t b = 0, issued = 0;
        while (x0 < w1) {
            const uint64_t x1 = std::min(w1, x0 + chunk);
            if (issued >= 2) HIP_CHECK(hipEventSynchronize(g->ev_cdone[b]));
            gather_chunk(g, rc->arrays, g->h_clist.p, g->h_cwpre.p, cc, x0, x1, g->h_cbuf_col[b].p,
                         rc->arrays == 2 ? g->h_cbuf_w[b].p : nullptr);
            HIP_CHECK(hipMemcpyAsync(g->d_cbuf_col[b].p, g->h_cbuf_col[b].p, (x1 - x0) * 4, hipMemcpyHostToDevice,
                                     g->s_c));
            if (rc->arrays == 2)
                HIP_CHECK(hipMemcpyAsync(g->d_cbuf_w[b].p, g->h_cbuf_w[b].p, (x1 - x0) * g->pk.wbytes,
                                         hipMemcpyHostToDevice, g->s_c));
            HIP_CHECK(g->timer.run(HYTM_K_PUSH_C, x1 - x0, g->s_c, [&] {
                return launch_push_edges(rc->as, g->d_list.p, g->d_wpre.p, cs, cs + cc, x0, x1, g->d_off.p,
                                         g->d_cbuf_col[b].p, g->d_cbuf_w[b].p, x0, true, g->s_c);
            }));
            HIP_CHECK(hipEventRecord(g->ev_cdone[b], g->s_c));
            *bytes += (x1 - x0) * edge_bytes(g, rc->arrays);
            *chunks += 1;
            issued++;
            b ^= 1;
            x0 = x1;
        }
        *st_out = HYTM_OK;
    } catch (const HipError& e) {
        *st_out = e.status;
    } catch (const std::bad_alloc&) {
        *st_out = fail(HYTM_E_NOMEM, "host allocation failed in the compaction engine");
    }
    *msg = g_err;  // the message is thread-local: hand it back to the calling thread
}

// Plan the edge budget for `plan_arrays` edge arrays and put the per-graph scratch, the
// engines' buffers and the resident cache in place.
hytm_status prepare_graph(hytm_graph* g, uint32_t plan_arrays, hipStream_t main, Plan* plan, Totals* tot) {
    hytm_status ps = make_plan(g, plan_arrays, plan);
    if (ps != HYTM_OK) return ps;
    const Plan& pl = *plan;
    const uint64_t n = g->n;
    const uint32_t npart = g->npart;
    g->d_list.ensure(n);
    g->d_wpre.ensure(n + 1);
    g->d_overflow.ensure(2);
    g->d_zcl.ensure(1);
    g->d_lanes.ensure(1);
    g->h_lanes.ensure(1);

    g->d_nA.ensure(npart);
    g->d_nF.ensure(npart);

    g->d_Ea.ensure(npart);
    g->d_Rq.ensure(npart);
    g->d_K.ensure(npart);
    // the selection that crosses to the host every iteration -- header, list and work bases,
    // engine codes -- is one block on each side, moved by one copy
    const size_t sel_bytes = sel_block_bytes(npart);
    // the views depend on npart (repartitioning changes it): re-derive them whenever it differs
    if (g->sel_npart != npart || g->d_sel.n < sel_bytes || g->h_sel.n < sel_bytes) {
        g->d_sel.ensure(sel_bytes);
        g->h_sel.ensure(sel_bytes);
        const SelLayout L = sel_layout(npart);
        g->d_hdr.view(g->d_sel.p, 1);
        g->d_wbase.view(g->d_sel.p + L.wbase, npart);
        g->d_lbase.view(g->d_sel.p + L.lbase, npart);
        g->d_mode.view(g->d_sel.p + L.mode, npart);
        g->h_hdr.view(g->h_sel.p, 1);
        g->h_wbase.view(g->h_sel.p + L.wbase, npart);
        g->h_lbase.view(g->h_sel.p + L.lbase, npart);
        g->h_mode.view(g->h_sel.p + L.mode, npart);
        g->sel_npart = npart;
    }

    // edge-budget buffers
    const bool fstream = g->params.filter_engine == HYTM_FILTER_STREAM;
    if (pl.allow_filter && !fstream)
        for (uint32_t s = 0; s < pl.nslots; s++) {
            g->d_slot_col[s].ensure(pl.slot_edges);
            if (plan_arrays == 2) g->d_slot_w[s].ensure(weight_words(g, pl.slot_edges));
        }
    if (pl.allow_filter && fstream) {
        g->d_tasks.ensure(npart);
        g->h_tasks.ensure(npart);
    }
    if (pl.allow_compact) {
        for (int b = 0; b < 2; b++) {
            g->d_cbuf_col[b].ensure(pl.cchunk);
            g->h_cbuf_col[b].ensure(pl.cchunk);
            if (plan_arrays == 2) {
                g->d_cbuf_w[b].ensure(weight_words(g, pl.cchunk));
                g->h_cbuf_w[b].ensure(weight_words(g, pl.cchunk));
            }
        }
        g->h_clist.ensure(n);
        g->h_cwpre.ensure(n + 1);
        if (!g->pool) {
            unsigned t = g->params.gather_threads;
            if (!t) t = std::max(1u, std::min(16u, std::thread::hardware_concurrency() / 2));
            g->pool = new Pool(t);
        }
    }

    // resident cache: partitions [0, nres) in the region, copying only what it lacks
    if (pl.nres > 0) {
        const uint64_t E = pl.res_edges;
        const uint64_t need = plan_arrays == 2 ? E + weight_words(g, E) : E;
        const uint64_t cap = std::max(need, pl.res_words);
        if (g->d_res.n < need || g->d_res.n > cap) {  // sized to this budget's region
            g->d_res_col.release();
            g->d_res_w.release();
            g->d_res.release();
            g->d_res.ensure(cap);
            g->res_valid = false;
        }
        if (!g->res_valid) {
            g->res_col = g->res_w = g->res_w_at = 0;
            g->res_valid = true;
        }
        const double t0 = now_ms();
        bool filled = false;
        if (g->res_col < E) {
            HIP_CHECK(hipMemcpyAsync(g->d_res.p + g->res_col, g->h_col + g->res_col, (E - g->res_col) * 4,
                                     hipMemcpyHostToDevice, main));
            tot->fill_bytes += (E - g->res_col) * 4;
            if (g->res_w && g->res_w_at < E && g->res_w_at + weight_words(g, g->res_w) > g->res_col) g->res_w = 0;
            g->res_col = E;
            filled = true;
        }
        if (plan_arrays == 2 && !(g->res_w >= E && g->res_w_at == E)) {
            HIP_CHECK(hipMemcpyAsync(g->d_res.p + E, g->h_w, E * g->pk.wbytes, hipMemcpyHostToDevice, main));
            tot->fill_bytes += E * g->pk.wbytes;
            g->res_w = E;
            g->res_w_at = E;
            g->res_col = std::min(g->res_col, E);  // the weights took the words past E
            filled = true;
        }
        if (filled) {
            HIP_CHECK(hipStreamSynchronize(main));
            tot->fill_ms += now_ms() - t0;
        }
        g->d_res_col.view(g->d_res.p, E);
        if (plan_arrays == 2)
            g->d_res_w.view(g->d_res.p + E, weight_words(g, E));
        else
            g->d_res_w.release();
        g->res_parts = pl.nres;
        g->res_edges = E;
        g->res_arrays = plan_arrays;
    }
    return HYTM_OK;
}

// The Tiz = Tef tie rule of a run.  zc_tie = 2 (automatic): zero-copy for PageRank without
// propagation blocking, filter otherwise.  Measured on MI355X, where a tie means that the
// two engines read the same lines: blocked PageRank's streamed pushes run from a 512-workgroup
// grid, in which the streaming filter (a chunk's loads issued before its vertices are
// located, each line read once) moves them faster than zero-copy's per-list passes (R-MAT 28
// at 8 GB: 3.82 s against 4.21 s); without blocking PageRank's pushes fill the GPU and zero-copy
// is the faster (R-MAT 24 at 25%: 313 against 340 ms).  Ties to filter are as fast or faster
// for BFS, SSSP and CC on both graphs.
uint32_t resolve_tie(const hytm_graph* g, int algo, bool pb_on) {
    const uint32_t t = g->params.zc_tie;
    if (t != 2) return t;
    return algo == HYTM_PAGERANK && !pb_on ? 1u : 0u;
}

// Engine choice inputs of a traversal under a plan made by prepare_graph.
void init_ctx(RunCtx& rc, hytm_graph* g, int algo, bool batched, const Plan& pl, hytm_run_stats* stats) {
    rc.g = g;
    rc.algo = algo;
    rc.arrays = edge_arrays(g, algo);
    rc.batched = batched;
    rc.plan = pl;
    rc.stats = stats;
    rc.sp = make_sel(g, rc.arrays);
    rc.sp.nres = pl.nres;
    rc.sp.allow_filter = pl.allow_filter || g->budget == UINT64_MAX;
    rc.sp.allow_compact = pl.allow_compact || g->budget == UINT64_MAX;
    rc.nwords = (uint32_t)((g->n + 31) / 32);
    rc.as.n = g->n;
    rc.as.overflow = g->d_overflow.p;
    rc.as.pk = g->pk;
    rc.as.far = nullptr;
    rc.as.bound = 0xFFFFFFFFu;  // no far set unless a single-source SSSP run asks for one
    rc.as.acc_copies = pr_acc_copies(false);  // a run decides once it knows whether it blocks
}

// One engine pass over the frontier `cur` (Algorithm 1 plus the engines of Sec. 6.2),
// joined into `main`.  *hout: the pass's selection header.  With lanes != null, *lanes =
// the union of the lane masks rc.mcur.  With stop_if_empty and an empty frontier, nothing
// is pushed.  Transfer and activity counts are added to *rec; trace_t >= 0 records the
// engine choice in the caller's mode trace.
hytm_status engine_pass(RunCtx& rc, const uint32_t* cur, hipStream_t main, Header* hout, uint64_t* lanes,
                        bool stop_if_empty, hytm_iter_stats* rec, int64_t trace_t, bool select_only = false) {
    hytm_graph* g = rc.g;
    KTimer& kt = g->timer;
    AlgoState& as = rc.as;
    const uint64_t n = g->n;
    const uint32_t npart = g->npart;
    const Plan& pl = rc.plan;
    const bool fstream = g->params.filter_engine == HYTM_FILTER_STREAM;
    const uint64_t d1b = edge_bytes(g, rc.arrays);
    // 1. statistics, engine selection, active lists (Algorithm 1, GPU part); timed on the
    // device from the statistics kernel to the end of the D2H copy, so the time the stream
    // spends finishing the previous iteration's pushes is not counted
    HIP_CHECK(hipEventRecord(g->ev_sel[0], main));
    HIP_CHECK(kt.run(HYTM_K_STATS, npart, main, [&] {
        return launch_stats_select(npart, g->d_pv.p, g->d_off.p, cur, rc.sp, g->d_mode.p, g->d_nA.p, g->d_nF.p,
                                   g->d_Ea.p, g->d_Rq.p, g->d_K.p, main);
    }));
    g->d_scan.ensure(scan_scratch_words(npart));
    HIP_CHECK(kt.run(HYTM_K_SCAN, npart, main, [&] {
        return launch_scan(npart, g->d_mode.p, g->d_nA.p, g->d_nF.p, g->d_Ea.p, g->d_Rq.p, g->d_K.p, g->d_lbase.p,
                           g->d_wbase.p, g->d_hdr.p, g->d_wpre.p, g->d_scan.p, main);
    }));
    HIP_CHECK(kt.run(HYTM_K_LISTS, npart, main, [&] {
        return launch_build_lists(npart, g->d_pv.p, g->d_off.p, cur, g->d_mode.p, g->d_lbase.p, g->d_wbase.p,
                                  g->d_list.p, g->d_wpre.p, main);
    }));
    // 2. selection back to the host (Algorithm 1: copy Vc, p and A to host)
    HIP_CHECK(hipMemcpyAsync(g->h_sel.p, g->d_sel.p, sel_block_bytes(npart), hipMemcpyDeviceToHost, main));
    if (lanes) {
        // which lanes have a non-empty frontier this iteration
        HIP_CHECK(launch_fill_u32((uint32_t*)g->d_lanes.p, 2, 0u, main));
        HIP_CHECK(launch_lane_union(rc.mcur, n, (unsigned long long*)g->d_lanes.p, main));
        HIP_CHECK(hipMemcpyAsync(g->h_lanes.p, g->d_lanes.p, sizeof(uint64_t), hipMemcpyDeviceToHost, main));
    }
    HIP_CHECK(hipEventRecord(g->ev_sel[1], main));
    HIP_CHECK(hipStreamSynchronize(main));
    Totals& tt = rc.tot;
    tt.d2h += sizeof(Header) + npart * (1 + 4 + 8);
    const Header h = *g->h_hdr.p;
    *hout = h;
    float sel_ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&sel_ms, g->ev_sel[0], g->ev_sel[1]));
    tt.select_ms += sel_ms;
    if (lanes) *lanes = *g->h_lanes.p;
    if (stop_if_empty && h.frontier == 0) return HYTM_OK;

    // bookkeeping of the pass
    uint32_t scheduled = 0;
    for (int s = 0; s < NSEG; s++) {
        rec->parts[s + 1] += h.seg_parts[s];
        scheduled += h.seg_parts[s];
    }
    rec->parts[0] += npart - scheduled;
    rec->active_vertices += h.total_active;
    for (int s = 0; s < NSEG; s++) rec->active_edges += h.seg_edges[s];
    hytm_run_stats* stats = rc.stats;
    if (trace_t >= 0 && stats && stats->mode_trace && (uint64_t)(trace_t + 1) * npart <= stats->mode_trace_cap)
        memcpy(stats->mode_trace + (uint64_t)trace_t * npart, g->h_mode.p, npart);
    if (select_only) return HYTM_OK;

    // resident partitions: no transfer
    if (h.seg_list_count[SEG_R])
        HIP_CHECK(kt.run(HYTM_K_PUSH_RES, h.seg_work_total[SEG_R], main, [&] {
            return launch_push_edges(as, g->d_list.p, g->d_wpre.p, h.seg_list_start[SEG_R],
                                     h.seg_list_start[SEG_R] + h.seg_list_count[SEG_R], h.seg_work_start[SEG_R],
                                     h.seg_work_start[SEG_R] + h.seg_work_total[SEG_R], g->d_off.p, g->d_res_col.p,
                                     g->d_res_w.p, 0, false, main);
        }));
    // zero-copy: one kernel over all zero-copy vertices (Vz)
    if (h.seg_list_count[SEG_Z]) {
        HIP_CHECK(kt.run(HYTM_K_PUSH_ZC, h.seg_work_total[SEG_Z], g->s_zc, [&] {
            return launch_push_lines(as, g->d_list.p, g->d_wpre.p, h.seg_list_start[SEG_Z],
                                     h.seg_list_start[SEG_Z] + h.seg_list_count[SEG_Z], h.seg_work_start[SEG_Z],
                                     h.seg_work_start[SEG_Z] + h.seg_work_total[SEG_Z], g->d_off.p, g->d_col_map,
                                     g->d_w_map, (unsigned long long*)g->d_zcl.p, g->s_zc);
        }));
        rec->zc_lines += h.seg_work_total[SEG_Z];
    }
    // compaction: gathered by host threads, overlapping the filter tasks below
    std::thread cthread;
    hytm_status cst = HYTM_OK;
    std::string cmsg;
    uint64_t c_chunks = 0, c_bytes = 0, c_d2h = 0;
    if (h.seg_list_count[SEG_C])
        cthread = std::thread(run_compaction, &rc, h.seg_list_start[SEG_C], h.seg_list_count[SEG_C],
                              h.seg_work_start[SEG_C], h.seg_work_start[SEG_C] + h.seg_work_total[SEG_C], &c_chunks,
                              &c_bytes, &c_d2h, &cst, &cmsg);
    // filter: combine runs of <= k consecutive partitions (Sec. 5.2), then copy+push
    hytm_status fst = HYTM_OK;
    uint64_t f_bytes = 0;
    try {
        if (h.seg_list_count[SEG_F]) {
            const uint32_t k = g->params.combine_k;
            const uint64_t fend_list = h.seg_list_start[SEG_F] + h.seg_list_count[SEG_F];
            const uint64_t fend_work = h.seg_work_start[SEG_F] + h.seg_work_total[SEG_F];
            // the copy form keeps every task within one staging slot
            const uint64_t cap = fstream ? UINT64_MAX : pl.slot_edges;
            uint32_t gidx = 0;
            uint32_t i = 0;
            uint64_t chunks = 0;
            while (i < npart) {
                if (g->h_mode.p[i] != P_FILTER) {
                    i++;
                    continue;
                }
                // task = partitions [i, j): adjacent filter partitions, at most k
                uint32_t j = i + 1;
                uint64_t edges = g->pE[i];
                while (j < npart && j - i < k && g->h_mode.p[j] == P_FILTER && edges + g->pE[j] <= cap) {
                    edges += g->pE[j];
                    j++;
                }
                // list / work range of the task: up to the next filter partition's start
                uint32_t nx = j;
                while (nx < npart && g->h_mode.p[nx] != P_FILTER) nx++;
                const uint32_t ja = g->h_lbase.p[i];
                const uint32_t jb = nx < npart ? g->h_lbase.p[nx] : (uint32_t)fend_list;
                const uint64_t wa = g->h_wbase.p[i];
                const uint64_t wb = nx < npart ? g->h_wbase.p[nx] : fend_work;
                const uint64_t ebeg = g->h_off[g->pv[i]];
                f_bytes += edges * d1b;
                if (fstream) {
                    FTask& ft = g->h_tasks.p[gidx++];
                    ft.e0 = ebeg;
                    ft.e1 = ebeg + edges;
                    ft.ja = ja;
                    ft.jb = jb;
                    ft.chunk0 = chunks;
                    chunks += fstream_chunks(ft.e0, ft.e1);
                    i = j;
                    continue;
                }
                const uint32_t s = gidx % pl.nslots;
                if (gidx >= pl.nslots) HIP_CHECK(hipStreamWaitEvent(g->s_copy, g->ev_free[s], 0));
                HIP_CHECK(hipMemcpyAsync(g->d_slot_col[s].p, g->h_col + ebeg, edges * 4, hipMemcpyHostToDevice,
                                         g->s_copy));
                if (rc.arrays == 2)
                    HIP_CHECK(hipMemcpyAsync(g->d_slot_w[s].p, (const uint8_t*)g->h_w + ebeg * g->pk.wbytes,
                                             edges * g->pk.wbytes, hipMemcpyHostToDevice,
                                             g->s_copy));
                HIP_CHECK(hipEventRecord(g->ev_copied[s], g->s_copy));
                HIP_CHECK(hipStreamWaitEvent(g->s_fk, g->ev_copied[s], 0));
                HIP_CHECK(kt.run(HYTM_K_PUSH_F, wb - wa, g->s_fk, [&] {
                    return launch_push_edges(as, g->d_list.p, g->d_wpre.p, ja, jb, wa, wb, g->d_off.p,
                                             g->d_slot_col[s].p, g->d_slot_w[s].p, ebeg, false, g->s_fk);
                }));
                HIP_CHECK(hipEventRecord(g->ev_free[s], g->s_fk));
                gidx++;
                i = j;
            }
            rc.last_ftasks = fstream ? gidx : 0;
            rc.last_fchunks = fstream ? chunks : 0;
            if (fstream && gidx) {
                // one launch streams every filter task of the pass
                HIP_CHECK(hipMemcpyAsync(g->d_tasks.p, g->h_tasks.p, gidx * sizeof(FTask), hipMemcpyHostToDevice,
                                         g->s_fk));
                HIP_CHECK(kt.run(HYTM_K_PUSH_F, f_bytes / d1b, g->s_fk, [&] {
                    return launch_push_fstream(as, g->d_tasks.p, gidx, chunks, g->d_list.p, g->d_off.p,
                                               g->d_col_map, g->d_w_map, g->s_fk);
                }));
            }
            rec->filter_tasks += gidx;
        }
    } catch (const HipError& e) {
        fst = e.status;
    }
    if (cthread.joinable()) cthread.join();
    if (fst != HYTM_OK) return fst;
    if (cst != HYTM_OK) {
        g_err = cmsg;
        return cst;
    }
    rec->bytes_filter += f_bytes;
    rec->bytes_compact += c_bytes;
    tt.d2h += c_d2h;
    tt.cchunks += c_chunks;
    // 3. join every engine into the main stream
    HIP_CHECK(hipEventRecord(g->ev_join[0], g->s_fk));
    HIP_CHECK(hipEventRecord(g->ev_join[1], g->s_zc));
    HIP_CHECK(hipEventRecord(g->ev_join[2], g->s_c));
    for (int q = 0; q < 3; q++) HIP_CHECK(hipStreamWaitEvent(main, g->ev_join[q], 0));
    return HYTM_OK;
}

// Fold one iteration's record into the traversal's totals and the caller's stats.
void record_iteration(RunCtx& rc, hytm_iter_stats& rec, uint32_t t, double t_it) {
    Totals& tt = rc.tot;
    for (int s = 0; s < 5; s++) tt.part_iters[s] += rec.parts[s];
    tt.av += rec.active_vertices;
    tt.ae += rec.active_edges;
    tt.bf += rec.bytes_filter;
    tt.bc += rec.bytes_compact;
    tt.zcl += rec.zc_lines;
    tt.ftasks += rec.filter_tasks;
    rec.ms = now_ms() - t_it;
    hytm_run_stats* stats = rc.stats;
    if (stats && stats->iters && t < stats->iters_cap) {
        stats->iters[t] = rec;
        stats->iters_written = t + 1;
    }
}

// PageRank iterations after the first: the same pushes over the same lists and filter
// tasks, ordered after the main stream's prepare by an event instead of a host round trip.
hytm_status replay_pass(RunCtx& rc, hipStream_t main, hytm_iter_stats* rec, int64_t trace_t) {
    hytm_graph* g = rc.g;
    KTimer& kt = g->timer;
    AlgoState& as = rc.as;
    const uint32_t npart = g->npart;
    const Header& h = rc.replay.h;
    uint32_t scheduled = 0;
    for (int s = 0; s < NSEG; s++) {
        rec->parts[s + 1] += h.seg_parts[s];
        scheduled += h.seg_parts[s];
    }
    rec->parts[0] += npart - scheduled;
    rec->active_vertices += h.total_active;
    for (int s = 0; s < NSEG; s++) rec->active_edges += h.seg_edges[s];
    hytm_run_stats* stats = rc.stats;
    if (trace_t >= 0 && stats && stats->mode_trace && (uint64_t)(trace_t + 1) * npart <= stats->mode_trace_cap)
        memcpy(stats->mode_trace + (uint64_t)trace_t * npart, g->h_mode.p, npart);
    HIP_CHECK(hipEventRecord(g->ev_go, main));
    if (h.seg_list_count[SEG_R])
        HIP_CHECK(kt.run(HYTM_K_PUSH_RES, h.seg_work_total[SEG_R], main, [&] {
            return launch_push_edges(as, g->d_list.p, g->d_wpre.p, h.seg_list_start[SEG_R],
                                     h.seg_list_start[SEG_R] + h.seg_list_count[SEG_R], h.seg_work_start[SEG_R],
                                     h.seg_work_start[SEG_R] + h.seg_work_total[SEG_R], g->d_off.p, g->d_res_col.p,
                                     g->d_res_w.p, 0, false, main);
        }));
    if (h.seg_list_count[SEG_Z]) {
        HIP_CHECK(hipStreamWaitEvent(g->s_zc, g->ev_go, 0));
        HIP_CHECK(kt.run(HYTM_K_PUSH_ZC, h.seg_work_total[SEG_Z], g->s_zc, [&] {
            return launch_push_lines(as, g->d_list.p, g->d_wpre.p, h.seg_list_start[SEG_Z],
                                     h.seg_list_start[SEG_Z] + h.seg_list_count[SEG_Z], h.seg_work_start[SEG_Z],
                                     h.seg_work_start[SEG_Z] + h.seg_work_total[SEG_Z], g->d_off.p, g->d_col_map,
                                     g->d_w_map, (unsigned long long*)g->d_zcl.p, g->s_zc);
        }));
        rec->zc_lines += h.seg_work_total[SEG_Z];
    }
    if (rc.replay.ftasks) {
        HIP_CHECK(hipStreamWaitEvent(g->s_fk, g->ev_go, 0));
        HIP_CHECK(kt.run(HYTM_K_PUSH_F, rc.replay.fbytes / edge_bytes(g, rc.arrays), g->s_fk, [&] {
            return launch_push_fstream(as, g->d_tasks.p, rc.replay.ftasks, rc.replay.fchunks, g->d_list.p,
                                       g->d_off.p, g->d_col_map, g->d_w_map, g->s_fk);
        }));
        rec->filter_tasks += rc.replay.ftasks;
        rec->bytes_filter += rc.replay.fbytes;
    }
    HIP_CHECK(hipEventRecord(g->ev_join[0], g->s_fk));
    HIP_CHECK(hipEventRecord(g->ev_join[1], g->s_zc));
    for (int q = 0; q < 2; q++) HIP_CHECK(hipStreamWaitEvent(main, g->ev_join[q], 0));
    return HYTM_OK;
}

// ------------------------------------------------------ propagation blocking
// Workgroups of the streamed pushes beside the resident pieces.  Zero-copy line reads alone
// saturate the link from 128 workgroups of 256 threads up; the streamed PageRank pushes also
// wait on their atomic adds and need more, and every workgroup they hold is one the sorting
// passes lack.  Measured on MI355X, R-MAT 28 under an 8 GB budget, 20 steps, each engine on
// its own hardware queue and the streamed partitions read by the streaming filter: 192 ->
// 4.07 s, 256 -> 3.84-3.95 s, 320 -> 3.82-3.85 s, 384 -> 3.62-3.70 s, 448 -> 3.61 s, 512 ->
// 3.78 s, 768 -> 3.92 s, 1024 -> 4.08 s, 2048 -> 4.26 s.
constexpr uint32_t kPbLinkGrid = 384;

// PageRank's resident adds go through pair buckets (see PB_* in the kernel header) when it
// runs alone, some partitions are resident, the selection can contain no compaction
// partitions (their pushes are not replayed), filter partitions use the streaming engine,
// and the fine bins fit one LDS counting sort (n <= 2^24) or two sorting passes do
// (coarse bins, then fine bins: n <= 2^28).
constexpr bool kPbTwoPass = true;

// pr_blocking = 1 (automatic) also asks for at least 3/8 of the edges to be resident:
// below that the streamed atomics and the host link bound the iteration, and the sorting
// passes competing for CUs with the zero-copy kernel cost more than they save (measured on
// MI355X: a loss at 25% resident on R-MAT 24, 358 against 315 ms for 20 steps; a gain at
// 47% on R-MAT 28 under an 8 GB budget, 4.58 against 5.14 s).
bool pb_eligible(const RunCtx& rc) {
    const hytm_graph* g = rc.g;
    const uint32_t nfine = pb_fine_bins(g->n);
    const uint32_t nres = std::min(rc.plan.nres, g->npart);
    const bool wanted = g->params.pr_blocking == 2 || (g->params.pr_blocking == 1 && 8 * g->h_off[g->pv[nres]] >= 3 * g->m);
    return rc.algo == HYTM_PAGERANK && !rc.batched && wanted && g->m > 0 && rc.plan.nres > 0 &&
           nfine <= (kPbTwoPass ? PB_MAX_FINE : PB_LOCAL_BINS) && g->max_part_edges < (1ull << 31) &&
           g->n < (1ull << 31) && g->params.mode != HYTM_MODE_COMPACT &&
           g->params.filter_engine == HYTM_FILTER_STREAM;
}

// Pairs per piece buffer: by default one pair per vertex, so that a piece's bucket flushes
// (one read-modify-write of every accumulator slot) cost at most 8 bytes per pair; never
// less than the largest partition, never more than the resident edges.
uint64_t pb_capacity(const hytm_graph* g, uint64_t res_edges) {
    const uint64_t want = g->params.pr_block_pairs ? g->params.pr_block_pairs : std::max<uint64_t>(g->n, 1ull << 20);
    return std::max<uint64_t>(std::min<uint64_t>(std::max<uint64_t>(want, g->max_part_edges), res_edges), 1);
}

// Cut the resident partitions of the first iteration's selection into pieces, build the
// streaming filter tasks of the streamed partitions, and put the buffers and bucket plans
// in place.
hytm_status pb_plan(RunCtx& rc, const Header& h, hipStream_t main) {
    hytm_graph* g = rc.g;
    auto& pb = rc.pb;
    const uint32_t npart = g->npart;
    const uint8_t* md = g->h_mode.p;
    const uint32_t nres = std::min(rc.plan.nres, npart);
    pb.h = h;
    pb.cap = pb_capacity(g, g->h_off[g->pv[nres]]);
    pb.nfine = pb_fine_bins(g->n);
    pb.seg = pb_seg_len(pb.nfine, pb.cap);
    pb.max_segs = pb_max_segs(pb.nfine, pb.cap, pb.seg);
    pb.keys_a = pb.nfine > PB_LOCAL_BINS ? pb_coarse_bins(pb.nfine) : pb.nfine;
    pb.pieces.clear();
    pb.ftasks = 0;
    pb.fchunks = pb.fedges = 0;
    for (uint32_t p = 0; p < npart; p++) {
        if (md[p] == P_COMPACT) return fail(HYTM_E_STATE, "internal: compaction partition under PageRank blocking");
        if ((p < nres) != (md[p] == P_RES) && g->pE[p] > 0)
            return fail(HYTM_E_STATE, "internal: resident partitions are not the resident prefix");
    }
    // resident pieces: runs of partitions with at most cap edges
    uint64_t tj = 0;
    uint32_t pa = 0;
    while (pa < nres) {
        uint32_t pb_ = pa;
        uint64_t e = 0;
        while (pb_ < nres && (pb_ == pa || e + g->pE[pb_] <= pb.cap)) e += g->pE[pb_++];
        PbPiece pc;
        pc.e0 = g->h_off[g->pv[pa]];
        pc.cnt = g->h_off[g->pv[pb_]] - pc.e0;
        if (pc.cnt) {
            // the resident list holds the active vertices of the resident partitions in
            // order: the piece's entries run from its first resident partition's bases to
            // those of the next resident partition after it (or the segment's end)
            uint32_t p = pa;
            while (md[p] != P_RES) p++;  // a partition with edges is resident below nres
            pc.ja = g->h_lbase.p[p];
            pc.wa = g->h_wbase.p[p];
            uint32_t q = pb_;
            while (q < nres && md[q] != P_RES) q++;
            if (q < nres) {
                pc.jb = g->h_lbase.p[q];
                pc.wb = g->h_wbase.p[q];
            } else {
                pc.jb = h.seg_list_start[SEG_R] + h.seg_list_count[SEG_R];
                pc.wb = h.seg_work_start[SEG_R] + h.seg_work_total[SEG_R];
            }
            pc.tj = tj;
            tj += pb_tiles(pc.cnt);
            pb.pieces.push_back(pc);
        }
        pa = pb_;
    }
    // streamed filter partitions: tasks of <= k adjacent ones (Sec. 5.2), one launch per pass
    if (h.seg_list_count[SEG_F]) {
        g->h_tasks.ensure(npart);
        const uint32_t k = g->params.combine_k;
        const uint64_t fend_list = h.seg_list_start[SEG_F] + h.seg_list_count[SEG_F];
        uint32_t i = 0;
        while (i < npart) {
            if (md[i] != P_FILTER) {
                i++;
                continue;
            }
            uint32_t j = i + 1;
            uint64_t edges = g->pE[i];
            while (j < npart && j - i < k && md[j] == P_FILTER) edges += g->pE[j++];
            uint32_t nx = j;
            while (nx < npart && md[nx] != P_FILTER) nx++;
            FTask& ft = g->h_tasks.p[pb.ftasks++];
            ft.e0 = g->h_off[g->pv[i]];
            ft.e1 = ft.e0 + edges;
            ft.ja = g->h_lbase.p[i];
            ft.jb = nx < npart ? g->h_lbase.p[nx] : (uint32_t)fend_list;
            ft.chunk0 = pb.fchunks;
            pb.fchunks += fstream_chunks(ft.e0, ft.e1);
            pb.fedges += edges;
            i = j;
        }
        g->d_tasks.ensure(pb.ftasks);
        HIP_CHECK(hipMemcpyAsync(g->d_tasks.p, g->h_tasks.p, pb.ftasks * sizeof(FTask), hipMemcpyHostToDevice, main));
    }
    const uint32_t np = (uint32_t)pb.pieces.size();
    const uint32_t nbuf = std::min<uint32_t>(2, np);
    const bool two = pb.nfine > PB_LOCAL_BINS;  // the second pass writes destinations back
    for (uint32_t b = 0; b < nbuf; b++) {
        if (two) g->d_pb_v[b].ensure(pb.cap);
        g->d_pb_c[b].ensure(pb.cap);
    }
    g->d_pb_v[2].ensure(pb.cap);
    g->d_pb_c[2].ensure(pb.cap);
    g->d_pb_hist.ensure(pb.nfine);
    g->d_pb_foff.ensure((uint64_t)np * (pb.nfine + 1));
    g->d_pb_segs.ensure((uint64_t)np * 2 * pb.max_segs);
    g->d_pb_nsegs.ensure(std::max<uint32_t>(np, 1));
    g->d_pb_offa.ensure((uint64_t)np * pb_max_offa(pb.keys_a));
    g->d_pb_fcur.ensure(pb.nfine);
    g->d_pb_tj.ensure(std::max<uint64_t>(tj, 1));
    g->d_pb_err.ensure(1);
    HIP_CHECK(launch_fill_u32(g->d_pb_err.p, 1, 0u, main));
    return HYTM_OK;
}

// One PageRank push pass with propagation blocking over the resident partitions.  The
// streamed partitions are pushed as in every pass (zero-copy and streaming filter kernels
// with atomic adds into the per-XCD copies), while the resident pieces alternate between
// two buffers: a piece's push writes its contributions, then the bucketing stream sorts
// and sums the piece's pairs into the blocking copy and frees the buffer for the piece
// after next.  `first`: the bucket plans are counted (the same pairs recur every iteration).
hytm_status pb_pass(RunCtx& rc, hipStream_t main, hytm_iter_stats* rec, int64_t trace_t, bool first) {
    hytm_graph* g = rc.g;
    KTimer& kt = g->timer;
    const auto& pb = rc.pb;
    const Header& h = pb.h;
    const uint32_t npart = g->npart;
    if (!first) {
        uint32_t scheduled = 0;
        for (int s = 0; s < NSEG; s++) {
            rec->parts[s + 1] += h.seg_parts[s];
            scheduled += h.seg_parts[s];
        }
        rec->parts[0] += npart - scheduled;
        rec->active_vertices += h.total_active;
        for (int s = 0; s < NSEG; s++) rec->active_edges += h.seg_edges[s];
        hytm_run_stats* stats = rc.stats;
        if (trace_t >= 0 && stats && stats->mode_trace && (uint64_t)(trace_t + 1) * npart <= stats->mode_trace_cap)
            memcpy(stats->mode_trace + (uint64_t)trace_t * npart, g->h_mode.p, npart);
    }
    HIP_CHECK(hipEventRecord(g->ev_go, main));
    for (hipStream_t s : {g->s_c, g->s_zc, g->s_fk, g->s_pb}) HIP_CHECK(hipStreamWaitEvent(s, g->ev_go, 0));
    AlgoState& as = rc.as;
    // streamed partitions: atomic adds, at most at the host link's rate, from a grid that
    // keeps the link busy and leaves CUs to the resident pieces
    AlgoState al = as;
    al.link_grid = kPbLinkGrid;
    if (h.seg_list_count[SEG_Z]) {
        HIP_CHECK(kt.run(HYTM_K_PUSH_ZC, h.seg_work_total[SEG_Z], g->s_zc, [&] {
            return launch_push_lines(al, g->d_list.p, g->d_wpre.p, h.seg_list_start[SEG_Z],
                                     h.seg_list_start[SEG_Z] + h.seg_list_count[SEG_Z], h.seg_work_start[SEG_Z],
                                     h.seg_work_start[SEG_Z] + h.seg_work_total[SEG_Z], g->d_off.p, g->d_col_map,
                                     g->d_w_map, (unsigned long long*)g->d_zcl.p, g->s_zc);
        }));
        rec->zc_lines += h.seg_work_total[SEG_Z];
    }
    if (pb.ftasks) {
        HIP_CHECK(kt.run(HYTM_K_PUSH_F, pb.fedges, g->s_fk, [&] {
            return launch_push_fstream(al, g->d_tasks.p, pb.ftasks, pb.fchunks, g->d_list.p, g->d_off.p,
                                       g->d_col_map, g->d_w_map, g->s_fk);
        }));
        rec->filter_tasks += pb.ftasks;
        rec->bytes_filter += pb.fedges * 4;
    }
    // resident pieces
    const uint32_t nfine = pb.nfine;
    const bool two = nfine > PB_LOCAL_BINS;  // one pass when every fine bin fits the LDS sort
    const uint32_t shift_a = two ? PB_FINE_SHIFT + 5 : PB_FINE_SHIFT;
    const uint32_t stride_a = two ? PB_FINE_PER_COARSE : 1;
    float* acc_pb = as.acc + (uint64_t)as.acc_copies * acc_slots(g->n);  // the blocking copy
    hipStream_t sp = g->s_pb;
    uint32_t* err = g->d_pb_err.p;
    for (uint32_t pi = 0; pi < pb.pieces.size(); pi++) {
        const PbPiece& pc = pb.pieces[pi];
        const int buf = (int)(pi & 1);
        uint32_t* pv = g->d_pb_v[buf].p;
        float* pcv = g->d_pb_c[buf].p;
        if (pi >= 2) HIP_CHECK(hipStreamWaitEvent(g->s_c, g->ev_pbfree[buf], 0));  // summed already
        uint32_t* tjp = g->d_pb_tj.p + pc.tj;
        if (first) HIP_CHECK(launch_pb_tiles(g->d_wpre.p, pc.ja, pc.jb, pc.wa, pc.cnt, tjp, g->s_c));
        HIP_CHECK(kt.run(HYTM_K_PUSH_RES, pc.cnt, g->s_c, [&] {
            return launch_pb_expand(g->d_list.p, g->d_wpre.p, pc.jb, pc.wa, pc.cnt, tjp, as.contrib, pcv, g->s_c);
        }));
        HIP_CHECK(hipEventRecord(g->ev_pbpush, g->s_c));
        HIP_CHECK(hipStreamWaitEvent(sp, g->ev_pbpush, 0));
        uint32_t* foff = g->d_pb_foff.p + (uint64_t)pi * (nfine + 1);
        uint32_t* segs = g->d_pb_segs.p + (uint64_t)pi * 2 * pb.max_segs;
        uint32_t* nsegs = g->d_pb_nsegs.p + pi;
        uint32_t* offa = g->d_pb_offa.p + (uint64_t)pi * pb_max_offa(pb.keys_a);
        const uint32_t* in_v = g->d_res_col.p + pc.e0;  // destinations: the resident edge words
        const uint32_t vmask = g->pk.mask;
        HIP_CHECK(kt.run(HYTM_K_PR_BLOCK, pc.cnt, sp, [&]() -> hipError_t {
            hipError_t e;
            if (first) {
                if ((e = launch_fill_u32(g->d_pb_hist.p, nfine, 0u, sp)) != hipSuccess) return e;
                if ((e = launch_pb_hist(in_v, vmask, pc.cnt, nfine, g->d_pb_hist.p, err, sp)) != hipSuccess) return e;
                if ((e = launch_pb_plan(g->d_pb_hist.p, nfine, pb.seg, foff, segs, nsegs, sp)) != hipSuccess) return e;
                if ((e = launch_pb_plan_a(in_v, vmask, pc.cnt, shift_a, stride_a, nfine, foff, offa, err, sp)) !=
                    hipSuccess)
                    return e;
            }
            uint32_t* sv = g->d_pb_v[2].p;
            float* sc = g->d_pb_c[2].p;
            // first pass into the sort buffer (coarse bins, or fine bins when there is one pass)
            if ((e = launch_pb_scatter_a(in_v, vmask, pcv, pc.cnt, shift_a, stride_a, nfine, foff, offa, sv, sc,
                                         two ? g->d_pb_fcur.p : nullptr, err, sp)) != hipSuccess)
                return e;
            if (!two) return launch_pb_accum(sv, sc, foff, segs, nsegs, pb.max_segs, pb.seg, g->n, acc_pb, err, sp);
            // fine pass back into the piece buffer, then the sums
            if ((e = launch_pb_scatter(sv, sc, pc.cnt, PB_FINE_SHIFT, 1, nfine, foff, g->d_pb_fcur.p, pv, pcv, err,
                                       sp)) != hipSuccess)
                return e;
            return launch_pb_accum(pv, pcv, foff, segs, nsegs, pb.max_segs, pb.seg, g->n, acc_pb, err, sp);
        }));
        HIP_CHECK(hipEventRecord(g->ev_pbfree[buf], sp));
    }
    HIP_CHECK(hipEventRecord(g->ev_join[0], g->s_fk));
    HIP_CHECK(hipEventRecord(g->ev_join[1], g->s_zc));
    HIP_CHECK(hipEventRecord(g->ev_join[3], sp));
    for (int q : {0, 1, 3}) HIP_CHECK(hipStreamWaitEvent(main, g->ev_join[q], 0));
    return HYTM_OK;
}

// One iteration of a traversal.  *lanes_out: batched runs: the lanes with a non-empty
// frontier at the start of the iteration.  *empty_out: BFS/SSSP/CC only: the frontier was
// empty, nothing was pushed and the traversal is over.
hytm_status step_once(RunCtx& rc, hipStream_t main, uint64_t* lanes_out, bool* empty_out) {
    hytm_graph* g = rc.g;
    KTimer& kt = g->timer;
    AlgoState& as = rc.as;
    const uint64_t n = g->n;
    const uint32_t t = rc.t;
    const bool fixed_steps = rc.algo == HYTM_PAGERANK || rc.algo == HYTM_PPR;
    const double t_it = now_ms();
    const uint32_t copies = rc.pb_on ? as.acc_copies + 1 : as.acc_copies;  // + the blocking copy
    if (rc.algo == HYTM_PAGERANK)
        HIP_CHECK(kt.run(HYTM_K_OTHER, n, main, [&] {
            return launch_pr_prepare(n, g->d_off.p, g->d_x.p, g->d_contrib.p, g->d_acc.p, copies, main);
        }));
    if (rc.algo == HYTM_PPR)
        HIP_CHECK(kt.run(HYTM_K_OTHER, n, main, [&] { return launch_ppr_prepare(as, g->d_off.p, main); }));
    as.level_next = t + 1;
    hytm_iter_stats rec{};
    Header h;
    *lanes_out = 0;
    *empty_out = false;
    hytm_status st;
    if (rc.pb.ok) {
        st = pb_pass(rc, main, &rec, t, false);
        h = rc.pb.h;
    } else if (rc.pb_on) {
        st = engine_pass(rc, rc.cur, main, &h, nullptr, false, &rec, t, true);
        if (st == HYTM_OK) st = pb_plan(rc, h, main);
        if (st == HYTM_OK) {
            rc.pb.ok = true;
            st = pb_pass(rc, main, &rec, t, true);
        }
    } else if (rc.replay.ok) {
        st = replay_pass(rc, main, &rec, t);
        h = rc.replay.h;
    } else {
        st = engine_pass(rc, rc.cur, main, &h, rc.batched ? lanes_out : nullptr, !fixed_steps, &rec, t);
        // PageRank with every engine but compaction (whose host gather needs the host each
        // iteration), or with the copy-form filter (its per-task copies are host calls),
        // replays this selection from now on
        if (st == HYTM_OK && rc.algo == HYTM_PAGERANK && h.seg_list_count[SEG_C] == 0 &&
            (h.seg_list_count[SEG_F] == 0 || g->params.filter_engine == HYTM_FILTER_STREAM)) {
            rc.replay.ok = true;
            rc.replay.h = h;
            rc.replay.ftasks = rc.last_ftasks;
            rc.replay.fchunks = rc.last_fchunks;
            rc.replay.fbytes = rec.bytes_filter;
        }
    }
    if (st != HYTM_OK) return st;
    if (!fixed_steps && h.frontier == 0) {
        *empty_out = true;
        return HYTM_OK;
    }
    rc.tot.iters++;
    if (rc.reprocess) {
        // Sec. 6.1: the partitions just loaded are processed once more, from the vertices
        // the first pass improved; those stay in the next frontier
        HIP_CHECK(kt.run(HYTM_K_OTHER, g->npart, main, [&] {
            // reprocess 1: every loaded partition; 2: only those whose lists cost no host
            // transfer or only their own lines again (resident, zero-copy)
            const uint32_t mask = g->params.reprocess == 2
                                      ? (1u << P_RES) | (1u << P_ZC)
                                      : (1u << P_RES) | (1u << P_FILTER) | (1u << P_ZC) | (1u << P_COMPACT);
            return launch_loaded_frontier(g->npart, g->d_pv.p, g->d_mode.p, mask, rc.nxt, g->d_cur2.p, rc.nwords,
                                          main);
        }));
        Header h2;
        st = engine_pass(rc, g->d_cur2.p, main, &h2, nullptr, true, &rec, -1);
        if (st != HYTM_OK) return st;
    }
    if (rc.algo == HYTM_PAGERANK) {
        const float base = (float)((1.0 - g->params.pr_damping) / (double)n);
        const float d = (float)g->params.pr_damping;
        const float restart = (float)(1.0 - g->params.pr_damping);
        HIP_CHECK(kt.run(HYTM_K_OTHER, n, main, [&] {
            return launch_pr_apply(n, g->d_x.p, g->d_acc.p, copies, base, d, as.inv_n, restart, main);
        }));
    } else {
        if (rc.algo == HYTM_PPR) {
            const float d = (float)g->params.pr_damping;
            const float restart = (float)(1.0 - g->params.pr_damping);
            HIP_CHECK(kt.run(HYTM_K_OTHER, n, main, [&] { return launch_ppr_apply(as, d, main); }));
            HIP_CHECK(kt.run(HYTM_K_OTHER, 1, main, [&] { return launch_ppr_restart(as, rc.ppr, restart, main); }));
        }
        std::swap(rc.cur, rc.nxt);
        as.next = rc.nxt;
        HIP_CHECK(kt.run(HYTM_K_OTHER, rc.nwords, main, [&] { return launch_fill_u32(rc.nxt, rc.nwords, 0u, main); }));
        if (rc.batched) {
            std::swap(rc.mcur, rc.mnxt);
            as.mcur = rc.mcur;
            as.mnext = rc.mnxt;
            HIP_CHECK(kt.run(HYTM_K_OTHER, n, main,
                             [&] { return launch_fill_u32((uint32_t*)rc.mnxt, 2 * n, 0u, main); }));
        }
    }
    record_iteration(rc, rec, t, t_it);
    rc.t++;
    return HYTM_OK;
}

// Delta-based PageRank to convergence (Sec. 6.1, delta-driven priority): one iteration
// folds the pushed deltas in, reads the per-partition delta sums, schedules the partitions
// at or above the mean and pushes their vertices' deltas (twice with reprocessing).
// Returns the final total delta in *residual; x holds x + delta on return.
hytm_status run_delta_pagerank(RunCtx& rc, hipStream_t main, double* residual) {
    hytm_graph* g = rc.g;
    KTimer& kt = g->timer;
    const uint64_t n = g->n;
    const uint32_t npart = g->npart;
    const float d = (float)g->params.pr_damping;
    const uint32_t passes = rc.reprocess ? 2 : 1;
    double total = 0;
    for (;;) {
        const double t_it = now_ms();
        HIP_CHECK(kt.run(HYTM_K_OTHER, n, main, [&] {
            return launch_dpr_fold(npart, g->d_pv.p, n, g->d_acc.p, rc.as.acc_copies, g->d_delta.p, g->d_psum.p, main);
        }));
        HIP_CHECK(hipMemcpyAsync(g->h_psum.p, g->d_psum.p, npart * sizeof(double), hipMemcpyDeviceToHost, main));
        HIP_CHECK(hipStreamSynchronize(main));
        rc.tot.d2h += npart * sizeof(double);
        total = 0;
        for (uint32_t p = 0; p < npart; p++) total += g->h_psum.p[p];
        if (!(total > g->params.dpr_epsilon) || rc.t >= g->params.dpr_max_iterations) break;
        // delta-driven priority: the partitions holding at least the mean pending delta
        const double mean = total / npart;
        for (uint32_t p = 0; p < npart; p++) g->h_sched.p[p] = g->h_psum.p[p] > 0 && g->h_psum.p[p] >= mean;
        HIP_CHECK(hipMemcpyAsync(g->d_sched.p, g->h_sched.p, npart, hipMemcpyHostToDevice, main));
        hytm_iter_stats rec{};
        for (uint32_t pass = 0; pass < passes; pass++) {
            if (pass)
                HIP_CHECK(kt.run(HYTM_K_OTHER, n, main, [&] {
                    return launch_dpr_fold(npart, g->d_pv.p, n, g->d_acc.p, rc.as.acc_copies, g->d_delta.p, g->d_psum.p, main);
                }));
            HIP_CHECK(kt.run(HYTM_K_OTHER, n, main, [&] {
                return launch_dpr_activate(npart, g->d_pv.p, g->d_off.p, g->d_sched.p, g->d_delta.p, g->d_x.p,
                                           g->d_contrib.p, rc.cur, rc.nwords, d, main);
            }));
            Header h;
            hytm_status st = engine_pass(rc, rc.cur, main, &h, nullptr, true, &rec, pass ? -1 : (int64_t)rc.t);
            if (st != HYTM_OK) return st;
        }
        rc.tot.iters++;
        record_iteration(rc, rec, rc.t, t_it);
        rc.t++;
    }
    HIP_CHECK(kt.run(HYTM_K_OTHER, n, main, [&] { return launch_dpr_finish(n, g->d_x.p, g->d_delta.p, main); }));
    *residual = total;
    return HYTM_OK;
}

// Lane rows of a batched traversal: the power of two >= lanes.
uint32_t lane_shift(uint32_t lanes) {
    uint32_t sh = 0;
    while ((1u << sh) < lanes) sh++;
    return sh;
}

// Copy the lanes of `set` (values of n vertices each, in rows of 2^lshift) into
// consecutive n-value rows of the host buffer `out`, EXTRACT_LANES lanes per device pass.
constexpr uint32_t EXTRACT_LANES = 8;
void copy_lanes_out(hytm_graph* g, const uint32_t* vals, uint32_t lshift, const LaneSet& set, bool sub_base,
                    void* const* outs, hipStream_t main) {
    const uint64_t n = g->n;
    g->d_xout.ensure(n * EXTRACT_LANES);
    uint64_t rest = set.mask;
    uint32_t k = 0;
    while (rest) {
        LaneSet part = set;
        part.mask = 0;
        for (uint32_t c = 0; c < EXTRACT_LANES && rest; c++) {
            part.mask |= rest & (~rest + 1);
            rest &= rest - 1;
        }
        HIP_CHECK(launch_extract_lanes(vals, n, lshift, part, sub_base, g->hub_sorted() ? g->d_order.p : nullptr,
                                       g->d_xout.p, main));
        const uint32_t cnt = (uint32_t)__builtin_popcountll(part.mask);
        for (uint32_t c = 0; c < cnt; c++)
            HIP_CHECK(hipMemcpyAsync(outs[k + c], g->d_xout.p + (uint64_t)c * n, n * 4, hipMemcpyDeviceToHost, main));
        // the staging rows are reused by the next pass
        HIP_CHECK(hipStreamSynchronize(main));
        k += cnt;
    }
}

// One run.  lanes == 0: single source `sources[0]` (BFS/SSSP) or none (CC/PR), values_out
// holds n values, iterations_out one count.  lanes in 1..64: batched BFS/SSSP/PPR from
// sources[0..lanes), values_out holds lanes rows of n values, iterations_out one count per
// lane (the non-empty frontiers of that lane; PPR: its steps).
// SSSP with sssp_delta, once the frontier is empty: the bound rises to the smallest multiple
// of sssp_delta above the smallest distance waiting in the far set, and the far vertices
// below it become the frontier.  *more = false when nothing waits (the run is over).
hytm_status far_advance(RunCtx& rc, hipStream_t main, bool* more) {
    hytm_graph* g = rc.g;
    KTimer& kt = g->timer;
    HIP_CHECK(launch_fill_u32(g->d_farmin.p, 1, 0xFFFFFFFFu, main));
    HIP_CHECK(kt.run(HYTM_K_OTHER, rc.nwords, main, [&] {
        return launch_far_min(g->d_far.p, g->d_val.p, rc.nwords, g->d_farmin.p, main);
    }));
    HIP_CHECK(hipMemcpyAsync(g->h_farmin.p, g->d_farmin.p, sizeof(uint32_t), hipMemcpyDeviceToHost, main));
    HIP_CHECK(hipStreamSynchronize(main));
    rc.tot.d2h += sizeof(uint32_t);
    const uint32_t lo = *g->h_farmin.p;
    *more = lo != 0xFFFFFFFFu;
    if (!*more) return HYTM_OK;
    const uint64_t delta = g->params.sssp_delta;
    rc.as.bound = (uint32_t)std::min<uint64_t>((lo / delta + 1) * delta, 0xFFFFFFFFull);
    HIP_CHECK(kt.run(HYTM_K_OTHER, rc.nwords, main, [&] {
        return launch_far_move(g->d_far.p, g->d_val.p, rc.cur, rc.nwords, rc.as.bound, main);
    }));
    return HYTM_OK;
}

// SSSP overflow.  The push skips a candidate distance of 2^32-1 or more and raises its
// lane's flag; the flagged lanes whose converged distances leave an unreached vertex next
// to a reached one are those whose shortest distances do not all fit in uint32 (the
// oracle's rule: only a final distance decides).  Returns those lanes.
uint64_t sssp_overflow_lanes(hytm_graph* g, const uint32_t* dist, uint32_t lshift, uint64_t flagged, hipStream_t main) {
    if (!flagged) return 0;
    g->d_ovf.ensure(1);
    HIP_CHECK(launch_fill_u32((uint32_t*)g->d_ovf.p, 2, 0u, main));
    HIP_CHECK(launch_sssp_ovf_check(g->d_off.p, g->d_col_map, g->pk, dist, lshift, flagged, g->n,
                                    (unsigned long long*)g->d_ovf.p, main));
    uint64_t out = 0;
    HIP_CHECK(hipMemcpyAsync(&out, g->d_ovf.p, sizeof(out), hipMemcpyDeviceToHost, main));
    HIP_CHECK(hipStreamSynchronize(main));
    return out;
}

hytm_status run_impl(hytm_graph* g, hytm_algo algo, const uint32_t* sources, uint32_t lanes, void* values_out,
                     uint32_t* iterations_out, hytm_run_stats* stats, void* hip_stream) {
    HIP_CHECK(hipSetDevice(g->device));
    ensure_streams(g);
    const double t_begin = now_ms();
    const uint32_t arrays = edge_arrays(g, algo);
    const bool batched = lanes > 0;
    const uint32_t source = sources ? g->inner(sources[0]) : 0;
    hipStream_t main = hip_stream ? (hipStream_t)hip_stream : g->s_main;
    KTimer& kt = g->timer;
    kt.on = stats && stats->time_kernels;
    kt.recs.clear();
    kt.used = 0;

    RunCtx rc;
    Plan pl;
    hytm_status ps = prepare_graph(g, arrays, main, &pl, &rc.tot);
    if (ps != HYTM_OK) return ps;
    HIP_CHECK(hipEventRecord(g->ev_start, main));
    HIP_CHECK(launch_fill_u32((uint32_t*)g->d_zcl.p, 2, 0u, main));
    init_ctx(rc, g, algo, batched, pl, stats);
    rc.pb_on = pb_eligible(rc);
    rc.sp.zc_tie = resolve_tie(g, algo, rc.pb_on);
    rc.as.acc_copies = pr_acc_copies(rc.pb_on);

    const uint64_t n = g->n;
    const uint32_t nwords = rc.nwords;
    const uint32_t lsh = batched ? lane_shift(lanes) : 0;
    // vertex-associated device state (outside the budget)
    g->d_cur.ensure(nwords);
    g->d_next.ensure(nwords);
    rc.reprocess = g->params.reprocess && !batched &&
                   (algo == HYTM_BFS || algo == HYTM_SSSP || algo == HYTM_CC || algo == HYTM_PAGERANK_DELTA);
    const bool pr_like = algo == HYTM_PAGERANK || algo == HYTM_PAGERANK_DELTA;
    if (!batched) g->d_val.ensure(n);
    if (algo == HYTM_BFS && !batched && !rc.reprocess) g->d_visited.ensure(nwords);
    if (pr_like) {
        g->d_x.ensure(n);
        g->d_contrib.ensure(n);
        g->d_acc.ensure((rc.as.acc_copies + 1) * acc_slots(n));  // the adds' copies + the blocking copy
    }
    if (algo == HYTM_PAGERANK_DELTA) {
        g->d_delta.ensure(n);
        g->d_psum.ensure(g->npart);
        g->h_psum.ensure(g->npart);
        g->d_sched.ensure(g->npart);
        g->h_sched.ensure(g->npart);
    }
    if (rc.reprocess) g->d_cur2.ensure(nwords);
    const bool near_far = algo == HYTM_SSSP && !batched && g->params.sssp_delta > 0;
    if (near_far) {
        g->d_far.ensure(nwords);
        g->d_farmin.ensure(1);
        g->h_farmin.ensure(1);
        HIP_CHECK(launch_fill_u32(g->d_far.p, nwords, 0u, main));
    }
    if (batched) {
        g->d_mcur.ensure(n);
        g->d_mnext.ensure(n);
        if (algo == HYTM_BFS) g->d_mvis.ensure(n);
        if (algo == HYTM_PPR) {
            g->d_lx.ensure(n << lsh);
            g->d_lacc.ensure(n << lsh);
        } else {
            g->d_lval.ensure(n << lsh);
        }
    }

    AlgoState& as = rc.as;
    as.algo = batched                                   ? (algo == HYTM_BFS ? ALGO_MBFS : algo == HYTM_SSSP ? ALGO_MSSSP : ALGO_MPPR)
              : algo == HYTM_PAGERANK_DELTA              ? ALGO_PR
              : (algo == HYTM_BFS && rc.reprocess)       ? ALGO_BFS_RELAX
                                                         : (int)algo;
    as.val = g->d_val.p;
    as.visited = (algo == HYTM_BFS && !batched && !rc.reprocess) ? g->d_visited.p : nullptr;
    as.next = pr_like ? nullptr : g->d_next.p;
    as.acc = g->d_acc.p;
    as.contrib = g->d_contrib.p;
    as.inv_n = g->d_inv_n.p;  // null unless the graph is a union of graphs
    if (near_far) {
        as.far = g->d_far.p;
        as.bound = g->params.sssp_delta;  // the source's distance 0 lies below it
    }
    rc.cur = g->d_cur.p;
    rc.nxt = g->d_next.p;
    if (batched) {
        rc.mcur = g->d_mcur.p;
        rc.mnxt = g->d_mnext.p;
        as.mcur = rc.mcur;
        as.mnext = rc.mnxt;
        as.mvisited = algo == HYTM_BFS ? g->d_mvis.p : nullptr;
        as.lval = algo == HYTM_PPR ? nullptr : g->d_lval.p;
        as.lx = algo == HYTM_PPR ? g->d_lx.p : nullptr;
        as.lacc = algo == HYTM_PPR ? g->d_lacc.p : nullptr;
        as.lshift = lsh;
        LaneSources ls{};
        ls.count = lanes;
        for (uint32_t l = 0; l < lanes; l++) ls.src[l] = g->inner(sources[l]);
        HIP_CHECK(kt.run(HYTM_K_OTHER, n, main, [&] { return launch_init_lanes(as, ls, rc.cur, nwords, main); }));
        rc.ppr.mask = lanes == 64 ? ~0ull : (1ull << lanes) - 1;
        for (uint32_t l = 0; l < lanes; l++) rc.ppr.src[l] = ls.src[l];
    } else if (algo == HYTM_PAGERANK_DELTA) {
        // x = 0, every vertex holds delta = (1 - d) / n (n of its own graph), nothing pushed yet
        HIP_CHECK(launch_fill_u32((uint32_t*)g->d_x.p, n, 0u, main));
        HIP_CHECK(launch_dpr_init(n, g->d_delta.p, as.inv_n, (float)(1.0 - g->params.pr_damping), main));
        HIP_CHECK(launch_fill_u32((uint32_t*)g->d_acc.p, rc.as.acc_copies * acc_slots(n), 0u, main));
    } else {
        const float x0 = n ? (float)(1.0 / (double)n) : 0.f;
        HIP_CHECK(kt.run(HYTM_K_OTHER, n, main,
                         [&] { return launch_init(as, n, source, x0, g->d_x.p, rc.cur, nwords, main); }));
    }
    uint32_t lane_iters[MAX_LANES] = {};
    const uint32_t T = algo == HYTM_PAGERANK ? g->params.pr_iterations
                       : algo == HYTM_PPR    ? g->params.ppr_iterations
                                             : UINT32_MAX;
    double residual = 0;
    if (algo == HYTM_PAGERANK_DELTA) {
        hytm_status st = run_delta_pagerank(rc, main, &residual);
        if (st != HYTM_OK) return st;
    }
    while (algo != HYTM_PAGERANK_DELTA && rc.t < T) {
        uint64_t active = 0;
        bool empty = false;
        hytm_status st = step_once(rc, main, &active, &empty);
        if (st != HYTM_OK) return st;
        if (empty && near_far) {
            bool more = false;
            if ((st = far_advance(rc, main, &more)) != HYTM_OK) return st;
            if (more) continue;
        }
        if (empty) break;
        for (uint32_t l = 0; l < lanes; l++) lane_iters[l] += (uint32_t)((active >> l) & 1);
    }
    HIP_CHECK(hipStreamSynchronize(main));
    if (rc.pb.ok) {
        uint32_t perr = 0;
        HIP_CHECK(hipMemcpy(&perr, g->d_pb_err.p, sizeof(perr), hipMemcpyDeviceToHost));
        if (perr) return fail(HYTM_E_DEVICE, "internal: PageRank pair buckets did not match the pushed pairs");
    }
    if (algo == HYTM_SSSP) {
        uint32_t of[2] = {0, 0};
        HIP_CHECK(hipMemcpy(of, g->d_overflow.p, sizeof(of), hipMemcpyDeviceToHost));
        const uint64_t flagged = batched ? ((uint64_t)of[0] | ((uint64_t)of[1] << 32)) & rc.ppr.mask : (of[0] ? 1ull : 0ull);
        if (sssp_overflow_lanes(g, batched ? g->d_lval.p : g->d_val.p, batched ? lsh : 0, flagged, main))
            return fail(HYTM_E_RANGE, "an SSSP distance reaches 2^32-1 and does not fit in uint32");
    }
    if (batched) {
        // lane l of the value rows -> row l of the caller's buffer
        LaneSet all{};
        all.mask = rc.ppr.mask;
        std::vector<void*> outs(lanes);
        for (uint32_t l = 0; l < lanes; l++) outs[l] = (uint32_t*)values_out + (uint64_t)l * n;
        const uint32_t* vals = algo == HYTM_PPR ? (const uint32_t*)g->d_lx.p : g->d_lval.p;
        copy_lanes_out(g, vals, lsh, all, false, outs.data(), main);
    } else {
        const uint32_t* src = pr_like ? (const uint32_t*)g->d_x.p : g->d_val.p;
        if (g->hub_sorted()) {
            // back to the caller's ids (CC: labels become the smallest original id)
            g->d_xout.ensure(n);
            if (algo == HYTM_CC) {
                g->d_minold.ensure(n);
                HIP_CHECK(launch_cc_relabel(src, g->d_order.p, g->d_rank.p, n, g->d_minold.p, g->d_xout.p, main));
            } else {
                HIP_CHECK(launch_gather_u32(src, g->d_rank.p, n, g->d_xout.p, main));
            }
            src = g->d_xout.p;
        }
        HIP_CHECK(hipMemcpyAsync(values_out, src, n * 4, hipMemcpyDeviceToHost, main));
    }
    HIP_CHECK(hipStreamSynchronize(main));
    const double t_end = now_ms();
    if (iterations_out) {
        if (batched)
            for (uint32_t l = 0; l < lanes; l++) iterations_out[l] = lane_iters[l];
        else
            *iterations_out = rc.tot.iters;
    }
    if (stats) {
        if (kt.on) {
            // every engine joined the main stream before it was synchronised above
            for (int c = 0; c < kClasses; c++) {
                stats->kernel_ms[c] = 0;
                stats->kernel_launches[c] = 0;
                stats->kernel_items[c] = 0;
            }
            kt.collect(stats->kernel_ms, stats->kernel_launches, stats->kernel_items);
            kt.on = false;
        }
        const Totals& tt = rc.tot;
        stats->iterations = tt.iters;
        stats->npart = g->npart;
        stats->nres = pl.nres;
        for (int s = 0; s < 5; s++) stats->part_iters[s] = tt.part_iters[s];
        stats->active_vertices = tt.av;
        stats->active_edges = tt.ae;
        stats->bytes_filter = tt.bf;
        stats->bytes_compact = tt.bc;
        uint64_t zcd = 0;
        HIP_CHECK(hipMemcpy(&zcd, g->d_zcl.p, sizeof(zcd), hipMemcpyDeviceToHost));
        stats->zc_lines = tt.zcl;
        stats->zc_lines_distinct = zcd;
        stats->bytes_zerocopy = zcd * 32 * edge_bytes(g, arrays);  // 32 edges of d1 bytes per zero-copy line
        stats->bytes_d2h = tt.d2h;
        stats->bytes_resident_fill = tt.fill_bytes;
        stats->filter_tasks = tt.ftasks;
        stats->compact_chunks = tt.cchunks;
        stats->ms_total = t_end - t_begin;
        stats->ms_fill = tt.fill_ms;
        stats->ms_select = tt.select_ms;
        stats->residual = residual;
    }
    return HYTM_OK;
}

template <class F>
hytm_status guarded(F&& f) {
    try {
        return f();
    } catch (const HipError& e) {
        return e.status;
    } catch (const std::bad_alloc&) {
        return fail(HYTM_E_NOMEM, "host allocation failed");
    }
}

}  // namespace

// ============================================================== query server
namespace {

struct Query {
    int algo = 0;
    uint32_t source = 0;
    void* out = nullptr;
    double t_submit = 0, t_admit = 0, t_done = 0;
    uint32_t iterations = 0;
    hytm_status status = HYTM_OK;
    std::string msg;
    bool done = false;
};

// The lanes of one algorithm: own frontier bitmaps, lane masks and value rows; the
// graph's scratch and engines are shared with the other groups.
struct LaneGroup {
    int algo = -1;  // hytm_algo; -1 = no group
    uint32_t lanes = 0, lshift = 0;
    RunCtx rc;
    DevBuf<uint32_t> cur, nxt, lval;
    DevBuf<uint64_t> mcur, mnxt, mvis;
    DevBuf<float> lx;
    DevBuf<double> lacc;
    uint64_t occupied = 0;  // lanes holding a query (changed by the worker only, under the lock)
    uint64_t fresh = 0;     // lanes admitted since the last step
    double vtime = 0;       // worker time spent on this group (fair sharing between groups)
    bool was_busy = false;
    std::shared_ptr<Query> q[MAX_LANES];
    uint32_t src[MAX_LANES] = {}, base[MAX_LANES] = {}, iters[MAX_LANES] = {}, left[MAX_LANES] = {};

    uint64_t all() const { return lanes == 64 ? ~0ull : (1ull << lanes) - 1; }
    void release() {
        for (auto* b : {&cur, &nxt, &lval}) b->release();
        for (auto* b : {&mcur, &mnxt, &mvis}) b->release();
        lx.release();
        lacc.release();
    }
};

int group_index(int algo) { return algo == HYTM_BFS ? 0 : algo == HYTM_SSSP ? 1 : algo == HYTM_PPR ? 2 : -1; }

uint64_t group_state_bytes(uint64_t n, int algo, uint32_t lanes) {
    const uint64_t rows = n << lane_shift(lanes);
    uint64_t b = 2 * ((n + 31) / 32) * 4 + 2 * n * 8;  // union bitmaps, lane masks
    if (algo == HYTM_BFS) b += n * 8;                   // lanes that reached each vertex
    return b + rows * (algo == HYTM_PPR ? 4 + 8 : 4);  // PPR: FP32 x and FP64 accumulators
}

}  // namespace

struct hytm_server {
    hytm_graph* g = nullptr;
    hytm_server_config cfg{};
    LaneGroup grp[3];  // BFS, SSSP, PPR
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Query>> pending;
    std::unordered_map<uint64_t, std::shared_ptr<Query>> tickets;
    uint64_t next_ticket = 1;
    bool stop = false;
    hytm_status fatal = HYTM_OK;
    std::string fatal_msg;
    std::thread worker;
};

namespace {

// Hand the values of the lanes in `mask` to their queries and free the lanes.
void retire_lanes(hytm_server* s, LaneGroup& gr, uint64_t mask, hipStream_t main) {
    hytm_graph* g = s->g;
    uint64_t over = 0;
    if (gr.algo == HYTM_SSSP) {
        HIP_CHECK(hipStreamSynchronize(main));
        uint32_t of[2] = {0, 0};
        HIP_CHECK(hipMemcpy(of, g->d_overflow.p, sizeof(of), hipMemcpyDeviceToHost));
        over = sssp_overflow_lanes(g, gr.lval.p, gr.lshift, ((uint64_t)of[0] | ((uint64_t)of[1] << 32)) & mask, main);
    }
    LaneSet set{};
    set.mask = mask & ~over;
    void* outs[MAX_LANES];
    uint32_t k = 0;
    for (uint64_t m = set.mask; m; m &= m - 1) {
        const uint32_t l = (uint32_t)__builtin_ctzll(m);
        set.base[l] = gr.base[l];
        outs[k++] = gr.q[l]->out;
    }
    if (set.mask) {
        const uint32_t* vals = gr.algo == HYTM_PPR ? (const uint32_t*)gr.lx.p : gr.lval.p;
        copy_lanes_out(g, vals, gr.lshift, set, gr.algo == HYTM_BFS, outs, main);
    }
    HIP_CHECK(launch_reset_lanes(gr.rc.as, mask, main));
    const double now = now_ms();
    std::lock_guard<std::mutex> lk(s->mu);
    for (uint64_t m = mask; m; m &= m - 1) {
        const uint32_t l = (uint32_t)__builtin_ctzll(m);
        Query& q = *gr.q[l];
        q.iterations = gr.iters[l];
        if ((over >> l) & 1) {
            q.status = HYTM_E_RANGE;
            q.msg = "an SSSP distance reaches 2^32-1 and does not fit in uint32";
        }
        q.t_done = now;
        q.done = true;
        gr.q[l].reset();
    }
    gr.occupied &= ~mask;
    s->cv_done.notify_all();
}

// The worker: admit queued queries into free lanes, step every group that holds
// queries by one iteration, retire the lanes whose traversal ended.
void serve_loop(hytm_server* s) {
    hytm_graph* g = s->g;
    hipStream_t main = g->s_main;
    hytm_status st = HYTM_OK;
    try {
        HIP_CHECK(hipSetDevice(g->device));
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(s->mu);
                auto busy = [&] { return (s->grp[0].occupied | s->grp[1].occupied | s->grp[2].occupied) != 0; };
                s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty() || busy(); });
                if (s->pending.empty() && !busy()) break;  // stopped and drained
                // oldest first, each into the lowest free lane of its group
                const double now = now_ms();
                for (auto it = s->pending.begin(); it != s->pending.end();) {
                    LaneGroup& gr = s->grp[group_index((*it)->algo)];
                    const uint64_t free_lanes = gr.all() & ~gr.occupied;
                    if (!free_lanes) {
                        ++it;
                        continue;
                    }
                    const uint32_t l = (uint32_t)__builtin_ctzll(free_lanes);
                    gr.occupied |= 1ull << l;
                    gr.fresh |= 1ull << l;
                    gr.q[l] = *it;
                    gr.src[l] = (*it)->source;
                    gr.base[l] = gr.rc.t;
                    gr.iters[l] = 0;
                    gr.left[l] = g->params.ppr_iterations;
                    (*it)->t_admit = now;
                    it = s->pending.erase(it);
                }
            }
            // Fair sharing: step only the busy group that has used the least worker time, so
            // short BFS/SSSP steps interleave with long dense PPR steps instead of waiting
            // behind them; a group that turns busy starts at the current minimum.
            double base = 1e300;
            for (const LaneGroup& gr : s->grp)
                if (gr.was_busy && gr.occupied) base = std::min(base, gr.vtime);
            LaneGroup* pick = nullptr;
            for (LaneGroup& gr : s->grp) {
                if (!gr.occupied) {
                    gr.was_busy = false;
                    continue;
                }
                if (!gr.was_busy && base < 1e300) gr.vtime = std::max(gr.vtime, base);
                gr.was_busy = true;
                if (!pick || gr.vtime < pick->vtime) pick = &gr;
            }
            for (LaneGroup* pg : {pick}) {
                if (!pg) continue;
                LaneGroup& gr = *pg;
                struct Clock {
                    double& acc;
                    double t0 = now_ms();
                    ~Clock() { acc += now_ms() - t0; }
                } clock{gr.vtime};
                if (gr.fresh) {
                    LaneSet set{};
                    set.mask = gr.fresh;
                    for (uint64_t m = gr.fresh; m; m &= m - 1) {
                        const uint32_t l = (uint32_t)__builtin_ctzll(m);
                        set.src[l] = gr.src[l];
                        set.base[l] = gr.base[l];
                    }
                    HIP_CHECK(launch_admit_lanes(gr.rc.as, set, gr.rc.cur, main));
                    gr.fresh = 0;
                }
                if (gr.algo == HYTM_PPR) {
                    uint64_t due = 0;  // nothing left to step (ppr_iterations = 0)
                    for (uint64_t m = gr.occupied; m; m &= m - 1)
                        if (!gr.left[__builtin_ctzll(m)]) due |= m & (~m + 1);
                    if (due) retire_lanes(s, gr, due, main);
                    if (!gr.occupied) continue;
                    gr.rc.ppr.mask = gr.occupied;
                    for (uint64_t m = gr.occupied; m; m &= m - 1) gr.rc.ppr.src[__builtin_ctzll(m)] = gr.src[__builtin_ctzll(m)];
                }
                uint64_t active = 0;
                bool empty = false;
                st = step_once(gr.rc, main, &active, &empty);
                if (st != HYTM_OK) throw HipError{st};
                uint64_t done = 0;
                if (gr.algo == HYTM_PPR) {
                    for (uint64_t m = gr.occupied; m; m &= m - 1) {
                        const uint32_t l = (uint32_t)__builtin_ctzll(m);
                        gr.iters[l]++;
                        if (--gr.left[l] == 0) done |= 1ull << l;
                    }
                } else {
                    for (uint64_t m = gr.occupied & active; m; m &= m - 1) gr.iters[__builtin_ctzll(m)]++;
                    done = gr.occupied & ~active;
                }
                if (done) retire_lanes(s, gr, done, main);
            }
        }
        return;
    } catch (const HipError& e) {
        st = e.status;
    } catch (const std::bad_alloc&) {
        st = fail(HYTM_E_NOMEM, "host allocation failed in the query server");
    }
    // a failed step leaves the lane state undefined: fail every query, accept no more
    std::lock_guard<std::mutex> lk(s->mu);
    s->fatal = st;
    s->fatal_msg = g_err;
    auto fail_query = [&](Query& q) {
        q.status = st;
        q.msg = s->fatal_msg;
        q.t_done = now_ms();
        q.done = true;
    };
    for (auto& q : s->pending) fail_query(*q);
    s->pending.clear();
    for (LaneGroup& gr : s->grp)
        for (uint32_t l = 0; l < MAX_LANES; l++)
            if (gr.q[l]) {
                fail_query(*gr.q[l]);
                gr.q[l].reset();
            }
    for (LaneGroup& gr : s->grp) gr.occupied = 0;
    s->cv_done.notify_all();
}

hytm_status server_setup(hytm_server* s) {
    hytm_graph* g = s->g;
    HIP_CHECK(hipSetDevice(g->device));
    ensure_streams(g);
    hipStream_t main = g->s_main;
    g->timer.on = false;
    const uint64_t n = g->n;
    const uint32_t nwords = (uint32_t)((n + 31) / 32);
    Plan pl;
    Totals tot;
    const uint32_t plan_arrays = s->cfg.lanes[1] ? edge_arrays(g, HYTM_SSSP) : 1;
    hytm_status ps = prepare_graph(g, plan_arrays, main, &pl, &tot);
    if (ps != HYTM_OK) return ps;
    static const int algos[3] = {HYTM_BFS, HYTM_SSSP, HYTM_PPR};
    for (int k = 0; k < 3; k++) {
        LaneGroup& gr = s->grp[k];
        if (!s->cfg.lanes[k]) continue;
        gr.algo = algos[k];
        gr.lanes = s->cfg.lanes[k];
        gr.lshift = lane_shift(gr.lanes);
        gr.cur.ensure(nwords);
        gr.nxt.ensure(nwords);
        gr.mcur.ensure(n);
        gr.mnxt.ensure(n);
        if (gr.algo == HYTM_BFS) gr.mvis.ensure(n);
        if (gr.algo == HYTM_PPR) {
            gr.lx.ensure(n << gr.lshift);
            gr.lacc.ensure(n << gr.lshift);
        } else {
            gr.lval.ensure(n << gr.lshift);
        }
        init_ctx(gr.rc, g, gr.algo, true, pl, nullptr);
        AlgoState& as = gr.rc.as;
        as.algo = gr.algo == HYTM_BFS ? ALGO_MBFS : gr.algo == HYTM_SSSP ? ALGO_MSSSP : ALGO_MPPR;
        as.next = gr.nxt.p;
        as.mcur = gr.mcur.p;
        as.mnext = gr.mnxt.p;
        as.mvisited = gr.mvis.p;
        as.lval = gr.lval.p;
        as.lx = gr.lx.p;
        as.lacc = gr.lacc.p;
        as.lshift = gr.lshift;
        gr.rc.cur = gr.cur.p;
        gr.rc.nxt = gr.nxt.p;
        gr.rc.mcur = gr.mcur.p;
        gr.rc.mnxt = gr.mnxt.p;
        HIP_CHECK(launch_fill_u32(gr.cur.p, nwords, 0u, main));
        HIP_CHECK(launch_fill_u32(gr.nxt.p, nwords, 0u, main));
        HIP_CHECK(launch_fill_u32((uint32_t*)gr.mcur.p, 2 * n, 0u, main));
        HIP_CHECK(launch_fill_u32((uint32_t*)gr.mnxt.p, 2 * n, 0u, main));
        if (gr.mvis.p) HIP_CHECK(launch_fill_u32((uint32_t*)gr.mvis.p, 2 * n, 0u, main));
        HIP_CHECK(launch_reset_lanes(as, gr.all(), main));
    }
    HIP_CHECK(launch_fill_u32(g->d_overflow.p, 2, 0u, main));
    g->d_xout.ensure(n * EXTRACT_LANES);
    HIP_CHECK(hipStreamSynchronize(main));
    return HYTM_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

void hytm_default_params(hytm_params* p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(hytm_params);
    p->mode = HYTM_MODE_HYBRID;
    p->partition_edges = 32768;
    p->combine_k = 4;
    p->alpha_num = 4;
    p->alpha_den = 5;
    p->beta_num = 2;
    p->beta_den = 5;
    p->gamma_num = 5;
    p->gamma_den = 8;
    p->line_bytes = 128;
    p->max_outstanding = 256;
    p->index_bytes = 4;
    p->pr_iterations = 20;
    p->pr_damping = 0.85;
    p->ppr_iterations = 10;
    p->reprocess = 0;
    p->dpr_max_iterations = 10000;
    p->dpr_epsilon = 1e-7;
    p->compact_gather_num = 0;
    p->compact_gather_den = 1;
    p->rq_distinct_lines = 0;
    p->zc_tie = 0;
    p->pr_blocking = 1;
    p->pr_block_pairs = 0;
    p->sssp_delta = 0;
    p->streams = 4;
    p->gather_threads = 0;
    p->compact_chunk_edges = 0;
}

const char* hytm_last_error(void) { return g_err.c_str(); }

hytm_status hytm_graph_create(uint64_t n, uint64_t m, const void* offsets, uint32_t offset_bytes, const uint32_t* col,
                              const uint32_t* weights, uint32_t flags, int hip_device, hytm_graph** out) {
    g_err.clear();
    if (!out) return fail(HYTM_E_INVAL, "out is NULL");
    if (!offsets) return fail(HYTM_E_INVAL, "offsets is NULL");
    if (m > 0 && !col) return fail(HYTM_E_INVAL, "col is NULL");
    if (offset_bytes != 4 && offset_bytes != 8) return fail(HYTM_E_INVAL, "offset_bytes must be 4 or 8");
    if (n == 0) return fail(HYTM_E_INVAL, "graph has no vertices");
    if (n >= 0xFFFFFFFFull) return fail(HYTM_E_RANGE, "n = %llu: vertex ids must fit below 2^32-1", (unsigned long long)n);
    if (offset_bytes == 4 && m > 0xFFFFFFFFull) return fail(HYTM_E_INVAL, "m does not fit 4-byte offsets");
    if (flags & ~(uint32_t)(HYTM_GRAPH_SYMMETRIC | HYTM_GRAPH_SKIP_COL_CHECK | HYTM_GRAPH_HUB_SORT |
                            HYTM_GRAPH_NO_PACK | HYTM_GRAPH_WIDE_WEIGHTS))
        return fail(HYTM_E_INVAL, "unknown flag bits 0x%x", flags);
    const bool hub_sort = flags & HYTM_GRAPH_HUB_SORT;
    hytm_graph* g = nullptr;
    try {
        g = new hytm_graph();
        g->n = n;
        g->m = m;
        g->flags = flags;
        g->device = hip_device;
        hytm_default_params(&g->params);
        g->h_off.resize(n + 1);
        for (uint64_t v = 0; v <= n; v++)
            g->h_off[v] = offset_bytes == 8 ? ((const uint64_t*)offsets)[v] : ((const uint32_t*)offsets)[v];
        if (g->h_off[0] != 0) {
            delete g;
            return fail(HYTM_E_INVAL, "offsets[0] must be 0");
        }
        for (uint64_t v = 0; v < n; v++)
            if (g->h_off[v + 1] < g->h_off[v]) {
                delete g;
                return fail(HYTM_E_INVAL, "offsets decrease at vertex %llu", (unsigned long long)v);
            }
        if (g->h_off[n] != m) {
            delete g;
            return fail(HYTM_E_INVAL, "offsets[n] = %llu but m = %llu", (unsigned long long)g->h_off[n],
                        (unsigned long long)m);
        }
        if (!(flags & HYTM_GRAPH_SKIP_COL_CHECK) || hub_sort) {
            for (uint64_t e = 0; e < m; e++)
                if (col[e] >= n) {
                    delete g;
                    return fail(HYTM_E_INVAL, "col[%llu] = %u is not a vertex", (unsigned long long)e, col[e]);
                }
        }
    } catch (const std::bad_alloc&) {
        delete g;
        return fail(HYTM_E_NOMEM, "host allocation failed");
    }
    hytm_status st = guarded([&]() -> hytm_status {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || count == 0)
            return fail(HYTM_E_DEVICE, "no HIP device available: %s", hipGetErrorString(e));
        if (hip_device < 0 || hip_device >= count)
            return fail(HYTM_E_DEVICE, "HIP device %d does not exist (%d visible)", hip_device, count);
        HIP_CHECK(hipSetDevice(hip_device));
        // edge arrays: pinned host memory mapped into the device address space.  When the
        // neighbour ids and the weight range fit one 32-bit word together, the weights
        // travel inside the neighbour words and SSSP moves 4 bytes per edge instead of 8.
        g->weighted = weights != nullptr;
        const unsigned threads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        uint32_t wmin = UINT32_MAX, wmax = 0;
        if (weights)
            for (uint64_t e = 0; e < m; e++) {
                wmin = std::min(wmin, weights[e]);
                wmax = std::max(wmax, weights[e]);
            }
        if (weights && m && !(flags & HYTM_GRAPH_NO_PACK)) {
            uint32_t vbits = 1, wbits = 0;
            while (vbits < 32 && (n - 1) >> vbits) vbits++;
            while (wbits < 32 && ((uint64_t)(wmax - wmin) >> wbits)) wbits++;
            if (vbits + wbits <= 32 && vbits < 32) g->pk = Pack{(1u << vbits) - 1, vbits, wmin, 4};
        }
        const bool packed = g->pk.shift < 32;
        // weights kept apart whose range fits a byte travel as one byte each (w - wmin): SSSP then
        // reads 5 bytes per edge instead of 8
        const bool narrow = weights && m && !packed && !(flags & HYTM_GRAPH_WIDE_WEIGHTS) && wmax - wmin <= 255;
        if (narrow) {
            g->pk.wmin = wmin;
            g->pk.wbytes = 1;
        }
        const size_t eb = std::max<uint64_t>(m, 1) * sizeof(uint32_t);
        HIP_CHECK(hipHostMalloc((void**)&g->h_col, eb, hipHostMallocMapped));
        HIP_CHECK(hipHostGetDevicePointer((void**)&g->d_col_map, g->h_col, 0));
        if (weights && !packed) {
            // padded to whole words: byte weights are loaded one byte at a time
            HIP_CHECK(hipHostMalloc((void**)&g->h_w, weight_words(g, std::max<uint64_t>(m, 1)) * 4, hipHostMallocMapped));
            HIP_CHECK(hipHostGetDevicePointer((void**)&g->d_w_map, g->h_w, 0));
        }
        std::vector<uint32_t> wtmp;  // relabelled weights on their way into packed words or bytes
        const uint32_t* wsrc = weights;
        if (hub_sort) {
            // relabel once, straight into the pinned arrays (Sec. 6.1)
            std::vector<uint32_t> order(n);
            g->h_rank.resize(n);
            g->hubs = hub_order(n, g->h_off.data(), col, 8, 100, threads, order.data(), g->h_rank.data());
            std::vector<uint64_t> off2(n + 1);
            uint32_t* w2 = g->h_w;
            if (weights && (packed || narrow)) {
                wtmp.resize(m);
                w2 = wtmp.data();
                wsrc = wtmp.data();
            }
            hub_relabel(n, g->h_off.data(), col, weights, order.data(), g->h_rank.data(), threads, off2.data(),
                        g->h_col, w2);
            g->h_off.swap(off2);
            g->d_rank.ensure(n);
            g->d_order.ensure(n);
            HIP_CHECK(hipMemcpy(g->d_rank.p, g->h_rank.data(), n * 4, hipMemcpyHostToDevice));
            HIP_CHECK(hipMemcpy(g->d_order.p, order.data(), n * 4, hipMemcpyHostToDevice));
        } else if (m) {
            parallel_copy(g->h_col, col, m * sizeof(uint32_t));
            if (weights && !packed && !narrow) parallel_copy(g->h_w, weights, m * sizeof(uint32_t));
        }
        if (narrow) {
            uint8_t* hw = (uint8_t*)g->h_w;
            const uint32_t base = wmin;
            const uint64_t step = (m + threads - 1) / threads;
            std::vector<std::thread> th;
            for (unsigned t = 0; t < threads; t++) {
                const uint64_t a = std::min<uint64_t>(m, t * step), b = std::min<uint64_t>(m, a + step);
                th.emplace_back([=] {
                    for (uint64_t e = a; e < b; e++) hw[e] = (uint8_t)(wsrc[e] - base);
                });
            }
            for (auto& x : th) x.join();
        }
        if (packed) {
            const Pack pk = g->pk;
            uint32_t* hc = g->h_col;
            const uint64_t step = (m + threads - 1) / threads;
            std::vector<std::thread> th;
            for (unsigned t = 0; t < threads; t++) {
                const uint64_t a = std::min<uint64_t>(m, t * step), b = std::min<uint64_t>(m, a + step);
                th.emplace_back([=] {
                    for (uint64_t e = a; e < b; e++) hc[e] |= (wsrc[e] - pk.wmin) << pk.shift;
                });
            }
            for (auto& x : th) x.join();
        }
        g->d_off.ensure(n + 1);
        HIP_CHECK(hipMemcpy(g->d_off.p, g->h_off.data(), (n + 1) * sizeof(uint64_t), hipMemcpyHostToDevice));
        partition_graph(g);
        return HYTM_OK;
    });
    if (st != HYTM_OK) {
        release_all(g);
        delete g;
        return st;
    }
    *out = g;
    return HYTM_OK;
}

hytm_status hytm_hub_order(uint64_t n, uint64_t m, const void* offsets, uint32_t offset_bytes, const uint32_t* col,
                           uint32_t* order_out, uint64_t* hubs_out) {
    g_err.clear();
    if (!offsets || !order_out || !hubs_out || (m && !col)) return fail(HYTM_E_INVAL, "NULL argument");
    if (offset_bytes != 4 && offset_bytes != 8) return fail(HYTM_E_INVAL, "offset_bytes must be 4 or 8");
    if (n >= 0xFFFFFFFFull) return fail(HYTM_E_RANGE, "n = %llu: vertex ids must fit below 2^32-1", (unsigned long long)n);
    try {
        std::vector<uint64_t> off(n + 1);
        for (uint64_t v = 0; v <= n; v++)
            off[v] = offset_bytes == 8 ? ((const uint64_t*)offsets)[v] : ((const uint32_t*)offsets)[v];
        if (off[0] != 0 || off[n] != m) return fail(HYTM_E_INVAL, "offsets must start at 0 and end at m");
        for (uint64_t v = 0; v < n; v++)
            if (off[v + 1] < off[v]) return fail(HYTM_E_INVAL, "offsets decrease at vertex %llu", (unsigned long long)v);
        for (uint64_t e = 0; e < m; e++)
            if (col[e] >= n) return fail(HYTM_E_INVAL, "col[%llu] = %u is not a vertex", (unsigned long long)e, col[e]);
        std::vector<uint32_t> rank(n);
        const unsigned threads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        *hubs_out = hub_order(n, off.data(), col, 8, 100, threads, order_out, rank.data());
    } catch (const std::bad_alloc&) {
        return fail(HYTM_E_NOMEM, "host allocation failed");
    }
    return HYTM_OK;
}

hytm_status hytm_graph_set_parts(hytm_graph* g, uint32_t count, const uint64_t* vertex_bounds) {
    g_err.clear();
    if (!g) return fail(HYTM_E_INVAL, "graph is NULL");
    if (g->server) return fail(HYTM_E_STATE, "a query server is open on this graph");
    if (count == 0) {
        g->parts.clear();
        g->d_inv_n.release();
        return HYTM_OK;
    }
    if (!vertex_bounds) return fail(HYTM_E_INVAL, "vertex_bounds is NULL");
    if (vertex_bounds[0] != 0 || vertex_bounds[count] != g->n)
        return fail(HYTM_E_INVAL, "vertex_bounds must run from 0 to n = %llu", (unsigned long long)g->n);
    for (uint32_t i = 0; i < count; i++)
        if (vertex_bounds[i + 1] <= vertex_bounds[i]) return fail(HYTM_E_INVAL, "graph %u has no vertices", i);
    return guarded([&]() -> hytm_status {
        // every edge must stay inside its graph (checked in the held order, mapped back)
        std::vector<uint32_t> order;
        if (g->hub_sorted()) {
            order.resize(g->n);
            for (uint64_t v = 0; v < g->n; v++) order[g->h_rank[v]] = (uint32_t)v;
        }
        auto caller = [&](uint64_t v) -> uint64_t { return order.empty() ? v : order[v]; };
        auto graph_of = [&](uint64_t v) -> uint32_t {
            return (uint32_t)(std::upper_bound(vertex_bounds, vertex_bounds + count + 1, v) - vertex_bounds - 1);
        };
        std::vector<float> inv(g->n);
        for (uint64_t v = 0; v < g->n; v++) {
            const uint64_t cv = caller(v);
            const uint32_t gi = graph_of(cv);
            inv[v] = (float)(1.0 / (double)(vertex_bounds[gi + 1] - vertex_bounds[gi]));
            for (uint64_t e = g->h_off[v]; e < g->h_off[v + 1]; e++) {
                const uint64_t cu = caller(g->h_col[e] & g->pk.mask);
                if (cu < vertex_bounds[gi] || cu >= vertex_bounds[gi + 1])
                    return fail(HYTM_E_INVAL, "edge %llu -> %llu leaves graph %u", (unsigned long long)cv,
                                (unsigned long long)cu, gi);
            }
        }
        HIP_CHECK(hipSetDevice(g->device));
        g->d_inv_n.ensure(g->n);
        HIP_CHECK(hipMemcpy(g->d_inv_n.p, inv.data(), g->n * sizeof(float), hipMemcpyHostToDevice));
        g->parts.assign(vertex_bounds, vertex_bounds + count + 1);
        return HYTM_OK;
    });
}

hytm_status hytm_set_device_budget(hytm_graph* g, uint64_t edge_bytes) {
    g_err.clear();
    if (!g) return fail(HYTM_E_INVAL, "graph is NULL");
    if (g->server) return fail(HYTM_E_STATE, "a query server is open on this graph");
    if (edge_bytes != g->budget) g->res_valid = false;
    g->budget = edge_bytes;
    return HYTM_OK;
}

hytm_status hytm_set_params(hytm_graph* g, const hytm_params* p) {
    g_err.clear();
    if (!g) return fail(HYTM_E_INVAL, "graph is NULL");
    if (g->server) return fail(HYTM_E_STATE, "a query server is open on this graph");
    hytm_params np;
    if (p) {
        if (p->struct_size != sizeof(hytm_params)) return fail(HYTM_E_INVAL, "params.struct_size mismatch");
        np = *p;
    } else {
        hytm_default_params(&np);
    }
    std::string why;
    if (!params_valid(np, &why)) return fail(HYTM_E_INVAL, "bad params: %s", why.c_str());
    const bool repart = np.partition_edges != g->params.partition_edges;
    g->params = np;
    if (repart)
        return guarded([&]() -> hytm_status {
            HIP_CHECK(hipSetDevice(g->device));
            partition_graph(g);
            return HYTM_OK;
        });
    // the resident cache stays valid: a run refills it only if its partition count or
    // edge arrays change under the new parameters
    return HYTM_OK;
}

hytm_status hytm_get_params(const hytm_graph* g, hytm_params* p) {
    g_err.clear();
    if (!g || !p) return fail(HYTM_E_INVAL, "NULL argument");
    *p = g->params;
    return HYTM_OK;
}

hytm_status hytm_staging_bytes(const hytm_graph* g, hytm_algo algo, uint64_t* bytes) {
    g_err.clear();
    if (!g || !bytes) return fail(HYTM_E_INVAL, "NULL argument");
    if (g->server) return fail(HYTM_E_STATE, "a query server is open on this graph");
    if (algo < HYTM_BFS || algo > HYTM_PAGERANK_DELTA) return fail(HYTM_E_INVAL, "unknown algorithm %d", (int)algo);
    const Staging s = staging_of(g, edge_arrays(g, algo));
    switch (g->params.mode) {
    case HYTM_MODE_FILTER: *bytes = s.f_bytes; break;
    case HYTM_MODE_COMPACT: *bytes = s.c_bytes; break;
    case HYTM_MODE_ZEROCOPY: *bytes = 0; break;
    default: *bytes = s.f_bytes + s.c_bytes;
    }
    return HYTM_OK;
}

hytm_status hytm_graph_info_get(const hytm_graph* g, hytm_graph_info* info) {
    g_err.clear();
    if (!g || !info) return fail(HYTM_E_INVAL, "NULL argument");
    info->n = g->n;
    info->m = g->m;
    info->npart = g->npart;
    info->max_partition_edges = (uint32_t)std::min<uint64_t>(g->max_part_edges, 0xFFFFFFFFull);
    info->hip_device = g->device;
    info->flags = g->flags;
    info->hubs = g->hubs;
    info->packed_weights = g->pk.shift < 32 ? 1u : 0u;
    info->weight_bytes = g->weighted && g->pk.shift == 32 ? g->pk.wbytes : 0u;
    return HYTM_OK;
}

hytm_status hytm_partition_bounds(const hytm_graph* g, uint64_t* bounds, uint64_t cap) {
    g_err.clear();
    if (!g || !bounds) return fail(HYTM_E_INVAL, "NULL argument");
    if (g->server) return fail(HYTM_E_STATE, "a query server is open on this graph");
    if (cap < g->pv.size()) return fail(HYTM_E_INVAL, "bounds buffer holds %llu entries, needs %zu",
                                        (unsigned long long)cap, g->pv.size());
    for (size_t i = 0; i < g->pv.size(); i++) bounds[i] = g->pv[i];
    return HYTM_OK;
}

hytm_status hytm_run(hytm_graph* g, hytm_algo algo, uint32_t source, void* values_out, uint32_t* iterations_out,
                     hytm_run_stats* stats, void* hip_stream) {
    g_err.clear();
    if (!g) return fail(HYTM_E_INVAL, "graph is NULL");
    if (g->server) return fail(HYTM_E_STATE, "a query server is open on this graph");
    if (!values_out) return fail(HYTM_E_INVAL, "values_out is NULL");
    if (algo < HYTM_BFS || algo > HYTM_PAGERANK_DELTA) return fail(HYTM_E_INVAL, "unknown algorithm %d", (int)algo);
    if (stats && stats->struct_size != sizeof(hytm_run_stats))
        return fail(HYTM_E_INVAL, "stats.struct_size mismatch");
    if ((algo == HYTM_BFS || algo == HYTM_SSSP || algo == HYTM_PPR) && source >= g->n)
        return fail(HYTM_E_RANGE, "source %u >= n = %llu", source, (unsigned long long)g->n);
    if (algo == HYTM_SSSP && !g->weighted) return fail(HYTM_E_INVAL, "SSSP needs edge weights");
    if (algo == HYTM_CC && !(g->flags & HYTM_GRAPH_SYMMETRIC))
        return fail(HYTM_E_INVAL, "CC needs a graph created with HYTM_GRAPH_SYMMETRIC");
    if (algo == HYTM_PAGERANK && g->params.pr_iterations == 0)
        return fail(HYTM_E_INVAL, "pr_iterations must be > 0");
    // personalized PageRank runs as one lane of the batched form
    const uint32_t lanes = algo == HYTM_PPR ? 1 : 0;
    return guarded([&] { return run_impl(g, algo, &source, lanes, values_out, iterations_out, stats, hip_stream); });
}

hytm_status hytm_run_batch(hytm_graph* g, hytm_algo algo, const uint32_t* sources, uint32_t nsources,
                           void* values_out, uint32_t* iterations_out, hytm_run_stats* stats, void* hip_stream) {
    g_err.clear();
    if (!g) return fail(HYTM_E_INVAL, "graph is NULL");
    if (g->server) return fail(HYTM_E_STATE, "a query server is open on this graph");
    if (!values_out || !sources) return fail(HYTM_E_INVAL, "NULL argument");
    if (algo != HYTM_BFS && algo != HYTM_SSSP && algo != HYTM_PPR)
        return fail(HYTM_E_INVAL, "batched runs support BFS, SSSP and PPR");
    if (nsources == 0 || nsources > MAX_LANES) return fail(HYTM_E_INVAL, "nsources must be in 1..64");
    if (stats && stats->struct_size != sizeof(hytm_run_stats))
        return fail(HYTM_E_INVAL, "stats.struct_size mismatch");
    for (uint32_t l = 0; l < nsources; l++)
        if (sources[l] >= g->n)
            return fail(HYTM_E_RANGE, "sources[%u] = %u >= n = %llu", l, sources[l], (unsigned long long)g->n);
    if (algo == HYTM_SSSP && !g->weighted) return fail(HYTM_E_INVAL, "SSSP needs edge weights");
    return guarded(
        [&] { return run_impl(g, algo, sources, nsources, values_out, iterations_out, stats, hip_stream); });
}

hytm_status hytm_select_engines(hytm_graph* g, uint64_t npart, const uint64_t* E, const uint64_t* nA,
                                const uint64_t* Ea, const uint64_t* Rq, uint64_t nres, uint32_t edge_arrays,
                                uint8_t* p_out) {
    g_err.clear();
    if (!g || (npart && (!E || !nA || !Ea || !Rq || !p_out))) return fail(HYTM_E_INVAL, "NULL argument");
    if (g->server) return fail(HYTM_E_STATE, "a query server is open on this graph");
    if (edge_arrays != 1 && edge_arrays != 2) return fail(HYTM_E_INVAL, "edge_arrays must be 1 or 2");
    for (uint64_t i = 0; i < npart; i++)
        if (E[i] >= (1ull << 40) || Ea[i] > E[i] || nA[i] > Ea[i] || Rq[i] >= (1ull << 44) ||
            (Ea[i] > 0 && nA[i] == 0))
            return fail(HYTM_E_INVAL, "partition %llu: statistics out of range", (unsigned long long)i);
    if (npart == 0) return HYTM_OK;
    return guarded([&]() -> hytm_status {
        HIP_CHECK(hipSetDevice(g->device));
        ensure_streams(g);
        SelParams sp = make_sel(g, edge_arrays);
        sp.nres = (uint32_t)std::min<uint64_t>(nres, 0xFFFFFFFFull);
        g->d_sel_in.ensure(4 * npart);
        g->d_sel_out.ensure(npart);
        const uint64_t* src[4] = {E, nA, Ea, Rq};
        for (int a = 0; a < 4; a++)
            HIP_CHECK(hipMemcpyAsync(g->d_sel_in.p + a * npart, src[a], npart * 8, hipMemcpyHostToDevice, g->s_main));
        HIP_CHECK(launch_select_only(npart, g->d_sel_in.p, g->d_sel_in.p + npart, g->d_sel_in.p + 2 * npart,
                                     g->d_sel_in.p + 3 * npart, sp, g->d_sel_out.p, g->s_main));
        HIP_CHECK(hipMemcpyAsync(p_out, g->d_sel_out.p, npart, hipMemcpyDeviceToHost, g->s_main));
        HIP_CHECK(hipStreamSynchronize(g->s_main));
        return HYTM_OK;
    });
}

hytm_status hytm_select_engines_static(hytm_graph* g, uint64_t npart, const uint64_t* E, const uint64_t* nA,
                                       const uint64_t* Ea, const uint64_t* Rq, uint64_t nres, uint32_t edge_arrays,
                                       uint8_t* p_out, void* hip_stream) {
    g_err.clear();
    if (!g || (npart && (!E || !nA || !Ea || !Rq || !p_out))) return fail(HYTM_E_INVAL, "NULL argument");
    if (g->server) return fail(HYTM_E_STATE, "a query server is open on this graph");
    if (edge_arrays != 1 && edge_arrays != 2) return fail(HYTM_E_INVAL, "edge_arrays must be 1 or 2");
    if (npart > STATIC_SEL_MAX_PARTS)
        return fail(HYTM_E_RANGE, "%llu partitions exceed the static scratch (at most %llu)",
                    (unsigned long long)npart, (unsigned long long)STATIC_SEL_MAX_PARTS);
    for (uint64_t i = 0; i < npart; i++)
        if (E[i] >= (1ull << 40) || Ea[i] > E[i] || nA[i] > Ea[i] || Rq[i] >= (1ull << 44) ||
            (Ea[i] > 0 && nA[i] == 0))
            return fail(HYTM_E_INVAL, "partition %llu: statistics out of range", (unsigned long long)i);
    if (npart == 0) return HYTM_OK;
    return guarded([&]() -> hytm_status {
        HIP_CHECK(hipSetDevice(g->device));
        uint64_t* scr = nullptr;  // this device's copy of the static array
        HIP_CHECK(static_select_scratch(g->device, &scr));
        hipStream_t st = (hipStream_t)hip_stream;
        SelParams sp = make_sel(g, edge_arrays);
        sp.nres = (uint32_t)std::min<uint64_t>(nres, 0xFFFFFFFFull);
        // every word the selection reads is written first, and every code it returns is
        // written by it, so nothing left by an earlier call is seen
        const uint64_t* src[4] = {E, nA, Ea, Rq};
        for (int a = 0; a < 4; a++)
            HIP_CHECK(hipMemcpyAsync(scr + a * npart, src[a], npart * 8, hipMemcpyHostToDevice, st));
        uint8_t* codes = (uint8_t*)(scr + 4 * npart);
        HIP_CHECK(launch_select_only(npart, scr, scr + npart, scr + 2 * npart, scr + 3 * npart, sp, codes, st));
        HIP_CHECK(hipMemcpyAsync(p_out, codes, npart, hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        return HYTM_OK;
    });
}

hytm_status hytm_link_probe(int hip_device, uint64_t bytes, hytm_link_probe_result* out) {
    g_err.clear();
    if (!out) return fail(HYTM_E_INVAL, "out is NULL");
    if (bytes < (1u << 20)) return fail(HYTM_E_INVAL, "probe size must be at least 1 MiB");
    bytes &= ~uint64_t(255);
    uint32_t* host = nullptr;
    void *dev = nullptr, *dev2 = nullptr;
    uint32_t* sink = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hytm_status status = guarded([&]() -> hytm_status {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
            return fail(HYTM_E_DEVICE, "HIP device %d is not available", hip_device);
        HIP_CHECK(hipSetDevice(hip_device));
        HIP_CHECK(hipHostMalloc((void**)&host, bytes, hipHostMallocMapped));
        memset(host, 1, bytes);
        uint32_t* dmap = nullptr;
        HIP_CHECK(hipHostGetDevicePointer((void**)&dmap, host, 0));
        HIP_CHECK(hipMalloc(&dev, bytes));
        HIP_CHECK(hipMalloc(&dev2, bytes));
        HIP_CHECK(hipMalloc((void**)&sink, 64));
        HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreate(&a));
        HIP_CHECK(hipEventCreate(&b));
        auto best_of = [&](auto&& op) {
            float best = 1e30f;
            for (int r = 0; r < 4; r++) {  // the first repetition warms up
                HIP_CHECK(hipEventRecord(a, st));
                HIP_CHECK(op());
                HIP_CHECK(hipEventRecord(b, st));
                HIP_CHECK(hipEventSynchronize(b));
                float ms = 0;
                HIP_CHECK(hipEventElapsedTime(&ms, a, b));
                if (r > 0) best = std::min(best, ms);
            }
            return (double)best;
        };
        const double gb = (double)bytes / 1e9;
        out->h2d_copy_gbps = gb / (best_of([&] { return hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, st); }) / 1e3);
        out->d2h_copy_gbps = gb / (best_of([&] { return hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, st); }) / 1e3);
        const uint32_t wpl[4] = {8, 16, 32, 0};
        for (int i = 0; i < 4; i++) {
            const double useful = wpl[i] ? gb * wpl[i] * 4 / 128.0 : gb;
            out->zc_read_gbps[i] = useful / (best_of([&] { return launch_zc_probe(dmap, bytes, wpl[i], sink, st); }) / 1e3);
        }
        out->hbm_copy_gbps = 2 * gb / (best_of([&] { return launch_copy_probe(dev2, dev, bytes, st); }) / 1e3);
        // host gather: the compaction engine's work, 16-word runs from random places
        {
            const uint64_t words = bytes / 4, runs = words / 2 / 16;
            std::vector<uint64_t> from(runs);
            uint64_t x = 0x9E3779B97F4A7C15ull;
            for (uint64_t r = 0; r < runs; r++) {
                x = x * 6364136223846793005ull + 1442695040888963407ull;
                from[r] = ((x >> 17) % (words / 16)) * 16;
            }
            uint32_t* dst = nullptr;
            HIP_CHECK(hipHostMalloc((void**)&dst, runs * 64, hipHostMallocDefault));
            const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency() / 2));
            Pool pool(nt);
            double best = 1e30;
            for (int rep = 0; rep < 3; rep++) {
                const double t0 = now_ms();
                const uint64_t step = (runs + nt * 4 - 1) / (nt * 4);
                pool.run(nt * 4, [&](unsigned t) {
                    const uint64_t r0 = std::min<uint64_t>(runs, t * step), r1 = std::min<uint64_t>(runs, r0 + step);
                    for (uint64_t r = r0; r < r1; r++) memcpy(dst + r * 16, host + from[r], 64);
                });
                best = std::min(best, now_ms() - t0);
            }
            (void)hipHostFree(dst);
            out->host_gather_gbps = (double)runs * 64 / 1e9 / (best / 1e3);
        }
        return HYTM_OK;
    });
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (st) (void)hipStreamDestroy(st);
    if (sink) (void)hipFree(sink);
    if (dev) (void)hipFree(dev);
    if (dev2) (void)hipFree(dev2);
    if (host) (void)hipHostFree(host);
    return status;
}

hytm_status hytm_host_alloc(int hip_device, uint64_t bytes, void** out) {
    g_err.clear();
    if (!out) return fail(HYTM_E_INVAL, "out is NULL");
    return guarded([&]() -> hytm_status {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
            return fail(HYTM_E_DEVICE, "HIP device %d is not available", hip_device);
        HIP_CHECK(hipSetDevice(hip_device));
        HIP_CHECK(hipHostMalloc(out, bytes ? bytes : 1, hipHostMallocDefault));
        return HYTM_OK;
    });
}

hytm_status hytm_host_free(void* p) {
    g_err.clear();
    if (!p) return HYTM_OK;
    hipError_t e = hipHostFree(p);
    if (e != hipSuccess) return fail(HYTM_E_DEVICE, "hipHostFree failed: %s", hipGetErrorString(e));
    return HYTM_OK;
}

hytm_status hytm_server_state_bytes(const hytm_graph* g, hytm_algo algo, uint32_t lanes, uint64_t* bytes) {
    g_err.clear();
    if (!g || !bytes) return fail(HYTM_E_INVAL, "NULL argument");
    if (group_index(algo) < 0) return fail(HYTM_E_INVAL, "the server runs BFS, SSSP and PPR");
    if (lanes == 0 || lanes > MAX_LANES) return fail(HYTM_E_INVAL, "lanes must be in 1..64");
    *bytes = group_state_bytes(g->n, algo, lanes);
    return HYTM_OK;
}

hytm_status hytm_server_open(hytm_graph* g, const hytm_server_config* cfg, hytm_server** out) {
    g_err.clear();
    if (!g || !cfg || !out) return fail(HYTM_E_INVAL, "NULL argument");
    *out = nullptr;
    if (cfg->struct_size != sizeof(hytm_server_config)) return fail(HYTM_E_INVAL, "config.struct_size mismatch");
    if (g->server) return fail(HYTM_E_STATE, "a query server is already open on this graph");
    static const hytm_algo algos[3] = {HYTM_BFS, HYTM_SSSP, HYTM_PPR};
    uint64_t need = g->n * EXTRACT_LANES * 4;  // extraction staging
    uint32_t groups = 0;
    for (int k = 0; k < 3; k++) {
        if (cfg->lanes[k] > MAX_LANES) return fail(HYTM_E_INVAL, "lanes[%d] = %u exceeds 64", k, cfg->lanes[k]);
        if (!cfg->lanes[k]) continue;
        groups++;
        need += group_state_bytes(g->n, algos[k], cfg->lanes[k]);
    }
    if (!groups) return fail(HYTM_E_INVAL, "no lane group: every lanes[] entry is 0");
    if (cfg->lanes[1] && !g->weighted) return fail(HYTM_E_INVAL, "an SSSP group needs edge weights");
    if (cfg->state_budget && need > cfg->state_budget)
        return fail(HYTM_E_BUDGET, "lane state needs %llu bytes, state_budget is %llu", (unsigned long long)need,
                    (unsigned long long)cfg->state_budget);
    std::unique_ptr<hytm_server> s(new (std::nothrow) hytm_server);
    if (!s) return fail(HYTM_E_NOMEM, "host allocation failed");
    s->g = g;
    s->cfg = *cfg;
    hytm_status st = guarded([&] { return server_setup(s.get()); });
    if (st != HYTM_OK) {
        for (LaneGroup& gr : s->grp) gr.release();
        return st;
    }
    g->server = s.get();
    s->worker = std::thread(serve_loop, s.get());
    *out = s.release();
    return HYTM_OK;
}

hytm_status hytm_server_submit(hytm_server* s, hytm_algo algo, uint32_t source, void* values_out,
                               uint64_t* ticket) {
    g_err.clear();
    if (!s || !values_out || !ticket) return fail(HYTM_E_INVAL, "NULL argument");
    const int k = group_index(algo);
    if (k < 0 || !s->cfg.lanes[k]) return fail(HYTM_E_INVAL, "the server has no lane group for algorithm %d", (int)algo);
    if (source >= s->g->n) return fail(HYTM_E_RANGE, "source %u >= n = %llu", source, (unsigned long long)s->g->n);
    std::shared_ptr<Query> q;
    try {
        q = std::make_shared<Query>();
    } catch (const std::bad_alloc&) {
        return fail(HYTM_E_NOMEM, "host allocation failed");
    }
    q->algo = algo;
    q->source = s->g->inner(source);
    q->out = values_out;
    q->t_submit = now_ms();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != HYTM_OK) {
        g_err = s->fatal_msg;
        return s->fatal;
    }
    if (s->stop) return fail(HYTM_E_STATE, "the server is closing");
    if (s->cfg.max_pending && s->pending.size() >= s->cfg.max_pending)
        return fail(HYTM_E_STATE, "the queue holds max_pending = %llu queries", (unsigned long long)s->cfg.max_pending);
    *ticket = s->next_ticket++;
    s->tickets[*ticket] = q;
    s->pending.push_back(q);
    s->cv_work.notify_one();
    return HYTM_OK;
}

hytm_status hytm_server_wait(hytm_server* s, uint64_t ticket, double timeout_ms, hytm_query_result* result) {
    g_err.clear();
    if (!s) return fail(HYTM_E_INVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(HYTM_E_STATE, "unknown ticket %llu", (unsigned long long)ticket);
    std::shared_ptr<Query> q = it->second;
    auto ready = [&] { return q->done; };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready))
        return fail(HYTM_E_STATE, "query %llu not done within %.1f ms", (unsigned long long)ticket, timeout_ms);
    s->tickets.erase(ticket);
    if (result) {
        result->status = q->status;
        result->iterations = q->iterations;
        result->queue_ms = q->t_admit ? q->t_admit - q->t_submit : 0.0;
        result->run_ms = q->t_admit ? q->t_done - q->t_admit : 0.0;
        result->total_ms = q->t_done - q->t_submit;
    }
    if (q->status != HYTM_OK) g_err = q->msg;
    return q->status;
}

hytm_status hytm_server_close(hytm_server* s) {
    g_err.clear();
    if (!s) return HYTM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    const hytm_status fatal = s->fatal;
    if (fatal != HYTM_OK) g_err = s->fatal_msg;
    (void)hipSetDevice(s->g->device);
    (void)hipDeviceSynchronize();
    for (LaneGroup& gr : s->grp) gr.release();
    s->g->server = nullptr;
    delete s;
    return fatal;
}

hytm_status hytm_graph_destroy(hytm_graph* g) {
    g_err.clear();
    if (!g) return HYTM_OK;
    if (g->server) return fail(HYTM_E_STATE, "close the query server on this graph first");
    (void)hipSetDevice(g->device);
    release_all(g);
    delete g;
    return HYTM_OK;
}

}  // extern "C"
