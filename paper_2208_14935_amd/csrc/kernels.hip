// Device side of the hybrid-transfer traversal, written for gfx950 (wave64).
//
// Per iteration (Sec. 4 overview, Algorithm 1):
//   k_stats_select  one wave per partition: active vertices, active edges and request
//                   lines from the frontier bitmap, then the engine choice of Sec. 5.1
//                   (Eq. 1-3, alpha/beta rule) in exact integer arithmetic;
//   k_scan_*        per-engine prefix sums over partitions (tile totals, tile bases,
//                   offsets), which place every partition's active vertices in one list
//                   ordered by engine segment and partition ("pre-combine" of Vc and Vz,
//                   Algorithm 1);
//   k_build_lists   one wave per scheduled partition: ordered compaction of its active
//                   vertices into the list plus the work prefix (edges, or 128-byte
//                   lines for zero-copy) used for load balancing;
//   k_push_edges    edge-balanced push over a list slice reading device memory
//                   (resident cache, filter staging, or compaction buffer);
//   k_push_lines    line-balanced push reading mapped pinned host memory: each half
//                   wave loads one whole 128-byte line (merged, aligned zero-copy
//                   access, Sec. 2.3 / Sec. 3.2);
// with push operators for BFS, SSSP (atomicMin), CC (atomicMin on labels) and
// PageRank (FP32 atomic add), and a bitmap-directed next frontier (Sec. 6.3).
#include <hip/hip_runtime.h>

#include <mutex>

#include "hytm_kernels.h"

namespace hytm {
namespace {

constexpr uint32_t UNREACHED = 0xFFFFFFFFu;
typedef unsigned __int128 u128;

__device__ __forceinline__ uint64_t lines_of(uint64_t s, uint64_t e, uint32_t sh) {
    // lines of 2^sh four-byte elements touched by elements [s, e), e > s
    return ((e - 1) >> sh) - (s >> sh) + 1;
}

// ------------------------------------------------------------ reductions / scans
__device__ __forceinline__ uint64_t wave_sum(uint64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Exclusive prefix sum over the wave; *total gets the wave's sum.
__device__ __forceinline__ uint64_t wave_exclusive_sum(uint64_t x, uint64_t* total) {
    const int lane = threadIdx.x & 63;
    uint64_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    *total = __shfl(v, 63, 64);
    return v - x;
}

// Exclusive prefix maximum over the wave (0 for lane 0); *total gets the wave's maximum.
__device__ __forceinline__ uint64_t wave_exclusive_max(uint64_t x, uint64_t* total) {
    const int lane = threadIdx.x & 63;
    uint64_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(v, d, 64);
        if (lane >= d) v = v > y ? v : y;
    }
    *total = __shfl(v, 63, 64);
    const uint64_t ex = __shfl_up(v, 1, 64);
    return lane ? ex : 0;
}

// ------------------------------------------------------------- engine selection
// Sec. 5.1 with RTT = 1 and every comparison cleared of denominators:
//   Tef = ceil(E*d1 / L), Tec = ceil((Ea*d1 + nA*d2) / L), Q = ceil(Rq / MR),
//   Tiz = Q * (gn*E + (gd-gn)*Ea) / (gd*E)
//   compaction iff ad*Tec < an*Tef  and  bd*gd*E*Tec < bn*Q*(gn*E + (gd-gn)*Ea);
//   else zero-copy iff Q*(gn*E + (gd-gn)*Ea) < gd*E*Tef; else filter.
__device__ __forceinline__ uint8_t select_engine(uint64_t E, uint64_t nA, uint64_t Ea, uint64_t Rq,
                                                 const SelParams& sp) {
    const uint64_t tef = (E * sp.d1 + sp.L - 1) / sp.L;
    uint64_t tec = (Ea * sp.d1 + nA * sp.d2 + sp.L - 1) / sp.L;
    if (sp.gn_c) {
        // the host gather runs as a pipeline with the copy: the slower of the two counts
        const u128 den = (u128)sp.L * sp.gd_c;
        const uint64_t tgc = (uint64_t)(((u128)Ea * sp.d1 * sp.gn_c + den - 1) / den);
        if (tgc > tec) tec = tgc;
    }
    const uint64_t q = (Rq + sp.MR - 1) / sp.MR;
    const u128 zfac = (u128)sp.gn * E + (u128)(sp.gd - sp.gn) * Ea;
    const bool c1 = (u128)sp.ad * tec < (u128)sp.an * tef;
    const bool c2 = (u128)sp.bd * sp.gd * E * tec < (u128)sp.bn * q * zfac;
    if (c1 && c2 && sp.allow_compact) return P_COMPACT;
    const u128 zl = (u128)q * zfac, zr = (u128)sp.gd * E * tef;
    if (zl < zr || (sp.zc_tie && zl == zr)) return P_ZC;
    return sp.allow_filter ? P_FILTER : P_ZC;
}

// ------------------------------------------------------------------- stats
// One wave per partition (four partitions per workgroup, no workgroup barriers).  The
// partition's vertices are taken in rounds of 64 aligned windows of 64 vertices: lane l loads
// the active bits of window l, a wave scan counts them, and then the round's active vertices
// are dealt out in order, one per lane, in batches of 64 (SEL_B batches with their offset
// loads in flight together).  Lanes are busy whatever the density, and where the frontier
// is dense consecutive lanes hold consecutive vertices, so the offset loads coalesce.
constexpr int SEL_B = 4;

// Active bits of window q (vertices 64 q .. 64 q + 63) restricted to [vb, ve).
__device__ __forceinline__ uint64_t window_bits(const uint32_t* __restrict__ bm, uint32_t q, uint32_t vb,
                                                uint32_t ve) {
    const uint32_t lo = q << 6;
    // word 2q+1 may lie past the bitmap when 64q + 32 >= ve; then its bits are masked off
    // below, and the load reads the partition's last word instead
    const uint32_t hi = min(2 * q + 1, (ve - 1) >> 5);
    uint64_t bits = bm[2 * q] | ((uint64_t)bm[hi] << 32);
    if (lo < vb) bits &= ~0ull << (vb - lo);
    if (ve - lo < 64) bits &= (1ull << (ve - lo)) - 1ull;
    return bits;
}

// Position of the r-th (from 0) set bit of x; r < popcount(x).
__device__ __forceinline__ uint32_t select_bit(uint64_t x, uint32_t r) {
    uint32_t pos = 0, c;
    c = __popc((uint32_t)x);
    if (r >= c) { r -= c; x >>= 32; pos += 32; }
    c = __popc((uint32_t)x & 0xFFFFu);
    if (r >= c) { r -= c; x >>= 16; pos += 16; }
    c = __popc((uint32_t)x & 0xFFu);
    if (r >= c) { r -= c; x >>= 8; pos += 8; }
    c = __popc((uint32_t)x & 0xFu);
    if (r >= c) { r -= c; x >>= 4; pos += 4; }
    c = __popc((uint32_t)x & 0x3u);
    if (r >= c) { r -= c; x >>= 2; pos += 2; }
    if (r >= ((uint32_t)x & 1u)) pos += 1;
    return pos;
}

// Inclusive prefix sum over the wave.
__device__ __forceinline__ uint32_t wave_inclusive_sum_u32(uint32_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// The vertex holding the k-th (from 0) active bit of the round: windows q0 + j, with
// incl the inclusive count of active bits over windows 0..lane; k < the round's total.
__device__ __forceinline__ uint32_t round_vertex(uint32_t k, uint32_t incl, uint32_t cnt, uint64_t wbits,
                                                 uint32_t q0) {
    uint32_t j = 0;
#pragma unroll
    for (uint32_t step = 32; step; step >>= 1)
        if (__shfl(incl, j + step - 1, 64) <= k) j += step;
    const uint64_t bj = __shfl(wbits, j, 64);
    const uint32_t before = __shfl(incl - cnt, j, 64);
    return ((q0 + j) << 6) + select_bit(bj, k - before);
}

// Running sums of a partition's statistics in one lane: active lists, their edges, request
// lines per list and distinct (Eq. 3), kernel lines; with a byte weight array its request
// lines are counted apart (a list of D edges spans D bytes there).  carry / carry_w: (line + 1)
// of the latest list's last line in each array, 0 = none.
struct SelAcc {
    uint64_t c = 0, ea = 0, rq = 0, kl = 0, rqd = 0, carry = 0;
    uint64_t rqw = 0, rqdw = 0, carry_w = 0;
};

// The lines of a list [s, e) in an array whose lines hold 2^sh entries: (first + 1, last + 1).
__device__ __forceinline__ void list_lines(uint64_t s, uint64_t e, uint32_t sh, uint64_t& fl, uint64_t& ll) {
    fl = (s >> sh) + 1;
    ll = ((e - 1) >> sh) + 1;
}

// Batches [b0, b0 + 64 G) of a round's active vertices: every lane loads (a lane past the
// round's end the round's last vertex), so the loads of all G batches are issued before the
// first is used.
template <int G>
__device__ __forceinline__ void stats_batches(uint32_t b0, uint32_t T, uint32_t incl, uint32_t cnt, uint64_t wbits,
                                              uint32_t q0, const uint64_t* __restrict__ off, const SelParams& sp,
                                              SelAcc& a) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t sh = sp.cost_shift, shw = sp.cost_shift + 2;  // byte weights: 4x the entries per line
    const bool bytew = sp.wbytes == 1;
    uint64_t s[G], e[G];
#pragma unroll
    for (int g = 0; g < G; g++) {
        const uint32_t k = b0 + 64 * g + lane;
        const uint32_t v = round_vertex(k < T ? k : T - 1, incl, cnt, wbits, q0);
        s[g] = off[v];
        e[g] = off[v + 1];
    }
#pragma unroll
    for (int g = 0; g < G; g++) {
        if (b0 + 64 * g >= T) break;
        const bool has = b0 + 64 * g + lane < T && e[g] > s[g];
        uint64_t fl = 0, ll = 0, flw = 0, llw = 0;
        if (has) {
            a.c += 1;
            a.ea += e[g] - s[g];
            a.rq += lines_of(s[g], e[g], sh);
            a.kl += lines_of(s[g], e[g], ZC_LINE_SHIFT);
            list_lines(s[g], e[g], sh, fl, ll);
            if (bytew) {
                a.rqw += lines_of(s[g], e[g], shw);
                list_lines(s[g], e[g], shw, flw, llw);
            }
        }
        // the last line of the latest earlier list (lists are in vertex order)
        uint64_t tot;
        const uint64_t ex = wave_exclusive_max(ll, &tot);
        const uint64_t prev = a.carry > ex ? a.carry : ex;
        if (has) a.rqd += ll - fl + 1 - (prev == fl ? 1 : 0);
        a.carry = a.carry > tot ? a.carry : tot;
        if (bytew) {  // uniform
            const uint64_t exw = wave_exclusive_max(llw, &tot);
            const uint64_t prevw = a.carry_w > exw ? a.carry_w : exw;
            if (has) a.rqdw += llw - flw + 1 - (prevw == flw ? 1 : 0);
            a.carry_w = a.carry_w > tot ? a.carry_w : tot;
        }
    }
}

__global__ __launch_bounds__(256) void k_stats_select(uint32_t npart, const uint32_t* __restrict__ pv,
                                                      const uint64_t* __restrict__ off,
                                                      const uint32_t* __restrict__ cur, SelParams sp,
                                                      uint8_t* __restrict__ mode, uint32_t* __restrict__ nA,
                                                      uint32_t* __restrict__ nF, uint64_t* __restrict__ Ea,
                                                      uint64_t* __restrict__ Rq, uint64_t* __restrict__ K) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wpb = blockDim.x >> 6, waves = gridDim.x * wpb;
    for (uint32_t i = blockIdx.x * wpb + (threadIdx.x >> 6); i < npart; i += waves) {
        const uint32_t vb = pv[i], ve = pv[i + 1];
        const uint32_t qb = vb >> 6, qe = (ve + 63) >> 6;
        SelAcc a;
        uint64_t f = 0;
        for (uint32_t q0 = qb; q0 < qe; q0 += 64) {  // uniform across the wave
            const uint64_t wbits = q0 + lane < qe ? window_bits(cur, q0 + lane, vb, ve) : 0ull;
            if (!__ballot(wbits != 0)) continue;
            const uint32_t cnt = __popcll(wbits);
            const uint32_t incl = wave_inclusive_sum_u32(cnt);
            const uint32_t T = __shfl(incl, 63, 64);
            f += cnt;
            // a round of at most 64 active vertices takes one batch, larger ones SEL_B at a time
            if (T <= 64)
                stats_batches<1>(0, T, incl, cnt, wbits, q0, off, sp, a);
            else
                for (uint32_t b0 = 0; b0 < T; b0 += 64 * SEL_B)
                    stats_batches<SEL_B>(b0, T, incl, cnt, wbits, q0, off, sp, a);
        }
        const uint64_t c = wave_sum(a.c);
        f = wave_sum(f);
        const uint64_t ea = wave_sum(a.ea);
        // request lines: the neighbour array, and the weight array beside it (Eq. 3)
        uint64_t rq = wave_sum(sp.rq_distinct ? a.rqd : a.rq);
        if (sp.wbytes == 1)
            rq += wave_sum(sp.rq_distinct ? a.rqdw : a.rqw);
        else if (sp.wbytes)
            rq *= 2;  // 4-byte weights: the neighbour array's lines again
        const uint64_t kl = wave_sum(a.kl);
        if (lane == 0) {
            uint8_t p;
            if (ea == 0)
                p = P_NONE;
            else if (i < sp.nres)
                p = P_RES;
            else if (sp.force)
                p = (uint8_t)sp.force;
            else
                p = select_engine(off[ve] - off[vb], c, ea, rq, sp);
            mode[i] = p;
            nA[i] = (uint32_t)c;
            nF[i] = (uint32_t)f;
            Ea[i] = ea;
            Rq[i] = rq;
            K[i] = kl;
        }
    }
}

__global__ void k_select_only(uint64_t npart, const uint64_t* __restrict__ E, const uint64_t* __restrict__ nA,
                              const uint64_t* __restrict__ Ea, const uint64_t* __restrict__ Rq, SelParams sp,
                              uint8_t* __restrict__ p) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < npart;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint8_t r;
        if (Ea[i] == 0)
            r = P_NONE;
        else if (i < sp.nres)
            r = P_RES;
        else if (sp.force)
            r = (uint8_t)sp.force;
        else
            r = select_engine(E[i], nA[i], Ea[i], Rq[i], sp);
        p[i] = r;
    }
}

// -------------------------------------------------------------------- scan
// The engine segments' list and work offsets and the selection header, in three launches:
// per tile of SCAN_TILE partitions the totals of every value (one workgroup per tile), then
// the segment starts and each tile's bases from the tile totals (one small workgroup), then
// per tile the offsets of each partition (one workgroup per tile).  Every thread takes a
// contiguous run of SCAN_PER partitions, so a workgroup needs one barrier per pass.
constexpr int SCAN_NV = 5 * NSEG + 1;  // cnt[4], work[4], parts[4], edges[4], lines[4], frontier
constexpr int SCAN_NB = 2 * NSEG;      // scanned per segment: list entries, work items
constexpr int SCAN_NW = SCAN_THREADS / 64;

// The values of partitions [i0, i1) summed into val[0, NV).
template <int NV>
__device__ __forceinline__ void scan_run_sums(uint32_t i0, uint32_t i1, const uint8_t* __restrict__ mode,
                                              const uint32_t* __restrict__ nA, const uint32_t* __restrict__ nF,
                                              const uint64_t* __restrict__ Ea, const uint64_t* __restrict__ Rq,
                                              const uint64_t* __restrict__ K, uint64_t (&val)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; k++) val[k] = 0;
    for (uint32_t i = i0; i < i1; i++) {
        if constexpr (NV == SCAN_NV) val[SCAN_NV - 1] += nF[i];
        const uint8_t m = mode[i];
        if (m == P_NONE) continue;
        const uint64_t ea = Ea[i], w = (m == P_ZC) ? K[i] : ea, na = nA[i];
#pragma unroll
        for (int sg = 0; sg < NSEG; sg++) {
            if (m != sg + 1) continue;
            val[sg] += na;
            val[NSEG + sg] += w;
            if (NV == SCAN_NV) {
                val[2 * NSEG + sg] += 1;
                val[3 * NSEG + sg] += ea;
                val[4 * NSEG + sg] += Rq[i];
            }
        }
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tot(uint32_t npart, const uint8_t* __restrict__ mode,
                                                   const uint32_t* __restrict__ nA, const uint32_t* __restrict__ nF,
                                                   const uint64_t* __restrict__ Ea, const uint64_t* __restrict__ Rq,
                                                   const uint64_t* __restrict__ K, uint64_t* __restrict__ tile_tot) {
    __shared__ uint64_t s_tot[SCAN_NW][SCAN_NV];
    const uint32_t i0 = min(blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER, npart), i1 = min(i0 + SCAN_PER, npart);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t val[SCAN_NV];
    scan_run_sums<SCAN_NV>(i0, i1, mode, nA, nF, Ea, Rq, K, val);
#pragma unroll
    for (int k = 0; k < SCAN_NV; k++) {
        const uint64_t v = wave_sum(val[k]);
        if (lane == 0) s_tot[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < SCAN_NV) {
        uint64_t t = 0;
        for (int w = 0; w < SCAN_NW; w++) t += s_tot[w][threadIdx.x];
        tile_tot[(uint64_t)blockIdx.x * SCAN_NV + threadIdx.x] = t;
    }
}

// One workgroup of 64 threads: grand totals, segment starts (segments lie one after another:
// RESIDENT, FILTER, ZEROCOPY, COMPACT), each tile's bases, the header, and the work prefix's
// closing entry.
__global__ __launch_bounds__(64) void k_scan_base(uint32_t ntiles, const uint64_t* __restrict__ tile_tot,
                                                  uint64_t* __restrict__ tile_base, Header* __restrict__ hdr,
                                                  uint64_t* __restrict__ wpre) {
    __shared__ uint64_t s_g[SCAN_NV];
    const uint32_t k = threadIdx.x;
    if (k < SCAN_NV) {
        uint64_t t = 0;
        for (uint32_t i = 0; i < ntiles; i++) t += tile_tot[(uint64_t)i * SCAN_NV + k];
        s_g[k] = t;
    }
    __syncthreads();
    if (k < SCAN_NB) {
        const uint32_t sg = k % NSEG, first = k - sg;  // first: 0 (list entries) or NSEG (work)
        uint64_t run = 0;
        for (uint32_t s2 = 0; s2 < sg; s2++) run += s_g[first + s2];
        for (uint32_t i = 0; i < ntiles; i++) {
            tile_base[(uint64_t)i * SCAN_NB + k] = run;
            run += tile_tot[(uint64_t)i * SCAN_NV + k];
        }
    }
    if (k == 0) {
        uint64_t la = 0, wa = 0;
#pragma unroll
        for (int sg = 0; sg < NSEG; sg++) {
            hdr->seg_parts[sg] = (uint32_t)s_g[2 * NSEG + sg];
            hdr->seg_list_start[sg] = (uint32_t)la;
            hdr->seg_list_count[sg] = (uint32_t)s_g[sg];
            hdr->seg_work_start[sg] = wa;
            hdr->seg_work_total[sg] = s_g[NSEG + sg];
            hdr->seg_edges[sg] = s_g[3 * NSEG + sg];
            hdr->seg_cost_lines[sg] = s_g[4 * NSEG + sg];
            la += s_g[sg];
            wa += s_g[NSEG + sg];
        }
        hdr->total_active = la;
        hdr->frontier = s_g[SCAN_NV - 1];
        wpre[la] = wa;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_write(uint32_t npart, const uint8_t* __restrict__ mode,
                                                     const uint32_t* __restrict__ nA, const uint64_t* __restrict__ Ea,
                                                     const uint64_t* __restrict__ K,
                                                     const uint64_t* __restrict__ tile_base,
                                                     uint32_t* __restrict__ lbase, uint64_t* __restrict__ wbase) {
    __shared__ uint64_t s_tot[SCAN_NW][SCAN_NB];
    const uint32_t i0 = min(blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER, npart), i1 = min(i0 + SCAN_PER, npart);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t val[SCAN_NB];
    scan_run_sums<SCAN_NB>(i0, i1, mode, nA, nullptr, Ea, nullptr, K, val);
    uint64_t ex[SCAN_NB];
#pragma unroll
    for (int k = 0; k < SCAN_NB; k++) {
        uint64_t v = val[k];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = __shfl_up(v, d, 64);
            if (lane >= d) v += y;
        }
        ex[k] = v - val[k];
        if (lane == 63) s_tot[wid][k] = v;
    }
    __syncthreads();
    uint64_t run[SCAN_NB];
#pragma unroll
    for (int k = 0; k < SCAN_NB; k++) {
        uint64_t before = 0;
        for (int w = 0; w < wid; w++) before += s_tot[w][k];
        run[k] = tile_base[(uint64_t)blockIdx.x * SCAN_NB + k] + before + ex[k];
    }
    for (uint32_t i = i0; i < i1; i++) {
        const uint8_t m = mode[i];
        uint32_t lb = 0xFFFFFFFFu;
        uint64_t wb = ~0ull;
#pragma unroll
        for (int sg = 0; sg < NSEG; sg++) {
            if (m != sg + 1) continue;
            lb = (uint32_t)run[sg];
            wb = run[NSEG + sg];
            run[sg] += nA[i];
            run[NSEG + sg] += (m == P_ZC) ? K[i] : Ea[i];
        }
        lbase[i] = lb;
        wbase[i] = wb;
    }
}

// ------------------------------------------------------------------ lists
// One wave per scheduled partition, dealing out each round's active vertices as in
// k_stats_select; a batch's entries are written in lane order, so the stores coalesce.
// Batches [b0, b0 + 64 G) of a round's active vertices, loaded as in stats_batches; the
// entries of vertices with edges go to list[pos...) in lane order with their work prefix.
template <int G>
__device__ __forceinline__ void list_batches(uint32_t b0, uint32_t T, uint32_t incl, uint32_t cnt, uint64_t wbits,
                                             uint32_t q0, const uint64_t* __restrict__ off, bool by_lines,
                                             uint32_t* __restrict__ list, uint64_t* __restrict__ wpre, uint64_t& pos,
                                             uint64_t& wp) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t s[G], e[G];
    uint32_t vv[G];
#pragma unroll
    for (int g = 0; g < G; g++) {
        const uint32_t k = b0 + 64 * g + lane;
        vv[g] = round_vertex(k < T ? k : T - 1, incl, cnt, wbits, q0);
        s[g] = off[vv[g]];
        e[g] = off[vv[g] + 1];
    }
#pragma unroll
    for (int g = 0; g < G; g++) {
        if (b0 + 64 * g >= T) break;
        const bool has = b0 + 64 * g + lane < T && e[g] > s[g];
        const uint64_t A = __ballot(has);
        const uint64_t wk = has ? (by_lines ? lines_of(s[g], e[g], ZC_LINE_SHIFT) : e[g] - s[g]) : 0;
        uint64_t tw;
        const uint64_t ew = wave_exclusive_sum(wk, &tw);
        if (has) {
            const uint64_t at = pos + __popcll(A & below);
            list[at] = vv[g];
            wpre[at] = wp + ew;
        }
        pos += __popcll(A);
        wp += tw;
    }
}

__global__ __launch_bounds__(256) void k_build_lists(uint32_t npart, const uint32_t* __restrict__ pv,
                                                     const uint64_t* __restrict__ off,
                                                     const uint32_t* __restrict__ cur,
                                                     const uint8_t* __restrict__ mode,
                                                     const uint32_t* __restrict__ lbase,
                                                     const uint64_t* __restrict__ wbase,
                                                     uint32_t* __restrict__ list, uint64_t* __restrict__ wpre) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wpb = blockDim.x >> 6, waves = gridDim.x * wpb;
    for (uint32_t i = blockIdx.x * wpb + (threadIdx.x >> 6); i < npart; i += waves) {
        const uint8_t m = mode[i];
        if (m == P_NONE) continue;
        const bool by_lines = m == P_ZC;
        const uint32_t vb = pv[i], ve = pv[i + 1];
        const uint32_t qb = vb >> 6, qe = (ve + 63) >> 6;
        uint64_t pos = lbase[i], wp = wbase[i];
        for (uint32_t q0 = qb; q0 < qe; q0 += 64) {  // uniform across the wave
            const uint64_t wbits = q0 + lane < qe ? window_bits(cur, q0 + lane, vb, ve) : 0ull;
            if (!__ballot(wbits != 0)) continue;
            const uint32_t cnt = __popcll(wbits);
            const uint32_t incl = wave_inclusive_sum_u32(cnt);
            const uint32_t T = __shfl(incl, 63, 64);
            if (T <= 64)
                list_batches<1>(0, T, incl, cnt, wbits, q0, off, by_lines, list, wpre, pos, wp);
            else
                for (uint32_t b0 = 0; b0 < T; b0 += 64 * SEL_B)
                    list_batches<SEL_B>(b0, T, incl, cnt, wbits, q0, off, by_lines, list, wpre, pos, wp);
        }
    }
}

// --------------------------------------------------------------- operators
// src(u): the value u pushes (read when the workgroup stages its vertices; it may
// already reflect updates made earlier in the same iteration, which only helps the
// monotone operators).  push(value, v, w): relax edge (u, v) with weight w.
struct OpBfs {
    static constexpr bool wave = false;
    static constexpr bool weighted = false;
    uint32_t* visited;
    uint32_t* next;
    uint32_t* lvl;
    uint32_t level_next;
    __device__ __forceinline__ uint32_t src(uint32_t) const { return 0; }
    __device__ __forceinline__ void push(uint32_t, uint32_t v, uint32_t) const {
        const uint32_t bit = 1u << (v & 31);
        uint32_t* wp = visited + (v >> 5);
        if (__builtin_nontemporal_load(wp) & bit) return;
        const uint32_t old = atomicOr(wp, bit);
        if (!(old & bit)) {  // exactly one thread discovers v
            lvl[v] = level_next;
            atomicOr(next + (v >> 5), bit);
        }
    }
};

struct OpSssp {
    static constexpr bool wave = false;
    static constexpr bool weighted = true;
    uint32_t* dist;
    uint32_t* next;
    uint32_t* overflow;
    uint32_t* far;   // improved vertices at or above `bound` wait here (bound 0xFFFFFFFF: never)
    uint32_t bound;
    __device__ __forceinline__ uint32_t src(uint32_t u) const { return dist[u]; }
    __device__ __forceinline__ void push(uint32_t du, uint32_t v, uint32_t w) const {
        const uint64_t nd = (uint64_t)du + w;
        if (nd >= UNREACHED) {
            *overflow = 1u;
            return;
        }
        if ((uint32_t)nd < dist[v]) {
            const uint32_t old = atomicMin(dist + v, (uint32_t)nd);
            if ((uint32_t)nd < old) atomicOr(((uint32_t)nd < bound ? next : far) + (v >> 5), 1u << (v & 31));
        }
    }
};

struct OpBfsRelax {
    static constexpr bool wave = false;
    static constexpr bool weighted = false;
    uint32_t* lvl;
    uint32_t* next;
    __device__ __forceinline__ uint32_t src(uint32_t u) const { return lvl[u]; }
    __device__ __forceinline__ void push(uint32_t lu, uint32_t v, uint32_t) const {
        const uint32_t nl = lu + 1;
        if (nl < lvl[v]) {
            const uint32_t old = atomicMin(lvl + v, nl);
            if (nl < old) atomicOr(next + (v >> 5), 1u << (v & 31));
        }
    }
};

struct OpCc {
    static constexpr bool wave = false;
    static constexpr bool weighted = false;
    uint32_t* lab;
    uint32_t* next;
    __device__ __forceinline__ uint32_t src(uint32_t u) const { return lab[u]; }
    __device__ __forceinline__ void push(uint32_t lu, uint32_t v, uint32_t) const {
        if (lu < lab[v]) {
            const uint32_t old = atomicMin(lab + v, lu);
            if (lu < old) atomicOr(next + (v >> 5), 1u << (v & 31));
        }
    }
};

// Accumulator copy of the XCD (accelerator complex die) the wave runs on, masked to the
// copies in use.  Any value in [0, copies) would be correct -- the adds are device-scope
// atomics and the copies are summed afterwards -- the die id just keeps each copy's lines in
// few dies' L2 and splits the adds aimed at one hub vertex `copies` ways.
__device__ __forceinline__ uint32_t acc_copy(uint32_t cmask) {
    uint32_t x;
    asm("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
    return x & cmask;
}

struct OpPr {
    static constexpr bool wave = false;
    static constexpr bool weighted = false;
    float* acc;
    uint64_t stride;  // floats per accumulator copy
    const float* contrib;
    uint32_t cmask;   // copies in use - 1
    __device__ __forceinline__ uint32_t src(uint32_t u) const { return __float_as_uint(contrib[u]); }
    __device__ __forceinline__ void push(uint32_t c, uint32_t v, uint32_t) const {
        unsafeAtomicAdd(acc + acc_copy(cmask) * stride + acc_slot(v), __uint_as_float(c));
    }
};

// Batched BFS: lanes of u's mask that have not reached v yet reach it now (one 64-bit
// atomicOr decides, per lane, which edge discovers v first).  The staged value is u.
struct OpMBfs {
    static constexpr bool wave = false;
    static constexpr bool weighted = false;
    const uint64_t* mcur;
    uint64_t* mnext;
    uint64_t* mvisited;
    uint32_t* lvl;   // n rows of 2^lshift lanes
    uint32_t* next;  // union of the next frontier
    uint32_t level_next;
    uint32_t lshift;
    __device__ __forceinline__ uint32_t src(uint32_t u) const { return u; }
    __device__ __forceinline__ void push(uint32_t u, uint32_t v, uint32_t) const {
        const uint64_t want = mcur[u] & ~mvisited[v];
        if (!want) return;
        const uint64_t old = atomicOr((unsigned long long*)(mvisited + v), (unsigned long long)want);
        uint64_t gained = want & ~old;
        if (!gained) return;
        atomicOr((unsigned long long*)(mnext + v), (unsigned long long)gained);
        atomicOr(next + (v >> 5), 1u << (v & 31));
        uint32_t* row = lvl + ((uint64_t)v << lshift);
        while (gained) {
            row[__ffsll((unsigned long long)gained) - 1] = level_next;
            gained &= gained - 1;
        }
    }
};

// Batched SSSP: every lane active at u relaxes (u, v) in its own distance row.
struct OpMSssp {
    static constexpr bool wave = true;
    static constexpr bool weighted = true;
    const uint64_t* mcur;
    uint64_t* mnext;
    uint32_t* dist;      // n rows of 2^lshift lanes
    uint32_t* next;      // union of the next frontier
    uint32_t* overflow;  // two words of lane bits: lanes whose distance would overflow
    uint32_t lshift;
    __device__ __forceinline__ uint32_t src(uint32_t u) const { return u; }
    __device__ __forceinline__ void push(uint32_t u, uint32_t v, uint32_t w) const {
        uint64_t m = mcur[u], gained = 0;
        const uint32_t* du = dist + ((uint64_t)u << lshift);
        uint32_t* dv = dist + ((uint64_t)v << lshift);
        while (m) {
            const uint32_t l = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const uint64_t nd = (uint64_t)du[l] + w;
            if (nd >= UNREACHED) {
                atomicOr(overflow + (l >> 5), 1u << (l & 31));
                continue;
            }
            if ((uint32_t)nd < dv[l]) {
                const uint32_t old = atomicMin(dv + l, (uint32_t)nd);
                if ((uint32_t)nd < old) gained |= 1ull << l;
            }
        }
        if (gained) {
            atomicOr((unsigned long long*)(mnext + v), (unsigned long long)gained);
            atomicOr(next + (v >> 5), 1u << (v & 31));
        }
    }
    // Wave form (see OpMPpr::push_wave): each pass gives 64 >> lshift of the wave's edges one
    // thread per lane, so an edge's relaxations are one atomicMin instruction over its
    // contiguous distance row; the lanes that improved are collected by ballot and one
    // thread per edge marks them.  It pays when the rows are dense (a batch started
    // together); when the wave's edges carry fewer than a quarter row of active lanes on
    // average (queries at different stages) each thread relaxes its own edge's lanes.
    // Called by every thread of the wave.
    __device__ __forceinline__ void push_wave(bool ok, uint32_t u, uint32_t v, uint32_t w) const {
        const uint64_t active = wave_sum(ok ? (uint64_t)__popcll(mcur[u]) : 0ull);
        const uint64_t edges = (uint64_t)__popcll(__ballot(ok));
        if (lshift < 3 || active * 4 < (edges << lshift)) {
            if (ok) push(u, v, w);
            return;
        }
        const uint32_t me = __lane_id();
        const uint32_t slot = me >> lshift, ln = me & ((1u << lshift) - 1);
        const uint32_t per = 64u >> lshift;
        const uint64_t rowmask = lshift >= 6 ? ~0ull : ((1ull << (1u << lshift)) - 1);
        uint64_t act = __ballot(ok);
        while (act) {
            uint64_t a = act;
            for (uint32_t k = 0; k < slot; k++) a &= a - 1;
            const int from = a ? (int)__ffsll((unsigned long long)a) - 1 : 0;
            const uint32_t uu = __shfl(u, from, 64), vv = __shfl(v, from, 64), ww = __shfl(w, from, 64);
            bool gained = false;
            if (a && ((mcur[uu] >> ln) & 1)) {
                const uint64_t nd = (uint64_t)dist[((uint64_t)uu << lshift) + ln] + ww;
                uint32_t* dv = dist + ((uint64_t)vv << lshift) + ln;
                if (nd >= UNREACHED) {
                    atomicOr(overflow + (ln >> 5), 1u << (ln & 31));
                } else if ((uint32_t)nd < *dv) {
                    const uint32_t old = atomicMin(dv, (uint32_t)nd);
                    gained = (uint32_t)nd < old;
                }
            }
            const uint64_t g = (__ballot(gained) >> (slot << lshift)) & rowmask;
            if (a && ln == 0 && g) {
                atomicOr((unsigned long long*)(mnext + vv), (unsigned long long)g);
                atomicOr(next + (vv >> 5), 1u << (vv & 31));
            }
            for (uint32_t k = 0; k < per && act; k++) act &= act - 1;
        }
    }
};

// Batched personalized PageRank: every lane active at u adds its share x_u / D_o(u)
// (prepared in place in u's row, FP32) into v's accumulator row (FP64: a hub's value is a
// sum of up to ~10^5 shares per step, which FP32 adds in atomic order would carry ~1e-4
// relative error; in FP64 only the FP32 rounding of x and of the shares remains).
struct OpMPpr {
    static constexpr bool wave = true;
    static constexpr bool weighted = false;
    const uint64_t* mcur;
    uint64_t* mnext;
    const float* share;  // n rows of 2^lshift lanes
    double* acc;         // n rows of 2^lshift lanes
    uint32_t* next;      // union of the next frontier
    uint32_t lshift;
    __device__ __forceinline__ uint32_t src(uint32_t u) const { return u; }
    __device__ __forceinline__ void push(uint32_t u, uint32_t v, uint32_t) const {
        const uint64_t m = mcur[u];
        if (!m) return;
        const float* su = share + ((uint64_t)u << lshift);
        double* av = acc + ((uint64_t)v << lshift);
        uint64_t b = m;
        while (b) {
            const uint32_t l = __ffsll((unsigned long long)b) - 1;
            b &= b - 1;
            unsafeAtomicAdd(av + l, (double)su[l]);
        }
        mark(m, v);
    }
    __device__ __forceinline__ void mark(uint64_t m, uint32_t v) const {
        if ((__builtin_nontemporal_load(mnext + v) & m) != m) atomicOr((unsigned long long*)(mnext + v), (unsigned long long)m);
        const uint32_t bit = 1u << (v & 31);
        if (!(__builtin_nontemporal_load(next + (v >> 5)) & bit)) atomicOr(next + (v >> 5), bit);
    }
    // The wave's edges (threads with ok) spread over the wave: each pass gives 64 >> lshift
    // edges one thread per lane, so the adds of one edge are one instruction over a
    // contiguous accumulator row instead of one instruction per lane.  Called by every
    // thread of the wave.
    __device__ __forceinline__ void push_wave(bool ok, uint32_t u, uint32_t v, uint32_t) const {
        if (lshift < 3) {  // rows of 1..4 lanes: one thread per edge
            if (ok) push(u, v, 0);
            return;
        }
        const uint32_t me = __lane_id();
        const uint32_t slot = me >> lshift, ln = me & ((1u << lshift) - 1);
        const uint32_t per = 64u >> lshift;
        uint64_t act = __ballot(ok);
        while (act) {
            uint64_t a = act;
            for (uint32_t k = 0; k < slot; k++) a &= a - 1;
            const int from = a ? (int)__ffsll((unsigned long long)a) - 1 : 0;
            const uint32_t uu = __shfl(u, from, 64), vv = __shfl(v, from, 64);
            if (a && ((mcur[uu] >> ln) & 1))
                unsafeAtomicAdd(acc + ((uint64_t)vv << lshift) + ln, (double)share[((uint64_t)uu << lshift) + ln]);
            for (uint32_t k = 0; k < per && act; k++) act &= act - 1;
        }
        if (ok) {
            const uint64_t m = mcur[u];
            if (m) mark(m, v);
        }
    }
};

// push(val, v, w) where ok holds, called by every thread of the wave together: operators
// with a wave form (Op::wave) share the work across the wave.
template <class Op>
__device__ __forceinline__ void push_if(const Op& op, bool ok, uint32_t val, uint32_t v, uint32_t w) {
    if constexpr (Op::wave)
        op.push_wave(ok, val, v, w);
    else if (ok)
        op.push(val, v, w);
}

// Largest j in [lo, hi) with pred(j) true, for a predicate that is true on a prefix of
// [lo, hi) and true at lo.  The whole workgroup searches together: each round every
// thread probes one of blockDim.x evenly spaced positions, so a range of N entries takes
// about log(N)/log(blockDim.x) rounds of independent loads instead of log2(N) dependent
// ones.  Every thread of the block must call it with the same arguments.
template <class Pred>
__device__ __forceinline__ uint32_t block_search_last(uint32_t lo, uint32_t hi, Pred pred, uint32_t* s_tmp) {
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + blockDim.x - 1) / blockDim.x;
        const uint32_t p = lo + threadIdx.x * step;
        const bool ok = p < hi && (threadIdx.x == 0 || pred(p));
        if (threadIdx.x == 0) *s_tmp = 0;
        __syncthreads();
        if (ok && threadIdx.x) atomicMax(s_tmp, threadIdx.x);
        __syncthreads();
        const uint32_t t = *s_tmp;
        __syncthreads();
        lo = lo + t * step;
        hi = min(lo + step, hi);
    }
    return lo;
}

// Inclusive prefix maximum of a[0 .. count) in LDS, count <= PER * blockDim.x, blockDim.x
// a multiple of 64 and at most 1024.  s_wave holds blockDim.x / 64 entries.
template <int PER = 4>
__device__ __forceinline__ void block_prefix_max_u16(uint16_t* a, uint32_t count, uint32_t* s_wave) {
    const uint32_t t = threadIdx.x, lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;
    uint32_t v[PER], m = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const uint32_t i = PER * t + q;
        v[q] = i < count ? a[i] : 0u;
        m = max(m, v[q]);
        v[q] = m;
    }
    uint32_t x = m;  // inclusive scan of thread maxima across the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d) x = max(x, y);
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    uint32_t before = __shfl_up(x, 1, 64);
    if (lane == 0) before = 0;
    for (uint32_t w = 0; w < wid; w++) before = max(before, s_wave[w]);
    (void)nw;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const uint32_t i = PER * t + q;
        if (i < count) a[i] = (uint16_t)max(v[q], before);
    }
    __syncthreads();
}

// ------------------------------------------------------------- edge push
// Decode an edge word (see Pack): the neighbour, and the weight from the word or from w.
__device__ __forceinline__ uint32_t pk_v(uint32_t c, const Pack& pk) { return c & pk.mask; }
__device__ __forceinline__ uint32_t pk_w(uint32_t c, uint32_t wraw, const Pack& pk) {
    return pk.shift < 32 ? (c >> pk.shift) + pk.wmin : wraw;
}
// A weight kept apart from the neighbour words: a uint32, or one byte holding w - wmin.
__device__ __forceinline__ uint32_t load_w(const uint32_t* __restrict__ w, uint64_t e, const Pack& pk) {
    return pk.wbytes == 1 ? (uint32_t)((const uint8_t*)w)[e] + pk.wmin : w[e];
}

constexpr int EDGE_THREADS = 256;
constexpr int EDGE_IPB = 1024;  // edge items per workgroup pass

template <class Op, bool COMPACTED>
__global__ __launch_bounds__(EDGE_THREADS) void k_push_edges(const uint32_t* __restrict__ list,
                                                             const uint64_t* __restrict__ wpre, uint32_t ja,
                                                             uint32_t jb, uint64_t item_lo, uint64_t item_hi,
                                                             const uint64_t* __restrict__ off,
                                                             const uint32_t* __restrict__ col,
                                                             const uint32_t* __restrict__ w, uint64_t shift,
                                                             Op op, Pack pk) {
    __shared__ uint64_t s_pre[EDGE_IPB];
    __shared__ uint64_t s_st[EDGE_IPB];
    __shared__ uint32_t s_val[EDGE_IPB];
    __shared__ uint16_t s_owner[EDGE_IPB];  // item -> staged vertex
    __shared__ uint32_t s_tmp, s_wave[EDGE_THREADS / 64];
    for (uint64_t blk = blockIdx.x;; blk += gridDim.x) {
        const uint64_t i0 = item_lo + blk * EDGE_IPB;
        if (i0 >= item_hi) break;
        const uint64_t i1 = min(i0 + (uint64_t)EDGE_IPB, item_hi);
        // list entries whose items meet [i0, i1): every one has at least one item there,
        // so there are at most EDGE_IPB of them
        const uint32_t j0 = block_search_last(ja, jb, [&](uint32_t j) { return wpre[j] <= i0; }, &s_tmp);
        const uint32_t j1 = block_search_last(j0, jb, [&](uint32_t j) { return wpre[j] < i1; }, &s_tmp);
        const uint32_t nv = j1 - j0 + 1;
        const uint32_t cnt = (uint32_t)(i1 - i0);
        for (uint32_t q = threadIdx.x; q < cnt; q += EDGE_THREADS) s_owner[q] = 0;
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < nv; k += EDGE_THREADS) {
            const uint32_t v = list[j0 + k];
            const uint64_t pre = wpre[j0 + k];
            s_pre[k] = pre;
            s_st[k] = (COMPACTED ? pre : off[v]) - shift;
            s_val[k] = op.src(v);
            if (k) s_owner[pre - i0] = (uint16_t)k;  // first item of every later vertex
        }
        __syncthreads();
        block_prefix_max_u16(s_owner, cnt, s_wave);
        for (uint32_t q0 = 0; q0 < cnt; q0 += EDGE_THREADS) {  // whole waves stay together
            const uint32_t q = q0 + threadIdx.x;
            const bool ok = q < cnt;
            uint32_t val = 0, v = 0, wt = 0;
            if (ok) {
                const uint32_t k = s_owner[q];
                const uint64_t e = s_st[k] + (i0 + q - s_pre[k]);
                v = col[e];
                if (Op::weighted && pk.shift == 32) wt = load_w(w, e, pk);
                val = s_val[k];
            }
            push_if(op, ok, val, pk_v(v, pk), Op::weighted ? pk_w(v, wt, pk) : 0u);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- line push
constexpr int LINE_THREADS = 256;
constexpr int LINE_HALVES = LINE_THREADS / 32;  // half waves per workgroup
constexpr int LINE_UNROLL = 8;                  // lines per half wave per pass
constexpr int LINE_IPB = LINE_HALVES * LINE_UNROLL;

template <class Op>
__global__ __launch_bounds__(LINE_THREADS) void k_push_lines(const uint32_t* __restrict__ list,
                                                             const uint64_t* __restrict__ wpre, uint32_t ja,
                                                             uint32_t jb, uint64_t item_lo, uint64_t item_hi,
                                                             const uint64_t* __restrict__ off,
                                                             const uint32_t* __restrict__ col,
                                                             const uint32_t* __restrict__ w, Op op,
                                                             unsigned long long* __restrict__ distinct, Pack pk) {
    __shared__ uint64_t s_pre[LINE_IPB];
    __shared__ uint64_t s_s[LINE_IPB];
    __shared__ uint64_t s_e[LINE_IPB];
    __shared__ uint32_t s_val[LINE_IPB];
    __shared__ uint32_t s_tmp;
    __shared__ uint64_t s_prev_end;  // end offset of the list entry before the staged ones
    __shared__ uint32_t s_cnt;
    uint32_t my_lines = 0;  // distinct lines of the items this half wave loaded
    const uint32_t half = threadIdx.x >> 5, lane = threadIdx.x & 31;
    for (uint64_t blk = blockIdx.x;; blk += gridDim.x) {
        const uint64_t i0 = item_lo + blk * LINE_IPB;
        if (i0 >= item_hi) break;
        const uint64_t i1 = min(i0 + (uint64_t)LINE_IPB, item_hi);
        const uint32_t j0 = block_search_last(ja, jb, [&](uint32_t j) { return wpre[j] <= i0; }, &s_tmp);
        const uint32_t j1 = block_search_last(j0, jb, [&](uint32_t j) { return wpre[j] < i1; }, &s_tmp);
        const uint32_t nv = j1 - j0 + 1;
        for (uint32_t k = threadIdx.x; k < nv; k += LINE_THREADS) {
            const uint32_t v = list[j0 + k];
            s_pre[k] = wpre[j0 + k];
            s_s[k] = off[v];
            s_e[k] = off[v + 1];
            s_val[k] = op.src(v);
        }
        if (distinct && threadIdx.x == 0) s_prev_end = j0 > ja ? off[list[j0 - 1] + 1] : UINT64_MAX;
        __syncthreads();
        uint32_t cv[LINE_UNROLL], wv[LINE_UNROLL], kk[LINE_UNROLL];
        bool ok[LINE_UNROLL];
#pragma unroll
        for (int r = 0; r < LINE_UNROLL; r++) {
            const uint64_t i = i0 + half + (uint64_t)LINE_HALVES * r;
            ok[r] = false;
            kk[r] = 0;
            cv[r] = 0;
            wv[r] = 0;
            if (i < i1) {
                uint32_t lo = 0, hi = nv;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_pre[mid] <= i)
                        lo = mid;
                    else
                        hi = mid;
                }
                const uint64_t s = s_s[lo];
                const uint64_t e = ((s >> ZC_LINE_SHIFT) << ZC_LINE_SHIFT) + ((i - s_pre[lo]) << ZC_LINE_SHIFT) + lane;
                if (distinct && lane == 0) {
                    // the first line of a vertex repeats when the previous active vertex
                    // (list order is CSR order) ends in it: count each line once
                    const uint64_t pe = lo ? s_e[lo - 1] : s_prev_end;
                    const bool dup = i == s_pre[lo] && pe != UINT64_MAX && pe > 0 &&
                                     ((pe - 1) >> ZC_LINE_SHIFT) == (s >> ZC_LINE_SHIFT);
                    my_lines += dup ? 0u : 1u;
                }
                if (e >= s && e < s_e[lo]) {
                    ok[r] = true;
                    kk[r] = lo;
                    cv[r] = col[e];
                    if (Op::weighted && pk.shift == 32) wv[r] = load_w(w, e, pk);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < LINE_UNROLL; r++)
            push_if(op, ok[r], s_val[kk[r]], pk_v(cv[r], pk), Op::weighted ? pk_w(cv[r], wv[r], pk) : 0u);
        __syncthreads();
    }
    if (distinct) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        if (lane == 0 && my_lines) atomicAdd(&s_cnt, my_lines);
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt) atomicAdd(distinct, (unsigned long long)s_cnt);
    }
}

// ------------------------------------------------------------- init etc.
__global__ void k_init(AlgoState s, uint64_t n, uint32_t source, float x0, float* __restrict__ x,
                       uint32_t* __restrict__ cur, uint32_t nwords) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
        if (s.algo == ALGO_PR)
            x[v] = s.inv_n ? s.inv_n[v] : x0;
        else if (s.algo == ALGO_CC)
            s.val[v] = (uint32_t)v;
        else
            s.val[v] = v == source ? 0u : UNREACHED;
    }
    for (uint64_t wi = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; wi < nwords; wi += stride) {
        uint32_t c;
        if (s.algo == ALGO_BFS || s.algo == ALGO_SSSP || s.algo == ALGO_BFS_RELAX) {
            c = (wi == (source >> 5)) ? (1u << (source & 31)) : 0u;
        } else {
            const uint64_t lo = wi << 5;
            c = lo + 32 <= n ? ~0u : (lo < n ? (1u << (uint32_t)(n - lo)) - 1u : 0u);
        }
        cur[wi] = c;
        if (s.next) s.next[wi] = 0;
        if (s.visited) s.visited[wi] = s.algo == ALGO_BFS ? c : 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && s.overflow) *s.overflow = 0;
}

// Batched runs: value rows to UNREACHED except each lane's own source, lane masks with
// each lane's bit at its source, the union frontier holding every source.
__global__ void k_init_lanes(AlgoState s, LaneSources src, uint32_t* __restrict__ cur, uint32_t nwords) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t cells = s.n << s.lshift;
    const uint32_t lmask = (1u << s.lshift) - 1;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cells; i += stride) {
        const uint32_t v = (uint32_t)(i >> s.lshift), l = (uint32_t)i & lmask;
        const bool at_src = l < src.count && src.src[l] == v;
        if (s.algo == ALGO_MPPR) {
            s.lx[i] = at_src ? 1.0f : 0.0f;
            s.lacc[i] = 0.0;
        } else {
            s.lval[i] = at_src ? 0u : UNREACHED;
        }
    }
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < s.n; v += stride) {
        uint64_t m = 0;
        for (uint32_t l = 0; l < src.count; l++)
            if (src.src[l] == v) m |= 1ull << l;
        ((uint64_t*)s.mcur)[v] = m;
        s.mnext[v] = 0;
        if (s.mvisited) s.mvisited[v] = m;
    }
    for (uint64_t wi = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; wi < nwords; wi += stride) {
        uint32_t c = 0;
        for (uint32_t l = 0; l < src.count; l++)
            if ((src.src[l] >> 5) == wi) c |= 1u << (src.src[l] & 31);
        cur[wi] = c;
        s.next[wi] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && s.overflow) s.overflow[0] = s.overflow[1] = 0;
}

__global__ __launch_bounds__(256) void k_lane_union(const uint64_t* __restrict__ mask, uint64_t n,
                                                    unsigned long long* __restrict__ lanes) {
    uint64_t m = 0;
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
        m |= mask[v];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m |= __shfl_xor(m, d, 64);
    if ((threadIdx.x & 63) == 0 && m) atomicOr(lanes, (unsigned long long)m);
}

// Lane extraction through LDS: a workgroup loads the rows of EX_V vertices with
// coalesced reads (row pitch padded by one word against bank conflicts), then writes
// each requested lane as a contiguous run of EX_V values.
constexpr uint32_t EX_V = 64;
__global__ __launch_bounds__(256) void k_extract_lanes(const uint32_t* __restrict__ vals, uint64_t n,
                                                       uint32_t lshift, LaneSet set, uint32_t nsel, bool sub_base,
                                                       const uint32_t* __restrict__ order,
                                                       uint32_t* __restrict__ out) {
    __shared__ uint32_t tile[EX_V * (MAX_LANES + 1)];
    __shared__ uint8_t s_lane[MAX_LANES];
    __shared__ uint32_t s_base[MAX_LANES];
    const uint32_t S = 1u << lshift, pitch = S + 1;
    if (threadIdx.x < MAX_LANES) {
        // k-th set lane of the mask, k = threadIdx.x
        uint64_t m = set.mask;
        for (uint32_t k = 0; k < threadIdx.x && m; k++) m &= m - 1;
        if (m) {
            const uint32_t l = __ffsll((unsigned long long)m) - 1;
            s_lane[threadIdx.x] = (uint8_t)l;
            s_base[threadIdx.x] = set.base[l];
        }
    }
    for (uint64_t v0 = (uint64_t)blockIdx.x * EX_V; v0 < n; v0 += (uint64_t)gridDim.x * EX_V) {
        const uint32_t nv = (uint32_t)(n - v0 < EX_V ? n - v0 : EX_V);
        __syncthreads();
        const uint32_t cells = nv << lshift;
        const uint32_t* src = vals + (v0 << lshift);
        for (uint32_t c = threadIdx.x; c < cells; c += blockDim.x) tile[(c >> lshift) * pitch + (c & (S - 1))] = src[c];
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < nsel * EX_V; q += blockDim.x) {
            const uint32_t k = q / EX_V, i = q % EX_V;
            if (i >= nv) continue;
            uint32_t x = tile[i * pitch + s_lane[k]];
            if (sub_base && x != UNREACHED) x -= s_base[k];
            out[(uint64_t)k * n + (order ? order[v0 + i] : v0 + i)] = x;
        }
    }
}

__global__ __launch_bounds__(256) void k_loaded_frontier(uint32_t npart, const uint32_t* __restrict__ pv,
                                                         const uint8_t* __restrict__ mode, uint32_t mode_mask,
                                                         const uint32_t* __restrict__ next, uint32_t* __restrict__ cur2) {
    for (uint32_t p = blockIdx.x; p < npart; p += gridDim.x) {
        if (!((mode_mask >> mode[p]) & 1)) continue;  // uniform across the workgroup
        for (uint32_t v = pv[p] + threadIdx.x; v < pv[p + 1]; v += blockDim.x)
            if ((next[v >> 5] >> (v & 31)) & 1) atomicOr(cur2 + (v >> 5), 1u << (v & 31));
    }
}

__global__ __launch_bounds__(256) void k_dpr_fold(uint32_t npart, const uint32_t* __restrict__ pv, uint64_t n,
                                                  float* __restrict__ acc, uint32_t copies,
                                                  float* __restrict__ delta, double* __restrict__ psum) {
    __shared__ double s_w[4];
    const uint64_t slots = acc_slots(n);
    for (uint32_t p = blockIdx.x; p < npart; p += gridDim.x) {
        double sum = 0.0;
        for (uint32_t v = pv[p] + threadIdx.x; v < pv[p + 1]; v += blockDim.x) {
            const uint32_t sl = acc_slot(v);
            float d = delta[v];
            for (uint32_t c = 0; c < copies; c++) {
                d += acc[c * slots + sl];
                acc[c * slots + sl] = 0.0f;
            }
            delta[v] = d;
            sum += (double)d;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = sum;
        __syncthreads();
        if (threadIdx.x == 0) psum[p] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_dpr_activate(uint32_t npart, const uint32_t* __restrict__ pv,
                                                      const uint64_t* __restrict__ off,
                                                      const uint8_t* __restrict__ sched, float* __restrict__ delta,
                                                      float* __restrict__ x, float* __restrict__ contrib,
                                                      uint32_t* __restrict__ cur, float damping) {
    for (uint32_t p = blockIdx.x; p < npart; p += gridDim.x) {
        if (!sched[p]) continue;  // uniform across the workgroup
        for (uint32_t v = pv[p] + threadIdx.x; v < pv[p + 1]; v += blockDim.x) {
            const float d = delta[v];
            if (!(d > 0.0f)) continue;
            x[v] += d;
            delta[v] = 0.0f;
            const uint64_t deg = off[v + 1] - off[v];
            if (deg) {
                contrib[v] = damping * d / (float)deg;
                atomicOr(cur + (v >> 5), 1u << (v & 31));
            }
        }
    }
}

__global__ void k_dpr_init(uint64_t n, float* __restrict__ delta, const float* __restrict__ inv_n, float restart,
                           float uniform) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
        delta[v] = inv_n ? restart * inv_n[v] : uniform;
}

__global__ void k_dpr_finish(uint64_t n, float* __restrict__ x, const float* __restrict__ delta) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
        x[v] += delta[v];
}

__global__ void k_gather_u32(const uint32_t* __restrict__ src, const uint32_t* __restrict__ rank, uint64_t n,
                             uint32_t* __restrict__ dst) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
        dst[v] = src[rank[v]];
}

// minold[label] = the smallest original id among the vertices holding that label.  Nearly
// every vertex of a graph with a giant component holds the same label, so one word would
// take an atomic per vertex: lanes holding the label of the wave's first lane fold their ids
// into one atomic, and no atomic is made when the slot already holds a smaller id (slots
// only decrease, so a stale read can only let an unneeded atomic through).
__global__ void k_cc_min_old(const uint32_t* __restrict__ lab, const uint32_t* __restrict__ order, uint64_t n,
                             uint32_t* minold) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < n; base += stride) {  // uniform per block
        const uint64_t v = base + threadIdx.x;
        const bool ok = v < n;
        const uint32_t l = ok ? lab[v] : UNREACHED;
        const uint32_t o = ok ? order[v] : UNREACHED;
        const uint32_t l0 = __shfl(l, 0, 64);  // lane 0 holds the wave's smallest v
        const bool same = ok && l == l0;
        uint32_t m = same ? o : UNREACHED;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) m = min(m, (uint32_t)__shfl_xor(m, d, 64));
        if (__lane_id() == 0 && m != UNREACHED && m < minold[l0]) atomicMin(minold + l0, m);
        if (ok && !same && o < minold[l]) atomicMin(minold + l, o);
    }
}

__global__ void k_cc_canon(const uint32_t* __restrict__ lab, const uint32_t* __restrict__ minold,
                           const uint32_t* __restrict__ rank, uint64_t n, uint32_t* __restrict__ dst) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
        dst[v] = minold[lab[rank[v]]];
}

// Smallest distance among the far vertices: one word of the far bitmap per thread, a wave
// minimum, one atomic per wave that holds any.
__global__ void k_far_min(const uint32_t* __restrict__ far, const uint32_t* __restrict__ dist, uint32_t nwords,
                          uint32_t* out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < nwords; base += stride) {  // uniform per block
        const uint64_t wd = base + threadIdx.x;
        uint32_t bits = wd < nwords ? far[wd] : 0u, m = UNREACHED;
        while (bits) {
            const uint32_t b = __ffs(bits) - 1;
            bits &= bits - 1;
            m = min(m, dist[wd * 32 + b]);
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) m = min(m, (uint32_t)__shfl_xor(m, d, 64));
        if (__lane_id() == 0 && m != UNREACHED) atomicMin(out, m);
    }
}

// Far vertices with distance below `bound` leave the far set and join the frontier; each
// thread owns one word of both bitmaps.
__global__ void k_far_move(uint32_t* __restrict__ far, const uint32_t* __restrict__ dist, uint32_t* __restrict__ cur,
                           uint32_t nwords, uint32_t bound) {
    for (uint64_t wd = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; wd < nwords;
         wd += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t f = far[wd];
        if (!f) continue;
        uint32_t bits = f, moved = 0;
        while (bits) {
            const uint32_t b = __ffs(bits) - 1;
            bits &= bits - 1;
            if (dist[wd * 32 + b] < bound) moved |= 1u << b;
        }
        if (moved) {
            far[wd] = f & ~moved;
            cur[wd] |= moved;
        }
    }
}

// SSSP overflow, decided after convergence.  A relaxation whose candidate reaches 2^32-1 is
// skipped and only raises a lane's flag; whether that lane's shortest distances really
// overflow is decided here.  After convergence every vertex whose shortest distance fits
// below 2^32-1 holds it, so a lane overflows exactly when some edge leads from a vertex it
// reached to one it did not.  One wave per vertex u (grid-stride): the lanes of `mask`
// that reached u read u's out-edges from the mapped host array `col` and check their
// targets; lanes that find an unreached target are ORed into *out.  dist: n rows of
// 2^lshift lanes (lshift 0: one distance per vertex).
__global__ __launch_bounds__(256) void k_sssp_ovf_check(const uint64_t* __restrict__ off,
                                                        const uint32_t* __restrict__ col, Pack pk,
                                                        const uint32_t* __restrict__ dist, uint32_t lshift,
                                                        uint64_t mask, uint64_t n, unsigned long long* out) {
    const uint32_t lane = __lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    uint64_t found = 0;
    for (uint64_t u = blockIdx.x * (uint64_t)(blockDim.x / 64) + threadIdx.x / 64; u < n; u += waves) {
        const bool mine = lane < (1u << lshift) && ((mask >> lane) & 1) && dist[(u << lshift) + lane] != UNREACHED;
        const uint64_t reached = __ballot(mine);
        if (!reached) continue;
        const uint64_t e1 = off[u + 1];
        for (uint64_t e = off[u] + lane; e < e1; e += 64) {
            const uint32_t* dv = dist + ((uint64_t)pk_v(col[e], pk) << lshift);
            for (uint64_t r = reached; r; r &= r - 1) {
                const uint32_t l = __ffsll((unsigned long long)r) - 1;
                if (dv[l] == UNREACHED) found |= 1ull << l;
            }
        }
    }
    if (found) atomicOr(out, (unsigned long long)found);
}

__global__ void k_admit_lanes(AlgoState s, LaneSet set, uint32_t* __restrict__ cur) {
    const uint32_t l = threadIdx.x;
    if (l >= MAX_LANES || !((set.mask >> l) & 1)) return;
    const uint32_t v = set.src[l];
    const uint64_t cell = ((uint64_t)v << s.lshift) + l;
    if (s.algo == ALGO_MPPR)
        s.lx[cell] = 1.0f;
    else
        s.lval[cell] = s.algo == ALGO_MBFS ? set.base[l] : 0u;
    atomicOr((unsigned long long*)(s.mcur + v), 1ull << l);
    if (s.mvisited) atomicOr((unsigned long long*)(s.mvisited + v), 1ull << l);
    atomicOr(cur + (v >> 5), 1u << (v & 31));
}

__global__ void k_reset_lanes(AlgoState s, uint64_t mask) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint32_t lmask = (1u << s.lshift) - 1;
    const uint64_t cells = s.n << s.lshift;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cells; i += stride) {
        if (!((mask >> ((uint32_t)i & lmask)) & 1)) continue;
        if (s.algo == ALGO_MPPR) {
            s.lx[i] = 0.0f;
            s.lacc[i] = 0.0;
        } else {
            s.lval[i] = UNREACHED;
        }
    }
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < s.n; v += stride) {
        ((uint64_t*)s.mcur)[v] &= ~mask;
        s.mnext[v] &= ~mask;
        if (s.mvisited) s.mvisited[v] &= ~mask;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && s.overflow) {
        s.overflow[0] &= ~(uint32_t)mask;
        s.overflow[1] &= ~(uint32_t)(mask >> 32);
    }
}

__global__ void k_ppr_prepare(AlgoState s, const uint64_t* __restrict__ off) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < s.n; v += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t m = s.mcur[v];
        const uint64_t d = off[v + 1] - off[v];
        if (!m || !d) continue;
        float* row = s.lx + (v << s.lshift);
        const float fd = (float)d;
        while (m) {
            const uint32_t l = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            row[l] = row[l] / fd;
        }
    }
}

__global__ void k_ppr_apply(AlgoState s, float damping) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < s.n; v += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t m = s.mcur[v] | s.mnext[v];
        if (!m) continue;
        float* x = s.lx + (v << s.lshift);
        double* a = s.lacc + (v << s.lshift);
        while (m) {
            const uint32_t l = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            x[l] = (float)((double)damping * a[l]);
            a[l] = 0.0;
        }
    }
}

__global__ void k_ppr_restart(AlgoState s, LaneSet set, float restart) {
    const uint32_t l = threadIdx.x;
    if (l >= MAX_LANES || !((set.mask >> l) & 1)) return;
    const uint32_t v = set.src[l];
    s.lx[((uint64_t)v << s.lshift) + l] += restart;
    atomicOr((unsigned long long*)(s.mnext + v), 1ull << l);
    atomicOr(s.next + (v >> 5), 1u << (v & 31));
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t count, uint32_t value) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_pr_prepare(uint64_t n, const uint64_t* __restrict__ off, const float* __restrict__ x,
                             float* __restrict__ contrib, float* __restrict__ acc, uint32_t copies) {
    const uint64_t slots = acc_slots(n);
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < slots;
         v += (uint64_t)gridDim.x * blockDim.x) {
        if (v < n) {
            const uint64_t d = off[v + 1] - off[v];
            contrib[v] = d ? x[v] / (float)d : 0.0f;
        }
        for (uint32_t c = 0; c < copies; c++) acc[c * slots + v] = 0.0f;
    }
}

__global__ void k_pr_apply(uint64_t n, float* __restrict__ x, const float* __restrict__ acc, uint32_t copies,
                           float base, float damping, const float* __restrict__ inv_n, float restart) {
    const uint64_t slots = acc_slots(n);
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t s = acc_slot((uint32_t)v);
        float sum = 0.0f;
        for (uint32_t c = 0; c < copies; c++) sum += acc[c * slots + s];
        x[v] = (inv_n ? restart * inv_n[v] : base) + damping * sum;
    }
}

// ---------------------------------------------------- propagation blocking
constexpr int PB_THREADS = 256;
constexpr int PB_PLAN_THREADS = 1024;
constexpr uint32_t PB_TILE = 2048;   // pairs per scatter tile, 8 per thread
constexpr uint32_t PB_LOCAL = PB_LOCAL_BINS;

// Exclusive sum of one value per thread over the workgroup (a multiple of 64 threads);
// *total = the sum of all.  s_w holds blockDim.x / 64 + 1 entries.  Every thread calls it.
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t x, uint32_t* s_w, uint32_t* total) {
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= (uint32_t)d) inc += y;
    }
    if (lane == 63) s_w[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (uint32_t w = 0; w < nw; w++) {
            const uint32_t t = s_w[w];
            s_w[w] = a;
            a += t;
        }
        s_w[nw] = a;
    }
    __syncthreads();
    const uint32_t r = s_w[wid] + inc - x;
    *total = s_w[nw];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(PB_THREADS) void k_pb_hist(const uint32_t* __restrict__ pv, uint32_t vmask, uint64_t cnt,
                                                        uint32_t nfine, uint32_t* __restrict__ hist,
                                                        uint32_t* __restrict__ err) {
    __shared__ uint32_t s_h[PB_MAX_FINE];
    for (uint32_t f = threadIdx.x; f < nfine; f += PB_THREADS) s_h[f] = 0;
    __syncthreads();
    bool bad = false;
    for (uint64_t i = blockIdx.x * (uint64_t)PB_THREADS + threadIdx.x; i < cnt;
         i += (uint64_t)gridDim.x * PB_THREADS) {
        const uint32_t f = (pv[i] & vmask) >> PB_FINE_SHIFT;
        if (f < nfine)
            atomicAdd(&s_h[f], 1u);
        else
            bad = true;
    }
    if (bad) atomicOr(err, 1u);
    __syncthreads();
    for (uint32_t f = threadIdx.x; f < nfine; f += PB_THREADS)
        if (s_h[f]) atomicAdd(hist + f, s_h[f]);
}

// One workgroup: bin starts and the accumulation segments of every non-empty bin.
__global__ __launch_bounds__(PB_PLAN_THREADS) void k_pb_plan(const uint32_t* __restrict__ hist, uint32_t nfine,
                                                             uint32_t seg, uint32_t* __restrict__ foff,
                                                             uint32_t* __restrict__ segs,
                                                             uint32_t* __restrict__ nsegs) {
    constexpr uint32_t PER = PB_MAX_FINE / PB_PLAN_THREADS;
    __shared__ uint32_t s_w[PB_PLAN_THREADS / 64 + 1];
    const uint32_t f0 = threadIdx.x * PER;
    uint32_t c[PER], sum = 0, ns = 0;
#pragma unroll
    for (uint32_t q = 0; q < PER; q++) {
        c[q] = f0 + q < nfine ? hist[f0 + q] : 0u;
        sum += c[q];
        ns += (c[q] + seg - 1) / seg;
    }
    uint32_t total, stotal;
    uint32_t base = block_excl_sum(sum, s_w, &total);
    uint32_t sb = block_excl_sum(ns, s_w, &stotal);
    for (uint32_t q = 0; q < PER; q++) {
        const uint32_t f = f0 + q;
        if (f >= nfine) break;
        foff[f] = base;
        base += c[q];
        for (uint32_t j = 0; (uint64_t)j * seg < c[q]; j++, sb++) {
            segs[2 * sb] = f;
            segs[2 * sb + 1] = j;
        }
    }
    if (threadIdx.x == 0) {
        foff[nfine] = total;
        *nsegs = stotal;
    }
}

// A tile whose keys span fewer than PB_LOCAL bins is counting-sorted in LDS: one cursor
// reservation per bin present, then the tile's pairs leave bin by bin in runs.  A tile
// spanning more (a stretch of nearly empty bins) reserves a position per pair.
__global__ __launch_bounds__(PB_THREADS) void k_pb_scatter(const uint32_t* __restrict__ in_v,
                                                           const float* __restrict__ in_c, uint64_t cnt,
                                                           uint32_t kshift, uint32_t stride, uint32_t nfine,
                                                           const uint32_t* __restrict__ foff,
                                                           uint32_t* __restrict__ cursor, uint32_t* __restrict__ out_v,
                                                           float* __restrict__ out_c, uint32_t* __restrict__ err) {
    constexpr uint32_t PER = PB_TILE / PB_THREADS;
    constexpr uint32_t LPER = PB_LOCAL / PB_THREADS;
    __shared__ uint32_t s_v[PB_TILE];
    __shared__ float s_c[PB_TILE];
    __shared__ uint16_t s_k[PB_TILE];
    __shared__ uint32_t s_cnt[PB_LOCAL], s_ofs[PB_LOCAL], s_g[PB_LOCAL], s_end[PB_LOCAL];
    __shared__ uint32_t s_kmin, s_kmax, s_w[PB_THREADS / 64 + 1];
    const uint32_t nkeys = (nfine + stride - 1) / stride;
    const uint32_t lane = threadIdx.x & 63;
    bool bad = false;
    // each workgroup walks tiles blockIdx.x, + gridDim.x, ...; the next tile's loads are
    // issued before the current tile is sorted
    const uint64_t step = (uint64_t)gridDim.x * PB_TILE;
    uint32_t v[PER], key[PER], rank[PER];
    float c[PER];
    {
        const uint64_t t0 = blockIdx.x * (uint64_t)PB_TILE;
        const uint32_t tc = (uint32_t)min((uint64_t)PB_TILE, cnt - t0);
#pragma unroll
        for (uint32_t r = 0; r < PER; r++) {
            const uint32_t i = r * PB_THREADS + threadIdx.x;
            v[r] = i < tc ? in_v[t0 + i] : 0u;
            c[r] = i < tc ? in_c[t0 + i] : 0.0f;
        }
    }
    for (uint64_t t0 = blockIdx.x * (uint64_t)PB_TILE; t0 < cnt; t0 += step) {
        const uint32_t tc = (uint32_t)min((uint64_t)PB_TILE, cnt - t0);
        uint32_t nv[PER];
        float nc[PER];
        {
            const uint64_t t1 = t0 + step;
            const uint32_t tc1 = t1 < cnt ? (uint32_t)min((uint64_t)PB_TILE, cnt - t1) : 0u;
#pragma unroll
            for (uint32_t r = 0; r < PER; r++) {
                const uint32_t i = r * PB_THREADS + threadIdx.x;
                nv[r] = i < tc1 ? in_v[t1 + i] : 0u;
                nc[r] = i < tc1 ? in_c[t1 + i] : 0.0f;
            }
        }
        uint32_t kmin = UINT32_MAX, kmax = 0;
        if (threadIdx.x == 0) {
            s_kmin = UINT32_MAX;
            s_kmax = 0;
        }
#pragma unroll
        for (uint32_t r = 0; r < PER; r++) {
            key[r] = 0;
            rank[r] = 0;
            if (r * PB_THREADS + threadIdx.x < tc) {
                key[r] = v[r] >> kshift;
                kmin = min(kmin, key[r]);
                kmax = max(kmax, key[r]);
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            kmin = min(kmin, (uint32_t)__shfl_xor(kmin, d, 64));
            kmax = max(kmax, (uint32_t)__shfl_xor(kmax, d, 64));
        }
        __syncthreads();
        if (lane == 0) {
            atomicMin(&s_kmin, kmin);
            atomicMax(&s_kmax, kmax);
        }
        __syncthreads();
        const uint32_t k0 = s_kmin, k1 = s_kmax;
        if (k1 < nkeys && k1 - k0 < PB_LOCAL) {  // uniform across the workgroup
#pragma unroll
            for (uint32_t q = 0; q < LPER; q++) s_cnt[LPER * threadIdx.x + q] = 0;
            __syncthreads();
#pragma unroll
            for (uint32_t r = 0; r < PER; r++)
                if (r * PB_THREADS + threadIdx.x < tc) rank[r] = atomicAdd(&s_cnt[key[r] - k0], 1u);
            __syncthreads();
            uint32_t loc[LPER], sum = 0, tot;
#pragma unroll
            for (uint32_t q = 0; q < LPER; q++) {
                loc[q] = s_cnt[LPER * threadIdx.x + q];
                sum += loc[q];
            }
            uint32_t base = block_excl_sum(sum, s_w, &tot);
#pragma unroll
            for (uint32_t q = 0; q < LPER; q++) {
                const uint32_t b = LPER * threadIdx.x + q;
                s_ofs[b] = base;
                base += loc[q];
                if (loc[q]) {
                    const uint32_t k = k0 + b;
                    s_g[b] = atomicAdd(cursor + k, loc[q]);
                    s_end[b] = foff[min((k + 1) * stride, nfine)];
                }
            }
            __syncthreads();
#pragma unroll
            for (uint32_t r = 0; r < PER; r++)
                if (r * PB_THREADS + threadIdx.x < tc) {
                    const uint32_t lk = key[r] - k0;
                    const uint32_t p = s_ofs[lk] + rank[r];
                    s_v[p] = v[r];
                    s_c[p] = c[r];
                    s_k[p] = (uint16_t)lk;
                }
            __syncthreads();
            for (uint32_t p = threadIdx.x; p < tc; p += PB_THREADS) {
                const uint32_t lk = s_k[p];
                const uint32_t gpos = s_g[lk] + (p - s_ofs[lk]);
                if (gpos < s_end[lk]) {
                    out_v[gpos] = s_v[p];
                    out_c[gpos] = s_c[p];
                } else {
                    bad = true;
                }
            }
        } else {
#pragma unroll
            for (uint32_t r = 0; r < PER; r++)
                if (r * PB_THREADS + threadIdx.x < tc) {
                    const uint32_t k = key[r];
                    if (k >= nkeys) {
                        bad = true;
                        continue;
                    }
                    const uint32_t gpos = atomicAdd(cursor + k, 1u);
                    if (gpos < foff[min((k + 1) * stride, nfine)]) {
                        out_v[gpos] = v[r];
                        out_c[gpos] = c[r];
                    } else {
                        bad = true;
                    }
                }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < PER; r++) {
            v[r] = nv[r];
            c[r] = nc[r];
        }
    }
    if (bad) atomicOr(err, 1u);
}

// Resident push of a piece (every vertex active): slot t of [0, cnt) gets the contribution
// of its edge's source, the list entry j in [ja, jb) whose work range holds wa + t.
// tj[k] = the last entry whose range starts at or before tile k's first slot (computed
// once per piece by k_pb_tiles); a workgroup marks, in an LDS owner map, where each later
// entry of its tile starts, takes prefix maxima, and writes the tile with coalesced stores.
constexpr uint32_t PB_EXP_TILE = 4096;

__global__ void k_pb_tiles(const uint64_t* __restrict__ wpre, uint32_t ja, uint32_t jb, uint64_t wa, uint64_t cnt,
                           uint32_t* __restrict__ tj) {
    const uint64_t ntiles = (cnt + PB_EXP_TILE - 1) / PB_EXP_TILE;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < ntiles;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t t = wa + k * PB_EXP_TILE;
        uint32_t lo = ja, hi = jb;  // wpre[ja] <= t < wpre[jb]
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (wpre[mid] <= t)
                lo = mid;
            else
                hi = mid;
        }
        tj[k] = lo;
    }
}

__global__ __launch_bounds__(256) void k_pb_expand(const uint32_t* __restrict__ list,
                                                   const uint64_t* __restrict__ wpre, uint32_t jb, uint64_t wa,
                                                   uint64_t cnt, const uint32_t* __restrict__ tj,
                                                   const float* __restrict__ contrib, float* __restrict__ pc) {
    constexpr uint32_t PER = PB_EXP_TILE / 256;
    __shared__ uint16_t s_owner[PB_EXP_TILE];
    __shared__ float s_val[PB_EXP_TILE + 1];
    __shared__ uint32_t s_wave[4];
    const uint64_t ntiles = (cnt + PB_EXP_TILE - 1) / PB_EXP_TILE;
    for (uint64_t k = blockIdx.x; k < ntiles; k += gridDim.x) {
        const uint64_t t0 = k * PB_EXP_TILE;
        const uint32_t tc = (uint32_t)min((uint64_t)PB_EXP_TILE, cnt - t0);
        const uint32_t j0 = tj[k];
        // entries that start inside the tile: j0 + 1 .. (the next tile's first entry), each
        // at most one per slot
        const uint32_t jl = k + 1 < ntiles ? tj[k + 1] : jb - 1;
        const uint32_t nv = jl - j0 + 1;  // <= PB_EXP_TILE + 1
#pragma unroll
        for (uint32_t r = 0; r < PER; r++) s_owner[r * 256 + threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nv; i += 256) {
            const uint32_t j = j0 + i;
            s_val[i] = contrib[list[j]];
            if (i) {
                const uint64_t st = wpre[j] - wa;
                if (st < t0 + tc) s_owner[st - t0] = (uint16_t)i;
            }
        }
        __syncthreads();
        block_prefix_max_u16<PER>(s_owner, tc, s_wave);
#pragma unroll
        for (uint32_t r = 0; r < PER; r++) {
            const uint32_t q = r * 256 + threadIdx.x;
            if (q < tc) pc[t0 + q] = s_val[s_owner[q]];
        }
        __syncthreads();
    }
}

// First sort pass with fixed output places: workgroup w of the pass takes input slice
// [w * range, (w + 1) * range), and the pairs of that slice in bin k go to
// offA[w * nkeys + k] onwards (the slice's pairs and their bins are the same in every
// PageRank iteration, so the places are counted once).  No global atomics.
__global__ __launch_bounds__(PB_THREADS) void k_pb_count_a(const uint32_t* __restrict__ in_v, uint32_t vmask,
                                                           uint64_t cnt, uint64_t range, uint32_t kshift,
                                                           uint32_t nkeys, uint32_t* __restrict__ cntA,
                                                           uint32_t* __restrict__ err) {
    __shared__ uint32_t s_cnt[PB_LOCAL];
    for (uint32_t b = threadIdx.x; b < nkeys; b += PB_THREADS) s_cnt[b] = 0;
    __syncthreads();
    const uint64_t lo = blockIdx.x * range, hi = min(cnt, lo + range);
    bool bad = false;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += PB_THREADS) {
        const uint32_t k = (in_v[i] & vmask) >> kshift;
        if (k < nkeys)
            atomicAdd(&s_cnt[k], 1u);
        else
            bad = true;
    }
    if (bad) atomicOr(err, 1u);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nkeys; b += PB_THREADS) cntA[(uint64_t)blockIdx.x * nkeys + b] = s_cnt[b];
}

// offA[w][k] = start of bin k + pairs of bin k in slices before w (in place over cntA).
// One workgroup of PB_A_WG threads per bin k, thread w holding slice w.
__global__ __launch_bounds__(PB_A_WG) void k_pb_scan_a(uint32_t* __restrict__ cntA, uint32_t nwg, uint32_t nkeys,
                                                       uint32_t stride, const uint32_t* __restrict__ foff) {
    __shared__ uint32_t s_w[PB_A_WG / 64 + 1];
    const uint32_t k = blockIdx.x, w = threadIdx.x;
    const uint64_t at = (uint64_t)w * nkeys + k;
    const uint32_t c = w < nwg ? cntA[at] : 0u;
    uint32_t tot;
    const uint32_t before = block_excl_sum(c, s_w, &tot);
    if (w < nwg) cntA[at] = foff[k * stride] + before;
}

__global__ __launch_bounds__(PB_THREADS) void k_pb_scatter_a(const uint32_t* __restrict__ in_v, uint32_t vmask,
                                                             const float* __restrict__ in_c, uint64_t cnt,
                                                             uint64_t range, uint32_t kshift, uint32_t stride,
                                                             uint32_t nfine, const uint32_t* __restrict__ foff,
                                                             const uint32_t* __restrict__ offA,
                                                             uint32_t* __restrict__ out_v, float* __restrict__ out_c,
                                                             uint32_t* __restrict__ fcur, uint32_t* __restrict__ err) {
    constexpr uint32_t PER = PB_TILE / PB_THREADS;
    constexpr uint32_t LPER = PB_LOCAL / PB_THREADS;
    __shared__ uint32_t s_v[PB_TILE];
    __shared__ float s_c[PB_TILE];
    __shared__ uint16_t s_k[PB_TILE];
    __shared__ uint32_t s_cnt[PB_LOCAL], s_ofs[PB_LOCAL], s_run[PB_LOCAL], s_end[PB_LOCAL];
    __shared__ uint32_t s_w[PB_THREADS / 64 + 1];
    const uint32_t nkeys = (nfine + stride - 1) / stride;
    // the second pass's cursors start at the fine bins' starts
    if (fcur)
        for (uint32_t f = blockIdx.x * PB_THREADS + threadIdx.x; f < nfine; f += gridDim.x * PB_THREADS)
            fcur[f] = foff[f];
    for (uint32_t b = threadIdx.x; b < PB_LOCAL; b += PB_THREADS) {
        s_run[b] = b < nkeys ? offA[(uint64_t)blockIdx.x * nkeys + b] : 0u;
        s_end[b] = b < nkeys ? foff[min((b + 1) * stride, nfine)] : 0u;
    }
    bool bad = false;
    const uint64_t lo = blockIdx.x * range, hi = min(cnt, lo + range);
    uint32_t v[PER], key[PER], rank[PER];
    float c[PER];
    // every load of a tile in flight before any is used; the next tile's loads are issued
    // before the current tile is sorted
#pragma unroll
    for (uint32_t r = 0; r < PER; r++) {
        const uint64_t i = lo + r * PB_THREADS + threadIdx.x;
        v[r] = i < hi ? in_v[i] & vmask : 0u;
        c[r] = i < hi ? in_c[i] : 0.0f;
    }
    for (uint64_t t0 = lo; t0 < hi; t0 += PB_TILE) {
        const uint32_t tc = (uint32_t)min((uint64_t)PB_TILE, hi - t0);
        uint32_t nv[PER];
        float nc[PER];
#pragma unroll
        for (uint32_t r = 0; r < PER; r++) {
            const uint64_t i = t0 + PB_TILE + r * PB_THREADS + threadIdx.x;
            nv[r] = i < hi ? in_v[i] & vmask : 0u;
            nc[r] = i < hi ? in_c[i] : 0.0f;
        }
#pragma unroll
        for (uint32_t q = 0; q < LPER; q++) s_cnt[LPER * threadIdx.x + q] = 0;
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < PER; r++) {
            key[r] = PB_LOCAL;
            rank[r] = 0;
            if (r * PB_THREADS + threadIdx.x < tc) {
                const uint32_t k = v[r] >> kshift;
                if (k < nkeys) {
                    key[r] = k;
                    rank[r] = atomicAdd(&s_cnt[k], 1u);
                } else {
                    bad = true;
                }
            }
        }
        __syncthreads();
        uint32_t loc[LPER], sum = 0, tot;
#pragma unroll
        for (uint32_t q = 0; q < LPER; q++) {
            loc[q] = s_cnt[LPER * threadIdx.x + q];
            sum += loc[q];
        }
        uint32_t base = block_excl_sum(sum, s_w, &tot);
#pragma unroll
        for (uint32_t q = 0; q < LPER; q++) {
            s_ofs[LPER * threadIdx.x + q] = base;
            base += loc[q];
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < PER; r++)
            if (key[r] < PB_LOCAL) {
                const uint32_t p = s_ofs[key[r]] + rank[r];
                s_v[p] = v[r];
                s_c[p] = c[r];
                s_k[p] = (uint16_t)key[r];
            }
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < tot; p += PB_THREADS) {
            const uint32_t k = s_k[p];
            const uint32_t gpos = s_run[k] + (p - s_ofs[k]);
            if (gpos < s_end[k]) {
                out_v[gpos] = s_v[p];
                out_c[gpos] = s_c[p];
            } else {
                bad = true;
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t q = 0; q < LPER; q++) s_run[LPER * threadIdx.x + q] += loc[q];
        // the next tile's count reset follows this update (barrier after the reset)
#pragma unroll
        for (uint32_t r = 0; r < PER; r++) {
            v[r] = nv[r];
            c[r] = nc[r];
        }
    }
    if (bad) atomicOr(err, 1u);
}

constexpr int PB_ACC_THREADS = 512;
constexpr uint32_t PB_ACC_BATCH = 8;  // pairs per thread with loads in flight together

__global__ __launch_bounds__(PB_ACC_THREADS) void k_pb_accum(const uint32_t* __restrict__ pv,
                                                             const float* __restrict__ pc,
                                                             const uint32_t* __restrict__ foff,
                                                             const uint32_t* __restrict__ segs,
                                                             const uint32_t* __restrict__ nsegs, uint32_t seg,
                                                             uint64_t n, float* __restrict__ acc,
                                                             uint32_t* __restrict__ err) {
    constexpr uint32_t Q4 = PB_FINE / 4 / PB_ACC_THREADS;  // float4 slots per thread
    __shared__ float4 s_a4[PB_FINE / 4];
    float* s_a = (float*)s_a4;
    const uint32_t s = blockIdx.x;
    if (s >= *nsegs) return;  // the same for every thread of the workgroup
    const uint32_t f = segs[2 * s], j = segs[2 * s + 1];
    const uint32_t b0 = foff[f], b1 = foff[f + 1];
    const uint32_t start = b0 + j * seg;
    const uint32_t end = min(b1, start + seg);
    const bool multi = b1 - b0 > seg;
#pragma unroll
    for (uint32_t q = 0; q < Q4; q++) s_a4[q * PB_ACC_THREADS + threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    bool bad = false;
    for (uint32_t i0 = start; i0 < end; i0 += PB_ACC_BATCH * PB_ACC_THREADS) {
        uint32_t v[PB_ACC_BATCH];
        float c[PB_ACC_BATCH];
#pragma unroll
        for (uint32_t r = 0; r < PB_ACC_BATCH; r++) {
            const uint32_t i = i0 + r * PB_ACC_THREADS + threadIdx.x;
            v[r] = i < end ? pv[i] : UINT32_MAX;
            c[r] = i < end ? pc[i] : 0.0f;
        }
#pragma unroll
        for (uint32_t r = 0; r < PB_ACC_BATCH; r++) {
            if (i0 + r * PB_ACC_THREADS + threadIdx.x >= end) continue;
            if ((v[r] >> PB_FINE_SHIFT) == f && v[r] < n)
                atomicAdd(&s_a[acc_slot(v[r]) & (PB_FINE - 1)], c[r]);
            else
                bad = true;
        }
    }
    if (bad) atomicOr(err, 1u);
    __syncthreads();
    // the bin's accumulator slots: [base, base + lim), lim a multiple of 4096
    const uint64_t base = (uint64_t)f << PB_FINE_SHIFT;
    const uint32_t lim4 = (uint32_t)min((uint64_t)PB_FINE, acc_slots(n) - base) / 4;
    if (!multi) {
        float4* a4 = (float4*)(acc + base);
        float4 x[Q4];
#pragma unroll
        for (uint32_t q = 0; q < Q4; q++) {
            const uint32_t k = q * PB_ACC_THREADS + threadIdx.x;
            if (k < lim4) x[q] = a4[k];
        }
#pragma unroll
        for (uint32_t q = 0; q < Q4; q++) {
            const uint32_t k = q * PB_ACC_THREADS + threadIdx.x;
            if (k < lim4) {
                const float4 y = s_a4[k];
                x[q].x += y.x;
                x[q].y += y.y;
                x[q].z += y.z;
                x[q].w += y.w;
                a4[k] = x[q];
            }
        }
    } else {
        for (uint32_t q = threadIdx.x; q < lim4 * 4; q += PB_ACC_THREADS)
            if (s_a[q] != 0.0f) unsafeAtomicAdd(acc + base + q, s_a[q]);
    }
}

// ---------------------------------------------------------- filter stream
// One workgroup pass = one chunk of FSTREAM_LINES lines of one task.  All lines of the
// chunk are loaded (the filter engine transfers whole partitions); an edge is pushed
// when it lies in the out-edge range of one of the task's active vertices.
// The chunk's host loads are issued as soon as the chunk is located, so the search for
// its active vertices and their staging overlap the link latency.  Staged ranges are
// chunk-relative 16-bit offsets, and each edge finds its vertex through an owner map
// (the index of the last active vertex starting at or before it, by prefix maximum).
template <class Op>
__global__ __launch_bounds__(LINE_THREADS) void k_push_fstream(const FTask* __restrict__ tasks, uint32_t ntasks,
                                                               uint64_t total_chunks,
                                                               const uint32_t* __restrict__ list,
                                                               const uint64_t* __restrict__ off,
                                                               const uint32_t* __restrict__ col,
                                                               const uint32_t* __restrict__ w, Op op, Pack pk) {
    constexpr uint32_t MAXE = FSTREAM_LINES * 32;  // edges per chunk (1536)
    constexpr int UNROLL = FSTREAM_LINES / LINE_HALVES;
    static_assert(MAXE <= 8 * LINE_THREADS, "owner map prefix covers 8 entries per thread");
    static_assert(FSTREAM_LINES % LINE_HALVES == 0, "whole lines per half wave");
    __shared__ uint16_t s_owner[MAXE];  // chunk position -> staged vertex
    __shared__ uint16_t s_s[MAXE];      // staged vertex range, relative to the chunk start
    __shared__ uint16_t s_e[MAXE];
    __shared__ uint32_t s_val[MAXE];
    __shared__ uint32_t s_tmp, s_wave[LINE_THREADS / 64];
    const uint32_t half = threadIdx.x >> 5, lane = threadIdx.x & 31;
    for (uint64_t c = blockIdx.x; c < total_chunks; c += gridDim.x) {
        // task of chunk c: last t with tasks[t].chunk0 <= c (tasks[0].chunk0 = 0)
        const uint32_t ti = block_search_last(0, ntasks, [&](uint32_t j) { return tasks[j].chunk0 <= c; }, &s_tmp);
        const FTask t = tasks[ti];
        const uint64_t line0 = (t.e0 >> ZC_LINE_SHIFT) + (c - t.chunk0) * FSTREAM_LINES;
        const uint64_t ce0 = max(t.e0, line0 << ZC_LINE_SHIFT);
        const uint64_t ce1 = min(t.e1, (line0 + FSTREAM_LINES) << ZC_LINE_SHIFT);
        const uint32_t cnt = (uint32_t)(ce1 - ce0);  // edges of the chunk, <= MAXE
        // the transfer: every line of the chunk, loads in flight from here on
        uint32_t cv[UNROLL], wv[UNROLL];
#pragma unroll
        for (int r = 0; r < UNROLL; r++) {
            const uint64_t e = ((line0 + half + (uint64_t)LINE_HALVES * r) << ZC_LINE_SHIFT) + lane;
            cv[r] = 0;
            wv[r] = 0;
            if (e >= ce0 && e < ce1) {
                cv[r] = col[e];
                if (Op::weighted && pk.shift == 32) wv[r] = load_w(w, e, pk);
            }
        }
        // active vertices whose out-edge ranges meet [ce0, ce1): list entries [j0, j0 + nv)
        // (the list is in vertex order, so both range ends increase with j)
        uint32_t j0 = t.ja, nv = 0;
        if (t.ja < t.jb && off[list[t.ja] + 1] <= ce0)
            j0 = block_search_last(t.ja, t.jb, [&](uint32_t j) { return off[list[j] + 1] <= ce0; }, &s_tmp) + 1;
        if (j0 < t.jb && off[list[j0]] < ce1)
            nv = block_search_last(j0, t.jb, [&](uint32_t j) { return off[list[j]] < ce1; }, &s_tmp) + 1 - j0;
        if (nv > 0) {  // uniform across the workgroup
            for (uint32_t q = threadIdx.x; q < cnt; q += LINE_THREADS) s_owner[q] = 0;
            __syncthreads();
            for (uint32_t k = threadIdx.x; k < nv; k += LINE_THREADS) {
                const uint32_t v = list[j0 + k];
                const uint64_t vs = off[v], ve = off[v + 1];
                const uint32_t rs = vs > ce0 ? (uint32_t)(vs - ce0) : 0u;
                s_s[k] = (uint16_t)rs;
                s_e[k] = (uint16_t)((ve < ce1 ? ve : ce1) - ce0);
                s_val[k] = op.src(v);
                if (k) s_owner[rs] = (uint16_t)k;  // later vertices start inside the chunk
            }
            __syncthreads();
            block_prefix_max_u16<8>(s_owner, cnt, s_wave);
#pragma unroll
            for (int r = 0; r < UNROLL; r++) {
                const uint64_t e = ((line0 + half + (uint64_t)LINE_HALVES * r) << ZC_LINE_SHIFT) + lane;
                bool ok = false;
                uint32_t val = 0;
                if (e >= ce0 && e < ce1) {
                    const uint32_t q = (uint32_t)(e - ce0);
                    const uint32_t k = s_owner[q];
                    ok = q >= s_s[k] && q < s_e[k];
                    val = s_val[k];
                }
                push_if(op, ok, val, pk_v(cv[r], pk), Op::weighted ? pk_w(cv[r], wv[r], pk) : 0u);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ probes
__global__ __launch_bounds__(256) void k_zc_probe_lines(const uint32_t* __restrict__ src, uint64_t nlines,
                                                        uint32_t wpl, uint32_t* __restrict__ sink) {
    const uint32_t lane = threadIdx.x & 31;
    const uint64_t half = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 5;
    const uint64_t halves = ((uint64_t)gridDim.x * blockDim.x) >> 5;
    uint32_t acc = 0;
    for (uint64_t line = half; line < nlines; line += halves)
        if (lane < wpl) acc += src[(line << 5) + lane];
    if (acc == 0x9E3779B9u) sink[0] = acc;  // keeps the loads; practically never true
}

__global__ __launch_bounds__(256) void k_zc_probe_stream(const uint4* __restrict__ src, uint64_t n16,
                                                         uint32_t* __restrict__ sink) {
    uint32_t acc = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n16;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 v = src[i];
        acc += v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;
}

__global__ __launch_bounds__(256) void k_copy_probe(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                    uint64_t n16) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n16;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

inline unsigned grid_for(uint64_t items, unsigned per_block, unsigned cap) {
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

constexpr unsigned GRID_CAP = 1u << 16;

}  // namespace

hipError_t launch_init(const AlgoState& s, uint64_t n, uint32_t source, float pr_x0, float* pr_x, uint32_t* cur,
                       uint32_t nwords, hipStream_t st) {
    k_init<<<grid_for(n > nwords ? n : nwords, 256, 8192), 256, 0, st>>>(s, n, source, pr_x0, pr_x, cur, nwords);
    return hipGetLastError();
}

hipError_t launch_init_lanes(const AlgoState& s, const LaneSources& src, uint32_t* cur_union, uint32_t nwords,
                             hipStream_t st) {
    k_init_lanes<<<grid_for(s.n << s.lshift, 256, 16384), 256, 0, st>>>(s, src, cur_union, nwords);
    return hipGetLastError();
}

hipError_t launch_lane_union(const uint64_t* mask, uint64_t n, unsigned long long* lanes, hipStream_t st) {
    k_lane_union<<<grid_for(n, 256, 2048), 256, 0, st>>>(mask, n, lanes);
    return hipGetLastError();
}

hipError_t launch_extract_lanes(const uint32_t* vals, uint64_t n, uint32_t lshift, const LaneSet& set, bool sub_base,
                                const uint32_t* order, uint32_t* out, hipStream_t st) {
    const uint32_t nsel = (uint32_t)__builtin_popcountll(set.mask);
    if (!n || !nsel || lshift > 6 || (set.mask >> 1 >> ((1u << lshift) - 1))) return n && nsel ? hipErrorInvalidValue : hipSuccess;
    k_extract_lanes<<<grid_for(n, EX_V, 16384), 256, 0, st>>>(vals, n, lshift, set, nsel, sub_base, order, out);
    return hipGetLastError();
}

hipError_t launch_loaded_frontier(uint32_t npart, const uint32_t* pv, const uint8_t* mode, uint32_t mode_mask,
                                  const uint32_t* next, uint32_t* cur2, uint32_t nwords, hipStream_t st) {
    hipError_t e = launch_fill_u32(cur2, nwords, 0u, st);
    if (e != hipSuccess || !npart) return e;
    k_loaded_frontier<<<npart < GRID_CAP ? npart : GRID_CAP, 256, 0, st>>>(npart, pv, mode, mode_mask, next, cur2);
    return hipGetLastError();
}

hipError_t launch_dpr_fold(uint32_t npart, const uint32_t* pv, uint64_t n, float* acc, uint32_t copies, float* delta,
                           double* psum, hipStream_t st) {
    if (!npart) return hipSuccess;
    if (copies < 1 || copies > ACC_COPIES) return hipErrorInvalidValue;
    k_dpr_fold<<<npart < GRID_CAP ? npart : GRID_CAP, 256, 0, st>>>(npart, pv, n, acc, copies, delta, psum);
    return hipGetLastError();
}

hipError_t launch_dpr_activate(uint32_t npart, const uint32_t* pv, const uint64_t* off, const uint8_t* sched,
                               float* delta, float* x, float* contrib, uint32_t* cur, uint32_t nwords, float damping,
                               hipStream_t st) {
    hipError_t e = launch_fill_u32(cur, nwords, 0u, st);
    if (e != hipSuccess || !npart) return e;
    k_dpr_activate<<<npart < GRID_CAP ? npart : GRID_CAP, 256, 0, st>>>(npart, pv, off, sched, delta, x, contrib,
                                                                         cur, damping);
    return hipGetLastError();
}

hipError_t launch_dpr_finish(uint64_t n, float* x, const float* delta, hipStream_t st) {
    if (!n) return hipSuccess;
    k_dpr_finish<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, x, delta);
    return hipGetLastError();
}

hipError_t launch_gather_u32(const uint32_t* src, const uint32_t* rank, uint64_t n, uint32_t* dst, hipStream_t st) {
    if (!n) return hipSuccess;
    k_gather_u32<<<grid_for(n, 256, 8192), 256, 0, st>>>(src, rank, n, dst);
    return hipGetLastError();
}

hipError_t launch_cc_relabel(const uint32_t* lab, const uint32_t* order, const uint32_t* rank, uint64_t n,
                             uint32_t* minold, uint32_t* dst, hipStream_t st) {
    if (!n) return hipSuccess;
    hipError_t e = launch_fill_u32(minold, n, UNREACHED, st);
    if (e != hipSuccess) return e;
    k_cc_min_old<<<grid_for(n, 256, 8192), 256, 0, st>>>(lab, order, n, minold);
    k_cc_canon<<<grid_for(n, 256, 8192), 256, 0, st>>>(lab, minold, rank, n, dst);
    return hipGetLastError();
}

hipError_t launch_far_min(const uint32_t* far, const uint32_t* dist, uint32_t nwords, uint32_t* out, hipStream_t st) {
    if (!nwords) return hipSuccess;
    k_far_min<<<grid_for(nwords, 256, 8192), 256, 0, st>>>(far, dist, nwords, out);
    return hipGetLastError();
}

hipError_t launch_far_move(uint32_t* far, const uint32_t* dist, uint32_t* cur, uint32_t nwords, uint32_t bound,
                           hipStream_t st) {
    if (!nwords) return hipSuccess;
    k_far_move<<<grid_for(nwords, 256, 8192), 256, 0, st>>>(far, dist, cur, nwords, bound);
    return hipGetLastError();
}

hipError_t launch_sssp_ovf_check(const uint64_t* off, const uint32_t* col, const Pack& pk, const uint32_t* dist,
                                 uint32_t lshift, uint64_t mask, uint64_t n, unsigned long long* out, hipStream_t st) {
    if (!n || !mask || lshift > 6) return lshift > 6 ? hipErrorInvalidValue : hipSuccess;
    k_sssp_ovf_check<<<grid_for(n, 4, 16384), 256, 0, st>>>(off, col, pk, dist, lshift, mask, n, out);
    return hipGetLastError();
}

hipError_t launch_admit_lanes(const AlgoState& s, const LaneSet& set, uint32_t* cur, hipStream_t st) {
    if (!set.mask) return hipSuccess;
    k_admit_lanes<<<1, MAX_LANES, 0, st>>>(s, set, cur);
    return hipGetLastError();
}

hipError_t launch_reset_lanes(const AlgoState& s, uint64_t mask, hipStream_t st) {
    if (!mask || !s.n) return hipSuccess;
    k_reset_lanes<<<grid_for(s.n << s.lshift, 256, 16384), 256, 0, st>>>(s, mask);
    return hipGetLastError();
}

hipError_t launch_ppr_prepare(const AlgoState& s, const uint64_t* off, hipStream_t st) {
    if (!s.n) return hipSuccess;
    k_ppr_prepare<<<grid_for(s.n, 256, 8192), 256, 0, st>>>(s, off);
    return hipGetLastError();
}

hipError_t launch_ppr_apply(const AlgoState& s, float damping, hipStream_t st) {
    if (!s.n) return hipSuccess;
    k_ppr_apply<<<grid_for(s.n, 256, 8192), 256, 0, st>>>(s, damping);
    return hipGetLastError();
}

hipError_t launch_ppr_restart(const AlgoState& s, const LaneSet& set, float restart, hipStream_t st) {
    if (!set.mask) return hipSuccess;
    k_ppr_restart<<<1, MAX_LANES, 0, st>>>(s, set, restart);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t st) {
    if (!count) return hipSuccess;
    k_fill_u32<<<grid_for(count, 256, 8192), 256, 0, st>>>(p, count, value);
    return hipGetLastError();
}

hipError_t launch_stats_select(uint32_t npart, const uint32_t* pv, const uint64_t* off, const uint32_t* cur,
                               const SelParams& sp, uint8_t* mode, uint32_t* nA, uint32_t* nF, uint64_t* Ea,
                               uint64_t* Rq, uint64_t* K, hipStream_t st) {
    if (!npart) return hipSuccess;
    k_stats_select<<<grid_for(npart, 4, GRID_CAP), 256, 0, st>>>(npart, pv, off, cur, sp, mode, nA, nF, Ea,
                                                                         Rq, K);
    return hipGetLastError();
}

hipError_t launch_scan(uint32_t npart, const uint8_t* mode, const uint32_t* nA, const uint32_t* nF,
                       const uint64_t* Ea, const uint64_t* Rq, const uint64_t* K, uint32_t* lbase, uint64_t* wbase,
                       Header* hdr, uint64_t* wpre, uint64_t* scratch, hipStream_t st) {
    const uint32_t ntiles = scan_tiles(npart);
    uint64_t* tile_tot = scratch;
    uint64_t* tile_base = scratch + (uint64_t)ntiles * SCAN_NV;
    if (ntiles) k_scan_tot<<<ntiles, SCAN_THREADS, 0, st>>>(npart, mode, nA, nF, Ea, Rq, K, tile_tot);
    k_scan_base<<<1, 64, 0, st>>>(ntiles, tile_tot, tile_base, hdr, wpre);
    if (ntiles) k_scan_write<<<ntiles, SCAN_THREADS, 0, st>>>(npart, mode, nA, Ea, K, tile_base, lbase, wbase);
    return hipGetLastError();
}

hipError_t launch_build_lists(uint32_t npart, const uint32_t* pv, const uint64_t* off, const uint32_t* cur,
                              const uint8_t* mode, const uint32_t* lbase, const uint64_t* wbase, uint32_t* list,
                              uint64_t* wpre, hipStream_t st) {
    if (!npart) return hipSuccess;
    k_build_lists<<<grid_for(npart, 4, GRID_CAP), 256, 0, st>>>(npart, pv, off, cur, mode, lbase, wbase,
                                                                        list, wpre);
    return hipGetLastError();
}

template <class Op>
static hipError_t push_edges_op(const Op& op, const uint32_t* list, const uint64_t* wpre, uint32_t ja, uint32_t jb,
                                uint64_t lo, uint64_t hi, const uint64_t* off, const uint32_t* col,
                                const uint32_t* w, uint64_t shift, bool compacted, const Pack& pk, hipStream_t st) {
    const unsigned g = grid_for(hi - lo, EDGE_IPB, GRID_CAP);
    if (compacted)
        k_push_edges<Op, true><<<g, EDGE_THREADS, 0, st>>>(list, wpre, ja, jb, lo, hi, off, col, w, shift, op, pk);
    else
        k_push_edges<Op, false><<<g, EDGE_THREADS, 0, st>>>(list, wpre, ja, jb, lo, hi, off, col, w, shift, op, pk);
    return hipGetLastError();
}

hipError_t launch_push_edges(const AlgoState& s, const uint32_t* list, const uint64_t* wpre, uint32_t ja,
                             uint32_t jb, uint64_t item_lo, uint64_t item_hi, const uint64_t* off,
                             const uint32_t* col, const uint32_t* w, uint64_t shift, bool compacted,
                             hipStream_t st) {
    if (item_hi <= item_lo || jb <= ja) return hipSuccess;
    switch (s.algo) {
    case ALGO_BFS:
        return push_edges_op(OpBfs{s.visited, s.next, s.val, s.level_next}, list, wpre, ja, jb, item_lo, item_hi,
                             off, col, w, shift, compacted, s.pk, st);
    case ALGO_SSSP:
        return push_edges_op(OpSssp{s.val, s.next, s.overflow, s.far, s.bound}, list, wpre, ja, jb, item_lo, item_hi, off, col, w,
                             shift, compacted, s.pk, st);
    case ALGO_CC:
        return push_edges_op(OpCc{s.val, s.next}, list, wpre, ja, jb, item_lo, item_hi, off, col, w, shift,
                             compacted, s.pk, st);
    case ALGO_BFS_RELAX:
        return push_edges_op(OpBfsRelax{s.val, s.next}, list, wpre, ja, jb, item_lo, item_hi, off, col, w, shift,
                             compacted, s.pk, st);
    case ALGO_MBFS:
        return push_edges_op(OpMBfs{s.mcur, s.mnext, s.mvisited, s.lval, s.next, s.level_next, s.lshift}, list, wpre, ja, jb,
                             item_lo, item_hi, off, col, w, shift, compacted, s.pk, st);
    case ALGO_MSSSP:
        return push_edges_op(OpMSssp{s.mcur, s.mnext, s.lval, s.next, s.overflow, s.lshift}, list, wpre, ja, jb, item_lo,
                             item_hi, off, col, w, shift, compacted, s.pk, st);
    case ALGO_MPPR:
        return push_edges_op(OpMPpr{s.mcur, s.mnext, s.lx, s.lacc, s.next, s.lshift}, list, wpre, ja, jb, item_lo,
                             item_hi, off, col, w, shift, compacted, s.pk, st);
    default:
        return push_edges_op(OpPr{s.acc, acc_slots(s.n), s.contrib, s.acc_copies - 1}, list, wpre, ja, jb, item_lo, item_hi, off, col, w, shift,
                             compacted, s.pk, st);
    }
}

template <class Op>
static hipError_t push_lines_op(const Op& op, const uint32_t* list, const uint64_t* wpre, uint32_t ja, uint32_t jb,
                                uint64_t lo, uint64_t hi, const uint64_t* off, const uint32_t* col,
                                const uint32_t* w, unsigned long long* distinct, const Pack& pk, hipStream_t st,
                                unsigned cap = GRID_CAP) {
    const unsigned g = grid_for(hi - lo, LINE_IPB, cap ? cap : GRID_CAP);
    k_push_lines<Op><<<g, LINE_THREADS, 0, st>>>(list, wpre, ja, jb, lo, hi, off, col, w, op, distinct, pk);
    return hipGetLastError();
}

hipError_t launch_push_lines(const AlgoState& s, const uint32_t* list, const uint64_t* wpre, uint32_t ja,
                             uint32_t jb, uint64_t item_lo, uint64_t item_hi, const uint64_t* off,
                             const uint32_t* col, const uint32_t* w, unsigned long long* distinct, hipStream_t st) {
    if (item_hi <= item_lo || jb <= ja) return hipSuccess;
    switch (s.algo) {
    case ALGO_BFS:
        return push_lines_op(OpBfs{s.visited, s.next, s.val, s.level_next}, list, wpre, ja, jb, item_lo, item_hi,
                             off, col, w, distinct, s.pk, st);
    case ALGO_SSSP:
        return push_lines_op(OpSssp{s.val, s.next, s.overflow, s.far, s.bound}, list, wpre, ja, jb, item_lo, item_hi, off, col, w, distinct, s.pk, st);
    case ALGO_CC:
        return push_lines_op(OpCc{s.val, s.next}, list, wpre, ja, jb, item_lo, item_hi, off, col, w, distinct, s.pk, st);
    case ALGO_BFS_RELAX:
        return push_lines_op(OpBfsRelax{s.val, s.next}, list, wpre, ja, jb, item_lo, item_hi, off, col, w, distinct, s.pk, st);
    case ALGO_MBFS:
        return push_lines_op(OpMBfs{s.mcur, s.mnext, s.mvisited, s.lval, s.next, s.level_next, s.lshift}, list, wpre, ja, jb,
                             item_lo, item_hi, off, col, w, distinct, s.pk, st);
    case ALGO_MSSSP:
        return push_lines_op(OpMSssp{s.mcur, s.mnext, s.lval, s.next, s.overflow, s.lshift}, list, wpre, ja, jb, item_lo,
                             item_hi, off, col, w, distinct, s.pk, st);
    case ALGO_MPPR:
        return push_lines_op(OpMPpr{s.mcur, s.mnext, s.lx, s.lacc, s.next, s.lshift}, list, wpre, ja, jb, item_lo,
                             item_hi, off, col, w, distinct, s.pk, st);
    default:
        return push_lines_op(OpPr{s.acc, acc_slots(s.n), s.contrib, s.acc_copies - 1}, list, wpre, ja, jb, item_lo, item_hi, off, col, w,
                             distinct, s.pk, st, s.link_grid);
    }
}

hipError_t launch_pr_prepare(uint64_t n, const uint64_t* off, const float* x, float* contrib, float* acc,
                             uint32_t copies, hipStream_t st) {
    if (!n) return hipSuccess;
    if (copies < 1 || copies > ACC_COPIES + 1) return hipErrorInvalidValue;
    k_pr_prepare<<<grid_for(acc_slots(n), 256, 8192), 256, 0, st>>>(n, off, x, contrib, acc, copies);
    return hipGetLastError();
}

hipError_t launch_pb_hist(const uint32_t* pv, uint32_t vmask, uint64_t cnt, uint32_t nfine, uint32_t* hist,
                          uint32_t* err, hipStream_t st) {
    if (!cnt) return hipSuccess;
    if (nfine == 0 || nfine > PB_MAX_FINE) return hipErrorInvalidValue;
    const unsigned g = (unsigned)std::min<uint64_t>(256, (cnt + 4095) / 4096);
    k_pb_hist<<<g, PB_THREADS, 0, st>>>(pv, vmask, cnt, nfine, hist, err);
    return hipGetLastError();
}

hipError_t launch_pb_plan(const uint32_t* hist, uint32_t nfine, uint32_t seg, uint32_t* foff, uint32_t* segs,
                          uint32_t* nsegs, hipStream_t st) {
    if (nfine == 0 || nfine > PB_MAX_FINE || seg == 0) return hipErrorInvalidValue;
    k_pb_plan<<<1, PB_PLAN_THREADS, 0, st>>>(hist, nfine, seg, foff, segs, nsegs);
    return hipGetLastError();
}

hipError_t launch_pb_scatter(const uint32_t* in_v, const float* in_c, uint64_t cnt, uint32_t kshift, uint32_t stride,
                             uint32_t nfine, const uint32_t* foff, uint32_t* cursor, uint32_t* out_v, float* out_c,
                             uint32_t* err, hipStream_t st) {
    if (!cnt) return hipSuccess;
    if (nfine == 0 || nfine > PB_MAX_FINE || (stride != 1 && stride != PB_FINE_PER_COARSE) ||
        (1u << kshift) != stride * PB_FINE)
        return hipErrorInvalidValue;
    k_pb_scatter<<<grid_for(cnt, PB_TILE, 2048), PB_THREADS, 0, st>>>(in_v, in_c, cnt, kshift, stride, nfine, foff,
                                                                      cursor, out_v, out_c, err);
    return hipGetLastError();
}

hipError_t launch_pb_tiles(const uint64_t* wpre, uint32_t ja, uint32_t jb, uint64_t wa, uint64_t cnt, uint32_t* tj,
                           hipStream_t st) {
    if (!cnt) return hipSuccess;
    if (jb <= ja) return hipErrorInvalidValue;
    const uint64_t ntiles = (cnt + PB_EXP_TILE - 1) / PB_EXP_TILE;
    k_pb_tiles<<<grid_for(ntiles, 256, 1024), 256, 0, st>>>(wpre, ja, jb, wa, cnt, tj);
    return hipGetLastError();
}

hipError_t launch_pb_expand(const uint32_t* list, const uint64_t* wpre, uint32_t jb, uint64_t wa, uint64_t cnt,
                            const uint32_t* tj, const float* contrib, float* pc, hipStream_t st) {
    if (!cnt) return hipSuccess;
    const uint64_t ntiles = (cnt + PB_EXP_TILE - 1) / PB_EXP_TILE;
    k_pb_expand<<<(unsigned)std::min<uint64_t>(ntiles, 4096), 256, 0, st>>>(list, wpre, jb, wa, cnt, tj, contrib, pc);
    return hipGetLastError();
}

// Slices of the first sort pass: `wg` workgroups of `range` pairs (a multiple of PB_TILE).
void pb_slices(uint64_t cnt, uint32_t* wg, uint64_t* range) {
    const uint64_t tiles = (cnt + PB_TILE - 1) / PB_TILE;
    const uint64_t per = (tiles + PB_A_WG - 1) / PB_A_WG;
    *range = std::max<uint64_t>(per, 1) * PB_TILE;
    *wg = (uint32_t)std::max<uint64_t>(1, (cnt + *range - 1) / *range);
}

hipError_t launch_pb_plan_a(const uint32_t* pv, uint32_t vmask, uint64_t cnt, uint32_t kshift, uint32_t stride,
                            uint32_t nfine, const uint32_t* foff, uint32_t* offA, uint32_t* err, hipStream_t st) {
    if (!cnt) return hipSuccess;
    const uint32_t nkeys = (nfine + stride - 1) / stride;
    if (nfine == 0 || nfine > PB_MAX_FINE || nkeys > PB_LOCAL || (1u << kshift) != stride * PB_FINE)
        return hipErrorInvalidValue;
    uint32_t wg;
    uint64_t range;
    pb_slices(cnt, &wg, &range);
    k_pb_count_a<<<wg, PB_THREADS, 0, st>>>(pv, vmask, cnt, range, kshift, nkeys, offA, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pb_scan_a<<<nkeys, PB_A_WG, 0, st>>>(offA, wg, nkeys, stride, foff);
    return hipGetLastError();
}

hipError_t launch_pb_scatter_a(const uint32_t* in_v, uint32_t vmask, const float* in_c, uint64_t cnt,
                               uint32_t kshift, uint32_t stride, uint32_t nfine, const uint32_t* foff,
                               const uint32_t* offA, uint32_t* out_v, float* out_c, uint32_t* fcur, uint32_t* err,
                               hipStream_t st) {
    if (!cnt) return hipSuccess;
    const uint32_t nkeys = (nfine + stride - 1) / stride;
    if (nfine == 0 || nfine > PB_MAX_FINE || nkeys > PB_LOCAL || (1u << kshift) != stride * PB_FINE)
        return hipErrorInvalidValue;
    uint32_t wg;
    uint64_t range;
    pb_slices(cnt, &wg, &range);
    k_pb_scatter_a<<<wg, PB_THREADS, 0, st>>>(in_v, vmask, in_c, cnt, range, kshift, stride, nfine, foff, offA, out_v,
                                              out_c, fcur, err);
    return hipGetLastError();
}

hipError_t launch_pb_accum(const uint32_t* pv, const float* pc, const uint32_t* foff, const uint32_t* segs,
                           const uint32_t* nsegs, uint32_t max_segs, uint32_t seg, uint64_t n, float* acc,
                           uint32_t* err, hipStream_t st) {
    if (!max_segs || !n) return hipSuccess;
    if (seg == 0) return hipErrorInvalidValue;
    k_pb_accum<<<max_segs, PB_ACC_THREADS, 0, st>>>(pv, pc, foff, segs, nsegs, seg, n, acc, err);
    return hipGetLastError();
}

template <class Op>
static hipError_t push_fstream_op(const Op& op, const FTask* tasks, uint32_t ntasks, uint64_t chunks,
                                  const uint32_t* list, const uint64_t* off, const uint32_t* col, const uint32_t* w,
                                  const Pack& pk, hipStream_t st, unsigned cap = GRID_CAP) {
    const unsigned c = cap ? cap : GRID_CAP;
    const unsigned g = (unsigned)(chunks < c ? chunks : c);
    k_push_fstream<Op><<<g, LINE_THREADS, 0, st>>>(tasks, ntasks, chunks, list, off, col, w, op, pk);
    return hipGetLastError();
}

hipError_t launch_push_fstream(const AlgoState& s, const FTask* tasks, uint32_t ntasks, uint64_t total_chunks,
                               const uint32_t* list, const uint64_t* off, const uint32_t* col, const uint32_t* w,
                               hipStream_t st) {
    if (!ntasks || !total_chunks) return hipSuccess;
    switch (s.algo) {
    case ALGO_BFS:
        return push_fstream_op(OpBfs{s.visited, s.next, s.val, s.level_next}, tasks, ntasks, total_chunks, list,
                               off, col, w, s.pk, st);
    case ALGO_SSSP:
        return push_fstream_op(OpSssp{s.val, s.next, s.overflow, s.far, s.bound}, tasks, ntasks, total_chunks, list, off, col, w, s.pk, st);
    case ALGO_CC:
        return push_fstream_op(OpCc{s.val, s.next}, tasks, ntasks, total_chunks, list, off, col, w, s.pk, st);
    case ALGO_BFS_RELAX:
        return push_fstream_op(OpBfsRelax{s.val, s.next}, tasks, ntasks, total_chunks, list, off, col, w, s.pk, st);
    case ALGO_MBFS:
        return push_fstream_op(OpMBfs{s.mcur, s.mnext, s.mvisited, s.lval, s.next, s.level_next, s.lshift}, tasks, ntasks,
                               total_chunks, list, off, col, w, s.pk, st);
    case ALGO_MSSSP:
        return push_fstream_op(OpMSssp{s.mcur, s.mnext, s.lval, s.next, s.overflow, s.lshift}, tasks, ntasks, total_chunks,
                               list, off, col, w, s.pk, st);
    case ALGO_MPPR:
        return push_fstream_op(OpMPpr{s.mcur, s.mnext, s.lx, s.lacc, s.next, s.lshift}, tasks, ntasks, total_chunks,
                               list, off, col, w, s.pk, st);
    default:
        return push_fstream_op(OpPr{s.acc, acc_slots(s.n), s.contrib, s.acc_copies - 1}, tasks, ntasks, total_chunks, list, off, col, w,
                               s.pk, st, s.link_grid);
    }
}

hipError_t launch_pr_apply(uint64_t n, float* x, const float* acc, uint32_t copies, float base, float damping,
                           const float* inv_n, float restart, hipStream_t st) {
    if (!n) return hipSuccess;
    if (copies < 1 || copies > ACC_COPIES + 1) return hipErrorInvalidValue;
    k_pr_apply<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, x, acc, copies, base, damping, inv_n, restart);
    return hipGetLastError();
}

hipError_t launch_dpr_init(uint64_t n, float* delta, const float* inv_n, float restart, hipStream_t st) {
    if (!n) return hipSuccess;
    k_dpr_init<<<grid_for(n, 256, 8192), 256, 0, st>>>(n, delta, inv_n, restart, (float)((double)restart / (double)n));
    return hipGetLastError();
}

hipError_t launch_zc_probe(const uint32_t* src, uint64_t bytes, uint32_t words_per_line, uint32_t* sink,
                           hipStream_t st) {
    if (words_per_line == 0)
        k_zc_probe_stream<<<4096, 256, 0, st>>>((const uint4*)src, bytes / 16, sink);
    else
        k_zc_probe_lines<<<4096, 256, 0, st>>>(src, bytes / 128, words_per_line, sink);
    return hipGetLastError();
}

hipError_t launch_copy_probe(void* dst, const void* src, uint64_t bytes, hipStream_t st) {
    k_copy_probe<<<8192, 256, 0, st>>>((uint4*)dst, (const uint4*)src, bytes / 16);
    return hipGetLastError();
}

hipError_t launch_select_only(uint64_t npart, const uint64_t* E, const uint64_t* nA, const uint64_t* Ea,
                              const uint64_t* Rq, const SelParams& sp, uint8_t* p, hipStream_t st) {
    if (!npart) return hipSuccess;
    k_select_only<<<grid_for(npart, 256, 4096), 256, 0, st>>>(npart, E, nA, Ea, Rq, sp, p);
    return hipGetLastError();
}

// Scratch of the allocation-free selection: the four statistics arrays (uint64 x npart
// each) followed by the engine codes (npart bytes), for at most STATIC_SEL_MAX_PARTS
// partitions.  Each device holds its own copy for the life of the process.  In host code
// the array's name stands for no device address; its address on the current device comes
// from hipGetSymbolAddress, once per device, below.
static __device__ __align__(256) uint64_t scratch[STATIC_SEL_WORDS];

hipError_t static_select_scratch(int device, uint64_t** out) {
    static std::mutex mu;
    static uint64_t* ptr[STATIC_SCRATCH_DEVICES] = {};
    if (device < 0 || device >= STATIC_SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
        void* at = nullptr;
        e = hipGetSymbolAddress(&at, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[device] = (uint64_t*)at;
    }
    *out = ptr[device];
    return hipSuccess;
}

}  // namespace hytm
