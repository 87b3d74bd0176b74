// Hub sorting (Sec. 6.1), host side.  See hubsort.h.
#include "hubsort.h"

#include <algorithm>
#include <thread>
#include <vector>

namespace hytm {
namespace {

template <class F>
void parallel_ranges(uint64_t count, unsigned threads, F&& f) {
    threads = std::max(1u, threads);
    if (count < (1u << 16) || threads == 1) {
        f(0, count);
        return;
    }
    std::vector<std::thread> th;
    const uint64_t step = (count + threads - 1) / threads;
    for (unsigned t = 0; t < threads; t++) {
        const uint64_t a = std::min(count, t * step), b = std::min(count, a + step);
        if (a < b) th.emplace_back([&f, a, b] { f(a, b); });
    }
    for (auto& x : th) x.join();
}

struct Scored {
    unsigned __int128 score;
    uint32_t v;
    bool operator<(const Scored& o) const {  // higher score first, then smaller id
        return score != o.score ? score > o.score : v < o.v;
    }
};

}  // namespace

uint64_t hub_order(uint64_t n, const uint64_t* off, const uint32_t* col, uint32_t num, uint32_t den,
                   unsigned threads, uint32_t* order, uint32_t* rank) {
    std::vector<uint32_t> din(n, 0);
    parallel_ranges(off[n], threads, [&](uint64_t a, uint64_t b) {
        for (uint64_t e = a; e < b; e++) __atomic_fetch_add(&din[col[e]], 1u, __ATOMIC_RELAXED);
    });
    std::vector<Scored> cand;
    for (uint64_t v = 0; v < n; v++) {
        const unsigned __int128 s = (unsigned __int128)(off[v + 1] - off[v]) * din[v];
        if (s) cand.push_back({s, (uint32_t)v});
    }
    const uint64_t k = std::min<uint64_t>(cand.size(), (uint64_t)(((unsigned __int128)n * num) / den));
    if (k < cand.size()) std::nth_element(cand.begin(), cand.begin() + k, cand.end());
    std::sort(cand.begin(), cand.begin() + k);
    for (uint64_t v = 0; v < n; v++) rank[v] = UINT32_MAX;
    for (uint64_t i = 0; i < k; i++) {
        order[i] = cand[i].v;
        rank[cand[i].v] = (uint32_t)i;
    }
    uint64_t i = k;
    for (uint64_t v = 0; v < n; v++)
        if (rank[v] == UINT32_MAX) {
            order[i] = (uint32_t)v;
            rank[v] = (uint32_t)i++;
        }
    return k;
}

void hub_relabel(uint64_t n, const uint64_t* off, const uint32_t* col, const uint32_t* w, const uint32_t* order,
                 const uint32_t* rank, unsigned threads, uint64_t* off2, uint32_t* col2, uint32_t* w2) {
    off2[0] = 0;
    for (uint64_t i = 0; i < n; i++) off2[i + 1] = off2[i] + (off[order[i] + 1] - off[order[i]]);
    // hubs, the longest lists, sit at the front: blocks of vertices are handed out on demand
    constexpr uint64_t kBlock = 4096;
    uint64_t next = 0;
    auto worker = [&] {
        std::vector<uint64_t> tmp;
        for (;;) {
            const uint64_t a = __atomic_fetch_add(&next, kBlock, __ATOMIC_RELAXED);
            if (a >= n) break;
            for (uint64_t i = a; i < std::min(n, a + kBlock); i++) {
                const uint32_t v = order[i];
                const uint64_t s = off[v], d = off[v + 1] - s;
                tmp.resize(d);
                // (new neighbour, weight) packed so that one sort orders by neighbour
                for (uint64_t j = 0; j < d; j++) tmp[j] = ((uint64_t)rank[col[s + j]] << 32) | (w ? w[s + j] : 0u);
                std::sort(tmp.begin(), tmp.end());
                uint32_t* c2 = col2 + off2[i];
                for (uint64_t j = 0; j < d; j++) c2[j] = (uint32_t)(tmp[j] >> 32);
                if (w) {
                    uint32_t* x2 = w2 + off2[i];
                    for (uint64_t j = 0; j < d; j++) x2[j] = (uint32_t)tmp[j];
                }
            }
        }
    };
    const unsigned t = n < (1u << 16) ? 1u : std::max(1u, threads);
    std::vector<std::thread> th;
    for (unsigned i = 1; i < t; i++) th.emplace_back(worker);
    worker();
    for (auto& x : th) x.join();
}

}  // namespace hytm
