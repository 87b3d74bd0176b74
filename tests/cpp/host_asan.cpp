// Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed): the
// input generator (gen.c) at vertex counts that are not powers of two -- its bucketed CSR
// build covers 2^ceil(log2 n) ids, so the buckets past n must be left alone -- and the
// runtime's hub sorting (hubsort.cpp) on the graphs it makes, with several threads.
// Built and run by tests/test_host_asan.py.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hubsort.h"

extern "C" {
struct gen_graph;
gen_graph* gen_er(uint64_t n, uint64_t nsamples, uint64_t seed);
gen_graph* gen_rmat(int scale, uint64_t nsamples, double a, double b, double c, uint64_t seed);
gen_graph* gen_symmetrize_csr(uint64_t n, const uint64_t* off, const uint32_t* col);
void gen_set_threads(int t);
uint64_t gen_num_vertices(const gen_graph* g);
uint64_t gen_num_edges(const gen_graph* g);
void gen_copy_out(const gen_graph* g, uint64_t* off, uint32_t* col);
void gen_free(gen_graph* g);
void gen_weights(uint64_t n, const uint64_t* off, const uint32_t* col, uint64_t seed, uint32_t maxw, uint32_t* w);
uint64_t gen_sources(uint64_t n, const uint64_t* off, uint64_t k, uint64_t seed, uint32_t* out);
}

static int fails = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::printf("check failed: %s (line %d)\n", #c, __LINE__);    \
            fails++;                                                      \
        }                                                                 \
    } while (0)

struct Csr {
    uint64_t n = 0, m = 0;
    std::vector<uint64_t> off;
    std::vector<uint32_t> col;
};

static Csr take(gen_graph* g) {
    Csr c;
    if (!g) {
        std::printf("generation failed\n");
        std::exit(1);
    }
    c.n = gen_num_vertices(g);
    c.m = gen_num_edges(g);
    c.off.resize(c.n + 1);
    c.col.resize(c.m ? c.m : 1);
    gen_copy_out(g, c.off.data(), c.col.data());
    gen_free(g);
    return c;
}

static void check_csr(const Csr& c) {
    CHECK(c.off[0] == 0 && c.off[c.n] == c.m);
    for (uint64_t u = 0; u < c.n; u++) {
        CHECK(c.off[u] <= c.off[u + 1]);
        for (uint64_t e = c.off[u]; e < c.off[u + 1]; e++) {
            CHECK(c.col[e] < c.n && c.col[e] != u);
            if (e > c.off[u]) CHECK(c.col[e - 1] < c.col[e]);  // sorted, no duplicates
        }
    }
}

static void check_hubsort(const Csr& c, unsigned threads) {
    std::vector<uint32_t> order(c.n), rank(c.n), w(c.m ? c.m : 1), col2(c.m ? c.m : 1), w2(c.m ? c.m : 1);
    std::vector<uint64_t> off2(c.n + 1);
    gen_weights(c.n, c.off.data(), c.col.data(), 7, 64, w.data());
    const uint64_t hubs = hytm::hub_order(c.n, c.off.data(), c.col.data(), 2, 25, threads, order.data(), rank.data());
    CHECK(hubs <= c.n * 2 / 25);
    for (uint64_t i = 0; i < c.n; i++) CHECK(rank[order[i]] == i);
    hytm::hub_relabel(c.n, c.off.data(), c.col.data(), w.data(), order.data(), rank.data(), threads, off2.data(),
                      col2.data(), w2.data());
    CHECK(off2[c.n] == c.m);
    for (uint64_t i = 0; i < c.n; i++) CHECK(off2[i + 1] - off2[i] == c.off[order[i] + 1] - c.off[order[i]]);
}

int main() {
    gen_set_threads(4);
    for (uint64_t n : {17000ull, 100003ull, 65537ull, 1ull << 16}) {
        Csr er = take(gen_er(n, 4 * n, 9));
        check_csr(er);
        Csr sym = take(gen_symmetrize_csr(er.n, er.off.data(), er.col.data()));
        check_csr(sym);
        check_hubsort(er, 4);
        std::vector<uint32_t> src(8);
        CHECK(gen_sources(er.n, er.off.data(), 8, 3, src.data()) <= 8);
    }
    Csr r = take(gen_rmat(17, 8ull << 17, 0.57, 0.19, 0.19, 17));
    check_csr(r);
    check_hubsort(r, 4);
    check_hubsort(r, 1);
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
