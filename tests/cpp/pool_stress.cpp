// Stress test of the compaction engine's thread pool (host only): thousands of short
// run() calls whose work items live on the caller's stack; every item must run exactly
// once per call.  Built with ThreadSanitizer by tests/test_host_pool.py.
#include <atomic>
#include <cstdio>
#include <vector>

#include "pool.h"

int main() {
    hytm::Pool pool(8);
    for (int rep = 0; rep < 3000; rep++) {
        const unsigned count = 1 + (rep * 7919) % 37;
        std::vector<std::atomic<int>> hits(count);
        for (auto& h : hits) h = 0;
        pool.run(count, [&](unsigned i) { hits[i].fetch_add(1); });
        for (unsigned i = 0; i < count; i++)
            if (hits[i] != 1) {
                std::printf("rep %d item %u ran %d times\n", rep, i, (int)hits[i]);
                return 1;
            }
    }
    std::printf("ok\n");
    return 0;
}
