// Hub sorting (Sec. 6.1): relabel a CSR graph so that its most important vertices come
// first.  Host code, run once when a graph is loaded.
#pragma once
#include <cstdint>

namespace hytm {

// order[i] = original id of new vertex i, rank[v] = new id of original vertex v.  The hubs
// are the floor(n * num / den) vertices with the largest D_o(v) * D_i(v) (the paper's
// H(v) up to its constant denominator) among those with a non-zero score, ties to the
// smaller id; they come first in decreasing score, then every other vertex in increasing
// id.  Returns the number of hubs.
uint64_t hub_order(uint64_t n, const uint64_t* off, const uint32_t* col, uint32_t num, uint32_t den,
                   unsigned threads, uint32_t* order, uint32_t* rank);

// The relabelled graph: new vertex i has the out-edges of order[i], each neighbour v
// written as rank[v], every list sorted by new neighbour id (weights follow their edge).
// off2 has n + 1 entries; w / w2 may be null.
void hub_relabel(uint64_t n, const uint64_t* off, const uint32_t* col, const uint32_t* w, const uint32_t* order,
                 const uint32_t* rank, unsigned threads, uint64_t* off2, uint32_t* col2, uint32_t* w2);

}  // namespace hytm
