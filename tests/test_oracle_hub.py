"""Pins for the oracle's hub sorting order (Sec. 6.1): closed forms on a star and a
bipartite graph, and the ranking by the paper's normalized score H(v) computed with
exact fractions, against an independent lexicographic sort."""
from fractions import Fraction

import numpy as np
from hypothesis import given, settings, strategies as st

import gen
import oracle


def csr(n, edges):
    return gen.from_pairs(n, np.array([e[0] for e in edges], np.uint32), np.array([e[1] for e in edges], np.uint32))


def test_star_center_first_then_smallest_leaves():
    n, c = 50, 5
    edges = [(c, i) for i in range(n) if i != c] + [(i, c) for i in range(n) if i != c]
    off, col = csr(n, edges)
    order, k = oracle.hub_order(off, col)
    assert k == 4  # floor(0.08 * 50)
    # the center scores 49 * 49; every leaf scores 1, ties to the smaller id
    np.testing.assert_array_equal(order[:4], [5, 0, 1, 2])
    np.testing.assert_array_equal(order[4:], [v for v in range(n) if v not in (5, 0, 1, 2)])


def test_no_vertex_with_both_in_and_out_edges_means_no_hubs():
    # edges only from {0..9} to {10..19}: every H(v) = 0
    n = 20
    off, col = csr(n, [(a, b) for a in range(10) for b in range(10, 20) if (a + b) % 3])
    order, k = oracle.hub_order(off, col)
    assert k == 0
    np.testing.assert_array_equal(order, np.arange(n))


@settings(max_examples=80, deadline=None)
@given(st.integers(1, 40).flatmap(lambda n: st.tuples(
    st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=120))))
def test_order_ranks_by_the_normalized_score(case):
    n, edges = case
    edges = sorted({e for e in edges if e[0] != e[1]})
    off, col = csr(n, edges)
    order, k = oracle.hub_order(off, col)
    assert sorted(order.tolist()) == list(range(n))  # a permutation
    dout = np.diff(off).astype(np.int64)
    din = np.bincount(col.astype(np.int64), minlength=n)
    # the score as the paper writes it, exactly
    dmo, dmi = max(dout.max(initial=0), 1), max(din.max(initial=0), 1)
    H = [Fraction(int(dout[v]) * int(din[v]), dmo * dmi) for v in range(n)]
    cand = [v for v in range(n) if H[v] > 0]
    want_k = min(len(cand), (8 * n) // 100)
    ranked = sorted(cand, key=lambda v: (-H[v], v))
    assert k == want_k
    assert order[:k].tolist() == ranked[:k]
    rest = order[k:].tolist()
    assert rest == sorted(rest)  # non-hubs keep their natural order


def test_rmat_hubs_have_the_largest_degree_products():
    off, col = gen.rmat(14, 16, seed=14)
    n = len(off) - 1
    order, k = oracle.hub_order(off, col)
    assert k == (8 * n) // 100 or k == int((np.diff(off) * np.bincount(col, minlength=n) > 0).sum())
    score = np.diff(off).astype(np.int64) * np.bincount(col, minlength=n).astype(np.int64)
    hub_min = score[order[:k]].min()
    nonhub = np.ones(n, bool)
    nonhub[order[:k]] = False
    assert hub_min >= score[nonhub].max()
    assert (np.diff(score[order[:k]]) <= 0).all()
