"""Pins for the CPU oracle's BFS, SSSP, CC and PageRank.

Each check compares the oracle with something other than itself: brute force over every
small digraph, closed forms, scipy's independent graph routines, certificates that
characterise the unique answer, or exact rational matrix powers.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
from hypothesis import given, settings, strategies as st

import gen
import oracle

U = oracle.UNREACHED


def csr_from_edges(n, edges):
    src = np.array([e[0] for e in edges], dtype=np.uint32)
    dst = np.array([e[1] for e in edges], dtype=np.uint32)
    return gen.from_pairs(n, src, dst)


def dense_reach_levels(n, adj, s):
    """Hop levels by boolean matrix powers: level = least k with (A^k)[s, v]."""
    lvl = [U] * n
    frontier = np.zeros(n, dtype=bool)
    frontier[s] = True
    seen = frontier.copy()
    k = 0
    while frontier.any():
        for v in np.nonzero(frontier)[0]:
            lvl[v] = k
        nxt = (adj[frontier].any(axis=0)) & ~seen
        seen |= nxt
        frontier = nxt
        k += 1
    return lvl


# ------------------------------------------------------------------ BFS
def test_bfs_every_digraph_up_to_4_vertices():
    n = 4
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        off, col = csr_from_edges(n, edges)
        adj = np.zeros((n, n), dtype=bool)
        for u, v in edges:
            adj[u, v] = True
        for s in range(n):
            lvl, it = oracle.bfs(off, col, s)
            want = dense_reach_levels(n, adj, s)
            assert list(lvl) == want, (edges, s)
            assert it == 1 + max(x for x in want if x != U)


def test_bfs_closed_forms():
    n = 50
    off, col = csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])  # path
    lvl, it = oracle.bfs(off, col, 0)
    assert list(lvl) == list(range(n)) and it == n
    lvl, it = oracle.bfs(off, col, 10)
    assert list(lvl[:10]) == [U] * 10 and list(lvl[10:]) == list(range(n - 10)) and it == n - 10
    off, col = csr_from_edges(n, [(0, i) for i in range(1, n)])  # star
    lvl, it = oracle.bfs(off, col, 0)
    assert lvl[0] == 0 and (lvl[1:] == 1).all() and it == 2
    n = 127  # complete binary tree in heap order: level = floor(log2(v + 1))
    off, col = csr_from_edges(n, [(v, c) for v in range(n) for c in (2 * v + 1, 2 * v + 2) if c < n])
    lvl, it = oracle.bfs(off, col, 0)
    assert list(lvl) == [int(np.floor(np.log2(v + 1))) for v in range(n)] and it == 7
    n = 9  # directed cycle
    off, col = csr_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    lvl, _ = oracle.bfs(off, col, 4)
    assert list(lvl) == [(v - 4) % n for v in range(n)]


def bfs_certificate(off, col, s, lvl):
    n = len(off) - 1
    deg = np.diff(off).astype(np.int64)
    u = np.repeat(np.arange(n, dtype=np.int64), deg)
    lu, lv = lvl[u].astype(np.int64), lvl[col].astype(np.int64)
    reached_u = lvl[u] != U
    assert lvl[s] == 0
    # no edge from a reached vertex skips a level, and it never leaves a vertex unreached
    assert (lv[reached_u] <= lu[reached_u] + 1).all()
    assert (lvl[col[reached_u]] != U).all()
    # every reached v != s has a parent one level up
    has_parent = np.zeros(n, dtype=bool)
    tight = reached_u & (lv == lu + 1)
    has_parent[col[tight]] = True
    reached = lvl != U
    reached[s] = False
    assert has_parent[reached].all()


def test_bfs_rmat16_certificate_and_scipy():
    off, col = gen.rmat(16, 16, seed=16)
    lvl, it = oracle.bfs(off, col, 0)
    bfs_certificate(off, col, 0, lvl)
    assert it == 1 + int(lvl[lvl != U].max())
    # scipy's unweighted shortest paths as an independent routine
    n = len(off) - 1
    A = sp.csr_matrix((np.ones(len(col)), col.astype(np.int64), off.astype(np.int64)), shape=(n, n))
    d = csg.shortest_path(A, method="D", unweighted=True, indices=0)
    want = np.where(np.isinf(d), U, d).astype(np.uint32)
    np.testing.assert_array_equal(lvl, want)


# ----------------------------------------------------------------- SSSP
def floyd_warshall(n, wedges):
    INF = float("inf")
    D = [[0 if i == j else INF for j in range(n)] for i in range(n)]
    for u, v, w in wedges:
        D[u][v] = min(D[u][v], w)
    for k in range(n):
        for i in range(n):
            for j in range(n):
                if D[i][k] + D[k][j] < D[i][j]:
                    D[i][j] = D[i][k] + D[k][j]
    return D


@settings(max_examples=150, deadline=None)
@given(st.integers(1, 9).flatmap(lambda n: st.tuples(
    st.just(n),
    st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1), st.integers(1, 64)), max_size=30),
    st.integers(0, n - 1))))
def test_sssp_matches_floyd_warshall(case):
    n, wedges, s = case
    # the CSR keeps one copy of each (u, v); give it that pair's weight
    wmap = {}
    for u, v, w in wedges:
        if u != v:
            wmap.setdefault((u, v), w)
    off, col = csr_from_edges(n, list(wmap))
    deg = np.diff(off).astype(np.int64)
    us = np.repeat(np.arange(n), deg)
    w = np.array([wmap[(int(a), int(b))] for a, b in zip(us, col)], dtype=np.uint32)
    dist = oracle.sssp(off, col, w, s)
    D = floyd_warshall(n, [(a, b, c) for (a, b), c in wmap.items()])
    want = [U if D[s][v] == float("inf") else D[s][v] for v in range(n)]
    assert list(dist) == want


def sssp_certificate(off, col, w, s, dist):
    n = len(off) - 1
    deg = np.diff(off).astype(np.int64)
    u = np.repeat(np.arange(n, dtype=np.int64), deg)
    du, dv = dist[u].astype(np.int64), dist[col].astype(np.int64)
    ru = dist[u] != U
    assert dist[s] == 0
    assert (dist[col[ru]] != U).all()
    assert (dv[ru] <= du[ru] + w[ru]).all()
    tight = ru & (dv == du + w)
    has_parent = np.zeros(n, dtype=bool)
    has_parent[col[tight]] = True
    reached = dist != U
    reached[s] = False
    assert has_parent[reached].all()


def test_sssp_rmat16_certificate_scipy_and_unit_weights():
    off, col = gen.rmat(16, 16, seed=16)
    w = gen.weights(off, col, 1016)
    dist = oracle.sssp(off, col, w, 0)
    sssp_certificate(off, col, w, 0, dist)
    n = len(off) - 1
    A = sp.csr_matrix((w.astype(np.float64), col.astype(np.int64), off.astype(np.int64)), shape=(n, n))
    d = csg.dijkstra(A, indices=0)
    np.testing.assert_array_equal(dist, np.where(np.isinf(d), U, d).astype(np.uint32))
    # unit weights reduce SSSP to BFS
    lvl, _ = oracle.bfs(off, col, 0)
    np.testing.assert_array_equal(oracle.sssp(off, col, np.ones_like(col), 0), lvl)


def test_sssp_check_accepts_exactly_the_shortest_distances():
    """The certificate is complete: on tiny graphs it accepts a proposed answer if and only
    if it equals Dijkstra's, over every answer with values in 0..6 or unreached."""
    import itertools
    rng = np.random.default_rng(5)
    for _ in range(12):
        n = 3
        pairs = [(a, b) for a in range(n) for b in range(n) if a != b and rng.random() < 0.5]
        off, col = csr_from_edges(n, pairs)
        w = rng.integers(1, 4, len(col)).astype(np.uint32)
        want = oracle.sssp(off, col, w, 0)
        for cand in itertools.product(list(range(7)) + [U], repeat=n):
            d = np.array(cand, dtype=np.uint32)
            ok = oracle.sssp_check(off, col, w, 0, d)[0] == 0
            assert ok == np.array_equal(d, want), (pairs, w, cand)


def test_sssp_check_rejects_every_single_change():
    off, col = gen.rmat(12, 8, seed=12)
    w = gen.weights(off, col, 1012)
    for s in (0, 17, 901):
        dist = oracle.sssp(off, col, w, s)
        assert oracle.sssp_check(off, col, w, s, dist) == (0, 0)
        rng = np.random.default_rng(s)
        for v in rng.integers(0, len(dist), 200):
            for new in {int(dist[v]) + 1, max(int(dist[v]) - 1, 0), U, 0}:
                if new == dist[v] or (new == U + 1):
                    continue
                bad = dist.copy()
                bad[v] = new & 0xFFFFFFFF
                if np.array_equal(bad, dist):
                    continue
                assert oracle.sssp_check(off, col, w, s, bad)[0] != 0, (s, v, new)


def test_sssp_closed_form_and_overflow():
    n = 20
    off, col = csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])
    w = np.arange(1, n, dtype=np.uint32)
    assert list(oracle.sssp(off, col, w, 0)) == [v * (v + 1) // 2 for v in range(n)]
    off, col = csr_from_edges(3, [(0, 1), (1, 2)])
    with pytest.raises(OverflowError):
        oracle.sssp(off, col, np.array([2**31, 2**31], dtype=np.uint32), 0)
    # 2^32 - 2 is the largest distance that fits
    d = oracle.sssp(off, col, np.array([2**31, 2**31 - 2], dtype=np.uint32), 0)
    assert int(d[2]) == 2**32 - 2
    # a path whose sum does not fit is no overflow when a shorter one reaches the same vertex
    off, col = csr_from_edges(5, [(0, 1), (0, 3), (1, 2), (3, 4), (4, 2)])
    w = np.array([2**31, 1, 2**31, 1, 1], dtype=np.uint32)  # in CSR order of the edges above
    assert list(oracle.sssp(off, col, w, 0)) == [0, 2**31, 3, 1, 2]


def test_sync_rounds_bounds_and_closed_forms():
    n = 30
    off, col = csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])
    assert oracle.sync_rounds(off, col, np.ones(n - 1, np.uint32), "sssp", 0) == n
    # a shortcut edge that is heavier than the path: synchronous rounds follow hop count
    # first, then the cheaper long path keeps improving the far end
    off, col = csr_from_edges(4, [(0, 1), (1, 2), (2, 3), (0, 3)])
    w = np.array([1, 100, 1, 1], dtype=np.uint32)  # CSR rows: 0->1, 0->3, 1->2, 2->3
    assert oracle.sync_rounds(off, col, w, "sssp", 0) == 4
    # label propagation on an undirected path settles after n rounds (n-1 hops + 1 quiet)
    off, col = gen.symmetrize(*csr_from_edges(n, [(i, i + 1) for i in range(n - 1)]))
    assert oracle.sync_rounds(off, col, None, "cc") == n


# ------------------------------------------------------------------- CC
@settings(max_examples=120, deadline=None)
@given(st.integers(1, 10).flatmap(lambda n: st.tuples(
    st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=20))))
def test_cc_matches_transitive_closure(case):
    n, edges = case
    off, col = gen.symmetrize(*csr_from_edges(n, [e for e in edges if e[0] != e[1]]))
    lab, k = oracle.cc(off, col)
    R = np.eye(n, dtype=bool)
    for u, v in edges:
        R[u, v] = R[v, u] = True
    for m in range(n):  # Warshall
        R |= R[:, [m]] & R[[m], :]
    want = [int(np.nonzero(R[v])[0].min()) for v in range(n)]
    assert list(lab) == want
    assert k == len(set(want))


def test_cc_rmat16_invariants_and_scipy():
    off, col = gen.symmetrize(*gen.rmat(16, 16, seed=16))
    lab, k = oracle.cc(off, col)
    n = len(off) - 1
    v = np.arange(n)
    u = np.repeat(v, np.diff(off).astype(np.int64))
    assert (lab[u] == lab[col]).all()
    assert (lab <= v).all()
    assert (lab[lab] == lab).all()
    assert len(np.unique(lab)) == k
    A = sp.csr_matrix((np.ones(len(col)), col.astype(np.int64), off.astype(np.int64)), shape=(n, n))
    ncomp, comp = csg.connected_components(A, directed=False)
    assert ncomp == k
    # same partition: map scipy's component id to its min vertex
    first = np.full(ncomp, n)
    np.minimum.at(first, comp, v)
    np.testing.assert_array_equal(lab, first[comp])
    deg = np.diff(off)
    assert (lab[deg == 0] == v[deg == 0]).all()  # isolated vertices label themselves


# ------------------------------------------------------------ PageRank
def exact_pagerank(n, edges, d, T):
    """Exact rational power iteration, dangling mass leaks."""
    out = {u: [] for u in range(n)}
    for u, v in edges:
        out[u].append(v)
    x = [Fraction(1, n)] * n
    for _ in range(T):
        acc = [Fraction(0)] * n
        for u in range(n):
            for v in out[u]:
                acc[v] += x[u] / len(out[u])
        x = [(1 - d) / n + d * a for a in acc]
    return x


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 8).flatmap(lambda n: st.tuples(
    st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=20),
    st.integers(0, 12))))
def test_pagerank_matches_exact_rationals(case):
    n, edges, T = case
    edges = sorted({e for e in edges if e[0] != e[1]})
    off, col = csr_from_edges(n, edges)
    x = oracle.pagerank(off, col, 0.85, T)
    want = exact_pagerank(n, edges, Fraction(85, 100), T)
    np.testing.assert_allclose(x, [float(f) for f in want], rtol=0, atol=1e-15)


def test_pagerank_closed_forms_and_mass_invariant():
    n = 11
    off, col = csr_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    np.testing.assert_allclose(oracle.pagerank(off, col, 0.85, 20), np.full(n, 1 / n), atol=1e-16)
    off, col = gen.rmat(16, 16, seed=16)
    n = len(off) - 1
    d = 0.85
    x19 = oracle.pagerank(off, col, d, 19)
    x20 = oracle.pagerank(off, col, d, 20)
    deg = np.diff(off)
    indeg = np.bincount(col, minlength=n)
    # no in-edges: only the teleport term
    np.testing.assert_allclose(x20[indeg == 0], (1 - d) / n, rtol=1e-15)
    # total mass after a step = (1-d) + d * mass held by vertices that have out-edges
    assert abs(x20.sum() - ((1 - d) + d * x19[deg > 0].sum())) < 1e-12
    # scipy sparse transpose product as an independent step
    A = sp.csr_matrix((np.ones(len(col)), col.astype(np.int64), off.astype(np.int64)), shape=(n, n))
    share = np.where(deg > 0, x19 / np.maximum(deg, 1), 0.0)
    np.testing.assert_allclose(x20, (1 - d) / n + d * (A.T @ share), rtol=1e-12, atol=1e-18)


# ------------------------------------------------- personalized PageRank
def test_ppr_closed_form_on_a_path():
    # path 0 -> 1 -> ... -> 14: the walk moves one hop per step, so after T steps
    # vertex j < T holds the restart mass that survived j hops and vertex T the
    # initial unit that survived T hops; the end of the path leaks.
    n, d = 15, 0.85
    off, col = csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])
    for T in (0, 1, 2, 5, 10, 14):
        want = np.zeros(n)
        want[:T] = (1 - d) * d ** np.arange(T)
        want[T] = d ** T
        np.testing.assert_allclose(oracle.ppr(off, col, 0, d, T), want, rtol=1e-14, atol=1e-300)
    # started mid-path, nothing flows backwards
    x = oracle.ppr(off, col, 9, d, 10)
    assert (x[:9] == 0).all()
    # the sink keeps receiving restart mass that made 5 hops (it passes nothing on)
    np.testing.assert_allclose(x[9:], (1 - d) * d ** np.arange(6), rtol=1e-14)


def test_ppr_averages_to_pagerank():
    # uniform start and uniform restart are the average of the point ones, and the
    # iteration is linear: PageRank = mean over sources of the personalized vectors
    off, col = gen.rmat(7, 6, seed=5)
    n = len(off) - 1
    for T in (1, 4, 10):
        mean = np.mean([oracle.ppr(off, col, s, 0.85, T) for s in range(n)], axis=0)
        np.testing.assert_allclose(mean, oracle.pagerank(off, col, 0.85, T), rtol=1e-12, atol=1e-17)


def test_ppr_converges_to_the_linear_solve():
    # x* = (1-d) (I - d P)^-1 e_s with P the column-substochastic transition matrix;
    # the step is a d-contraction in L1, so |x_T - x*|_1 <= d^T |x_0 - x*|_1 <= 2 d^T
    import scipy.sparse.linalg as spla
    off, col = gen.rmat(10, 8, seed=10)
    n, d = len(off) - 1, 0.85
    deg = np.diff(off).astype(np.float64)
    src = np.repeat(np.arange(n), np.diff(off).astype(np.int64))
    P = sp.csr_matrix((1.0 / deg[src], (col.astype(np.int64), src)), shape=(n, n))
    for s in (0, 3, 77):
        e = np.zeros(n)
        e[s] = 1.0
        xs = spla.spsolve((sp.identity(n) - d * P).tocsc(), (1 - d) * e)
        for T in (10, 60, 200):
            err = np.abs(oracle.ppr(off, col, s, d, T) - xs).sum()
            assert err <= 2 * d ** T + 1e-12, (s, T, err)


def test_ppr_mass_and_support():
    # on a graph without sinks the mass stays 1; the support after T steps is the set
    # of vertices within T hops of the source
    off, col = gen.symmetrize(*gen.rmat(9, 8, seed=3))
    deg = np.diff(off)
    s = int(np.nonzero(deg)[0][0])
    lvl, _ = oracle.bfs(off, col, s)
    comp = lvl != U
    assert (deg[comp] > 0).all()
    for T in (0, 1, 2, 3, 10):
        x = oracle.ppr(off, col, s, 0.85, T)
        assert abs(x.sum() - 1.0) < 1e-12
        np.testing.assert_array_equal(x > 0, lvl <= T)


@settings(max_examples=40, deadline=None)
@given(st.integers(1, 7).flatmap(lambda n: st.tuples(
    st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=16),
    st.integers(0, n - 1), st.integers(0, 10))))
def test_ppr_matches_matrix_powers(case):
    # x_T = d^T P^T e_s + (1-d) sum_{j<T} d^j P^j e_s, by exact dense rational powers
    n, edges, s, T = case
    edges = sorted({e for e in edges if e[0] != e[1]})
    off, col = csr_from_edges(n, edges)
    deg = [sum(1 for u, _ in edges if u == a) for a in range(n)]
    P = [[Fraction(0)] * n for _ in range(n)]
    for u, v in edges:
        P[v][u] += Fraction(1, deg[u])
    d = Fraction(85, 100)

    def mul(vec):
        return [sum(P[i][j] * vec[j] for j in range(n)) for i in range(n)]

    p = [Fraction(int(i == s)) for i in range(n)]
    want = [Fraction(0)] * n
    for j in range(T):
        want = [w + (1 - d) * d ** j * a for w, a in zip(want, p)]
        p = mul(p)
    want = [w + d ** T * a for w, a in zip(want, p)]
    np.testing.assert_allclose(oracle.ppr(off, col, s, 0.85, T), [float(f) for f in want], rtol=0, atol=1e-15)


def test_pagerank_long_run_is_the_linear_solve_fixed_point():
    # x* = (1-d)/n (I - d P)^-1 1 with P column-substochastic (sinks leak); the step is a
    # d-contraction in L1, so T = 300 steps are within 2 d^T of it
    import scipy.sparse.linalg as spla
    for off, col in (gen.rmat(11, 8, seed=11), gen.er(1500, 6000, seed=2)):
        n, d = len(off) - 1, 0.85
        deg = np.diff(off).astype(np.float64)
        src = np.repeat(np.arange(n), np.diff(off).astype(np.int64))
        P = sp.csr_matrix((1.0 / deg[src], (col.astype(np.int64), src)), shape=(n, n))
        xs = spla.spsolve((sp.identity(n) - d * P).tocsc(), np.full(n, (1 - d) / n))
        assert np.abs(oracle.pagerank(off, col, d, 300) - xs).sum() <= 2 * d ** 300 + 1e-13
