"""Hub-sorted graphs (Sec. 6.1): the library relabels the graph at creation; every result
must still equal the oracle's on the original graph, in the caller's ids -- BFS, SSSP and
CC bit for bit (CC labels = smallest original id of the component), PageRank and PPR
within 1e-6 -- through single runs, batched lanes and the query server."""
import sys

import numpy as np
import pytest

import gen
import oracle
import paper_2208_14935_amd as hy

pytestmark = pytest.mark.gpu
TOL = 1e-6


def note(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def case():
    off, col = gen.rmat(16, 16, seed=16)
    w = gen.weights(off, col, 1016)
    soff, scol = gen.symmetrize(off, col)
    return off, col, w, soff, scol


def want(case, algo, s=0):
    off, col, w, soff, scol = case
    if algo == "bfs":
        return oracle.bfs(off, col, s)[0]
    if algo == "sssp":
        return oracle.sssp(off, col, w, s)
    if algo == "cc":
        return oracle.cc(soff, scol)[0]
    if algo == "pagerank":
        return oracle.pagerank(off, col, 0.85, 20)
    return oracle.ppr(off, col, s, 0.85, 10)


def check(case, algo, got, s=0):
    ref = want(case, algo, s)
    if algo in ("pagerank", "ppr"):
        assert np.abs(got.astype(np.float64) - ref).max() <= TOL
    else:
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("algo", ["bfs", "sssp", "cc", "pagerank", "ppr"])
@pytest.mark.parametrize("mode,resident", [("hybrid", 0.25), ("hybrid", None), ("zerocopy", 0.0), ("filter", 0.0)])
def test_hub_sorted_results_in_original_ids(case, algo, mode, resident):
    off, col, w, soff, scol = case
    note(f"hub {algo} {mode} {resident}")
    if algo == "cc":
        g = hy.Graph(soff, scol, symmetric=True, hub_sort=True)
    else:
        g = hy.Graph(off, col, weights=w, hub_sort=True)
    with g:
        k = g.info()["hubs"]
        assert k == oracle.hub_order(soff, scol)[1] if algo == "cc" else k == oracle.hub_order(off, col)[1]
        g.set_params(mode=mode, partition_edges=4096)
        if resident is not None:
            g.set_resident_fraction(algo, resident)
        s = int(gen.sources(off, 1, 5)[0])
        r = g.run(algo, s)
        check(case, algo, r.values, s)
        if algo == "bfs":
            assert r.iterations == oracle.bfs(off, col, s)[1]


def test_hub_sorted_batch_and_server(case):
    off, col, w, _, _ = case
    srcs = gen.sources(off, 6, 66)
    with hy.Graph(off, col, weights=w, hub_sort=True) as g:
        g.set_params(partition_edges=4096)
        g.set_resident_fraction("sssp", 0.25)
        for algo in ("bfs", "sssp", "ppr"):
            vals, its, _ = g.run_batch(algo, srcs)
            for i, s in enumerate(srcs):
                check(case, algo, vals[i], int(s))
        with hy.Server(g, bfs=4, sssp=2, ppr=2) as srv:
            qs = [srv.submit(a, int(s)) for s in srcs for a in ("bfs", "sssp", "ppr")]
            for q in qs:
                srv.wait(q)
                check(case, q.algo, q.values, q.source)
