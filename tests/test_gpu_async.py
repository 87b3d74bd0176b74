"""The paper's asynchronous scheduling (Sec. 6.1) through the C ABI.

Reprocessing (a second pass over the partitions each iteration loaded) must leave BFS, SSSP
and CC results bit-identical to the oracle while not needing more iterations than the
synchronous runs.  Delta-based PageRank must land within d/(1-d) x its reported residual
(plus FP32 rounding) of the FP64 fixed point in L1, and within 1e-6 max-abs."""
import sys

import numpy as np
import pytest

import gen
import oracle
import paper_2208_14935_amd as hy

pytestmark = pytest.mark.gpu
D = 0.85


def note(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def case():
    off, col = gen.rmat(16, 16, seed=16)
    w = gen.weights(off, col, 1016)
    soff, scol = gen.symmetrize(off, col)
    return off, col, w, soff, scol


@pytest.fixture(scope="module")
def fixed_point(case):
    off, col = case[0], case[1]
    return oracle.pagerank(off, col, D, 300)  # within 2 * 0.85^300 of the fixed point


@pytest.mark.parametrize("algo", ["bfs", "sssp", "cc"])
@pytest.mark.parametrize("mode,resident,hub", [("hybrid", 0.25, False), ("hybrid", 0.25, True),
                                               ("zerocopy", 0.0, False), ("filter", 0.0, False),
                                               ("compact", 0.1, False), ("hybrid", None, False)])
def test_reprocessing_keeps_results_and_needs_no_more_iterations(case, algo, mode, resident, hub):
    off, col, w, soff, scol = case
    note(f"reprocess {algo} {mode} {resident} hub={hub}")
    s = int(gen.sources(off, 1, 9)[0])
    g = (hy.Graph(soff, scol, symmetric=True, hub_sort=hub) if algo == "cc"
         else hy.Graph(off, col, weights=w, hub_sort=hub))
    with g:
        g.set_params(mode=mode, partition_edges=4096, compact_chunk_edges=1 << 16)
        if resident is not None:
            g.set_resident_fraction(algo, resident)
        sync = g.run(algo, s)
        g.set_params(reprocess=1)
        r = g.run(algo, s, stats=True)
    if algo == "bfs":
        want, its = oracle.bfs(off, col, s)
        assert sync.iterations == its
    elif algo == "sssp":
        want = oracle.sssp(off, col, w, s)
    else:
        want = oracle.cc(soff, scol)[0]
    np.testing.assert_array_equal(r.values, want)
    np.testing.assert_array_equal(sync.values, want)
    assert r.iterations <= sync.iterations
    note(f"  iterations sync {sync.iterations} reprocess {r.iterations}")


@pytest.mark.parametrize("mode,resident,reprocess,hub", [("hybrid", 0.25, 0, False), ("hybrid", 0.25, 1, False),
                                                         ("hybrid", 0.25, 1, True), ("zerocopy", 0.0, 1, False),
                                                         ("filter", 0.0, 0, False), ("compact", 0.1, 1, False),
                                                         ("hybrid", None, 1, False)])
def test_delta_pagerank_reaches_the_fixed_point(case, fixed_point, mode, resident, reprocess, hub):
    off, col = case[0], case[1]
    note(f"dpr {mode} {resident} reprocess={reprocess} hub={hub}")
    with hy.Graph(off, col, hub_sort=hub) as g:
        g.set_params(mode=mode, partition_edges=4096, compact_chunk_edges=1 << 16, reprocess=reprocess)
        if resident is not None:
            g.set_resident_fraction("pagerank_delta", resident)
        r = g.run("pagerank_delta", stats=True)
    res = r.stats["residual"]
    assert 0 <= res <= 1e-7
    err = np.abs(r.values.astype(np.float64) - fixed_point)
    # the pending delta bounds the distance to the fixed point; FP32 accumulation adds a
    # few units in the last place of every value
    assert err.sum() <= D / (1 - D) * res + 4e-7 * fixed_point.sum() + 1e-9
    assert err.max() <= 1e-6
    note(f"  iterations {r.iterations} residual {res:.3g} l1 {err.sum():.3g}")


def test_delta_pagerank_epsilon_and_cap(case, fixed_point):
    off, col = case[0], case[1]
    with hy.Graph(off, col) as g:
        g.set_params(dpr_epsilon=1e-3)
        coarse = g.run("pagerank_delta", stats=True)
        assert coarse.stats["residual"] <= 1e-3
        err = np.abs(coarse.values.astype(np.float64) - fixed_point).sum()
        assert err <= D / (1 - D) * coarse.stats["residual"] + 1e-6
        g.set_params(dpr_epsilon=1e-7, dpr_max_iterations=3)
        capped = g.run("pagerank_delta", stats=True)
        assert capped.iterations == 3 and capped.stats["residual"] > 1e-7


@pytest.mark.parametrize("algo", ["bfs", "sssp", "cc"])
def test_reprocessing_resident_and_zero_copy_only(case, algo):
    off, col, w, soff, scol = case
    s = int(gen.sources(off, 1, 9)[0])
    g = hy.Graph(soff, scol, symmetric=True) if algo == "cc" else hy.Graph(off, col, weights=w)
    with g:
        g.set_params(partition_edges=4096, reprocess=2)
        g.set_resident_fraction(algo, 0.25)
        r = g.run(algo, s)
    want = (oracle.bfs(off, col, s)[0] if algo == "bfs" else oracle.sssp(off, col, w, s) if algo == "sssp"
            else oracle.cc(soff, scol)[0])
    np.testing.assert_array_equal(r.values, want)
