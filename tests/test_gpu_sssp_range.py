"""SSSP distances near the top of uint32, through the C ABI, against the oracle.

A shortest distance must fit below 2^32-1 (UINT32_MAX marks unreached), else the run
fails with E_RANGE -- but only a *final* distance decides, as in the oracle's Dijkstra
with 64-bit sums.  A longer path whose sum would not fit, relaxed before a shorter one
reaches the same vertex, is no error.  Every engine, the batched form and the query
server must agree with the oracle on that.
"""
import sys

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import gen
import oracle
import paper_2208_14935_amd as hy

pytestmark = pytest.mark.gpu
U = hy.UNREACHED
ENGINE_CASES = [("hybrid", "stream"), ("hybrid", "copy"), ("filter", "stream"), ("filter", "copy"),
                ("compact", "stream"), ("zerocopy", "stream")]


def note(*a):
    print(*a, flush=True, file=sys.stderr)


def transient_graph():
    """0->1 (2^31), 1->2 (2^31), 0->3 (1), 3->4 (1), 4->2 (1): vertex 1 offers vertex 2 the
    candidate 2^32 in the iteration before the path through 3 and 4 gives it 3."""
    src = np.array([0, 1, 0, 3, 4], np.uint32)
    dst = np.array([1, 2, 3, 4, 2], np.uint32)
    off, col = gen.from_pairs(5, src, dst)
    wmap = {(0, 1): 1 << 31, (1, 2): 1 << 31, (0, 3): 1, (3, 4): 1, (4, 2): 1}
    w = np.array([wmap[(u, int(col[e]))] for u in range(5) for e in range(int(off[u]), int(off[u + 1]))],
                 np.uint32)
    return off, col, w


@pytest.mark.parametrize("hub_sort", [False, True])
@pytest.mark.parametrize("resident", [0.0, 0.5])
@pytest.mark.parametrize("mode,fe", ENGINE_CASES)
def test_transient_candidate_overflow_is_no_error(mode, fe, resident, hub_sort):
    note(f"transient overflow single mode={mode} fe={fe} resident={resident} hub_sort={hub_sort}")
    off, col, w = transient_graph()
    with hy.Graph(off, col, weights=w, hub_sort=hub_sort) as g:
        g.set_params(partition_edges=1, mode=mode, filter_engine=fe, compact_chunk_edges=2)
        g.set_resident_fraction("sssp", resident)
        res = g.run("sssp", 0)
        np.testing.assert_array_equal(res.values, [0, 1 << 31, 3, 1, 2])
        assert 3 <= res.iterations <= oracle.sync_rounds(off, col, w, "sssp", 0)


@pytest.mark.parametrize("mode", ["hybrid", "zerocopy", "compact"])
def test_transient_candidate_overflow_batched(mode):
    note(f"transient overflow batched mode={mode}")
    off, col, w = transient_graph()
    srcs = [0, 1, 3, 0, 2, 4]
    with hy.Graph(off, col, weights=w) as g:
        g.set_params(partition_edges=1, mode=mode, compact_chunk_edges=2)
        g.set_resident_fraction("sssp", 0.0)
        vals, its, _ = g.run_batch("sssp", srcs)
        for k, s in enumerate(srcs):
            np.testing.assert_array_equal(vals[k], oracle.sssp(off, col, w, s))


def test_true_overflow_fails_the_batch():
    # 0 -> 1 -> 2 with weights 2^31: from 0 the distance of 2 is 2^32
    off, col = gen.from_pairs(3, np.array([0, 1], np.uint32), np.array([1, 2], np.uint32))
    w = np.array([1 << 31, 1 << 31], np.uint32)
    with hy.Graph(off, col, weights=w) as g:
        vals, _, _ = g.run_batch("sssp", [1, 2])
        np.testing.assert_array_equal(vals, [[U, 0, 1 << 31], [U, U, 0]])
        with pytest.raises(hy.HytmError) as ei:
            g.run_batch("sssp", [1, 0])
        assert ei.value.status == hy.E_RANGE


def test_transient_candidate_overflow_served():
    note("transient overflow served")
    off, col, w = transient_graph()
    with hy.Graph(off, col, weights=w) as g:
        g.set_params(partition_edges=1)
        g.set_resident_fraction("sssp", 0.0)
        with hy.Server(g, bfs=1, sssp=4, ppr=0) as srv:
            qs = [srv.submit("sssp", s) for s in (0, 3, 0, 1)]
            for q in qs:
                srv.wait(q)
                np.testing.assert_array_equal(q.values, oracle.sssp(off, col, w, q.source))


BIG = [1, 2, 7, (1 << 30) + 3, (1 << 31) - 1, 1 << 31, (1 << 31) + 5, (1 << 32) - 3, (1 << 32) - 2]


@st.composite
def heavy_graphs(draw):
    n = draw(st.integers(2, 10))
    m = draw(st.integers(1, 3 * n))
    src = np.array(draw(st.lists(st.integers(0, n - 1), min_size=m, max_size=m)), np.uint32)
    dst = np.array(draw(st.lists(st.integers(0, n - 1), min_size=m, max_size=m)), np.uint32)
    off, col = gen.from_pairs(n, src, dst)
    w = np.array(draw(st.lists(st.sampled_from(BIG), min_size=len(col), max_size=len(col))), np.uint32)
    mode = draw(st.sampled_from(["hybrid", "filter", "compact", "zerocopy"]))
    source = draw(st.integers(0, n - 1))
    return off, col, w, mode, source


@settings(max_examples=60, deadline=None, suppress_health_check=list(HealthCheck))
@given(heavy_graphs())
def test_heavy_weights_match_oracle(case):
    """Weights up to 2^32-2: values equal the oracle's, and E_RANGE exactly when the oracle
    finds a shortest distance that does not fit."""
    off, col, w, mode, source = case
    if len(col) == 0:
        return
    try:
        want = oracle.sssp(off, col, w, source)
    except OverflowError:
        want = None
    with hy.Graph(off, col, weights=w) as g:
        g.set_params(partition_edges=2, mode=mode, compact_chunk_edges=2)
        g.set_resident_fraction("sssp", 0.0)
        if want is None:
            with pytest.raises(hy.HytmError) as ei:
                g.run("sssp", source)
            assert ei.value.status == hy.E_RANGE
        else:
            np.testing.assert_array_equal(g.run("sssp", source).values, want)
        # batched: each lane against its own oracle run; one overflowing lane fails the batch
        srcs = sorted({source, 0, len(off) - 2})
        wants = []
        for s in srcs:
            try:
                wants.append(oracle.sssp(off, col, w, s))
            except OverflowError:
                wants.append(None)
        if any(x is None for x in wants):
            with pytest.raises(hy.HytmError) as ei:
                g.run_batch("sssp", srcs)
            assert ei.value.status == hy.E_RANGE
        else:
            vals, _, _ = g.run_batch("sssp", srcs)
            for k in range(len(srcs)):
                np.testing.assert_array_equal(vals[k], wants[k])
