"""GPU: single-source SSSP with a far set (`sssp_delta`): improved vertices at or above a
rising bound wait until the frontier empties.  Distances must equal the oracle's (Dijkstra)
bit for bit under every engine, budget, bound step, reprocessing and hub sorting; the
iteration count is bounded below by the BFS depth (every pushed hop takes an iteration) but,
unlike the synchronous push, not above by the synchronous round count.
"""
import sys

import numpy as np
import pytest

import gen
import oracle
import paper_2208_14935_amd as hy

pytestmark = pytest.mark.gpu
MODES = ["hybrid", "filter", "compact", "zerocopy"]
DELTAS = [1, 16, 64, 1000, 2**31]


def note(*a):
    print(*a, flush=True, file=sys.stderr)


class Case:
    def __init__(self, off, col, wseed, source=0):
        self.off, self.col, self.source = off, col, source
        self.w = gen.weights(off, col, wseed)
        self.dist = oracle.sssp(off, col, self.w, source)
        self.depth = oracle.bfs(off, col, source)[1]

    def check(self, res):
        bad = np.nonzero(res.values != self.dist)[0]
        assert len(bad) == 0, f"{len(bad)} mismatches, first at {bad[:5]}: got {res.values[bad[:5]]} " \
                              f"want {self.dist[bad[:5]]}"
        assert res.iterations >= self.depth


@pytest.fixture(scope="module")
def rmat12():
    off, col = gen.rmat(12, 16, seed=12)
    return Case(off, col, 1012)


@pytest.fixture(scope="module")
def rmat16():
    off, col = gen.rmat(16, 16, seed=16)
    return Case(off, col, 1016)


@pytest.fixture(scope="module")
def er_ragged():
    # 30001 vertices (no multiple of a 32-bit word of the bitmaps), average degree 3, from a
    # source in the middle
    off, col = gen.er(30001, 90000, seed=11)
    return Case(off, col, 2011, source=15000)


@pytest.mark.parametrize("delta", DELTAS)
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("resident", [0.25, None])
def test_far_set_matches_oracle(rmat12, mode, delta, resident):
    note(f"rmat12 sssp mode={mode} delta={delta} resident={resident}")
    with hy.Graph(rmat12.off, rmat12.col, weights=rmat12.w) as g:
        g.set_params(partition_edges=2048, mode=mode, compact_chunk_edges=4096, sssp_delta=delta)
        if resident is not None:
            g.set_resident_fraction("sssp", resident)
        rmat12.check(g.run("sssp", 0, stats=True))


@pytest.mark.parametrize("delta", DELTAS)
def test_far_set_on_ragged_graph(er_ragged, delta):
    note(f"er 30001 sssp delta={delta}")
    with hy.Graph(er_ragged.off, er_ragged.col, weights=er_ragged.w) as g:
        g.set_params(partition_edges=4096, sssp_delta=delta)
        g.set_resident_fraction("sssp", 0.3)
        er_ragged.check(g.run("sssp", er_ragged.source))


@pytest.mark.parametrize("delta", [0, 8, 64, 512])
def test_far_set_resident_and_work(rmat16, delta):
    """Resident 2^16-vertex graph; with a bound the pushed edges stay within twice the
    synchronous push's (printed for the record)."""
    note(f"rmat16 sssp delta={delta}")
    with hy.Graph(rmat16.off, rmat16.col, weights=rmat16.w) as g:
        g.set_params(sssp_delta=0)
        base = g.run("sssp", 0, stats=True)
        g.set_params(sssp_delta=delta)
        res = g.run("sssp", 0, stats=True)
    rmat16.check(base)
    rmat16.check(res)
    note(f"  pushed edges {res.stats['active_edges']} vs synchronous {base.stats['active_edges']}, "
         f"iterations {res.iterations} vs {base.iterations}")
    if delta == 0:
        assert res.iterations == base.iterations
    assert res.stats["active_edges"] <= 2 * base.stats["active_edges"]


@pytest.mark.parametrize("reprocess", [1, 2])
def test_far_set_with_reprocessing(rmat12, reprocess):
    with hy.Graph(rmat12.off, rmat12.col, weights=rmat12.w) as g:
        g.set_params(partition_edges=2048, sssp_delta=32, reprocess=reprocess)
        g.set_resident_fraction("sssp", 0.25)
        rmat12.check(g.run("sssp", 0))


def test_far_set_with_hub_sorting(rmat12):
    with hy.Graph(rmat12.off, rmat12.col, weights=rmat12.w, hub_sort=True) as g:
        g.set_params(partition_edges=2048, sssp_delta=32)
        g.set_resident_fraction("sssp", 0.25)
        rmat12.check(g.run("sssp", 0))


def test_batched_runs_ignore_the_bound(rmat12):
    srcs = [0, 5, 77, 1000]
    with hy.Graph(rmat12.off, rmat12.col, weights=rmat12.w) as g:
        g.set_params(partition_edges=2048, sssp_delta=16)
        vals, its, _ = g.run_batch("sssp", srcs)
    for i, s in enumerate(srcs):
        np.testing.assert_array_equal(vals[i], oracle.sssp(rmat12.off, rmat12.col, rmat12.w, s))


def test_far_set_keeps_overflow_reporting():
    off = np.array([0, 1, 2, 2], np.uint64)
    col = np.array([1, 2], np.uint32)
    with hy.Graph(off, col, weights=np.array([2**31, 2**31], np.uint32)) as g:
        for delta in (1, 2**30, 2**32 - 1):
            g.set_params(sssp_delta=delta)
            with pytest.raises(hy.HytmError) as ei:
                g.run("sssp", 0)
            assert ei.value.status == hy.E_RANGE
