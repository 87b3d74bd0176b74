"""The resident cache shared by one- and two-array runs: on a graph with separate weights
the budget's resident share holds either the neighbour prefix col[0, E1) (BFS, CC,
PageRank) or a shorter prefix col[0, E2) followed by w[0, E2) (SSSP).  Alternating runs
must stay exact against the oracle, copy only the part of the region that differs at each
switch, and nothing at all when the algorithm repeats."""
import sys

import numpy as np
import pytest

import gen
import oracle
import paper_2208_14935_amd as hy

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def case():
    off, col = gen.rmat(14, 16, seed=14)
    w = gen.weights(off, col, 1014)
    return off, col, w


def resident_edges(g, off, nres):
    return int(off[int(g.partition_bounds()[nres])])


@pytest.mark.parametrize("narrow", [True, False])
@pytest.mark.parametrize("frac", [0.3, 0.7])
def test_switching_copies_only_the_difference(case, frac, narrow):
    off, col, w = case
    note(f"rmat14 alternating bfs/sssp, resident share {frac}, byte weights {narrow}")
    want_bfs = oracle.bfs(off, col, 0)[0]
    want_sssp = oracle.sssp(off, col, w, 0)
    with hy.Graph(off, col, weights=w, pack=False, narrow=narrow) as g:
        assert not g.info()["packed_weights"]
        wb = g.info()["weight_bytes"]
        assert wb == (1 if narrow else 4)
        g.set_params(partition_edges=2048, compact_chunk_edges=4096)
        stage = max(g.staging_bytes("bfs"), g.staging_bytes("sssp"))
        g.set_budget(stage + int(frac * 4 * g.m))
        fills = []
        e1 = e2 = None
        for algo in ("bfs", "sssp", "bfs", "sssp", "sssp", "pagerank", "bfs"):
            r = g.run(algo, 0, stats=True)
            if algo == "bfs":
                np.testing.assert_array_equal(r.values, want_bfs)
                e1 = resident_edges(g, off, r.stats["nres"])
            elif algo == "sssp":
                np.testing.assert_array_equal(r.values, want_sssp)
                e2 = resident_edges(g, off, r.stats["nres"])
            fills.append(r.stats["bytes_resident_fill"])
        assert 0 < e2 < e1
        # both layouts fit the one region: 4 E1 and (4 + wb) E2 bytes are within a partition
        maxpart = int(np.diff(off[g.partition_bounds().astype(np.int64)]).max())
        assert (4 + wb) * e2 <= 4 * e1 + (4 + wb) * maxpart
        # bfs: col[0, E1); sssp: w[0, E2) only, placed right after col[0, E2); bfs: col[E2, E1)
        # again (the neighbour prefix kept is col[0, E2)); sssp: w again; sssp: nothing;
        # pagerank after sssp: as bfs; bfs after pagerank: nothing
        back = 4 * (e1 - e2)
        assert fills == [4 * e1, wb * e2, back, wb * e2, 0, back, 0], (fills, e1, e2)


def test_budget_change_resizes_the_region(case):
    off, col, w = case
    want_sssp = oracle.sssp(off, col, w, 0)
    want_bfs = oracle.bfs(off, col, 0)[0]
    with hy.Graph(off, col, weights=w, pack=False) as g:
        g.set_params(partition_edges=2048, compact_chunk_edges=4096)
        stage = max(g.staging_bytes("bfs"), g.staging_bytes("sssp"))
        for frac in (0.6, 0.2, 0.9, None):
            g.set_budget(stage + int(frac * 8 * g.m) if frac is not None else 2**64 - 1)
            np.testing.assert_array_equal(g.run("sssp", 0).values, want_sssp)
            np.testing.assert_array_equal(g.run("bfs", 0).values, want_bfs)
