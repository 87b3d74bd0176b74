"""Batched multi-source BFS/SSSP (up to 64 lanes in one traversal): every lane must equal
the oracle's single-source result bit for bit, under every transfer engine and budget."""
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
def g16():
    off, col = gen.rmat(16, 16, seed=16)
    w = gen.weights(off, col, 1016)
    return off, col, w


@pytest.mark.parametrize("algo", ["bfs", "sssp"])
@pytest.mark.parametrize("mode,fe,resident", [("hybrid", "stream", None), ("hybrid", "stream", 0.25),
                                              ("hybrid", "copy", 0.25), ("zerocopy", "stream", 0.0),
                                              ("compact", "stream", 0.1), ("filter", "stream", 0.0)])
def test_batch_lanes_match_single_source_oracle(g16, algo, mode, fe, resident):
    off, col, w = g16
    n = len(off) - 1
    srcs = np.concatenate([[0], gen.sources(off, 62, 77), [0]]).astype(np.uint32)  # 64 lanes, a repeat
    note(f"batch {algo} {mode} {fe} resident={resident} lanes={len(srcs)}")
    with hy.Graph(off, col, weights=w) as g:
        g.set_params(mode=mode, filter_engine=fe, partition_edges=4096, compact_chunk_edges=1 << 16)
        if resident is not None:
            g.set_resident_fraction(algo, resident)
        vals, its, st = g.run_batch(algo, srcs, stats=True)
    assert vals.shape == (len(srcs), n)
    for l, s in enumerate(srcs):
        if algo == "bfs":
            want, it = oracle.bfs(off, col, int(s))
            assert its[l] == it, (l, s)
        else:
            want = oracle.sssp(off, col, w, int(s))
            lo = oracle.bfs(off, col, int(s))[1]
            assert lo <= its[l] <= oracle.sync_rounds(off, col, w, "sssp", int(s)), (l, s)
        bad = np.nonzero(vals[l] != want)[0]
        assert len(bad) == 0, f"lane {l} source {s}: {len(bad)} mismatches at {bad[:5]}"


def test_batch_small_sizes_and_errors(g16):
    off, col, w = g16
    with hy.Graph(off, col, weights=w) as g:
        vals, its, _ = g.run_batch("bfs", [5])
        want, it = oracle.bfs(off, col, 5)
        np.testing.assert_array_equal(vals[0], want)
        assert its[0] == it
        with pytest.raises(hy.HytmError) as ei:
            g.run_batch("bfs", np.arange(65))
        assert ei.value.status == hy.E_INVAL
        with pytest.raises(hy.HytmError) as ei:
            g.run_batch("bfs", [len(off)])
        assert ei.value.status == hy.E_RANGE
        with pytest.raises(hy.HytmError) as ei:
            g.run_batch("pagerank", [0])
        assert ei.value.status == hy.E_INVAL


def test_batch_equals_single_runs_on_random_graph():
    rng = np.random.default_rng(3)
    n = 300
    src = rng.integers(0, n, 2000).astype(np.uint32)
    dst = rng.integers(0, n, 2000).astype(np.uint32)
    off, col = gen.from_pairs(n, src, dst)
    w = gen.weights(off, col, 9)
    srcs = rng.integers(0, n, 17).astype(np.uint32)
    with hy.Graph(off, col, weights=w) as g:
        g.set_params(partition_edges=64, combine_k=2, compact_chunk_edges=128)
        g.set_resident_fraction("sssp", 0.2)
        for algo in ("bfs", "sssp"):
            vals, its, _ = g.run_batch(algo, srcs)
            for l, s in enumerate(srcs):
                np.testing.assert_array_equal(vals[l], g.run(algo, int(s)).values)
