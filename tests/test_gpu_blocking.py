"""GPU: PageRank with propagation blocking -- the pushes emit one (destination, contribution)
pair per edge, each piece of partitions has its pairs bucketed by destination in two
counting-sort passes and summed in LDS -- against the FP64 oracle (1e-6 max-abs) and the
atomic path.  Piece sizes down to one partition cut the graph into many pieces in both
lanes (resident and streamed), so the double-buffered piece pipeline and both sort
levels (graphs of more than 2^19 vertices) are exercised.
"""
import sys

import numpy as np
import pytest

import gen
import oracle
import paper_2208_14935_amd as hy

pytestmark = pytest.mark.gpu
PR_TOL = 1e-6
BLOCK = hy.KERNEL_CLASSES.index("pr_blocking")


def note(*a):
    print(*a, flush=True, file=sys.stderr)


class PrCase:
    def __init__(self, off, col):
        self.off, self.col = off, col
        self.want = oracle.pagerank(off, col, 0.85, 20)

    def check(self, res):
        err = np.abs(res.values.astype(np.float64) - self.want).max()
        assert err <= PR_TOL, f"pagerank max-abs error {err}"
        assert res.iterations == 20


@pytest.fixture(scope="module")
def rmat12():
    return PrCase(*gen.rmat(12, 16, seed=12))


@pytest.fixture(scope="module")
def er_odd():
    # 20001 vertices (no multiple of a 4096-slot block or a 16384-slot bin), many without
    # out-edges, average degree 4: every contribution is far above the tolerance
    return PrCase(*gen.er(20001, 80000, seed=7))


@pytest.fixture(scope="module")
def rmat20():
    return PrCase(*gen.rmat(20, 16, seed=20))


def budget(g, resident):
    if resident is not None:
        g.set_resident_fraction("pagerank", resident)


@pytest.mark.parametrize("mode", ["hybrid", "filter", "zerocopy", "compact"])
@pytest.mark.parametrize("pairs", [0, 4096, 1])
@pytest.mark.parametrize("resident", [0.25, 0.0, None])
def test_blocked_pagerank_matches_oracle(rmat12, mode, pairs, resident):
    note(f"rmat12 pagerank blocking mode={mode} pairs={pairs} resident={resident}")
    with hy.Graph(rmat12.off, rmat12.col) as g:
        g.set_params(partition_edges=2048, mode=mode, pr_block_pairs=pairs)
        budget(g, resident)
        res = g.run("pagerank", stats=True, time_kernels=True)
        rmat12.check(res)
        launches = res.stats["kernel_launches"][BLOCK]
        if mode == "compact":
            assert launches == 0  # compaction pushes do not know an edge's CSR index
        else:
            # one bucketing launch group per piece and iteration
            assert launches >= 20


def test_blocked_and_atomic_paths_agree(er_odd):
    note("er_odd pagerank blocking on / off")
    with hy.Graph(er_odd.off, er_odd.col) as g:
        g.set_params(partition_edges=1024, pr_block_pairs=5000)
        g.set_resident_fraction("pagerank", 0.3)
        on = g.run("pagerank", stats=True, time_kernels=True)
        g.set_params(pr_blocking=0)
        g.set_resident_fraction("pagerank", 0.3)
        off = g.run("pagerank", stats=True, time_kernels=True)
    er_odd.check(on)
    er_odd.check(off)
    assert on.stats["kernel_launches"][BLOCK] > 0
    assert off.stats["kernel_launches"][BLOCK] == 0
    assert np.abs(on.values.astype(np.float64) - off.values).max() <= PR_TOL
    # the same engines moved the same bytes: only the adds changed
    for k in ("bytes_filter", "bytes_zerocopy", "active_edges"):
        assert on.stats[k] == off.stats[k], k


@pytest.mark.parametrize("mode", ["hybrid", "zerocopy"])
@pytest.mark.parametrize("resident", [0.25, None])
def test_two_level_buckets_match_oracle(rmat20, mode, resident):
    """2^20 vertices: 64 fine bins in 2 coarse bins, pieces of 300000 pairs."""
    note(f"rmat20 pagerank blocking mode={mode} resident={resident}")
    with hy.Graph(rmat20.off, rmat20.col) as g:
        g.set_params(mode=mode, pr_block_pairs=300000)
        budget(g, resident)
        res = g.run("pagerank", stats=True, time_kernels=True)
        rmat20.check(res)
        assert res.stats["kernel_launches"][BLOCK] >= 20 * (len(rmat20.col) // 300000)


def test_default_piece_size_matches_oracle(rmat20):
    note("rmat20 pagerank blocking default pieces, hybrid at a quarter budget")
    with hy.Graph(rmat20.off, rmat20.col) as g:
        g.set_params(gamma=(1, 1), zc_tie=1)
        g.set_resident_fraction("pagerank", 0.25)
        res = g.run("pagerank", stats=True, time_kernels=True)
        rmat20.check(res)
        assert res.stats["kernel_launches"][BLOCK] > 0


def test_piece_size_limit_is_checked(rmat12):
    with hy.Graph(rmat12.off, rmat12.col) as g:
        with pytest.raises(hy.HytmError) as ei:
            g.set_params(pr_block_pairs=1 << 31)
        assert ei.value.status == hy.E_INVAL
        with pytest.raises(hy.HytmError):
            g.set_params(pr_blocking=2)
