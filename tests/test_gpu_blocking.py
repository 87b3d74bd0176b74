"""GPU: PageRank with propagation blocking over the resident partitions -- their pushes
write one contribution per edge, each piece of resident partitions has its (destination,
contribution) pairs bucketed by destination and summed in LDS, while streamed partitions
keep their atomic adds -- against the FP64 oracle (1e-6 max-abs) and the all-atomic path.
Piece sizes down to one partition cut the resident prefix into many pieces, exercising
the double-buffered piece pipeline; graphs of up to 2^24 vertices bucket in one
counting-sort pass, larger ones in two (coarse, then fine bins).
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


@pytest.fixture(scope="module")
def er_big():
    # 17M vertices: 1038 fine bins, more than one LDS sort holds, so two passes
    note("er_big: generating")
    off, col = gen.er(17_000_000, 34_000_000, seed=9)
    note("er_big: oracle")
    case = PrCase(off, col)
    note("er_big: ready")
    return case


def budget(g, resident):
    if resident is not None:
        g.set_resident_fraction("pagerank", resident)


@pytest.mark.parametrize("mode", ["hybrid", "filter", "zerocopy", "compact"])
@pytest.mark.parametrize("pairs", [0, 4096, 1])
@pytest.mark.parametrize("resident", [0.25, 0.0, None])
def test_blocked_pagerank_matches_oracle(rmat12, mode, pairs, resident):
    note(f"rmat12 pagerank blocking mode={mode} pairs={pairs} resident={resident}")
    with hy.Graph(rmat12.off, rmat12.col) as g:
        g.set_params(partition_edges=2048, mode=mode, pr_block_pairs=pairs, pr_blocking=2)
        budget(g, resident)
        res = g.run("pagerank", stats=True, time_kernels=True)
        rmat12.check(res)
        launches = res.stats["kernel_launches"][BLOCK]
        if mode == "compact" or res.stats["nres"] == 0:
            # compaction pushes are not replayed; without resident partitions nothing is blocked
            assert launches == 0
        else:
            # one bucketing launch group per piece and iteration
            assert launches >= 20
            if pairs:
                assert launches >= 40  # several pieces: the two buffers alternate


def test_blocked_and_atomic_paths_agree(er_odd):
    note("er_odd pagerank blocking on / off")
    with hy.Graph(er_odd.off, er_odd.col) as g:
        g.set_params(partition_edges=1024, pr_block_pairs=5000, pr_blocking=2)
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
def test_many_pieces_match_oracle(rmat20, mode, resident):
    """2^20 vertices, pieces of 300000 pairs."""
    note(f"rmat20 pagerank blocking mode={mode} resident={resident}")
    with hy.Graph(rmat20.off, rmat20.col) as g:
        g.set_params(mode=mode, pr_block_pairs=300000, pr_blocking=2)
        budget(g, resident)
        res = g.run("pagerank", stats=True, time_kernels=True)
        rmat20.check(res)
        assert res.stats["kernel_launches"][BLOCK] >= 20 * 3


@pytest.mark.parametrize("resident,blocked", [(0.25, False), (0.6, True), (None, True)])
def test_automatic_blocking_follows_resident_share(rmat20, resident, blocked):
    """Default piece size and pr_blocking = 1: blocking only with at least 3/8 of the
    edges resident."""
    note(f"rmat20 pagerank automatic blocking resident={resident}")
    with hy.Graph(rmat20.off, rmat20.col) as g:
        g.set_params(gamma=(1, 1), zc_tie=1)
        budget(g, resident)
        res = g.run("pagerank", stats=True, time_kernels=True)
        rmat20.check(res)
        assert (res.stats["kernel_launches"][BLOCK] > 0) == blocked


@pytest.mark.parametrize("resident", [0.5, None])
def test_two_pass_buckets_match_oracle(er_big, resident):
    note(f"er 17M pagerank two-pass blocking resident={resident}")
    with hy.Graph(er_big.off, er_big.col) as g:
        g.set_params(pr_block_pairs=4_000_000, pr_blocking=2)
        budget(g, resident)
        note("er 17M: graph loaded, running")
        res = g.run("pagerank", stats=True, time_kernels=True)
        note("er 17M: run done")
        er_big.check(res)
        assert res.stats["kernel_launches"][BLOCK] >= 20 * 2


def test_piece_size_limit_is_checked(rmat12):
    with hy.Graph(rmat12.off, rmat12.col) as g:
        with pytest.raises(hy.HytmError) as ei:
            g.set_params(pr_block_pairs=1 << 31)
        assert ei.value.status == hy.E_INVAL
        with pytest.raises(hy.HytmError):
            g.set_params(pr_blocking=3)
