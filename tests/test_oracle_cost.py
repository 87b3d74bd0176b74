"""Pins for the oracle's partitioning, activity statistics, engine selection (Eq. 1-3 and
the alpha/beta rule of Sec. 5.1), task combination (Sec. 5.2) and compaction output.

The selection cases below were worked by hand from the equations; the numbers in each
comment are the hand computation, not the oracle's output.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import gen
import oracle
from oracle import COMPACT, FILTER, NONE, RESIDENT, ZEROCOPY, CostParams


def off_from_degrees(deg):
    return np.concatenate([[0], np.cumsum(np.asarray(deg, dtype=np.uint64))]).astype(np.uint64)


def lines_brute(start_edge, deg, line_bytes=128, entry_bytes=4):
    """Distinct `line_bytes` lines touched by entries start_edge..start_edge+deg-1 of an array
    of `entry_bytes`-byte entries (every byte of each entry)."""
    return len({(entry_bytes * e + b) // line_bytes for e in range(start_edge, start_edge + deg)
                for b in range(entry_bytes)})


# ------------------------------------------------------------- partition
def test_partition_hand_cases():
    assert list(oracle.partition(off_from_degrees([3, 3, 3]), 6)) == [0, 2, 3]
    assert list(oracle.partition(off_from_degrees([10]), 4)) == [0, 1]
    assert list(oracle.partition(off_from_degrees([2, 0, 0, 2, 2]), 4)) == [0, 4, 5]
    # an oversize vertex sits alone; the zero-degree vertices after it open the next one
    assert list(oracle.partition(off_from_degrees([1, 9, 0, 0, 1]), 4)) == [0, 1, 2, 5]
    assert list(oracle.partition(off_from_degrees([0, 0, 0]), 4)) == [0, 3]


@settings(max_examples=200, deadline=None)
@given(st.lists(st.integers(0, 40), min_size=1, max_size=60), st.integers(1, 64))
def test_partition_is_greedy_and_covers(deg, target):
    off = off_from_degrees(deg)
    b = [int(x) for x in oracle.partition(off, target)]
    assert b[0] == 0 and b[-1] == len(deg) and all(x < y for x, y in zip(b, b[1:]))
    for i in range(len(b) - 1):
        E = sum(deg[b[i]:b[i + 1]])
        # within target, unless it holds a single vertex with edges and that one exceeds it
        nz = [d for d in deg[b[i]:b[i + 1]] if d > 0]
        assert E <= target or (len(nz) == 1 and nz[0] > target)
        if i + 1 < len(b) - 1:
            # maximal: the next partition's first vertex did not fit
            assert E > 0 and E + deg[b[i + 1]] > target


# ------------------------------------------------------------------ stats
@settings(max_examples=200, deadline=None)
@given(st.lists(st.integers(0, 80), min_size=1, max_size=40), st.integers(1, 100), st.data())
def test_stats_match_brute_force_line_count(deg, target, data):
    off = off_from_degrees(deg)
    n = len(deg)
    active = np.array(data.draw(st.lists(st.booleans(), min_size=n, max_size=n)), dtype=np.uint8)
    b = oracle.partition(off, target)
    for arrays in (1, 2):
        nA, Ea, Rq = oracle.partition_stats(b, off, active, arrays=arrays)
        for i in range(len(b) - 1):
            vs = [v for v in range(int(b[i]), int(b[i + 1])) if active[v] and deg[v] > 0]
            assert nA[i] == len(vs)
            assert Ea[i] == sum(deg[v] for v in vs)
            assert Rq[i] == arrays * sum(lines_brute(int(off[v]), deg[v]) for v in vs)
    # byte weights: the weight lists are deg[v] bytes at byte offset off[v]
    _, _, Rq1 = oracle.partition_stats(b, off, active, arrays=2, weight_bytes=1)
    for i in range(len(b) - 1):
        vs = [v for v in range(int(b[i]), int(b[i + 1])) if active[v] and deg[v] > 0]
        assert Rq1[i] == sum(lines_brute(int(off[v]), deg[v]) + lines_brute(int(off[v]), deg[v], entry_bytes=1)
                             for v in vs)


def test_fig4_toy_graph_request_counts():
    # Sec. 3.3 / Fig. 4: 9 vertices and 128 edges in two 64-edge halves; every neighbour
    # list fits in one 128-byte line.  With each half fully active (half of all edges),
    # the 6-vertex half costs 6 zero-copy requests and the 3-vertex half costs 3.
    deg = [16, 16, 8, 8, 8, 8, 32, 16, 16]
    off = off_from_degrees(deg)
    b = oracle.partition(off, 64)
    assert list(b) == [0, 6, 9]
    nA, Ea, Rq = oracle.partition_stats(b, off, np.ones(9, np.uint8))
    assert list(Ea) == [64, 64] and list(nA) == [6, 3] and list(Rq) == [6, 3]
    # both fit one TLP window: ceil(6/256) = ceil(3/256) = 1, so Tiz ties; ratio 1 -> RTTzc = RTT
    E = [64, 64]
    p = oracle.select(E, nA, Ea, Rq)
    assert p[0] == p[1]


# ---------------------------------------------------------------- select
def one_partition(deg, active_mask, arrays=1, weight_bytes=None, distinct=False):
    off = off_from_degrees(deg)
    E = int(off[-1])
    b = np.array([0, len(deg)], dtype=np.uint64)
    nA, Ea, Rq = oracle.partition_stats(b, off, np.asarray(active_mask, np.uint8), arrays=arrays,
                                        weight_bytes=weight_bytes, distinct=distinct)
    return [E], nA, Ea, Rq


def test_requests_count_each_array_with_its_own_entry_size():
    # Three active lists of 40, 8 and 100 edges at edge offsets 0, 40, 48, 128-byte lines.
    # Neighbour array (4-byte entries): bytes [0,160) [160,192) [192,592) touch lines
    # {0,1} {1} {1,2,3,4}: 2 + 1 + 4 = 7 transactions per list, 5 distinct lines.
    # Byte weights: bytes [0,40) [40,48) [48,148) touch lines {0} {0} {0,1}: 1 + 1 + 2 = 4
    # transactions, 2 distinct lines.  4-byte weights repeat the neighbour array's counts.
    deg, act = [40, 8, 100], [1, 1, 1]
    for distinct, col, wb1 in ((False, 7, 4), (True, 5, 2)):
        assert one_partition(deg, act, distinct=distinct)[3][0] == col
        assert one_partition(deg, act, arrays=2, distinct=distinct)[3][0] == 2 * col
        assert one_partition(deg, act, arrays=2, weight_bytes=4, distinct=distinct)[3][0] == 2 * col
        assert one_partition(deg, act, arrays=2, weight_bytes=1, distinct=distinct)[3][0] == col + wb1
    with pytest.raises(ValueError):
        one_partition(deg, act, arrays=1, weight_bytes=1)
    with pytest.raises(ValueError):
        one_partition(deg, act, arrays=2, weight_bytes=2)


def test_select_w1_fully_active_goes_filter():
    # 1024 vertices x 32 edges, aligned: E = 32768, Tef = ceil(131072/32768) = 4,
    # Tec = ceil((131072 + 4096)/32768) = 5 (not < 3.2), Rq = 1024 -> ceil(1024/256) = 4,
    # RTTzc = RTT (ratio 1) -> Tiz = 4 = Tef: the tie goes to filter.
    E, nA, Ea, Rq = one_partition([32] * 1024, [1] * 1024)
    assert (int(nA[0]), int(Ea[0]), int(Rq[0])) == (1024, 32768, 1024)
    assert oracle.select(E, nA, Ea, Rq)[0] == FILTER


def test_select_w2_single_small_vertex_goes_zerocopy():
    # one active vertex of degree 10 at offset 0: Tec = 1 < 0.8*4; Tiz = 1*(5/8 + 3/8*10/32768)
    # ~ 0.6251, beta*Tiz ~ 0.25 < Tec -> not compaction; Tiz < Tef -> zero-copy
    deg = [10] + [32758]
    E, nA, Ea, Rq = one_partition(deg, [1, 0])
    assert oracle.select(E, nA, Ea, Rq)[0] == ZEROCOPY


def test_select_w3_many_tiny_active_vertices_go_compaction():
    # 8192 vertices x 4 edges, first 4096 active: Ea = 16384, Tec = ceil(81920/32768) = 3
    # < 3.2; every 16-byte list sits inside one line: Rq = 4096 -> 16; RTTzc = 5/8 + 3/8*1/2
    # = 13/16 -> Tiz = 13, beta*Tiz = 5.2 > 3 -> compaction
    E, nA, Ea, Rq = one_partition([4] * 8192, [1] * 4096 + [0] * 4096)
    assert int(Rq[0]) == 4096
    assert oracle.select(E, nA, Ea, Rq)[0] == COMPACT


def test_select_w5_w6_zerocopy_versus_filter():
    # 2048 vertices x 16 edges (64 B, never crossing a line).
    # Half active: Tec = ceil((65536+4096)/32768) = 3; Rq = 1024 -> 4; Tiz = 4*13/16 = 3.25;
    # beta*Tiz = 1.3 < 3 -> not compaction; 3.25 < 4 -> zero-copy.
    E, nA, Ea, Rq = one_partition([16] * 2048, [1] * 1024 + [0] * 1024)
    assert oracle.select(E, nA, Ea, Rq)[0] == ZEROCOPY
    # All active: Tec = 5; Rq = 2048 -> 8; Tiz = 8 > 4 -> filter.
    E, nA, Ea, Rq = one_partition([16] * 2048, [1] * 2048)
    assert oracle.select(E, nA, Ea, Rq)[0] == FILTER


def test_select_w7_gamma_weights_the_fixed_part():
    # 2048 x 16 edges, 1126 active: Ea = 18016, ratio 0.5498; Rq = 1126 -> 5;
    # Tiz = 5*(5/8 + 3/8*0.5498) = 4.156 >= 4 -> filter.  With gamma and 1-gamma swapped it
    # would be 5*(3/8 + 5/8*0.5498) = 3.59 < 4 -> zero-copy.
    E, nA, Ea, Rq = one_partition([16] * 2048, [1] * 1126 + [0] * 922)
    assert int(Rq[0]) == 1126
    assert oracle.select(E, nA, Ea, Rq)[0] == FILTER


def test_select_w8_index_bytes_count_in_tec():
    # 2730 x 12 edges + one x 8 edges = 32768; first 2000 active: Ea = 24000, |A| = 2000,
    # Tec = ceil((96000 + 8000)/32768) = 4 (3 without the index term), not < 3.2.
    # 48-byte lists cross a line 2 times in 8 -> Rq = 2500 -> 10; RTTzc = 5/8 + 3/8*24000/32768
    # -> Tiz = 8.997 > 4 -> filter.  Dropping |A|*d2 would make it compaction.
    deg = [12] * 2730 + [8]
    E, nA, Ea, Rq = one_partition(deg, [1] * 2000 + [0] * 731)
    assert (int(nA[0]), int(Ea[0]), int(Rq[0])) == (2000, 24000, 2500)
    assert oracle.select(E, nA, Ea, Rq)[0] == FILTER
    assert oracle.select(E, nA, Ea, Rq, params=CostParams(d2=0))[0] == COMPACT


def test_select_two_edge_arrays():
    # SSSP reads neighbours and weights: d1 = 8 and every list costs its lines twice.
    # W3 with weights: Tef = ceil(262144/32768) = 8, Tec = ceil((131072+16384)/32768) = 5
    # < 6.4; Rq = 8192 -> 32; Tiz = 32*13/16 = 26, beta*Tiz = 10.4 > 5 -> compaction.
    E, nA, Ea, Rq = one_partition([4] * 8192, [1] * 4096 + [0] * 4096, arrays=2)
    assert int(Rq[0]) == 8192
    assert oracle.select(E, nA, Ea, Rq, params=CostParams(d1=8))[0] == COMPACT


def test_select_byte_weights():
    # SSSP with weights stored as bytes reads d1 = 5 bytes per edge; Eq. 3's per-list requests
    # still count one transaction of each array per list (a 2-byte weight run costs one).
    # 16384 vertices of degree 2 (E = 32768), half of them active (Ea = 16384, nA = 8192),
    # 8-byte and 2-byte lists aligned within lines -> Rq = 2 * 8192 = 16384 -> ceil(/256) = 64,
    # RTTzc = 5/8 + 3/8 * 1/2 = 13/16, Tiz = 52.
    #   d1 = 8: Tef = 8, Tec = ceil((131072 + 32768)/32768) = 5 < 6.4 and < 20.8 -> compaction.
    #   d1 = 5: Tef = 5, Tec = ceil((81920 + 32768)/32768) = 4, not < alpha*Tef = 4; Tiz = 52
    #           is not < 5 either -> filter.  The index term weighs more against fewer bytes.
    E, nA, Ea, Rq = one_partition([2] * 16384, [1] * 8192 + [0] * 8192, arrays=2, weight_bytes=1)
    assert (int(E[0]), int(nA[0]), int(Ea[0]), int(Rq[0])) == (32768, 8192, 16384, 16384)
    assert oracle.select(E, nA, Ea, Rq, params=CostParams(d1=8))[0] == COMPACT
    assert oracle.select(E, nA, Ea, Rq, params=CostParams(d1=5))[0] == FILTER


def test_select_inactive_resident_and_forced():
    E = [100, 100, 100, 100]
    nA, Ea, Rq = [0, 3, 3, 3], [0, 30, 30, 30], [0, 3, 3, 3]
    assert list(oracle.select(E, nA, Ea, Rq, nres=2)) == [NONE, RESIDENT, ZEROCOPY, ZEROCOPY]
    assert list(oracle.select(E, nA, Ea, Rq, nres=0, force=COMPACT)) == [NONE, COMPACT, COMPACT, COMPACT]
    assert list(oracle.select(E, nA, Ea, Rq, nres=1, force=FILTER)) == [NONE, FILTER, FILTER, FILTER]


# --------------------------------------------------------------- combine
def test_combine_hand_cases():
    F, N, Z, C = FILTER, NONE, ZEROCOPY, COMPACT
    E = [1] * 9
    assert oracle.combine([F] * 5, E[:5], k=4) == [(0, 4), (4, 5)]
    assert oracle.combine([F, N, F], E[:3], k=4) == [(0, 1), (2, 3)]
    assert oracle.combine([F, F, F], E[:3], k=1) == [(0, 1), (1, 2), (2, 3)]
    assert oracle.combine([F, F, Z, F, F, F, C, F, F], E, k=2) == [(0, 2), (3, 5), (5, 6), (7, 9)]
    assert oracle.combine([N, Z, C, RESIDENT], E[:4], k=4) == []
    # an edge cap closes a task early; an oversize partition sits alone
    assert oracle.combine([F] * 4, [3, 3, 3, 9], k=4, max_edges=6) == [(0, 2), (2, 3), (3, 4)]


@settings(max_examples=200, deadline=None)
@given(st.lists(st.sampled_from([NONE, RESIDENT, FILTER, ZEROCOPY, COMPACT]), max_size=50),
       st.integers(1, 6))
def test_combine_covers_every_filter_partition_once(p, k):
    tasks = oracle.combine(p, [1] * len(p), k=k)
    covered = [i for a, b in tasks for i in range(a, b)]
    assert covered == [i for i, x in enumerate(p) if x == FILTER]
    for a, b in tasks:
        assert 1 <= b - a <= k
    # maximal: two tasks touch only when the first is full
    for (a0, b0), (a1, b1) in zip(tasks, tasks[1:]):
        if b0 == a1:
            assert b0 - a0 == k


# ---------------------------------------------------------------- gather
def test_gather_matches_slicing():
    off, col = gen.rmat(10, 8, seed=3)
    rng = np.random.default_rng(0)
    vc = np.sort(rng.choice(len(off) - 1, 200, replace=False)).astype(np.uint32)
    packed, newoff = oracle.gather(vc, off, col)
    want = np.concatenate([col[off[v]:off[v + 1]] for v in vc])
    np.testing.assert_array_equal(packed, want)
    np.testing.assert_array_equal(np.diff(newoff), np.diff(off)[vc])
    assert newoff[0] == 0


def test_select_gather_term_hand_case():
    # the w3 partition: Ea = 16384 edges, d1 = 4 -> 65536 gathered bytes.  Tec = 3, Tef = 4,
    # Tiz = 13.  gather = 1 (host gathers as fast as the link): Tgc = ceil(65536/32768) = 2
    # -> max(3, 2) = 3, still compaction.  gather = 2: Tgc = 4 -> not < 0.8*4 -> the rule
    # falls through to Tiz < Tef? 13 >= 4 -> filter.
    E, nA, Ea, Rq = one_partition([4] * 8192, [1] * 4096 + [0] * 4096)
    base = oracle.CostParams()
    assert oracle.select(E, nA, Ea, Rq, params=oracle.CostParams(gather=(1, 1)))[0] == COMPACT
    assert oracle.select(E, nA, Ea, Rq, params=oracle.CostParams(gather=(2, 1)))[0] == FILTER
    assert oracle.select(E, nA, Ea, Rq, params=oracle.CostParams(gather=(0, 1)))[0] == \
        oracle.select(E, nA, Ea, Rq, params=base)[0] == COMPACT


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 64), st.integers(1, 16), st.integers(0, 2 ** 32 - 1))
def test_select_gather_term_only_moves_partitions_off_compaction(gn, gd, seed):
    # a costlier gather can only turn compaction into filter or zero-copy, never the reverse,
    # and it never touches a partition that was not compaction
    rng = np.random.default_rng(seed)
    npart = 200
    E = rng.integers(1, 1 << 18, size=npart).astype(np.uint64)
    Ea = (E * rng.random(npart)).astype(np.uint64)
    nA = np.minimum(Ea, rng.integers(1, 1 << 12, size=npart)).astype(np.uint64)
    nA[Ea == 0] = 0
    Rq = (nA + Ea // 32 + rng.integers(0, 64, size=npart)).astype(np.uint64)
    a = oracle.select(E, nA, Ea, Rq)
    b = oracle.select(E, nA, Ea, Rq, params=oracle.CostParams(gather=(gn, gd)))
    changed = a != b
    assert (a[changed] == COMPACT).all()
    assert (b != COMPACT)[changed].all()
    assert not ((b == COMPACT) & (a != COMPACT)).any()


@settings(max_examples=60, deadline=None)
@given(st.lists(st.integers(0, 70), min_size=1, max_size=60), st.integers(1, 300), st.data())
def test_distinct_lines_match_a_set_of_touched_lines(deg, target, data):
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.uint64)
    n = len(deg)
    active = np.array(data.draw(st.lists(st.booleans(), min_size=n, max_size=n)))
    bounds = oracle.partition(off, target)
    for arrays in (1, 2):
        _, _, rq = oracle.partition_stats(bounds, off, active, arrays=arrays, distinct=True)
        _, _, rq_pv = oracle.partition_stats(bounds, off, active, arrays=arrays)
        for i in range(len(bounds) - 1):
            lines = set()
            for v in range(int(bounds[i]), int(bounds[i + 1])):
                if active[v] and deg[v]:
                    lines.update(range(int(off[v]) * 4 // 128, (int(off[v + 1]) * 4 - 1) // 128 + 1))
            assert rq[i] == arrays * len(lines)
            assert rq[i] <= rq_pv[i]  # never more than one request per vertex line
    _, _, rq1 = oracle.partition_stats(bounds, off, active, arrays=2, weight_bytes=1, distinct=True)
    for i in range(len(bounds) - 1):
        lines, wlines = set(), set()
        for v in range(int(bounds[i]), int(bounds[i + 1])):
            if active[v] and deg[v]:
                lines.update(range(int(off[v]) * 4 // 128, (int(off[v + 1]) * 4 - 1) // 128 + 1))
                wlines.update(range(int(off[v]) // 128, (int(off[v + 1]) - 1) // 128 + 1))
        assert rq1[i] == len(lines) + len(wlines)


def test_select_tie_rule_parameter():
    # the w1 tie (Tiz = Tef = 4) goes to zero-copy with zc_tie; a strict Tef < Tiz stays filter
    E, nA, Ea, Rq = one_partition([32] * 1024, [1] * 1024)
    assert oracle.select(E, nA, Ea, Rq, params=CostParams(zc_tie=1))[0] == ZEROCOPY
    E2, nA2, Ea2, Rq2 = one_partition([33] * 1024, [1] * 1024)  # misaligned lists: Rq > lines
    assert int(Rq2[0]) > (int(Ea2[0]) * 4 + 127) // 128
    assert oracle.select(E2, nA2, Ea2, Rq2, params=CostParams(zc_tie=1))[0] == FILTER
