"""Personalized PageRank lanes and the query server, through the C ABI.

PPR (single source and batched lanes) must stay within 1e-6 max-abs of the FP64 oracle.
Queries served in a mix must give what the oracle gives (BFS/SSSP bit for bit, PPR within
1e-6) and what the same query gives when run alone."""
import sys
import threading
import time

import numpy as np
import pytest

import gen
import oracle
import paper_2208_14935_amd as hy

pytestmark = pytest.mark.gpu
PPR_TOL = 1e-6


def note(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def g16():
    off, col = gen.rmat(16, 16, seed=16)
    w = gen.weights(off, col, 1016)
    return off, col, w


def ppr_err(got, off, col, s, T=10):
    want = oracle.ppr(off, col, int(s), 0.85, T)
    return float(np.abs(got.astype(np.float64) - want).max())


@pytest.mark.parametrize("mode,fe,resident", [("hybrid", "stream", None), ("hybrid", "stream", 0.25),
                                              ("hybrid", "copy", 0.25), ("zerocopy", "stream", 0.0),
                                              ("compact", "stream", 0.1), ("filter", "stream", 0.0)])
def test_ppr_single_and_batched_match_oracle(g16, mode, fe, resident):
    off, col, w = g16
    srcs = np.concatenate([[0], gen.sources(off, 8, 91), [0]]).astype(np.uint32)  # 10 lanes, a repeat
    note(f"ppr {mode} {fe} resident={resident} lanes={len(srcs)}")
    with hy.Graph(off, col) as g:
        g.set_params(mode=mode, filter_engine=fe, partition_edges=4096, compact_chunk_edges=1 << 16)
        if resident is not None:
            g.set_resident_fraction("ppr", resident)
        r = g.run("ppr", int(srcs[1]))
        assert r.values.dtype == np.float32 and r.iterations == 10
        assert ppr_err(r.values, off, col, srcs[1]) <= PPR_TOL
        vals, its, _ = g.run_batch("ppr", srcs)
    assert vals.shape == (len(srcs), len(off) - 1)
    assert (its == 10).all()
    for i, s in enumerate(srcs):
        assert ppr_err(vals[i], off, col, s) <= PPR_TOL, (i, s)


def test_ppr_iteration_count_parameter(g16):
    off, col, _ = g16
    with hy.Graph(off, col) as g:
        g.set_params(ppr_iterations=0)
        r = g.run("ppr", 7)
        want = np.zeros(len(off) - 1, dtype=np.float32)
        want[7] = 1.0
        np.testing.assert_array_equal(r.values, want)
        assert r.iterations == 0
        g.set_params(ppr_iterations=3)
        g.set_resident_fraction("ppr", 0.0)
        vals, its, _ = g.run_batch("ppr", [3, 11])
        assert (its == 3).all()
        for i, s in enumerate((3, 11)):
            assert ppr_err(vals[i], off, col, s, T=3) <= PPR_TOL


@pytest.mark.parametrize("algo", ["bfs", "sssp"])
def test_batch_with_a_narrow_lane_row(g16, algo):
    # 5 lanes use rows of 8 values instead of 64
    off, col, w = g16
    srcs = gen.sources(off, 5, 55)
    with hy.Graph(off, col, weights=w) as g:
        g.set_params(partition_edges=4096)
        g.set_resident_fraction(algo, 0.25)
        vals, its, _ = g.run_batch(algo, srcs)
    for i, s in enumerate(srcs):
        want = oracle.bfs(off, col, int(s))[0] if algo == "bfs" else oracle.sssp(off, col, w, int(s))
        np.testing.assert_array_equal(vals[i], want)


def mixed_queries(off, count, seed):
    """Seeded mix: half BFS, 30% SSSP, 20% PPR, sources over vertices with out-edges."""
    rng = np.random.default_rng(seed)
    kinds = rng.choice(["bfs", "sssp", "ppr"], size=count, p=[0.5, 0.3, 0.2])
    srcs = gen.sources(off, count, seed)
    return [(str(k), int(s)) for k, s in zip(kinds, srcs)]


@pytest.mark.parametrize("lanes,resident", [((4, 4, 2), 0.25), ((64, 64, 64), 0.0), ((1, 2, 1), None)])
def test_server_mix_matches_oracle_and_runs_alone(g16, lanes, resident):
    off, col, w = g16
    queries = mixed_queries(off, 40, 4000 + sum(lanes))
    note(f"serve lanes={lanes} resident={resident} queries={len(queries)}")
    with hy.Graph(off, col, weights=w) as g:
        g.set_params(partition_edges=4096)
        if resident is not None:
            g.set_resident_fraction("sssp", resident)
        alone = {}
        for a, s in queries:
            if (a, s) not in alone:
                r = g.run(a, s)
                alone[(a, s)] = (r.values.copy(), r.iterations)
        with hy.Server(g, bfs=lanes[0], sssp=lanes[1], ppr=lanes[2]) as srv:
            with pytest.raises(hy.HytmError) as e:
                g.run("bfs", 0)
            assert e.value.status == hy.E_STATE
            # arrivals spread over time from another thread, so queries join running groups
            subs = []
            rng = np.random.default_rng(7)

            def producer():
                for a, s in queries:
                    subs.append(srv.submit(a, s))
                    time.sleep(float(rng.uniform(0, 0.002)))

            th = threading.Thread(target=producer)
            th.start()
            th.join()
            done = [srv.wait(q) for q in subs]
        g.run("bfs", 0)  # the graph is free again
    for q in done:
        got = q.values
        want_alone, it_alone = alone[(q.algo, q.source)]
        assert q.result["status"] == hy.OK
        assert q.result["total_ms"] >= q.result["run_ms"] >= 0 and q.result["queue_ms"] >= 0
        if q.algo == "bfs":
            lvl, it = oracle.bfs(off, col, q.source)
            np.testing.assert_array_equal(got, lvl)
            np.testing.assert_array_equal(got, want_alone)
            assert q.result["iterations"] == it == it_alone
        elif q.algo == "sssp":
            np.testing.assert_array_equal(got, oracle.sssp(off, col, w, q.source))
            np.testing.assert_array_equal(got, want_alone)
            lo = oracle.bfs(off, col, q.source)[1]
            hi = oracle.sync_rounds(off, col, w, "sssp", q.source)
            assert lo <= q.result["iterations"] <= hi
        else:
            assert ppr_err(got, off, col, q.source) <= PPR_TOL
            assert np.abs(got - want_alone).max() <= PPR_TOL
            assert q.result["iterations"] == 10 == it_alone


def test_server_sssp_overflow_stays_in_its_lane():
    # 0 -> 1 -> 2 with weights 2^31: from 0 the distance of 2 overflows uint32, from 1 it does not
    off, col = gen.from_pairs(4, np.array([0, 1, 2], np.uint32), np.array([1, 2, 3], np.uint32))
    w = np.array([1 << 31, 1 << 31, 5], dtype=np.uint32)
    with hy.Graph(off, col, weights=w) as g:
        with hy.Server(g, bfs=2, sssp=4, ppr=0) as srv:
            qa = srv.submit("sssp", 0)
            qb = srv.submit("sssp", 1)
            qc = srv.submit("bfs", 0)
            with pytest.raises(hy.HytmError) as e:
                srv.wait(qa)
            assert e.value.status == hy.E_RANGE
            srv.wait(qb)
            srv.wait(qc)
            np.testing.assert_array_equal(qb.values, [hy.UNREACHED, 0, 1 << 31, (1 << 31) + 5])
            np.testing.assert_array_equal(qc.values, [0, 1, 2, 3])
            # the lane is clean for the next query
            qd = srv.submit("sssp", 2)
            srv.wait(qd)
            np.testing.assert_array_equal(qd.values, [hy.UNREACHED, hy.UNREACHED, 0, 5])


def test_server_argument_and_state_errors(g16):
    off, col, w = g16
    with hy.Graph(off, col) as g:
        for kw, status in (({"bfs": 0, "sssp": 0, "ppr": 0}, hy.E_INVAL), ({"bfs": 65, "sssp": 0, "ppr": 0}, hy.E_INVAL),
                           ({"bfs": 1, "sssp": 1, "ppr": 0}, hy.E_INVAL),  # no weights
                           ({"bfs": 64, "sssp": 0, "ppr": 64, "state_budget": 1 << 20}, hy.E_BUDGET)):
            with pytest.raises(hy.HytmError) as e:
                hy.Server(g, **kw)
            assert e.value.status == status, kw
        need = hy.Server.state_bytes(g, "bfs", 64) + hy.Server.state_bytes(g, "ppr", 3)
        assert hy.Server.state_bytes(g, "ppr", 3) == hy.Server.state_bytes(g, "ppr", 4)  # rows of 4
        with hy.Server(g, bfs=64, sssp=0, ppr=3, state_budget=need + (len(off) - 1) * 32) as srv:
            with pytest.raises(hy.HytmError) as e:
                hy.Server(g, bfs=1, sssp=0, ppr=0)
            assert e.value.status == hy.E_STATE
            for call in (lambda: g.set_params(combine_k=2), lambda: g.set_budget(1 << 20),
                         lambda: g.run_batch("bfs", [0])):
                with pytest.raises(hy.HytmError) as e:
                    call()
                assert e.value.status == hy.E_STATE
            with pytest.raises(hy.HytmError) as e:
                srv.submit("sssp", 0)
            assert e.value.status == hy.E_INVAL
            with pytest.raises(hy.HytmError) as e:
                srv.submit("bfs", len(off) - 1)
            assert e.value.status == hy.E_RANGE
            with pytest.raises(ValueError):
                srv.submit("ppr", 0, out=np.zeros(len(off) - 1, dtype=np.uint32))
            q = srv.submit("ppr", 0)
            srv.wait(q)
            assert ppr_err(q.values, off, col, 0) <= PPR_TOL
            with pytest.raises(hy.HytmError) as e:
                srv.wait(q)  # already waited for
            assert e.value.status == hy.E_STATE
        g.set_params(combine_k=2)  # released by close
