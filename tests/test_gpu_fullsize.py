"""GPU parity at the benchmark's full size and launch configuration (R-MAT scale 24,
edge budget 25% of the bytes each algorithm reads, 32768-edge partitions, hybrid engines),
under two cost-model settings: the paper's (zero-copy damping 5/8, per-vertex requests,
ties to filter) and the one the benchmark uses on MI355X (no damping, since full-line
zero-copy reads run at the copy rate; distinct-line requests; ties to zero-copy).  They
pick different engines for many partitions.

BFS and CC are compared with the oracle element by element; SSSP by its certificate
(distance 0 at the source, no edge can still relax, every reached vertex has a tight parent
edge, reachability equal to BFS's), which pins the unique distances; PageRank element by
element within 1e-6 of the FP64 oracle's 20 steps.
"""
import os
import sys

import numpy as np
import pytest

import gen
import oracle
import oracle_cache
import paper_2208_14935_amd as hy

pytestmark = pytest.mark.gpu
SCALE = int(os.environ.get("HYTM_FULLSIZE_SCALE", "24"))


def note(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def big():
    gen.set_threads(min(16, os.cpu_count() or 1))
    off, col = gen.rmat_cached(SCALE, 16, seed=SCALE)
    w = gen.weights(off, col, 1000 + SCALE)
    srcs = gen.sources(off, 8, 2000 + SCALE)
    g = hy.Graph(off, col, weights=w, check_col=False)
    note(f"rmat{SCALE}: n={g.n} m={g.m}")
    yield off, col, w, srcs, g
    g.close()


SETTINGS = {
    "paper": dict(gamma=(5, 8), rq_distinct_lines=0, zc_tie=0),
    "bench": dict(gamma=(64, 64), rq_distinct_lines=1, zc_tie=1),
}
_want = {}


def cached(key, fn):
    """The oracle's answer for key, computed once per process (and kept on disk across
    processes when HYTM_ORACLE_CACHE names a directory)."""
    if key not in _want:
        _want[key] = oracle_cache.cached(f"rmat{SCALE}-" + "-".join(str(k) for k in key), fn)
    return _want[key]


def budget(g, arrays, setting):
    g.set_params(**SETTINGS[setting])
    g.set_budget(int(0.25 * 4 * arrays * g.m))


@pytest.mark.parametrize("setting", list(SETTINGS))
def test_bfs_fullsize_exact(big, setting):
    off, col, w, srcs, g = big
    budget(g, 1, setting)
    for s in srcs[:2]:
        note(f"bfs from {s}, {setting} cost model")
        r = g.run("bfs", int(s), stats=True)
        want, it = cached(("bfs", int(s)), lambda: oracle.bfs(off, col, int(s)))
        np.testing.assert_array_equal(r.values, want)
        assert r.iterations == it
        assert r.stats["nres"] < r.stats["npart"]  # oversubscribed


@pytest.mark.parametrize("setting", list(SETTINGS))
def test_sssp_fullsize_certificate(big, setting):
    off, col, w, srcs, g = big
    budget(g, g.edge_arrays("sssp"), setting)
    s = int(srcs[0])
    note(f"sssp from {s}, {setting} cost model")
    r = g.run("sssp", s)
    lvl, it_bfs = cached(("bfs", s), lambda: oracle.bfs(off, col, s))
    sssp_certificate(off, col, w, r.values, s, lvl)
    assert r.iterations >= it_bfs


def sssp_certificate(off, col, w, dist, s, lvl):
    """Distance 0 at the source, reachability equal to BFS's, no edge can still relax and
    every reached vertex but the source has a tight in-edge: together they fix the unique
    shortest distances (weights >= 1)."""
    n = len(off) - 1
    assert dist[s] == 0
    assert ((dist != hy.UNREACHED) == (lvl != hy.UNREACHED)).all()
    u = np.repeat(np.arange(n, dtype=np.uint32), np.diff(off).astype(np.int64))
    du = dist[u].astype(np.int64)
    dv = dist[col].astype(np.int64)
    reached = dist[u] != hy.UNREACHED
    del u
    assert (dv[reached] <= du[reached] + w[reached]).all()
    tight = reached & (dv == du + w.astype(np.int64))
    has_parent = np.zeros(n, dtype=bool)
    has_parent[col[tight]] = True
    need = dist != hy.UNREACHED
    need[s] = False
    assert has_parent[need].all()


def test_batched_fullsize_lanes(big):
    """64 BFS and 64 SSSP sources in one traversal each, as the batch benchmark runs them
    (bench cost-model settings, 25% budget): sampled lanes against the oracle (BFS element by
    element, SSSP by its certificate)."""
    off, col, w, srcs, g = big
    budget(g, 1, "bench")
    lanes = gen.sources(off, 64, 3000 + SCALE)
    check = [0, 1, 63]
    note("batched bfs, 64 sources")
    vals, its, _ = g.run_batch("bfs", lanes)
    for i in check:
        s = int(lanes[i])
        want, it = cached(("bfs", s), lambda: oracle.bfs(off, col, s))
        np.testing.assert_array_equal(vals[i], want, err_msg=f"bfs lane {i} source {s}")
        assert its[i] == it
    note("batched sssp, 64 sources")
    vals, its, _ = g.run_batch("sssp", lanes)
    for i in (0, 63):
        s = int(lanes[i])
        lvl, it_bfs = cached(("bfs", s), lambda: oracle.bfs(off, col, s))
        sssp_certificate(off, col, w, vals[i], s, lvl)
        assert its[i] >= it_bfs


def test_server_fullsize_queries(big):
    """The query server as the serving benchmark runs it (64 lanes per group, budget planned
    for SSSP's edge words at 25%, bench cost-model settings): BFS queries exact against the
    oracle, SSSP queries by the certificate, a PPR query within 1e-6 max-abs of the FP64
    oracle.  PPR keeps its mass near the source (values up to ~3e-2, sums of up to ~2.4e5
    shares per step): the per-step sums are accumulated in FP64, so only the FP32 rounding
    of the values and shares (~1e-7 relative per step) remains."""
    off, col, w, srcs, g = big
    budget(g, g.edge_arrays("sssp"), "bench")
    queries = [("bfs", int(srcs[0])), ("sssp", int(srcs[0])), ("ppr", int(srcs[0])), ("bfs", int(srcs[1])),
               ("sssp", int(srcs[1]))]
    note("server, 5 queries")
    with hy.Server(g, bfs=64, sssp=64, ppr=64) as srv:
        subs = [srv.submit(a, s) for a, s in queries]
        done = [srv.wait(q) for q in subs]
    for q in done:
        assert q.result["status"] == hy.OK
        lvl, it = cached(("bfs", q.source), lambda: oracle.bfs(off, col, q.source))
        if q.algo == "bfs":
            np.testing.assert_array_equal(q.values, lvl)
            assert q.result["iterations"] == it
        elif q.algo == "sssp":
            sssp_certificate(off, col, w, q.values, q.source, lvl)
            assert q.result["iterations"] >= it
        else:
            want = oracle.ppr(off, col, q.source, 0.85, 10)
            err = np.abs(q.values.astype(np.float64) - want)
            assert err.max() <= 1e-6, (float(err.max()), int(err.argmax()), float(want[err.argmax()]))
            assert q.result["iterations"] == 10


def test_cc_fullsize_exact():
    off, col = gen.rmat(SCALE, 16, seed=SCALE)
    soff, scol = gen.symmetrize(off, col)
    del off, col
    got = {}
    with hy.Graph(soff, scol, symmetric=True, check_col=False) as g:
        for setting in SETTINGS:
            note(f"cc, {setting} cost model")
            budget(g, 1, setting)
            got[setting] = g.run("cc").values.copy()
    want, _ = oracle.cc(soff, scol)
    for setting, vals in got.items():
        np.testing.assert_array_equal(vals, want, err_msg=setting)


@pytest.mark.parametrize("setting", list(SETTINGS))
def test_pagerank_fullsize_matches_oracle(big, setting):
    """All 20 steps from x_0 = 1/n, element by element against the FP64 oracle."""
    off, col, w, srcs, g = big
    budget(g, 1, setting)
    note(f"pagerank, {setting} cost model")
    r = g.run("pagerank")
    assert r.iterations == 20
    want = cached(("pagerank", 20), lambda: oracle.pagerank(off, col, 0.85, 20))
    err = np.abs(r.values.astype(np.float64) - want)
    assert err.max() <= 1e-6, (float(err.max()), int(err.argmax()))
