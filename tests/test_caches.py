"""The binary CSR cache of the generators and the oracle result cache of the large tests:
round trips, rejection of damaged files, and keys that follow the sources."""
import os

import numpy as np
import pytest

import gen
import oracle
import oracle_cache


def test_csr_round_trip(tmp_path):
    off, col = gen.rmat(10, 8, seed=3)
    p = str(tmp_path / "g.csr")
    gen.save_csr(p, off, col)
    for mm in (False, True):
        o2, c2 = gen.load_csr(p, mmap=mm)
        np.testing.assert_array_equal(o2, off)
        np.testing.assert_array_equal(c2, col)
    assert os.path.getsize(p) == 24 + 8 * len(off) + 4 * len(col)


def test_csr_rejects_damaged_files(tmp_path):
    off, col = gen.rmat(8, 4, seed=1)
    p = str(tmp_path / "g.csr")
    gen.save_csr(p, off, col)
    with open(p, "r+b") as fh:
        fh.truncate(os.path.getsize(p) - 4)
    with pytest.raises(ValueError):
        gen.load_csr(p)
    q = str(tmp_path / "h.csr")
    with open(q, "wb") as fh:
        fh.write(b"NOTACSR!" + bytes(16))
    with pytest.raises(ValueError):
        gen.load_csr(q)
    with pytest.raises(ValueError):
        gen.save_csr(p, off, col[:-1])


def test_rmat_cached_matches_and_reuses(tmp_path):
    d = str(tmp_path / "graphs")
    a = gen.rmat_cached(9, 8, seed=5, cache_dir=d)
    files = os.listdir(d)
    assert len(files) == 1 and gen.source_tag() in files[0]
    b = gen.rmat_cached(9, 8, seed=5, cache_dir=d)
    ref = gen.rmat(9, 8, seed=5)
    for x in (a, b):
        np.testing.assert_array_equal(x[0], ref[0])
        np.testing.assert_array_equal(x[1], ref[1])


def test_oracle_cache_round_trip(tmp_path, monkeypatch):
    off, col = gen.rmat(9, 8, seed=2)
    calls = []

    def compute():
        calls.append(1)
        return oracle.bfs(off, col, 0)

    monkeypatch.delenv("HYTM_ORACLE_CACHE", raising=False)
    want = oracle_cache.cached("t-bfs", compute)
    monkeypatch.setenv("HYTM_ORACLE_CACHE", str(tmp_path / "oc"))
    first = oracle_cache.cached("t-bfs", compute)
    again = oracle_cache.cached("t-bfs", compute)
    assert len(calls) == 2  # uncached, then computed once and read back
    for got in (first, again):
        np.testing.assert_array_equal(got[0], want[0])
        assert got[1] == want[1] and isinstance(got[1], int)
    pr = oracle_cache.cached("t-pr", lambda: oracle.pagerank(off, col, 0.85, 3))
    np.testing.assert_array_equal(oracle_cache.cached("t-pr", lambda: None), pr)
