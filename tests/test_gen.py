"""The seeded input generators: well-formed CSR, determinism, symmetrization, weights."""
import numpy as np

import gen


def edges_of(off, col):
    u = np.repeat(np.arange(len(off) - 1, dtype=np.uint64), np.diff(off).astype(np.int64))
    return u, col.astype(np.uint64)


def check_csr(off, col):
    n = len(off) - 1
    assert off[0] == 0 and off[-1] == len(col) and (np.diff(off.astype(np.int64)) >= 0).all()
    u, v = edges_of(off, col)
    assert (v < n).all() and (u != v).all()
    key = (u << np.uint64(32)) | v
    assert (np.diff(key.astype(np.int64)) > 0).all()  # rows sorted, no duplicates


def test_rmat_wellformed_deterministic_skewed():
    off, col = gen.rmat(14, 16, seed=7)
    check_csr(off, col)
    off2, col2 = gen.rmat(14, 16, seed=7)
    np.testing.assert_array_equal(off, off2)
    np.testing.assert_array_equal(col, col2)
    off3, _ = gen.rmat(14, 16, seed=8)
    assert not np.array_equal(off, off3)
    deg = np.diff(off)
    assert deg[0] == deg.max()  # no label permutation: vertex 0 is the top hub
    assert len(col) < 16 << 14  # duplicates were removed


def test_er_and_pairs():
    off, col = gen.er(1000, 20000, seed=1)
    check_csr(off, col)
    assert 19000 < len(col) <= 20000
    off, col = gen.from_pairs(4, [0, 0, 1, 2, 2, 3], [1, 1, 2, 2, 0, 3])
    assert list(off) == [0, 1, 2, 3, 3] and list(col) == [1, 2, 0]


def test_symmetrize():
    off, col = gen.rmat(12, 8, seed=3)
    so, sc = gen.symmetrize(off, col)
    check_csr(so, sc)
    u, v = edges_of(off, col)
    su, sv = edges_of(so, sc)
    want = set(zip(u.tolist(), v.tolist())) | set(zip(v.tolist(), u.tolist()))
    assert set(zip(su.tolist(), sv.tolist())) == want


def test_weights_depend_on_edge_only():
    off, col = gen.rmat(12, 8, seed=3)
    w = gen.weights(off, col, 1016)
    assert w.min() >= 1 and w.max() <= 64 and len(np.unique(w)) == 64
    # the symmetrized graph keeps the weight of every original (u, v)
    so, sc = gen.symmetrize(off, col)
    sw = gen.weights(so, sc, 1016)
    u, v = edges_of(off, col)
    su, sv = edges_of(so, sc)
    lookup = dict(zip(zip(su.tolist(), sv.tolist()), sw.tolist()))
    assert all(lookup[(a, b)] == c for a, b, c in zip(u.tolist(), v.tolist(), w.tolist()))


def test_sources():
    off, col = gen.rmat(12, 8, seed=3)
    s = gen.sources(off, 8, 2024)
    assert len(s) == 8 and len(set(s.tolist())) == 8
    assert (np.diff(off)[s] > 0).all()
    np.testing.assert_array_equal(s, gen.sources(off, 8, 2024))


def test_disjoint_union_layout():
    a = gen.rmat(6, 4, seed=1)
    b = gen.from_pairs(3, np.array([0, 2], np.uint32), np.array([1, 0], np.uint32))
    off, col, w, bounds = gen.disjoint_union([a, b])
    na = len(a[0]) - 1
    np.testing.assert_array_equal(bounds, [0, na, na + 3])
    np.testing.assert_array_equal(off[: na + 1], a[0])
    np.testing.assert_array_equal(col[: len(a[1])], a[1])
    np.testing.assert_array_equal(off[na:] - off[na], b[0])
    np.testing.assert_array_equal(col[len(a[1]):], b[1] + na)
    assert w is None
