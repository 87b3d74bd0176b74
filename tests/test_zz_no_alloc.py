"""The allocation-free selection entry point (hytm_select_engines_static) against the
allocating one (hytm_select_engines), through the C ABI: engine codes equal byte for byte
on two calls in a row, the second with fewer partitions (the static scratch keeps the
first call's contents), under each engine mode and both edge-array counts, and a size past
the static limit refused on the host."""
import numpy as np
import pytest

import gen
import paper_2208_14935_amd as hy

pytestmark = pytest.mark.gpu


def stats(rng, npart):
    """Per-partition statistics in the ranges the selection accepts, with some inactive
    partitions, some fully active ones and the rest in between."""
    E = rng.integers(1, 1 << 20, npart, dtype=np.uint64)
    frac = rng.random(npart)
    frac[rng.random(npart) < 0.2] = 0.0
    frac[rng.random(npart) < 0.1] = 1.0
    Ea = np.minimum(E, np.ceil(E * frac)).astype(np.uint64)
    nA = np.where(Ea > 0, np.maximum(1, (Ea // rng.integers(1, 64, npart, dtype=np.uint64))), 0).astype(np.uint64)
    nA = np.minimum(nA, Ea)
    Rq = (Ea * 4 // 128 + nA + rng.integers(0, 3, npart, dtype=np.uint64) * (nA > 0)).astype(np.uint64)
    return E, nA, Ea, Rq


@pytest.fixture(scope="module")
def graph():
    off, col = gen.rmat(10, 8, seed=10)
    with hy.Graph(off, col) as g:
        yield g


@pytest.mark.parametrize("mode", ["hybrid", "zerocopy"])
@pytest.mark.parametrize("arrays", [1, 2])
def test_static_selection_matches_allocating_one(graph, mode, arrays):
    g = graph
    g.set_params(mode=mode)
    try:
        rng = np.random.default_rng(7 + arrays)
        for npart, nres in ((hy.STATIC_SELECT_MAX_PARTS, 1000), (70_001, 17)):
            E, nA, Ea, Rq = stats(rng, npart)
            want = g.select_engines(E, nA, Ea, Rq, nres=nres, edge_arrays=arrays)
            got = g.select_engines_static(E, nA, Ea, Rq, nres=nres, edge_arrays=arrays)
            assert got.shape == (npart,)
            np.testing.assert_array_equal(got, want)
            assert len(np.unique(want)) >= 2
    finally:
        g.reset_params()


def test_static_selection_limits(graph):
    g = graph
    empty = np.zeros(0, dtype=np.uint64)
    assert g.select_engines_static(empty, empty, empty, empty).shape == (0,)
    n = hy.STATIC_SELECT_MAX_PARTS + 1
    big = np.ones(n, dtype=np.uint64)
    with pytest.raises(hy.HytmError) as ei:
        g.select_engines_static(big, big, big, big)
    assert ei.value.status == 2  # HYTM_E_RANGE, refused before any device work
