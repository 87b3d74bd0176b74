"""The autotuner's search (host logic) on a synthetic cost surface, and on the GPU a real
tuning run whose chosen parameters keep the results oracle-exact."""
import numpy as np
import pytest

import gen
import oracle
from paper_2208_14935_amd.tune import coordinate_descent


def test_coordinate_descent_finds_separable_minimum():
    grid = {"a": [1, 2, 3, 4], "b": ["x", "y", "z"], "c": [10, 20]}
    target = {"a": 3, "b": "z", "c": 20}
    cost = lambda cfg: sum(cfg[k] != v for k, v in target.items()) + 0.1 * cfg["a"]
    best, c, trials = coordinate_descent({"a": 1, "b": "x", "c": 10}, grid, cost)
    assert best == target
    assert c == cost(target)
    assert all(t[1] >= c for t in trials)


def test_coordinate_descent_keeps_start_when_it_is_best():
    grid = {"a": [1, 2, 3]}
    best, c, trials = coordinate_descent({"a": 2}, grid, lambda cfg: abs(cfg["a"] - 2))
    assert best == {"a": 2} and c == 0 and len(trials) == 3


def test_autotune_budgets_by_the_algorithms_bytes_per_edge():
    # budget_frac is a share of the bytes per edge the algorithm reads (SSSP with byte
    # weights: 5), not of 4 bytes per edge array
    from types import SimpleNamespace
    from paper_2208_14935_amd.tune import autotune

    class FakeGraph:
        m = 1000

        def __init__(self):
            self.budgets, self.applied = [], []

        def params(self):
            return SimpleNamespace(partition_edges=32768, combine_k=4, alpha_num=4, alpha_den=5, beta_num=2,
                                   beta_den=5, gamma_num=5, gamma_den=8, filter_engine=0)

        def edge_bytes(self, algo):
            return 5 if algo == "sssp" else 4

        def set_params(self, **kw):
            self.applied.append(kw)

        def set_budget(self, b):
            self.budgets.append(b)

    for algo, per_edge in (("sssp", 5), ("bfs", 4)):
        g = FakeGraph()
        res = autotune(g, algo, 0, budget_frac=0.25, grid={"combine_k": [1, 4]}, rounds=1,
                       runner=lambda gg, a, s: 1.0 + gg.applied[-1]["combine_k"] / 100)
        assert set(g.budgets) == {int(0.25 * per_edge * g.m)}
        assert res["best"]["combine_k"] == 1


@pytest.mark.gpu
def test_autotune_on_rmat16_keeps_results_exact():
    import paper_2208_14935_amd as hy
    from paper_2208_14935_amd.tune import autotune
    off, col = gen.rmat(16, 16, seed=16)
    w = gen.weights(off, col, 1016)
    grid = {"partition_edges": [8192, 32768, 131072], "combine_k": [4, 32], "gamma": [(5, 8), (1, 1)],
            "ab": [((4, 5), (2, 5))], "filter_engine": ["stream", "copy"]}
    with hy.Graph(off, col, weights=w) as g:
        res = autotune(g, "sssp", 0, budget_frac=0.25, grid=grid, repeats=1, rounds=1)
        assert res["best"]["partition_edges"] in grid["partition_edges"]
        assert len(res["trials"]) >= 5 and res["seconds"] > 0
        np.testing.assert_array_equal(g.run("sssp", 0).values, oracle.sssp(off, col, w, 0))
