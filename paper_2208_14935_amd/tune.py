"""Autotuner for the hybrid-transfer parameters.

Coordinate descent over the knobs that shape a run without changing its results:
partition size (8K..256K edges, the granularity of the cost model, Sec. 4/5.2), the
task-combination width k (Sec. 5.2), the selection constants alpha/beta (Sec. 5.1 rule)
and gamma (the zero-copy round-trip damping of Eq. 3), and the filter engine form.
Each candidate is timed with real library runs on the caller's graph, algorithm, source
and budget; the best setting is left on the graph and returned with the table of trials.

The kernels here map work to threads by edges (edge- and line-balanced), so there is no
separate threads-per-vertex knob to tune.
"""
from __future__ import annotations

import time

import numpy as np

DEFAULT_GRID = {
    "partition_edges": [8192, 16384, 32768, 65536, 131072, 262144],
    "combine_k": [1, 4, 16, 64],
    "ab": [((4, 5), (2, 5)), ((1, 1), (1, 2)), ((3, 5), (1, 5))],
    "gamma": [(5, 8), (1, 1), (3, 4)],
    "filter_engine": ["stream", "copy"],
}


def coordinate_descent(start: dict, grid: dict, cost, rounds: int = 2):
    """Minimise cost(config) one knob at a time, `rounds` passes over the knobs.
    Returns (best config, best cost, list of (config, cost) trials)."""
    best = dict(start)
    best_cost = cost(best)
    trials = [(dict(best), best_cost)]
    for _ in range(rounds):
        improved = False
        for knob, values in grid.items():
            for v in values:
                if best.get(knob) == v:
                    continue
                cand = dict(best)
                cand[knob] = v
                c = cost(cand)
                trials.append((dict(cand), c))
                if c < best_cost:
                    best, best_cost, improved = cand, c, True
        if not improved:
            break
    return best, best_cost, trials


def _apply(graph, cfg: dict):
    (an, ad), (bn, bd) = cfg["ab"]
    graph.set_params(partition_edges=cfg["partition_edges"], combine_k=cfg["combine_k"],
                     alpha=(an, ad), beta=(bn, bd), gamma=tuple(cfg["gamma"]),
                     filter_engine=cfg["filter_engine"])


def autotune(graph, algo: str, source: int = 0, budget_frac: float | None = 0.25, grid: dict | None = None,
             repeats: int = 2, rounds: int = 2, runner=None):
    """Tune `graph` (a paper_2208_14935_amd.Graph) for `algo` from `source` at a budget of
    `budget_frac` of the edge bytes the algorithm reads (staging included; None = keep the
    graph's budget).  runner(graph, algo, source) -> seconds may replace the timed run.
    Returns {"best": config, "seconds": t, "trials": [(config, seconds), ...]}."""
    grid = grid or DEFAULT_GRID
    p = graph.params()
    start = {
        "partition_edges": p.partition_edges, "combine_k": p.combine_k,
        "ab": ((p.alpha_num, p.alpha_den), (p.beta_num, p.beta_den)),
        "gamma": (p.gamma_num, p.gamma_den),
        "filter_engine": "stream" if p.filter_engine == 0 else "copy",
    }
    ebytes = graph.edge_bytes(algo)  # SSSP: 4 when packed, 5 with byte weights, else 8

    def timed(g, a, s):
        # results into a pinned buffer: a pageable one adds the same staged copy to every
        # candidate and blurs their differences
        from . import ALGOS, FLOAT_ALGOS, pinned_empty
        out = pinned_empty(max(g.n, 1), np.float32 if ALGOS[a] in FLOAT_ALGOS else np.uint32)[: g.n]
        g.run(a, s, out=out)  # warm caches and allocations
        t = float("inf")
        for _ in range(repeats):
            t0 = time.perf_counter()
            g.run(a, s, out=out)
            t = min(t, time.perf_counter() - t0)
        return t

    run = runner or timed

    def cost(cfg):
        _apply(graph, cfg)
        if budget_frac is not None:
            graph.set_budget(int(budget_frac * ebytes * graph.m))
        return run(graph, algo, source)

    best, t, trials = coordinate_descent(start, grid, cost, rounds=rounds)
    _apply(graph, best)
    if budget_frac is not None:
        graph.set_budget(int(budget_frac * ebytes * graph.m))
    return {"best": best, "seconds": t, "trials": trials}
