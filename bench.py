"""Benchmark: hybrid-transfer graph traversal on one MI355X.

Workload (default, "oversubscribed"): R-MAT scale 28 (268M vertices, edge factor 16,
a/b/c = .57/.19/.19, self-loops and duplicates removed, ~4.3B edges), uint64 offsets,
uint32 neighbours and weights in [1, 64] held in pinned host memory (~34 GB); device edge
budget capped at 8 GB; 32768-edge partitions.  One step = BFS and SSSP from one seeded
source (the step's index picks one of 8 seeded sources in turn), CC on the symmetrized
graph and 20 synchronous PageRank iterations.  "--workload quarter-budget" is the R-MAT
scale-24 configuration at 25% of each algorithm's edge bytes with all 8 sources per step.

Prints one JSON line with GTEPS (algorithmic edges: reached out-edges for BFS/SSSP, m_sym
for CC, 20 m for PageRank), host-link GB/s against the measured pinned-copy peak, the
dominant kernel's roofline from live HIP-event timings, and the single-threaded CPU
oracle's rate on a bounded sample of the same workload (run before any GPU call, on one
core the process pins its thread to).
"""
import os

# The engine issues each pass's work on six HIP streams (selection, resident pushes, zero-copy,
# streaming filter, compaction copies, PageRank pair sorting).  HIP maps streams onto
# GPU_MAX_HW_QUEUES hardware queues (4 by default), and two streams that share a queue run
# their kernels one after the other.  The benchmark gives each stream its own queue (at least
# 8 queues, also where the environment sets fewer); it must be set before the process makes
# its first HIP call.
os.environ["GPU_MAX_HW_QUEUES"] = str(max(8, int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4)))

import argparse  # noqa: E402
import hashlib  # noqa: E402
import json  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import paper_2208_14935_amd as hy  # noqa: E402

HBM_PEAK_GBPS = 8000.0
# HBM traffic of the dominant kernel, from two rocprofv3 PMC passes over this benchmark
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB, the factors read off the probe's device copy of
# known size), mean per launch of the timed step.  It holds only for the kernel source and
# workload it was measured on; otherwise the roofline reports traffic null.
PMC_TRAFFIC = {"kernel": "k_push_fstream<OpPr>",
               "workload": "rmat28-ef16-budget8GB-hybrid-src1perstep-w8-rqdistinct-autotie",
               "kernels_sha256": "7fc92fe00bd43dd6d387b06d39c1643cbf3bec19e808d55180efbbe71fa48e7e",
               "bytes_per_launch": (2.0 * 14162316.25625 + 1.0 * 70101049.3125) * 1024.0,
               "summary": "profiles/pmc_traffic_rmat28_budget8GB_hybrid.md"}
PCIE_GEN5_X16_GBPS = 63.0
# hipHostMalloc fails past ~64 GiB per process on the MI355X hosts measured (295 GiB of RAM);
# the engine's own pinned buffers (compaction lists, selection mirrors, result buffers) need
# a few GB beside the edge arrays
PINNED_CEILING = 64 << 30
PINNED_HEADROOM = 10 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except Exception:
        pass


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=None,
                    help="R-MAT scale (default 28 for the oversubscribed workload, else 24)")
    ap.add_argument("--edge-factor", type=float, default=16)
    ap.add_argument("--sources", type=int, default=8)
    ap.add_argument("--sources-per-step", type=int, default=None,
                    help="BFS/SSSP sources per step, taken in turn from the seeded sources "
                         "(default 1 for the oversubscribed workload, all for quarter-budget)")
    ap.add_argument("--budget-frac", type=float, default=0.25)
    ap.add_argument("--mode", default="hybrid", choices=list(hy.MODES))
    ap.add_argument("--partition-edges", type=int, default=32768)
    ap.add_argument("--combine-k", type=int, default=4)
    ap.add_argument("--filter-engine", default="stream", choices=list(hy.FILTER_ENGINES))
    ap.add_argument("--gamma", default="probe",
                    help="zero-copy damping: 'probe' (from the measured partial-line cost), "
                         "'paper' (5/8) or num/den")
    ap.add_argument("--algos", default="bfs,sssp,cc,pagerank")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--probe-bytes", type=int, default=1 << 30)
    ap.add_argument("--workload", default="oversubscribed",
                    choices=["oversubscribed", "quarter-budget", "batch", "serve", "modes", "multigraph"],
                    help="oversubscribed: the headline step (R-MAT 28 at an 8 GB edge budget); quarter-budget: "
                         "R-MAT 24 at 25%% of the edge bytes; batch: 64-source BFS/SSSP in one traversal "
                         "against 64 sequential single-source runs; serve: Poisson arrivals of a BFS/SSSP/PPR "
                         "mix through the query server against one query at a time")
    ap.add_argument("--lanes", type=int, default=64)
    ap.add_argument("--qps", type=float, default=50.0, help="serve: mean arrival rate")
    ap.add_argument("--graph", default="rmat", choices=["rmat", "er"],
                    help="rmat: R-MAT at --scale; er: uniform G(n, m) with --er-vertices and --er-degree")
    ap.add_argument("--er-vertices", type=int, default=200_000_000)
    ap.add_argument("--er-degree", type=float, default=20.0)
    ap.add_argument("--pinned-ceiling", type=float, default=PINNED_CEILING,
                    help="pinned host bytes one process may hold; above it the headline step runs phased")
    ap.add_argument("--budget-bytes", type=float, default=None,
                    help="absolute device budget for edge data (default 8e9 for the oversubscribed workload, "
                         "else 0 = --budget-frac of each algorithm's bytes)")
    ap.add_argument("--modes", default="filter,filter-copy,compact,zerocopy,hybrid",
                    help="modes: transfer modes to compare (filter-copy = the explicit-copy filter engine)")
    ap.add_argument("--repeats", type=int, default=5, help="modes: timed runs per cell (median reported)")
    ap.add_argument("--copy-k", type=int, default=64,
                    help="modes: adjacent partitions per explicit copy of the filter-copy column")
    ap.add_argument("--queries", type=int, default=200, help="serve: queries in the arrival trace")
    ap.add_argument("--graphs", type=int, default=32, help="multigraph: R-MAT graphs of scales 16..22")
    ap.add_argument("--reprocess", type=int, nargs="?", const=1, default=0,
                    help="second pass over each iteration's loaded partitions (the paper's asynchronous "
                         "scheduling); 2 = only resident and zero-copy partitions")
    ap.add_argument("--hub-sort", action="store_true", help="relabel hubs to the front when the graphs are loaded")
    ap.add_argument("--no-pack", action="store_true",
                    help="keep SSSP weights in their own array instead of packing them into the neighbour words")
    ap.add_argument("--rq-per-vertex", dest="rq_distinct", action="store_false",
                    help="zero-copy requests of the cost model as Eq. 3's per-vertex lines (default: the distinct "
                         "lines the zero-copy kernel actually reads)")
    ap.add_argument("--rq-distinct", dest="rq_distinct", action="store_true")
    ap.add_argument("--zc-tie", default="auto",
                    help="where a Tiz = Tef tie goes: 'auto' (zero-copy for PageRank without propagation blocking, "
                         "filter otherwise), 'filter' (the paper), 'zerocopy', or 'probe' (zero-copy when full-line "
                         "zero-copy reads reach 95%% of the measured copy rate)")
    ap.add_argument("--sssp-delta", type=int, default=0,
                    help="SSSP far set: bound step (0 = the paper's synchronous push)")
    ap.add_argument("--pr-blocking", type=int, default=1, choices=[0, 1, 2],
                    help="PageRank over resident partitions: bucket the (destination, contribution) pairs and sum "
                         "them in LDS (propagation blocking) -- 1 = when at least half of the edges are resident, "
                         "2 = always, 0 = never (random float atomics into per-XCD accumulator copies)")
    ap.add_argument("--compact-gather", default="off",
                    help="host-gather term of the compaction cost: 'off' (the paper's rule), 'probe' (link rate / "
                         "measured gather rate) or num/den")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the engine runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is a design only)", file=sys.stderr)
        sys.exit(2)
    algos = args.algos.split(",")
    headline = args.workload in ("oversubscribed", "quarter-budget")
    if args.scale is None:
        args.scale = 28 if args.workload == "oversubscribed" else 24
    if args.budget_bytes is None:
        args.budget_bytes = 8e9 if args.workload == "oversubscribed" else 0
    if args.sources_per_step is None:
        args.sources_per_step = 1 if args.workload == "oversubscribed" else args.sources

    gen.set_threads(min(16, len(os.sched_getaffinity(0)) or 1))
    if args.workload == "multigraph":
        return multigraph_workload(args)
    t0 = time.time()
    if args.graph == "er":
        off, col = gen.er(args.er_vertices, int(args.er_vertices * args.er_degree), seed=7)
    else:
        off, col = gen.rmat_cached(args.scale, args.edge_factor, seed=args.scale)  # HYTM_GRAPH_CACHE: reuse
    n, m = len(off) - 1, len(col)
    log(f"generated n={n} m={m} in {time.time() - t0:.1f}s")
    w = gen.weights(off, col, 1000 + args.scale)
    log(f"weights done {time.time() - t0:.1f}s")
    srcs = gen.sources(off, args.sources, 2000 + args.scale)
    need_sym = "cc" in algos and (headline or args.workload == "modes")
    soff, scol = gen.symmetrize(off, col) if need_sym else (None, None)
    deg = np.diff(off).astype(np.int64)
    gname = f"er{n}-d{args.er_degree:g}" if args.graph == "er" else f"rmat{args.scale}"
    log(f"graph: {gname} n={n} m={m} m_sym={len(scol) if scol is not None else 0} "
        f"max_deg={deg.max()} gen {time.time() - t0:.1f}s")

    # the oracle's leg runs first, before this process makes any GPU call, on one pinned core
    cpu = None
    if headline and not args.no_cpu_baseline:
        cpu = cpu_baseline(off, col, w, soff, scol, srcs, algos, large=n > (1 << 26))

    probe = hy.link_probe(args.probe_bytes)
    log(f"probe: {json.dumps(probe)}")

    t0 = time.time()
    g = hy.Graph(off, col, weights=w, check_col=False, hub_sort=args.hub_sort, pack=not args.no_pack)
    ginfo = g.info()
    packed = bool(ginfo["packed_weights"])
    # Both graphs of the headline step stay pinned at once only when their edge arrays fit
    # under the host's pinned-memory ceiling with room for the engine's own pinned buffers;
    # otherwise the step runs phased: every timed pass over the directed graph, then the
    # directed graph's pinned copy is released, the symmetrized graph is pinned, and every
    # timed CC pass follows.  Swapping the pinned copies is excluded like graph loading.
    g_bytes = m * g.edge_bytes("sssp" if w is not None else "bfs")
    sym_bytes = 4 * len(scol) if scol is not None else 0
    phased = (headline and scol is not None
              and g_bytes + sym_bytes + PINNED_HEADROOM > args.pinned_ceiling)
    # the per-mode workload loads the symmetrized graph only after the directed one is
    # closed, so that the two never hold pinned host memory at once
    gs = (hy.Graph(soff, scol, symmetric=True, check_col=False, hub_sort=args.hub_sort)
          if scol is not None and args.workload != "modes" and not phased else None)
    log(f"pinned graph copies {time.time() - t0:.1f}s"
        + (f" (phased: {g_bytes / 1e9:.1f} + {sym_bytes / 1e9:.1f} GB of edges over a "
           f"{args.pinned_ceiling / 2**30:.0f} GiB pinned ceiling)" if phased else ""))
    if headline:
        del col, w  # the graphs hold their own pinned copies (at R-MAT 28 these were ~70 GB)
        if not phased:
            del scol
    gamma = gamma_from(args.gamma, probe)
    log(f"gamma = {gamma[0]}/{gamma[1]}")
    if args.compact_gather == "off":
        cgather = (0, 1)
    elif args.compact_gather == "probe":
        cgather = (max(1, int(round(64 * probe["h2d_copy_gbps"] / probe["host_gather_gbps"]))), 64)
    else:
        a, b_ = args.compact_gather.split("/")
        cgather = (int(a), int(b_))
    log(f"compaction gather cost = {cgather[0]}/{cgather[1]}")
    # a tie means equal bytes by either engine; rates within 5% of each other count as equal
    zc_tie = {"filter": 0, "zerocopy": 1, "auto": 2}.get(args.zc_tie,
                                              int(probe["zc_read_gbps"]["128B"] >= 0.95 * probe["h2d_copy_gbps"]))
    log(f"tie to zero-copy = {zc_tie}")

    def configure(h):
        h.set_params(mode=args.mode, partition_edges=args.partition_edges, combine_k=args.combine_k,
                     filter_engine=args.filter_engine, gamma=gamma, reprocess=int(args.reprocess),
                     compact_gather=cgather, rq_distinct_lines=int(args.rq_distinct), zc_tie=zc_tie,
                     pr_blocking=args.pr_blocking, sssp_delta=args.sssp_delta)

    for h in (g, gs):
        if h is not None:
            configure(h)
    if args.workload == "batch":
        return batch_workload(args, g, off, col, deg, gamma, probe)
    if args.workload == "serve":
        return serve_workload(args, g, off, gamma, probe)
    if args.workload == "modes":
        return modes_workload(args, gname, g, (soff, scol), deg, srcs[:1], algos, gamma, probe, cgather, zc_tie)

    def budget(h, algo):
        # an absolute edge budget, or a fraction of the edge bytes the graph holds for the
        # algorithm (SSSP: neighbours and weights, or one packed word per edge)
        if args.budget_bytes:
            h.set_budget(int(args.budget_bytes))
        else:
            h.set_budget(int(args.budget_frac * h.edge_bytes(algo) * h.m))

    kt = not args.no_kernel_timing

    # algorithmic edges of BFS and SSSP from s: out-edges of the vertices reachable from s
    # (SSSP reaches exactly the vertices BFS reaches), counted outside the timed region
    reach_edges = {}
    budget(g, "bfs")
    for s in srcs:
        lv = g.run("bfs", int(s)).values
        reach_edges[int(s)] = int(deg[lv != hy.UNREACHED].sum())

    # results land in pinned host buffers (direct DMA); each run overwrites the previous one
    out_u32 = hy.pinned_empty(n, np.uint32)
    out_f32 = hy.pinned_empty(n, np.float32)

    k_src = max(1, min(args.sources_per_step, len(srcs)))
    step_no = [0]
    ebytes = {a: g.edge_bytes(a) for a in ("bfs", "sssp", "pagerank")}  # bytes per edge read

    def step_sources():
        # step i takes sources i*k .. i*k+k-1 of the seeded list, wrapping around
        i = step_no[0]
        step_no[0] += 1
        return [srcs[(i * k_src + j) % len(srcs)] for j in range(k_src)]

    def step_directed(record):
        runs = []
        ss = step_sources()
        if "bfs" in algos:
            budget(g, "bfs")
            for s in ss:
                r = g.run("bfs", int(s), stats=True, time_kernels=kt and record, out=out_u32)
                runs.append(("bfs", r, reach_edges[int(s)]))
        if "pagerank" in algos:
            budget(g, "pagerank")
            r = g.run("pagerank", stats=True, time_kernels=kt and record, out=out_f32)
            runs.append(("pagerank", r, 20 * m))
        if "sssp" in algos:
            budget(g, "sssp")
            for s in ss:
                r = g.run("sssp", int(s), stats=True, time_kernels=kt and record, out=out_u32)
                runs.append(("sssp", r, reach_edges[int(s)]))
        return runs

    def step_cc(record):
        if "cc" not in algos:
            return []
        budget(gs, "cc")
        r = gs.run("cc", stats=True, time_kernels=kt and record, out=out_u32)
        return [("cc", r, gs.m)]

    def timed(step):
        for i in range(args.warmup):
            t = time.time()
            step(False)
            log(f"warmup step {i}: {time.time() - t:.2f}s")
        runs = []
        sync()
        t_start = time.perf_counter()
        for i in range(args.steps):
            t = time.time()
            runs += step(True)
            log(f"step {i}: {time.time() - t:.2f}s")
        sync()
        return runs, time.perf_counter() - t_start

    if not phased:
        all_runs, elapsed = timed(lambda record: step_directed(record) + step_cc(record))
        m_sym = int(gs.m) if gs is not None else None
    else:
        all_runs, elapsed = timed(step_directed)
        log(f"phase 1 (directed graph): {elapsed:.2f}s")
        g.close()
        t = time.time()
        gs = hy.Graph(soff, scol, symmetric=True, check_col=False, hub_sort=args.hub_sort)
        configure(gs)
        del scol
        log(f"pinned symmetrized copy {time.time() - t:.1f}s")
        runs_cc, elapsed_cc = timed(step_cc)
        log(f"phase 2 (symmetrized graph): {elapsed_cc:.2f}s")
        all_runs += runs_cc
        elapsed += elapsed_cc
        m_sym = int(gs.m)
    ebytes["cc"] = gs.edge_bytes("cc") if gs is not None else 4

    edges = sum(e for _, _, e in all_runs)
    value = edges / elapsed / 1e9
    per_algo = {}
    for a in algos:
        rs = [(r, e) for name, r, e in all_runs if name == a]
        if not rs:
            continue
        ms = sum(r.stats["ms_total"] for r, _ in rs)
        per_algo[a] = {
            "gteps": sum(e for _, e in rs) / (ms / 1e3) / 1e9,
            "ms_per_run": ms / len(rs),
            "iterations": rs[0][0].iterations,
            "engine_partition_iters": dict(zip(hy.ENGINE_NAMES, rs[0][0].stats["part_iters"])),
            "bytes_filter": sum(r.stats["bytes_filter"] for r, _ in rs) // len(rs),
            "bytes_compact": sum(r.stats["bytes_compact"] for r, _ in rs) // len(rs),
            "bytes_zerocopy": sum(r.stats["bytes_zerocopy"] for r, _ in rs) // len(rs),
            "ms_select": sum(r.stats["ms_select"] for r, _ in rs) / len(rs),
            "ms_fill": sum(r.stats["ms_fill"] for r, _ in rs) / len(rs),
        }
    moved = sum(r.stats["bytes_filter"] + r.stats["bytes_compact"] + r.stats["bytes_zerocopy"]
                + r.stats["bytes_resident_fill"] for _, r, _ in all_runs)
    link_gbps = moved / elapsed / 1e9
    host_link = {"gbps": link_gbps, "peak_gbps": probe["h2d_copy_gbps"],
                 "frac": link_gbps / probe["h2d_copy_gbps"],
                 "explicit_bytes": sum(r.stats["bytes_filter"] + r.stats["bytes_compact"] + r.stats["bytes_resident_fill"]
                                       for _, r, _ in all_runs),
                 "zerocopy_bytes": sum(r.stats["bytes_zerocopy"] for _, r, _ in all_runs)}

    workload = (gname + (f"-ef{args.edge_factor:g}" if args.graph == "rmat" else "")
                + (f"-budget{args.budget_bytes / 1e9:g}GB" if args.budget_bytes else f"-budget{args.budget_frac:g}")
                + f"-{args.mode}" + (f"-src{k_src}perstep" if k_src != len(srcs) else "")
                + (f"-reprocess{args.reprocess}" if args.reprocess else "") + ("-hubsort" if args.hub_sort else "")
                + ("" if packed else {1: "-w8", 4: "-unpacked"}.get(ginfo["weight_bytes"], ""))
                + ("" if cgather[0] == 0 else "-gathercost") + ("-rqdistinct" if args.rq_distinct else "")
                + {0: "", 1: "-zctie", 2: "-autotie"}[zc_tie] + ("-prblock" if args.pr_blocking == 2 and "pagerank" in algos else "")
                + (f"-delta{args.sssp_delta}" if args.sssp_delta and "sssp" in algos else ""))
    roofline = None
    kernels = {}
    if kt:
        # per (algorithm, kernel class): event ms, launches, items, items x edge arrays, and
        # the distinct lines the zero-copy kernel read (a line two lists share counts once)
        per = {}
        for name, r, _ in all_runs:
            a = ebytes[name]
            for c, cls in enumerate(hy.KERNEL_CLASSES):
                nl = r.stats["kernel_launches"][c]
                if not nl:
                    continue
                e = per.setdefault((name, cls), [0.0, 0, 0, 0, 0])
                e[0] += r.stats["kernel_ms"][c]
                e[1] += nl
                e[2] += r.stats["kernel_items"][c]
                e[3] += r.stats["kernel_items"][c] * a  # bytes of the edge arrays
                if cls == "push_zerocopy":
                    e[4] += r.stats["zc_lines_distinct"] * 32 * a  # a line of each array
        for cls in hy.KERNEL_CLASSES:
            es = [v for (al, c), v in per.items() if c == cls]
            kernels[cls] = {"ms": sum(v[0] for v in es) / args.steps,
                            "launches": sum(v[1] for v in es) // args.steps,
                            "items": sum(v[2] for v in es) // args.steps}
        (dalgo, name), (d_ms, d_launches, d_items, d_aitems, d_zc) = max(per.items(), key=lambda kv: kv[1][0])
        avg_ms = d_ms / max(d_launches, 1)
        # algorithmic bytes per launch.  Kernels reading the mapped host arrays are priced
        # against the host link: the zero-copy kernel moves 128 B per distinct line it reads
        # per edge array, the streaming filter kernel the bytes per edge (4, 5 with byte weights,
        # 8) of its tasks' edges.  Kernels reading device memory are priced against HBM: the
        # bytes per edge plus one 4-byte vertex value touched per edge.
        if name == "push_zerocopy":
            per_launch = d_zc / max(d_launches, 1)
            bound, peak = "pcie", PCIE_GEN5_X16_GBPS
        elif name == "push_filter" and args.filter_engine == "stream":
            per_launch = d_aitems / max(d_launches, 1)
            bound, peak = "pcie", PCIE_GEN5_X16_GBPS
        elif name.startswith("push"):
            per_launch = (d_aitems + d_items * 4) / max(d_launches, 1)
            bound, peak = "hbm", HBM_PEAK_GBPS
        elif name == "pr_blocking":
            # per pair: each counting-sort pass reads and writes 8 B, the summing pass reads
            # 8 B; per piece: one read-modify-write of every accumulator slot
            passes = 2 if (n + 16383) // 16384 > 1024 else 1
            slots = (n + 4095) // 4096 * 4096
            per_launch = (d_items * (16 * passes + 8) + d_launches * 8 * slots) / max(d_launches, 1)
            bound, peak = "hbm", HBM_PEAK_GBPS
        else:
            per_launch = d_items * 16 / max(d_launches, 1)
            bound, peak = "hbm", HBM_PEAK_GBPS
        achieved = per_launch / (avg_ms / 1e3) / 1e9
        op = {"bfs": "OpBfs", "sssp": "OpSssp", "cc": "OpCc", "pagerank": "OpPr"}[dalgo]
        symbol = {"push_zerocopy": f"k_push_lines<{op}>", "push_filter": f"k_push_fstream<{op}>",
                  "push_resident": f"k_push_edges<{op}, false>", "push_compact": f"k_push_edges<{op}, true>",
                  "stats": "k_stats_select", "lists": "k_build_lists"}.get(name, name)
        traffic = None
        src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2208_14935_amd", "csrc", "kernels.hip")
        with open(src, "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
        if (symbol == PMC_TRAFFIC["kernel"] and sha == PMC_TRAFFIC["kernels_sha256"]
                and workload == PMC_TRAFFIC["workload"]):
            traffic = PMC_TRAFFIC["bytes_per_launch"]
        roofline = {"kernel": symbol, "algorithm": dalgo, "class": name, "bound": bound, "achieved": achieved,
                    "peak": peak, "unit": "GB/s", "frac": achieved / peak, "traffic": traffic,
                    "traffic_unit": "bytes per launch (HBM, PMC)", "algorithmic_bytes_per_launch": per_launch,
                    "avg_launch_ms": avg_ms, "launches_per_step": d_launches // args.steps,
                    "measured_link_peak_gbps": probe["h2d_copy_gbps"]}

    out = {
        "metric": "GTEPS for BFS/SSSP/CC/PR at capped HBM budget; host-link GB/s vs peak",
        "value": value,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 (BFS/SSSP/CC), f32 (PageRank)",
        "data": "synthetic R-MAT, seeded",
        "config": {"workload": workload,
                   "n": n, "m": m, "m_sym": m_sym, "phased": phased,
                   "sources": [int(s) for s in srcs], "sources_per_step": k_src,
                   "budget_bytes": int(args.budget_bytes) if args.budget_bytes else None,
                   "budget_frac_of_edge_bytes": None if args.budget_bytes else args.budget_frac,
                   "partition_edges": args.partition_edges, "combine_k": args.combine_k, "mode": args.mode,
                   "filter_engine": args.filter_engine, "gamma": list(gamma), "algos": algos,
                   "compact_gather": list(cgather), "zc_tie": zc_tie,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host_link": host_link,
        "per_algo": per_algo,
        "kernels": kernels,
        "probe": probe,
    }
    print(json.dumps(out), flush=True)


def batch_workload(args, g, off, col, deg, gamma, probe):
    """64-source BFS and SSSP in one traversal each, against the same 64 sources run one
    at a time, at the same budget and parameters.  GTEPS counts, per source, the out-edges
    of the vertices it reaches."""
    n, m = len(off) - 1, len(col)
    srcs = gen.sources(off, args.lanes, 3000 + args.scale)
    reach = []
    g.set_budget(int(args.budget_frac * 4 * g.m))
    for s in srcs:
        lv = g.run("bfs", int(s)).values
        reach.append(int(deg[lv != hy.UNREACHED].sum()))
    edges = sum(reach)
    res = {}
    out_b = hy.pinned_empty((len(srcs), g.n), np.uint32)
    out_1 = hy.pinned_empty(g.n, np.uint32)
    for algo in ("bfs", "sssp"):
        g.set_budget(int(args.budget_frac * g.edge_bytes(algo) * g.m))
        g.run_batch(algo, srcs, out=out_b)  # warm-up
        times = []
        for _ in range(args.steps):
            sync()
            t = time.perf_counter()
            vals, its, st = g.run_batch(algo, srcs, stats=True, out=out_b)
            sync()
            times.append(time.perf_counter() - t)
        tb = min(times)
        sync()
        t = time.perf_counter()
        for s in srcs:
            g.run(algo, int(s), out=out_1)
        sync()
        ts = time.perf_counter() - t
        res[algo] = {"batched_ms": tb * 1e3, "sequential_ms": ts * 1e3, "speedup": ts / tb,
                     "batched_gteps": edges / tb / 1e9, "sequential_gteps": edges / ts / 1e9,
                     "iterations": int(max(its)),
                     "host_link_gbps": (st["bytes_filter"] + st["bytes_compact"] + st["bytes_zerocopy"]) / tb / 1e9}
        log(f"{algo}: batched {tb * 1e3:.1f} ms, sequential {ts * 1e3:.1f} ms")
    value = 2 * edges / (res["bfs"]["batched_ms"] + res["sssp"]["batched_ms"]) / 1e6
    out = {
        "metric": "multi-source GTEPS (64 BFS + 64 SSSP sources, one traversal each) vs one source at a time",
        "value": value, "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": res["bfs"]["batched_ms"] + res["sssp"]["batched_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic R-MAT, seeded",
        "config": {"workload": f"rmat{args.scale}-batch{len(srcs)}-budget{args.budget_frac:g}", "n": n, "m": m,
                   "lanes": len(srcs), "mode": args.mode, "filter_engine": args.filter_engine, "gamma": list(gamma)},
        "batch": res, "probe": probe,
    }
    print(json.dumps(out), flush=True)


def modes_workload(args, gname, g, sym, deg, srcs, algos, gamma, probe, cgather, zc_tie):
    """Every algorithm under each transfer mode at one device budget (one warm-up run, then
    --repeats timed runs that reuse the resident prefix, reported as median, min and max;
    absolute --budget-bytes, else --budget-frac of the algorithm's edge bytes): GTEPS and
    the host link's achieved GB/s (explicit + zero-copy + resident-fill bytes over run time)
    against the measured pinned-copy peak.  Modes: filter (the streaming form), filter-copy
    (the explicit-copy form, SDMA copies of up to --copy-k adjacent partitions into staging),
    compact, zerocopy, hybrid."""
    s = int(srcs[0])
    # results land in pinned buffers, as in the other workloads (a pageable one makes the
    # final copy of n values go through staging: ~90 ms more at RMAT-28)
    n_max = max(g.n, len(sym[0]) - 1 if sym[0] is not None else 0)
    outs = {np.uint32: hy.pinned_empty(n_max, np.uint32), np.float32: hy.pinned_empty(n_max, np.float32)}
    lv = g.run("bfs", s).values  # reach of the source, outside the timed runs
    reach = int(deg[lv != hy.UNREACHED].sum())
    m_directed, m_sym = int(g.m), (len(sym[1]) if sym[1] is not None else 0)
    work = {"bfs": reach, "sssp": reach, "cc": m_sym, "pagerank": 20 * g.m}
    table = {}
    order = [a for a in algos if a != "cc"] + (["cc"] if "cc" in algos else [])
    gs = None
    for a in order:
        if a == "cc" and gs is None:
            g.close()
            gs = hy.Graph(sym[0], sym[1], symmetric=True, check_col=False, hub_sort=args.hub_sort)
            gs.set_params(partition_edges=args.partition_edges, combine_k=args.combine_k,
                          filter_engine=args.filter_engine, gamma=gamma, reprocess=int(args.reprocess),
                          compact_gather=cgather, rq_distinct_lines=int(args.rq_distinct), zc_tie=zc_tie)
        for mode in args.modes.split(","):
            h = gs if a == "cc" else g
            if mode == "filter-copy":
                h.set_params(mode="filter", filter_engine="copy", combine_k=args.copy_k)
            else:
                h.set_params(mode=mode, filter_engine=args.filter_engine, combine_k=args.combine_k)
            h.set_budget(int(args.budget_bytes) if args.budget_bytes else int(args.budget_frac * h.edge_bytes(a) * h.m))
            out = outs[np.float32 if a == "pagerank" else np.uint32][: h.n]
            try:
                h.run(a, s, out=out)  # warm-up: staging buffers and the resident prefix of this plan
                rs = [h.run(a, s, stats=True, out=out) for _ in range(max(1, args.repeats))]
            except hy.HytmError as e:  # a forced engine whose staging does not fit
                table[f"{mode}/{a}"] = {"error": str(e)}
                log(f"{mode:9s} {a:9s} {e}")
                continue
            times = sorted(x.stats["ms_total"] for x in rs)
            r = sorted(rs, key=lambda x: x.stats["ms_total"])[len(rs) // 2]  # the median run
            st = r.stats
            sec = st["ms_total"] / 1e3
            moved = st["bytes_filter"] + st["bytes_compact"] + st["bytes_zerocopy"] + st["bytes_resident_fill"]
            row = {"ms": st["ms_total"], "ms_min": times[0], "ms_max": times[-1], "runs": len(times),
                   "gteps": work[a] / sec / 1e9, "iterations": r.iterations,
                   "link_gbps": moved / sec / 1e9, "link_frac": moved / sec / 1e9 / probe["h2d_copy_gbps"],
                   "bytes_filter": st["bytes_filter"], "bytes_compact": st["bytes_compact"],
                   "bytes_zerocopy": st["bytes_zerocopy"], "bytes_resident_fill": st["bytes_resident_fill"],
                   "nres": st["nres"], "npart": st["npart"],
                   "engine_partition_iters": dict(zip(hy.ENGINE_NAMES, st["part_iters"]))}
            table[f"{mode}/{a}"] = row
            log(f"{mode:11s} {a:9s} {row['ms']:9.1f} ms [{times[0]:.1f}, {times[-1]:.1f}]  {row['gteps']:6.2f} GTEPS  "
                f"link {row['link_gbps']:5.1f} GB/s "
                f"({row['link_frac'] * 100:4.1f}%)  iters {r.iterations}")
    hyb = [v for k, v in table.items() if k.startswith("hybrid/") and "ms" in v]
    tot_ms = sum(v["ms"] for v in hyb)
    value = sum(work[k.split("/")[1]] for k, v in table.items() if k.startswith("hybrid/") and "ms" in v) / (tot_ms / 1e3) / 1e9 if hyb else None
    out = {
        "metric": "GTEPS for BFS/SSSP/CC/PR at capped HBM budget; host-link GB/s vs peak",
        "value": value, "unit": "GTEPS", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": tot_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 (BFS/SSSP/CC), f32 (PageRank)", "data": "synthetic, seeded",
        "config": {"workload": (f"{gname}-budget{args.budget_bytes / 1e9:g}GB-modes" if args.budget_bytes
                                else f"{gname}-budget{args.budget_frac:g}-modes")
                               + ("-rqdistinct" if args.rq_distinct else ""), "n": len(deg), "m": m_directed,
                   "m_sym": m_sym, "source": s, "gamma": list(gamma)},
        "modes": table, "probe": probe,
    }
    print(json.dumps(out), flush=True)


def multigraph_workload(args):
    """--graphs seeded R-MAT graphs of uneven size (scales 16..22), device-resident: CC on
    their symmetrized forms and 20-step PageRank, once as one traversal over the disjoint
    union (hytm_graph_set_parts) and once graph by graph.  GTEPS counts m_sym per CC run
    and 20 m per PageRank run."""
    rng = np.random.default_rng(3200)
    scales = sorted(int(x) for x in rng.integers(16, 23, size=args.graphs))
    t0 = time.time()
    directed = [gen.rmat(s, args.edge_factor, seed=3300 + i) for i, s in enumerate(scales)]
    sym = [gen.symmetrize(o, c) for o, c in directed]
    off, col, _, b = gen.disjoint_union(directed)
    soff, scol, _, sb = gen.disjoint_union(sym)
    log(f"{args.graphs} graphs, scales {scales}, union n={len(off) - 1} m={len(col)} m_sym={len(scol)}, "
        f"gen {time.time() - t0:.1f}s")
    work = 20 * len(col) + len(scol)
    u = hy.Graph(off, col, check_col=False)
    us = hy.Graph(soff, scol, symmetric=True, check_col=False)
    u.set_parts(b)
    us.set_parts(sb)
    singles = [(hy.Graph(o, c, check_col=False), hy.Graph(so, sc, symmetric=True, check_col=False))
               for (o, c), (so, sc) in zip(directed, sym)]
    u_out = hy.pinned_empty(len(off) - 1, np.float32)
    us_out = hy.pinned_empty(len(soff) - 1, np.uint32)
    big = max(len(o) - 1 for o, _ in directed)
    s_pr, s_cc = hy.pinned_empty(big, np.float32), hy.pinned_empty(big, np.uint32)

    def union_step():
        u.run("pagerank", out=u_out)
        us.run("cc", out=us_out)

    def single_step():
        for gd, gsym in singles:
            gd.run("pagerank", out=s_pr[: gd.n])
            gsym.run("cc", out=s_cc[: gsym.n])

    res = {}
    for name, fn in (("union", union_step), ("one_by_one", single_step)):
        for _ in range(args.warmup):
            fn()
        sync()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        sync()
        sec = (time.perf_counter() - t) / args.steps
        res[name] = {"ms": sec * 1e3, "gteps": work / sec / 1e9}
        log(f"{name}: {sec * 1e3:.1f} ms per CC+PR pass over all graphs")
    out = {
        "metric": f"GTEPS of CC + PageRank over {args.graphs} uneven R-MAT graphs in one traversal vs one by one",
        "value": res["union"]["gteps"], "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["union"]["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 (CC), f32 (PageRank)", "data": "synthetic R-MAT, seeded",
        "config": {"workload": f"multigraph-{args.graphs}-rmat16to22-resident", "scales": scales,
                   "n": len(off) - 1, "m": len(col), "m_sym": len(scol)},
        "multigraph": res, "speedup": res["one_by_one"]["ms"] / res["union"]["ms"],
    }
    print(json.dumps(out), flush=True)


def serve_workload(args, g, off, gamma, probe):
    """A seeded trace of Poisson arrivals (mean rate --qps) carrying 50% BFS, 30% SSSP and
    20% personalized PageRank (10 steps, restart 0.15) queries.  The server run submits
    each query at its arrival time and measures submit-to-result latency inside the
    library.  The one-at-a-time reference runs the same queries back to back through
    hytm_run and replays the trace through a single FIFO server with those service times.
    --budget-bytes sets the edge budget, else --budget-frac of SSSP's edge bytes; --budget-frac < 0
    keeps the graph device-resident."""
    n = len(off) - 1
    rng = np.random.default_rng(6000 + args.scale)
    kinds = rng.choice(["bfs", "sssp", "ppr"], size=args.queries, p=[0.5, 0.3, 0.2])
    srcs = gen.sources(off, args.queries, 6100 + args.scale)
    arrivals = np.cumsum(rng.exponential(1.0 / args.qps, size=args.queries))
    if args.budget_bytes:
        g.set_budget(int(args.budget_bytes))
    elif args.budget_frac >= 0:
        g.set_budget(int(args.budget_frac * g.edge_bytes("sssp") * g.m))  # planned for SSSP's edge bytes
    outs = {k: hy.pinned_empty(n, np.float32 if k == "ppr" else np.uint32) for k in ("bfs", "sssp", "ppr")}
    for k in ("bfs", "sssp", "ppr"):
        g.run(k, int(srcs[0]), out=outs[k])  # warm-up: buffers and resident cache
    service = []
    for k, s in zip(kinds, srcs):
        t = time.perf_counter()
        g.run(str(k), int(s), out=outs[str(k)])
        service.append(time.perf_counter() - t)
    finish, seq_lat = 0.0, []
    for a, sv in zip(arrivals, service):
        finish = max(finish, a) + sv
        seq_lat.append(finish - a)
    seq_span = finish - arrivals[0]
    log(f"one at a time: service p50 {np.percentile(service, 50) * 1e3:.1f} ms, busy {sum(service):.2f}s "
        f"for a {arrivals[-1]:.2f}s trace")

    lanes = min(64, args.lanes)
    # result buffers per kind: enough for every query of the kind in flight or queued, up to
    # 2 x lanes; latency counts from the scheduled arrival, so a submit held back by a
    # missing buffer is charged to the server
    # (pinned result memory is capped at about 16 GB in all)
    per_kind = max(4, int(16e9 // (3 * 4 * max(n, 1))))
    bufs = {k: [hy.pinned_empty(n, np.float32 if k == "ppr" else np.uint32)
                for _ in range(min(2 * lanes, per_kind, int((kinds == k).sum()) or 1))] for k in ("bfs", "sssp", "ppr")}
    with hy.Server(g, bfs=lanes, sssp=lanes, ppr=lanes) as srv:
        warm = [srv.submit(k, int(srcs[0])) for k in ("bfs", "sssp", "ppr")]
        for q in warm:
            srv.wait(q)
        subs = []
        free = {k: list(range(len(bufs[k]))) for k in bufs}
        t0 = time.perf_counter()
        pending = []
        for i, (k, s) in enumerate(zip(kinds, srcs)):
            k = str(k)
            while time.perf_counter() - t0 < arrivals[i] - arrivals[0]:
                time.sleep(0.0002)
            if not free[k]:  # every buffer of this kind is busy: wait for the oldest query of the kind
                j = next(x for x in range(len(pending)) if pending[x][1] == k)
                q, _, b, lag = pending.pop(j)
                srv.wait(q)
                subs.append((q.result, lag))
                free[k].append(b)
            b = free[k].pop()
            lag = (time.perf_counter() - t0 - (arrivals[i] - arrivals[0])) * 1e3
            pending.append((srv.submit(k, int(s), out=bufs[k][b]), k, b, lag))
        for q, k, b, lag in pending:
            srv.wait(q)
            subs.append((q.result, lag))
        span = time.perf_counter() - t0
    lat = np.array([r["total_ms"] + lag for r, lag in subs])
    subs = [r for r, _ in subs]
    seq = np.array(seq_lat) * 1e3
    res = {
        "server": {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                   "qps": args.queries / span, "queue_p99_ms": float(np.percentile([r["queue_ms"] for r in subs], 99))},
        "one_at_a_time": {"p50_ms": float(np.percentile(seq, 50)), "p99_ms": float(np.percentile(seq, 99)),
                          "qps": args.queries / seq_span, "service_p50_ms": float(np.percentile(service, 50)) * 1e3},
    }
    log(json.dumps(res))
    out = {
        "metric": f"serving p99 latency, Poisson arrivals at {args.qps:g} QPS, 50/30/20 BFS/SSSP/PPR",
        "value": res["server"]["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": args.queries, "warmup": 3,
        "ms_per_step": span * 1e3 / args.queries, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32+f32", "data": "synthetic R-MAT, seeded arrivals",
        "config": {"workload": f"rmat{args.scale}-serve-{args.qps:g}qps"
                               + (f"-budget{args.budget_bytes / 1e9:g}GB" if args.budget_bytes else ""),
                   "n": n, "m": int(g.m), "lanes": lanes, "budget_frac": args.budget_frac,
                   "budget_bytes": args.budget_bytes, "gamma": list(gamma)},
        "serve": res, "probe": probe,
    }
    print(json.dumps(out), flush=True)


def gamma_from(spec, probe):
    """RTTzc = gamma*RTT + (1-gamma)*ratio*RTT prices a zero-copy request as a fixed part
    plus a part proportional to its payload.  From the probe, a line read for a fraction f
    of its bytes takes time proportional to f*U(1)/U(f) (U = useful GB/s); solving
    gamma + (1-gamma)*f = f*U(1)/U(f) at f = 1/4 and 1/2 and averaging gives gamma."""
    if spec == "paper":
        return (5, 8)
    if spec != "probe":
        a, b = spec.split("/")
        return (int(a), int(b))
    u = probe["zc_read_gbps"]
    est = []
    for f, key in ((0.25, "32B"), (0.5, "64B")):
        t = f * u["128B"] / u[key]
        est.append((t - f) / (1 - f))
    gam = min(1.0, max(0.0, sum(est) / len(est)))
    return (int(round(gam * 64)), 64)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(off, col, w, soff, scol, srcs, algos, large=False):
    """The oracle, single-threaded, on a bounded sample of the step: BFS and SSSP from the
    first source, CC on the symmetrized graph and 2 PageRank iterations; on graphs above
    2^26 vertices (about 10-40 s per algorithm there) BFS from the first source only.  It
    runs in a thread pinned to one core (the last one this process may use) before the
    process makes any GPU call; the rest of the process keeps its own affinity."""
    import threading

    import oracle
    deg = np.diff(off).astype(np.int64)
    m = len(col)
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    res = {}

    def work():
        os.sched_setaffinity(0, {core})  # this thread only
        res["affinity"] = sorted(os.sched_getaffinity(0))
        edges, secs, parts = 0, 0.0, []
        s = int(srcs[0])
        if "bfs" in algos:
            t = time.perf_counter()
            lvl, _ = oracle.bfs(off, col, s)
            secs += time.perf_counter() - t
            edges += int(deg[lvl != hy.UNREACHED].sum())
            parts.append("bfs(src0)")
        if "sssp" in algos and not large:
            t = time.perf_counter()
            d = oracle.sssp(off, col, w, s)
            secs += time.perf_counter() - t
            edges += int(deg[d != hy.UNREACHED].sum())
            parts.append("sssp(src0)")
        if "cc" in algos and soff is not None and not large:
            t = time.perf_counter()
            oracle.cc(soff, scol)
            secs += time.perf_counter() - t
            edges += len(scol)
            parts.append("cc")
        if "pagerank" in algos and not large:
            t = time.perf_counter()
            oracle.pagerank(off, col, 0.85, 2)
            secs += time.perf_counter() - t
            edges += 2 * m
            parts.append("pagerank(2 iterations)")
        res.update(edges=edges, secs=secs, parts=parts)

    th = threading.Thread(target=work)
    th.start()
    th.join()
    edges, secs = res["edges"], res["secs"]
    log(f"cpu oracle: {edges} edges in {secs:.1f}s on core {res['affinity']}")
    return {"value": edges / secs / 1e9 if secs else None, "unit": "GTEPS", "cores": len(res["affinity"]),
            "kind": "oracle",
            "sample": " + ".join(res["parts"]) + " on the same graph, single thread pinned to one core",
            "seconds": secs, "core": res["affinity"], "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "cores_allowed": len(allowed)}


if __name__ == "__main__":
    main()
