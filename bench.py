"""Throughput benchmark: edges featurized per second on one MI355X.

One step = build the device graph store from the edge list already resident
in HBM, then mine every pattern column (FAN_OUT, FAN_IN, SG_k, GS_k,
CYC_2..CYC_L) for every edge.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges/sec featurized (all patterns, exact) learned vs static sched; p99 stream lat"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (generator, kwargs, delta, L, k)
    "large": ("large", {"seed": 404}, 86400, 6, 2),
    "mid": ("mid", {"seed": 202}, 86400, 6, 2),
    "tiny": ("tiny", {"seed": 101}, 86400, 4, 3),
    # a 5M-edge graph of a seed the cost model is not trained on (202..205)
    "mid_heldout": ("mid", {"seed": 206}, 86400, 6, 2),
}


MINING_SOURCES = ("mine.hip", "mine.h", "common.h", "internal.h")
# the mining stages (HIP event times) after the graph build; "mine" spans them
# all, first mining kernel to last (the cycle kernel overlaps other stages)
MINE_STAGES = ("anchor", "lists", "model", "units", "sg", "cyc")


def mining_source_sha1():
    """sha1 (12 hex digits) over the sources the mining kernels are built
    from, in the order of MINING_SOURCES."""
    import hashlib
    h = hashlib.sha1()
    for name in MINING_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_12241_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def recorded_traffic(kernel):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3
    summary, or None if the mining sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_large32M.json")
    try:
        rec = json.load(open(path))
        sha = mining_source_sha1()
    except (OSError, ValueError):
        return None
    if rec.get("mining_sources_sha1") != sha:
        return None
    return rec.get("traffic_bytes_per_dispatch", {}).get(kernel)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2604_12241_amd import workloads as W
    gen, kw, delta, L, k = WORKLOADS[name]
    t0 = time.time()
    g = getattr(W, gen)(**kw)
    log(f"[bench] generated {name}: {g.n_edges} edges, {g.n_vertices} accounts in {time.time() - t0:.1f}s")
    return g, delta, L, k


def train_cost_model(delta, L, k, n_graphs=4, cache=None):
    """Cost model trained (untimed) on graphs of the 5M-edge generator
    (seeds 202..), labels from the plain miner's work counters."""
    import paper_2604_12241_amd as A
    from paper_2604_12241_amd import workloads as W
    if cache and os.path.exists(cache):
        A.amlm_costmodel_load(cache)
        log(f"[bench] cost model loaded from {cache}")
        return
    t0 = time.time()
    Gs = []
    for i in range(n_graphs):
        g = W.mid(202 + i)
        Gs.append(A.Graph(g.src, g.dst, g.ts, g.n_vertices))
    A.amlm_costmodel_train(Gs, [A.params(A.AMLM_ALL, delta, L, k)] * n_graphs, epochs=4, batch=4096, seed=1)
    for G in Gs:
        G.close()
    log(f"[bench] cost model trained on {n_graphs} graphs of 5M edges in {time.time() - t0:.1f}s")
    if cache:
        A.amlm_costmodel_save(cache)


def _stream_source(g, n_pool, seed=505):
    """Endless stream after the end of g: a pool of generated batches
    (log-uniform 1e3..1e5 edges, the graph's account activity) replayed with
    their timestamps shifted past everything before."""
    from paper_2604_12241_amd import workloads as W
    pool = W.stream_batches(g, seed=seed, n_batches=n_pool)
    t_first = int(pool[0].ts.min())
    span = int(pool[-1].ts.max()) - t_first + 1
    rep = 0
    while True:
        for b in pool:
            yield b.src, b.dst, b.ts + rep * span, b.n_edges
        rep += 1


def bench_serving(A, G, g, p, n_batches=6100, skip=100, slots=4, n_pool=300, inflight=64, loads=(0.5, 0.8)):
    """Config-5 style serving: the graph resident, stream batches of 1k-100k
    edges (log-uniform) strictly after its end.  A saturation run (every
    batch queued as fast as the server takes it) gives the sustained rate;
    then Poisson arrivals at 50 % and 80 % of it, n_batches each, give the
    p50 / p99 batch latency (submit -> results ready) over all but the first
    `skip` batches of each load."""
    t0 = time.time()
    src = _stream_source(g, n_pool)
    log(f"[bench] generated a pool of {n_pool} stream batches in {time.time() - t0:.1f}s")
    S = A.Server(G, p, hbm_budget=0, max_slots=slots)
    for _ in range(8):                       # warm the slots
        a, b, c, _ = next(src)
        S.wait(S.submit(a, b, c, wait=True))
    # saturation: batches queued as fast as the server accepts them
    n_sat = n_batches // 2
    t_a = time.perf_counter()
    tk, done, edges = [], 0, 0
    for _ in range(n_sat):
        a, b, c, n = next(src)
        tk.append(S.submit(a, b, c, wait=True))
        edges += n
        while len(tk) - done > inflight:     # keep the results flowing
            S.wait(tk[done])
            done += 1
    for t in tk[done:]:
        S.wait(t)
    t_b = time.perf_counter()
    sustained = edges / (t_b - t_a)
    log(f"[bench] serving saturation: {n_sat} batches, {sustained / 1e6:.1f} M edges/s")
    mean_edges = edges / n_sat
    rng = np.random.default_rng(7)
    res = {"sustained_edges_per_s": sustained, "saturation_batches": n_sat, "slots": slots,
           "batches_per_load": n_batches, "latency_excludes_first": skip,
           "batch_edges": "log-uniform 1e3..1e5"}
    for frac in loads:
        rate = frac * sustained / mean_edges          # batches per second
        gaps = rng.exponential(1.0 / rate, n_batches)
        tk = []
        lat = []
        due = time.perf_counter()
        for gap in gaps:
            due += gap
            a, b, c, _ = next(src)
            while time.perf_counter() < due:
                time.sleep(min(0.0002, max(0.0, due - time.perf_counter())))
            tk.append(S.submit(a, b, c, wait=True))
            while len(tk) - len(lat) > inflight:
                t = tk[len(lat)]
                S.wait(t)
                x, _, z = S.times(t)
                lat.append((z - x) * 1e3)
        for t in tk[len(lat):]:
            S.wait(t)
            x, _, z = S.times(t)
            lat.append((z - x) * 1e3)
        lat = lat[skip:]
        res[f"load_{int(frac * 100)}"] = {"p50_ms": float(np.percentile(lat, 50)),
                                          "p99_ms": float(np.percentile(lat, 99)),
                                          "max_ms": float(np.max(lat)),
                                          "offered_edges_per_s": frac * sustained, "batches_timed": len(lat)}
        log(f"[bench] serving at {int(frac * 100)}%: p50 {res[f'load_{int(frac * 100)}']['p50_ms']:.2f} ms, "
            f"p99 {res[f'load_{int(frac * 100)}']['p99_ms']:.2f} ms")
    res["window_store"] = S.stats()
    S.close()
    return res


def bench_batching(A, n_graphs=256, steps=5):
    """Config-3 style batching: 256 independent graphs of 1k-200k edges
    (log-uniform), windows of 6 h / 24 h / 72 h, in one batched store mined by
    one captured launch; chunk / grid autotuned (cached per device)."""
    import torch
    from paper_2604_12241_amd import workloads as W
    t0 = time.time()
    subs = W.batch_subgraphs(n_graphs)
    log(f"[bench] generated {n_graphs} sub-graphs ({sum(g.n_edges for g, _ in subs)} edges) in "
        f"{time.time() - t0:.1f}s")
    B = A.Batch([(g.src, g.dst, g.ts, g.n_vertices) for g, _ in subs])
    ps = [A.params(A.AMLM_ALL, d, 6, 2) for _, d in subs]
    outs = [torch.empty((A.amlm_num_columns(q), int(B.sizes[i])), dtype=torch.int32, device="cuda")
            for i, q in enumerate(ps)]
    chosen = A.amlm_autotune(B, ps, outs, os.path.join(os.environ.get("TMPDIR", "/tmp"), "amlm_autotune.json"))
    A.amlm_mine_batch(B, ps, outs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        A.amlm_mine_batch(B, ps, outs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / steps
    E = B.n_edges
    n, captures = B.info_batch()
    B.close()
    return {"edges_per_s": E / dt, "ms_per_launch": dt * 1e3, "graphs": n, "edges": E,
            "autotuned": {"chunk": chosen[0], "sg_blocks": chosen[1], "cyc_blocks": chosen[2]},
            "hipgraph_captures": captures}


def bench_variants(A, g, reps=3):
    """The paper's variants on a 5M-edge graph: the pattern modifiers (whole
    mining) and the stage-cell interpreter on patterns the fixed kernels
    also compute (same counts checked), each timed with HIP events."""
    import torch
    PROGS = {
        # cells: (op, node, peer, tlo, tref, thi, skip, distinct, agg, threshold)
        "fan_out": [(A.AMLM_CELL_FOR_OUT, A.VAR_U, 0, A.AMLM_T_WINDOW, 0, A.AMLM_T_THROUGH, (), False,
                     A.AMLM_AGG_SUM, 0)],
        "sg": [(A.AMLM_CELL_FOR_IN, A.VAR_U, 0, A.AMLM_T_WINDOW, 0, A.AMLM_T_BEFORE, (A.VAR_V,), True,
                A.AMLM_AGG_AT_LEAST_K, 0),
               (A.AMLM_CELL_FOR_OUT, 2, 0, A.AMLM_T_WINDOW, 0, A.AMLM_T_BEFORE, (), True, A.AMLM_AGG_AT_LEAST, 1),
               (A.AMLM_CELL_PROBE, 3, A.VAR_V, A.AMLM_T_AFTER, 1, A.AMLM_T_THROUGH, (), False, A.AMLM_AGG_SUM, 0)],
    }
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    E = g.n_edges

    def tm(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    res = {"graph": f"{E} edges, {g.n_vertices} accounts, delta=86400s (5M-edge generator, seed 206)"}
    mods = (("default", A.AMLM_ALL, 6, 2), ("sg_unordered", A.AMLM_ALL | A.AMLM_SG_UNORDERED, 6, 2),
            ("sg_phase", A.AMLM_ALL | A.AMLM_SG_PHASE, 6, 2),
            ("deg_columns", A.AMLM_ALL | A.AMLM_DEG_OUT | A.AMLM_DEG_IN, 6, 2),
            ("participation", A.AMLM_ALL | A.AMLM_PART, 6, 2),
            ("cycles_L4", A.AMLM_CYCLES, 4, 2), ("cycles_any_order_L4", A.AMLM_CYCLES | A.AMLM_CYC_ANY_ORDER, 4, 2))
    for name, pat, L, k in mods:
        p = A.params(pat, 86400, L, k)
        out = torch.empty((A.amlm_num_columns(p), E), dtype=torch.int32, device="cuda")
        ms = tm(lambda: A.amlm_mine(G, p, out))
        res[name] = {"ms": ms, "edges_per_s": E / (ms * 1e-3), "L": L, "k": k}
    fixed = A.amlm_mine(G, A.params(A.AMLM_FAN_OUT | A.AMLM_SG, 86400, 2, 2))
    for (name, cells), col in zip(PROGS.items(), (0, 1)):
        cc = [A.cell(*c) for c in cells]
        out = torch.empty(E, dtype=torch.int32, device="cuda")
        ms = tm(lambda: A.amlm_mine_program(G, cc, 86400, 2, out))
        p1 = A.params(A.AMLM_FAN_OUT if name == "fan_out" else A.AMLM_SG, 86400, 2, 2)
        o1 = torch.empty((1, E), dtype=torch.int32, device="cuda")
        ms_fixed = tm(lambda: A.amlm_mine(G, p1, o1))
        res[f"program_{name}"] = {"ms": ms, "fixed_kernel_ms": ms_fixed,
                                  "identical_to_fixed": bool(torch.equal(out, fixed[col]))}
    A.amlm_graph_sync(G)
    G.close()
    return res


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def oracle_full(g, delta, L, k, unordered=False, procs=None):
    """The oracle (plain single-threaded C) over the whole graph, as `procs`
    processes on disjoint anchor ranges; returns its counts and the
    cpu_baseline record.  Runs before anything touches the GPU (the workers
    are forked)."""
    import oracle
    from oracle.parallel import default_procs, mine_parallel
    procs = procs or default_procs()
    pats = oracle.ALL | (oracle.SG_UNORDERED if unordered else 0)
    t0 = time.perf_counter()
    counts, info = mine_parallel(g.src, g.dst, g.ts, g.n_vertices, pats, delta, L, k, procs=procs,
                                 progress=lambda lo, hi, s: log(f"[bench] oracle anchors [{lo}, {hi}) done in {s:.1f} s"))
    wall = time.perf_counter() - t0
    n = g.n_edges
    loop = max(info["loop_s"])
    per_core = float(np.mean([(hi - lo) / s for (lo, hi), s in zip(info["ranges"], info["loop_s"]) if s > 0]))
    rec = {"value": n / loop, "unit": "edges/s", "cores": procs, "kind": "oracle",
           "sample": f"all {n} anchors in {procs} processes over disjoint edge-id ranges; value = edges / "
                     f"slowest process's anchor loop ({loop:.1f} s; graph set-up excluded, "
                     f"{wall:.1f} s wall with set-up)",
           "per_core_edges_per_s": per_core, "cpu": cpu_model(), "host_cpus": os.cpu_count()}
    return counts, rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["large", "mid", "tiny"])
    ap.add_argument("--schedule", default="learned", choices=["static", "learned"])
    ap.add_argument("--sg-order", default="ordered", choices=["ordered", "unordered"],
                    help="scatter-gather legs of an intermediate strictly ordered (default) or window-only")
    ap.add_argument("--train-graphs", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle run (and with it the full-graph parity check)")
    ap.add_argument("--oracle-procs", type=int, default=0, help="oracle processes (0: host cores, at most 16)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serve-slots", type=int, default=4, help="server slots (batches mined concurrently)")
    ap.add_argument("--serve-inflight", type=int, default=64, help="batches submitted and not yet collected")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="HIP hardware queues of this process (GPU_MAX_HW_QUEUES, set before the runtime starts): "
                         "the server runs one stream per slot plus its committer's; 0 leaves the environment alone")
    ap.add_argument("--model-cache", default=None, help="load / save the trained cost model here")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: no comparisons, plus a 1 GiB copy of known size")
    ap.add_argument("--profile-serve", type=int, default=0, metavar="N",
                    help="with --profile: then a serving saturation run of N batches (its dispatches "
                         "follow the copy kernel in a trace)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU "
              "time-sharded path is a design, not built", file=sys.stderr)
        sys.exit(2)
    if args.profile:
        args.no_serve = args.no_batch = args.no_cpu_baseline = True
    if args.hw_queues > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)

    g, delta, L, k = make_workload(args.workload)
    gh = make_workload("mid_heldout")[0] if not args.profile else None
    ref = cpu_rec = None
    if not args.no_cpu_baseline:
        # the oracle first: its workers are forked, before this process
        # initialises the GPU
        log("[bench] running the oracle over the whole graph ...")
        ref, cpu_rec = oracle_full(g, delta, L, k, args.sg_order == "unordered", args.oracle_procs or None)
        log(f"[bench] oracle: {cpu_rec['sample']}")

    import torch
    import paper_2604_12241_amd as A

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    src = torch.from_numpy(g.src.view(np.int32)).to(dev)
    dst = torch.from_numpy(g.dst.view(np.int32)).to(dev)
    ts = torch.from_numpy(g.ts).to(dev)
    sched = A.AMLM_SCHED_LEARNED if args.schedule == "learned" else A.AMLM_SCHED_STATIC
    if sched == A.AMLM_SCHED_LEARNED:
        train_cost_model(delta, L, k, args.train_graphs, args.model_cache)
    pats = A.AMLM_ALL | (A.AMLM_SG_UNORDERED if args.sg_order == "unordered" else 0)
    p = A.params(pats, delta, L, k, sched)
    p_static = A.params(pats, delta, L, k, A.AMLM_SCHED_STATIC)
    G = A.Graph(src, dst, ts, g.n_vertices)
    E = g.n_edges
    counts = torch.empty((A.amlm_num_columns(p), E), dtype=torch.int32, device=dev)

    # the method's algorithmic bytes per anchor (untimed accounting run):
    # rows B_io, B_sg/gs, B_cyc
    _, work = A.amlm_mine_work(G, p)
    torch.cuda.synchronize()
    wk = work.cpu().numpy().view(np.uint64)
    b_io, b_sg, b_cyc = (int(wk[r].sum()) for r in range(3))
    del work

    def step(pp=p):
        G.rebuild(src, dst, ts, g.n_vertices)
        A.amlm_mine(G, pp, counts)

    def timed(pp, steps):
        A.amlm_set_timing(G, True)
        stage_ms = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(pp)
            for kname, v in A.amlm_stage_times(G).items():
                stage_ms.setdefault(kname, []).append(v)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        A.amlm_set_timing(G, False)
        A.amlm_graph_sync(G)
        return (t1 - t0) / steps, {kname: float(np.mean(v)) for kname, v in stage_ms.items()}

    for _ in range(args.warmup):
        step()
    A.amlm_graph_sync(G)
    dt, avg = timed(p, args.steps)
    mine_ms = avg.get("mine", 0.0)
    parity = None
    if ref is not None:
        got = counts.cpu().numpy().view(np.uint32)
        bad = (got != ref)
        parity = {"edges": E, "columns": int(got.shape[0]), "mismatches": int(bad.sum()),
                  "mismatches_per_column": [int(x) for x in bad.sum(axis=1)],
                  "against": "oracle over all anchors (cpu_baseline run)"}
        del got, bad
    static = None
    if args.profile:
        # copy probe: 1 GiB read + 1 GiB written by the library's copy kernel
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        A.amlm_copy(b, a)
        torch.cuda.synchronize()
    elif sched == A.AMLM_SCHED_LEARNED:
        # the other schedules on the same graph and clock: static (no
        # slicing), the length rule (slicing without the network) and the
        # true per-anchor costs (headroom only: never shipped)
        check = counts.clone()
        _, wk_l = A.amlm_mine_work(G, p)
        torch.cuda.synchronize()
        true_cost = torch.log1p(wk_l[3].to(torch.float64)).to(torch.float32).contiguous()
        del wk_l
        A.amlm_graph_set_costs(G, true_cost)
        schedules = {}
        for name, sc in (("static", A.AMLM_SCHED_STATIC), ("length_rule", A.AMLM_SCHED_LENGTH),
                         ("oracle_cost", A.AMLM_SCHED_GIVEN)):
            px = A.params(pats, delta, L, k, sc)
            step(px)
            A.amlm_graph_sync(G)
            same = bool(torch.equal(check, counts))
            dtx, avgx = timed(px, args.steps)
            schedules[name] = {"value": E / dtx, "ms_per_step": dtx * 1e3, "stage_ms": avgx,
                               "counts_identical_to_learned": same}
        A.amlm_graph_set_costs(G, None)
        del check, true_cost
        static = schedules["static"]
        schedules["learned"] = {"value": E / dt, "ms_per_step": dt * 1e3, "stage_ms": avg}
        # rank correlation of the predicted against the true scatter-gather
        # bytes, on graphs the model was not trained on
        from scipy.stats import spearmanr
        heldout = {}
        Gh = A.Graph(gh.src, gh.dst, gh.ts, gh.n_vertices)
        for name, GG in (("mid_seed206", Gh), (args.workload, G)):
            pr, lb, wl = A.amlm_costmodel_eval(GG, p)
            heldout[name] = {"anchors": int(pr.shape[0]),
                             "spearman_model": float(spearmanr(pr, lb).correlation),
                             "spearman_window_length": float(spearmanr(wl, lb).correlation)}
        Gh.close()
        schedules["heldout_rank_correlation"] = heldout
        schedules["length_rule_bytes_per_entry"] = A.amlm_costmodel_length_coef()

    # the dominant kernel (k_sg) against the HBM roofline: the method's
    # scatter-gather bytes over its mean event time; and the whole mining
    # (B_io + B_sg/gs + B_cyc) over the summed mining stages
    achieved = b_sg / (avg["sg"] * 1e-3) / 1e9
    traffic = recorded_traffic("k_sg")
    roof = {"kernel": "k_sg", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes": b_sg, "avg_ms": avg["sg"],
            "traffic": traffic,
            "traffic_over_algorithmic": (traffic / b_sg) if traffic and b_sg else None,
            "traffic_source": "profiles/mining_large32M.md (FETCH_SIZE x2.0 + WRITE_SIZE, copy-kernel calibrated)",
            "bytes_definition": "B_sg/gs: sender scan, per distinct sender min(scan to the (k-1)-th other "
                                "intermediate, v's in-window), GS scatter scan; 8 B per element"}
    b_alg = b_io + b_sg + b_cyc
    mining_roof = {"algorithmic_bytes": b_alg, "b_io": b_io, "b_sg_gs": b_sg, "b_cyc": b_cyc,
                   "mine_ms": mine_ms, "achieved": b_alg / (mine_ms * 1e-3) / 1e9 if mine_ms else None,
                   "frac": b_alg / (mine_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if mine_ms else None,
                   "span": "HIP events around the whole mining launch sequence (stage 'mine')"}

    out = {
        "metric": METRIC, "value": E / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {E} edges, {g.n_vertices} accounts, "
                               f"delta={delta}s, L={L}, k={k}", "schedule": args.schedule,
                   "sg_order": args.sg_order, "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
                   "n_edges": E, "n_vertices": g.n_vertices, "delta": delta, "L": L, "k": k},
        "mine_only_edges_per_s": E / (mine_ms * 1e-3) if mine_ms > 0 else None,
        "stage_ms": avg,
        "roofline": roof,
        "mining_roofline": mining_roof,
    }
    if parity is not None:
        out["parity"] = parity
    if static is not None:
        out["static_schedule"] = static
        out["learned_over_static"] = (E / dt) / static["value"]
        out["schedules"] = schedules
        out["learned_over_length_rule"] = (E / dt) / schedules["length_rule"]["value"]
    if not args.no_serve:
        out["stream"] = bench_serving(A, G, g, p, slots=args.serve_slots, inflight=args.serve_inflight)
        out["p99_stream_latency_ms"] = out["stream"]["load_80"]["p99_ms"]
    elif args.profile and args.profile_serve > 0:
        out["stream"] = bench_serving(A, G, g, p, n_batches=2 * args.profile_serve, slots=args.serve_slots,
                                      inflight=args.serve_inflight, loads=())
    if not args.no_batch:
        out["batching"] = bench_batching(A)
    if gh is not None and not args.no_variants:
        log("[bench] variants and stage-cell programs on the 5M-edge graph ...")
        out["variants"] = bench_variants(A, gh)
    if cpu_rec is not None:
        out["cpu_baseline"] = cpu_rec
    print(json.dumps(out), flush=True)
    G.close()


if __name__ == "__main__":
    main()
