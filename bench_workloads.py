"""The non-default measurements of bench.py: implicit inference and
execution (--workload implicit), 4096 independent graphs in one launch
(batch) and the serving replay (serving).  Each returns one
JSON-serialisable record."""
from __future__ import annotations

import sys
import threading
import time

import numpy as np

from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl

METRIC = "tasks/sec + per-task overhead (ns) + min effective task granularity, 1 GPU"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _base(value, ms, steps, warmup, config, **extra):
    return {"metric": METRIC, "value": value, "unit": "tasks/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
            "data": "synthetic", "config": config, **extra}


def run_implicit(args, stream):
    """2^16 tasks over 2^24 elements in 1024 subregions, halos 1..64, R = 64:
    device inference (timed), then execution."""
    ig = wl.halo_graph(1024, 16384, 64, seed=0, rounds=64)
    t0 = time.perf_counter()
    g = tg.graph_from_implicit(ig)
    host_s = time.perf_counter() - t0
    tm = tg.tg_graph_timings(g.handle)
    E = tg.tg_graph_num_edges(g.handle)
    log(f"implicit: inferred {E} edges, inference {tm['infer_ms']:.2f} ms, compile {tm['compile_ms']:.1f} ms")
    cfg, ms = tg.tg_graph_autotune(g.handle, reps=1)
    log(f"implicit: tuned {cfg} {ms:.2f} ms")
    for _ in range(args.warmup):
        tg.tg_graph_execute(g.handle, None, stream)
    tg.tg_graph_wait(g.handle)
    for _ in range(args.steps):
        tg.tg_graph_execute(g.handle, None, stream)
    kt = tg.tg_graph_kernel_times(g.handle, args.steps)
    ms = float(np.mean(kt))
    word_rounds = 64 * 16384 * 64 * 1024
    # the same program on its two-hop-reduced DAG (the exact transitive
    # reduction here): fewer counter decrements, identical results
    t1 = time.perf_counter()
    removed = tg.tg_graph_reduce_edges(g.handle)
    reduce_ms = (time.perf_counter() - t1) * 1e3
    rcfg, _ = tg.tg_graph_autotune(g.handle, reps=1)
    for _ in range(args.warmup):
        tg.tg_graph_execute(g.handle, None, stream)
    tg.tg_graph_wait(g.handle)
    for _ in range(args.steps):
        tg.tg_graph_execute(g.handle, None, stream)
    rms = float(np.mean(tg.tg_graph_kernel_times(g.handle, args.steps)))
    log(f"implicit: reduced DAG {E - removed} edges ({reduce_ms:.0f} ms host), {rms:.2f} ms ({rcfg})")
    return _base(ig.N / (ms * 1e-3), ms, args.steps, args.warmup,
                 {"workload": "implicit halo program: 65536 tasks, 2^24 u32 in 1024 subregions, halos 1..64, R=64",
                  "launch": cfg},
                 inferred_edges=E, edges_expected=6254592, infer_ms=tm["infer_ms"], compile_ms=tm["compile_ms"],
                 host_build_s=host_s, word_rounds_per_s=word_rounds / (ms * 1e-3),
                 reduced={"edges": E - removed, "reduce_ms": reduce_ms, "ms": rms, "launch": rcfg})


def run_batch(args, stream):
    """4096 independent graphs (frozen manifest) in one persistent launch, vs
    the same graphs launched one after another."""
    import oracle
    specs = wl.batch_manifest(args.graphs, seed=0)
    t0 = time.perf_counter()
    egs, gs = [], []
    for i, sp in enumerate(specs):
        eg = wl.pattern_graph(sp.pattern, sp.W, sp.T, seed=sp.seed, n=sp.n, rounds=sp.rounds)
        egs.append(eg)
        gs.append(tg.graph_from_explicit(eg))
        if i % 512 == 0:
            log(f"batch: built {i} graphs, {time.perf_counter() - t0:.0f} s")
    N = sum(eg.N for eg in egs)
    U = sum(eg.N * eg.n * eg.rounds for eg in egs)
    log(f"batch: {len(gs)} graphs, {N} tasks, {U:.3e} word-rounds; host build {time.perf_counter() - t0:.0f} s")
    # launch shape and schedule: autotuned on a seeded sample of 256 graphs
    # (re-planning the full batch for every candidate would take minutes)
    tune = None
    if not args.no_tune:
        rng = np.random.default_rng(7)
        sub = rng.choice(len(gs), size=min(256, len(gs)), replace=False)
        bs = tg.tg_batch_create([gs[i].handle for i in sub])
        tune, tms = tg.tg_batch_autotune(bs, reps=1)
        tg.tg_batch_destroy(bs)
        log(f"batch: autotuned on {len(sub)} graphs: {tune} ({tms:.1f} ms)")
    cfg = None if tune is None else tg.make_config(
        mapping=tune["mapping"], workers=tune["workers"], wg_waves=tune["wg_waves"], notify=tune["notify"],
        gang=tune.get("gang", 0),
        schedule=tune["schedule"])
    t1 = time.perf_counter()
    b = tg.tg_batch_create([g.handle for g in gs], cfg)
    layout_s = time.perf_counter() - t1
    bcfg, _, btimes = tg.tg_batch_info(b, with_times=True)
    log(f"batch: layout {layout_s:.1f} s ({btimes}), launch {bcfg}")
    for _ in range(args.warmup):
        tg.tg_batch_execute(b, stream)
    tg.tg_batch_wait(b)
    for _ in range(args.steps):
        tg.tg_batch_execute(b, stream)
    kt = tg.tg_batch_kernel_times(b, args.steps)
    ms = float(np.mean(kt))
    log(f"batch: batched {ms:.1f} ms")
    # parity on the 16 cheapest graphs (oracle, bit-exact digests)
    order = np.argsort([eg.N * eg.n * max(eg.rounds, 1) for eg in egs])[:16]
    parity = True
    for i in order:
        eg = egs[i]
        ref = oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, eg.rounds, seed=eg.seed, want_payload=False)
        parity &= bool(np.array_equal(tg.tg_graph_read_digests(gs[i].handle), ref["digest"]))
    # the same graphs launched one after another (a seeded sample of 256)
    rng = np.random.default_rng(0)
    sample = rng.choice(len(gs), size=min(256, len(gs)), replace=False)
    tg.tg_batch_destroy(b)
    seq_ms, seq_tasks = 0.0, 0
    for i in sample:
        tg.tg_graph_execute(gs[i].handle, None, stream)
        tg.tg_graph_wait(gs[i].handle)
        tg.tg_graph_execute(gs[i].handle, None, stream)
        seq_ms += float(tg.tg_graph_kernel_times(gs[i].handle, 1)[0])
        seq_tasks += egs[i].N
    return _base(N / (ms * 1e-3), ms, args.steps, args.warmup,
                 {"workload": f"{len(gs)} independent graphs: W~U[8,512], T~U[8,256], five patterns, "
                              "n~U{64..1024}, R~LogNormal(ln 64, 1); one persistent launch", "launch": bcfg},
                 tasks=N, word_rounds=U, word_rounds_per_s=U / (ms * 1e-3), layout_s=layout_s,
                 layout_ms=btimes, tuned_on_sample=tune,
                 parity_16_graphs=parity,
                 one_launch_per_graph={"sample_graphs": len(sample), "tasks": seq_tasks,
                                       "tasks_per_s": seq_tasks / (seq_ms * 1e-3)})


def run_serving(args, stream):
    """Poisson stream of graph submissions (frozen manifest) replayed in real
    time into the continuous-batching server; latency p50/p99 and sustained
    tasks/s."""
    import oracle
    warm = max(args.requests // 10, 1)
    reqs = wl.serving_manifest(warm + args.requests, rate=args.rate, seed=0)
    t0 = time.perf_counter()
    graphs, handles = [], []
    for i, r in enumerate(reqs):
        x = wl.build_request(r)
        graphs.append(x)
        handles.append(tg.graph_from_implicit(x) if isinstance(x, wl.ImplicitGraph) else tg.graph_from_explicit(x))
        if i % 1000 == 0:
            log(f"serving: built {i} requests, {time.perf_counter() - t0:.0f} s")
    srv = tg.tg_server_create(64 << 30, slots=args.slots, max_batch=64)
    tickets = [None] * len(reqs)

    def client():
        start = time.perf_counter()
        for i, r in enumerate(reqs):
            dt = r.arrival_s - (time.perf_counter() - start)
            if dt > 0:
                time.sleep(dt)
            tickets[i] = tg.tg_server_submit(srv, handles[i].handle)

    th = threading.Thread(target=client)
    th.start()
    th.join()
    lat, done = [], []
    for i, t in enumerate(tickets):
        s_ns, a_ns, d_ns = tg.tg_server_wait(srv, t)
        if i >= warm:
            lat.append((d_ns - s_ns) * 1e-6)
            done.append((s_ns, d_ns, graphs[i].N))
    stats = tg.tg_server_stats(srv)
    tg.tg_server_destroy(srv)
    first = min(x[0] for x in done)
    last = max(x[1] for x in done)
    tasks = sum(x[2] for x in done)
    span_s = (last - first) * 1e-9
    lat = np.array(lat)
    # parity on a sample of requests
    rng = np.random.default_rng(1)
    parity = True
    for i in rng.choice(len(reqs), size=32, replace=False):
        x = graphs[i]
        if isinstance(x, wl.ImplicitGraph):
            ref = oracle.implicit_program_order(x.N, x.req_ptr, x.lo, x.hi, x.priv, x.rounds, x.space, seed=x.seed)
        else:
            ref = oracle.exec_explicit(x.N, x.n, x.pred_ptr, x.preds, x.rounds, seed=x.seed, want_payload=False)
        parity &= bool(np.array_equal(tg.tg_graph_read_digests(handles[i].handle), ref["digest"]))
    return _base(tasks / span_s, span_s * 1e3, len(lat), warm,
                 {"workload": f"serving: Poisson {args.rate:.0f} req/s, sizes LogNormal(median 4096, sigma 1) in "
                              f"[64, 2^20], explicit/implicit 1:1, 64 GB budget, {args.slots} launch slots"},
                 latency_ms={"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "max": float(lat.max())},
                 offered_req_per_s=args.rate, server=stats, parity_32_requests=parity)
