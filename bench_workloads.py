"""The configuration legs of bench.py beyond the headline step: the implicit
halo program (inference and execution), 4096 independent graphs in one
launch with their comparators, and the serving replay.  Each leg returns a
JSON-serialisable record; bench.py puts them all on its one output line (and
`--workload implicit|batch|serving` prints one of them alone as a full line).

Parity in these legs is checked against the oracle: stored values written by
a script that calls only the oracle (the halo program), or the oracle run in
parallel worker processes on a seeded sample (batch, serving)."""
from __future__ import annotations

import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl

METRIC = "tasks/sec + per-task overhead (ns) + min effective task granularity, 1 GPU"
ROOT = os.path.dirname(os.path.abspath(__file__))
# integer-VALU peak of the task body from the unit counts: the published
# fp32 vector peak (157.3 TFLOP/s = 256 CUs x 2.4 GHz x 128 lanes x 2 flops
# per fused multiply-add) gives 128 32-bit lanes per clock per CU; the
# compiled mix is 8 VALU instructions per word-round (3 shifts, 3 xors, one
# 32-bit multiply, one add), so 256 x 2.4e9 x 128 / 8 word-rounds/s.  (64
# lanes per clock would give half this, which the measured mix rate exceeds.)
ALU_PEAK_WORD_ROUNDS = 256 * 2.4e9 * 128 / 8


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def base_line(value, ms, steps, warmup, config, **extra):
    return {"metric": METRIC, "value": value, "unit": "tasks/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
            "data": "synthetic", "config": config, **extra}


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


def _timed_graph(g, cfg, stream, warmup, steps):
    for _ in range(max(warmup, 1)):
        tg.tg_graph_execute(g.handle, cfg, stream)
    tg.tg_graph_wait(g.handle)
    for _ in range(steps):
        tg.tg_graph_execute(g.handle, cfg, stream)
    return float(np.mean(tg.tg_graph_kernel_times(g.handle, steps)))


# ------------------------------------------------------------------ alone

def run_alone(args, stream, probes=None):
    """One Task Bench shaped graph alone (1024 x 1000, 256-word payloads,
    0 mix rounds) with the static lists (wavefronts x 1024, level order) or
    the ready queue (wavefronts x 2048, tile 1): for kernel traces and
    counters of one dispatch on one pattern."""
    eg = wl.pattern_graph(args.pattern, 1024, 1000, seed=0, n=256, rounds=0)
    g = tg.graph_from_explicit(eg)
    if args.dispatch == "queue":
        cfg = tg.make_config(mapping=1, workers=2048, dispatch=tg.TG_DISPATCH_QUEUE, tile=1)
    else:
        cfg = tg.make_config(mapping=1, workers=1024, schedule=tg.TG_SCHED_LEVEL)
    ms = _timed_graph(g, cfg, stream, args.warmup, args.steps)
    import oracle
    ref = oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, 0, want_payload=False)
    ok = bool(np.array_equal(tg.tg_graph_read_digests(g.handle), ref["digest"]))
    # edges signalled by a counter atomic in this launch shape (a one-graph
    # batch plans the same layout)
    b = tg.tg_batch_create([g.handle], cfg)
    try:
        signalled = tg.tg_batch_signalled_edges(b)
    finally:
        tg.tg_batch_destroy(b)
    log(f"alone: {signalled} of {eg.E} edges signalled")
    return {"workload": f"{args.pattern} 1024 x 1000 alone, n=256, R=0, {args.dispatch}", "tasks": eg.N,
            "edges": eg.E, "signalled_edges": signalled, "exec_ms": ms, "tasks_per_s": eg.N / (ms * 1e-3),
            "parity": ok, "launch": tg.tg_graph_exec_info(g.handle)[0]}


def oracle_rate(tasks, refs, wall_s, processes):
    """The oracle's throughput on a parity sample: tasks over the summed
    single-process oracle seconds (one core), and over the pool's wall time
    with `processes` worker processes side by side."""
    busy = sum(r[2] for r in refs)
    return {"kind": "oracle", "tasks": int(tasks), "tasks_per_s_one_core": tasks / busy if busy else None,
            "tasks_per_s_pool": tasks / wall_s if wall_s else None, "processes": processes,
            "oracle_s": busy, "wall_s": wall_s}


# ---------------------------------------------------------------- implicit

RETENTION = {"all": tg.TG_KEEP_ALL, "sinks": tg.TG_KEEP_SINKS}


def request_graph(x, retention="sinks", reduce_implicit=True):
    """A graph of the batch or serving workloads in the form the benchmark
    runs it: explicit graphs reuse payload memory once every reader has run
    (keeping the sinks' payloads) unless retention is "all"; implicit graphs
    execute the two-hop reduction of their last-user DAG unless
    reduce_implicit is false (the inferred DAG is kept for reading)."""
    if isinstance(x, wl.ImplicitGraph):
        h = tg.graph_from_implicit(x)
        h.inferred_edges = tg.tg_graph_num_edges(h.handle)
        if reduce_implicit:
            tg.tg_graph_reduce_edges(h.handle)
        return h
    h = tg.graph_from_explicit(x, retention=RETENTION[retention])
    h.inferred_edges = x.E
    return h


def run_implicit(args, stream, probes=None):
    """2^16 tasks over 2^24 elements in 1024 subregions, halos 1..64, R = 64:
    device inference (timed), then execution (autotuned launch shape), on
    the full and on the reduced DAG; every digest and the whole array
    against the oracle's stored values."""
    t0 = time.perf_counter()
    ig = wl.halo_graph(1024, 16384, 64, seed=0, rounds=64)
    # the first inference of a process also allocates the inference's
    # device region (kept for later ones): finalize once to warm up, then
    # time the program's inference on a second graph
    first = tg.tg_graph_timings(tg.graph_from_implicit(ig).handle)["infer_ms"]
    g = tg.graph_from_implicit(ig)
    host_s = time.perf_counter() - t0
    tm = tg.tg_graph_timings(g.handle)
    E = tg.tg_graph_num_edges(g.handle)
    log(f"implicit: inferred {E} edges, inference {tm['infer_ms']:.2f} ms, compile {tm['compile_ms']:.1f} ms")
    with open(os.path.join(ROOT, "tests", "golden", "halo_program_r64.json")) as f:
        gold = json.load(f)

    def parity():
        d = tg.tg_graph_read_digests(g.handle)
        A = tg.tg_graph_read_data(g.handle, 0, ig.space)
        return bool(_sha(d) == gold["digest_sha256"] and _sha(A) == gold["array_sha256"] and
                    f"{tg.tg_graph_checksum(g.handle):#018x}" == gold["checksum"])

    if getattr(args, "no_tune", False):
        # the shape the autotuner picked for this program: 96 gangs of four
        # 16-wave workgroups, column order
        cfg = dict(mapping=3, workers=96, wg_waves=16, schedule=tg.TG_SCHED_COLUMN, gang=4)
        ms = _timed_graph(g, tg.make_config(**cfg), stream, args.warmup, args.steps)
    else:
        cfg, tms = tg.tg_graph_autotune(g.handle, reps=1)
        log(f"implicit: tuned {cfg} {tms:.2f} ms")
        ms = _timed_graph(g, None, stream, args.warmup, args.steps)
    ok = parity()
    word_rounds = 64 * 16384 * 64 * 1024
    t1 = time.perf_counter()
    removed = tg.tg_graph_reduce_edges(g.handle)
    reduce_ms = (time.perf_counter() - t1) * 1e3
    if getattr(args, "no_tune", False):
        rcfg = cfg
        rms = _timed_graph(g, tg.make_config(**rcfg), stream, args.warmup, args.steps)
    else:
        # the reduced DAG has its own best launch shape (a gang signals every
        # executed edge once per member, so fewer edges favour other shapes)
        rcfg, rtms = tg.tg_graph_autotune(g.handle, reps=1)
        log(f"implicit: reduced DAG tuned {rcfg} {rtms:.2f} ms")
        rms = _timed_graph(g, None, stream, args.warmup, args.steps)
    rok = parity()
    log(f"implicit: {ms:.2f} ms (parity {ok}); reduced DAG {E - removed} edges, {rms:.2f} ms (parity {rok})")
    pi = (probes or {}).get("mix_word_rounds_per_s")
    cpu = None
    if "cpu" not in getattr(args, "skipset", set()):
        # the oracle on the program's first sweep (1024 tasks, the same
        # requirements and seed; about 4 s on one core), one thread pinned
        # to one core; its digests must equal the stored first-sweep hash
        import oracle
        ig1 = wl.halo_graph(1024, 16384, 1, seed=0, rounds=64)
        allowed = sorted(os.sched_getaffinity(0))
        old = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {allowed[0]})
        try:
            tc = time.perf_counter()
            r1 = oracle.implicit_program_order(ig1.N, ig1.req_ptr, ig1.lo, ig1.hi, ig1.priv, ig1.rounds, ig1.space,
                                               seed=ig1.seed)
            cs = time.perf_counter() - tc
        finally:
            os.sched_setaffinity(0, old)
        cpu = {"kind": "oracle", "cores": 1, "sample": "the first sweep: 1024 tasks over 2^24 u32, R=64",
               "tasks_per_s": ig1.N / cs, "word_rounds_per_s": 16384 * 64 * ig1.N / cs, "oracle_s": cs,
               "matches_stored_first_sweep": _sha(r1["digest"]) == gold["sweep_digest_sha256"][0]}
        log(f"implicit: oracle first sweep {cs:.1f} s on one core")
    return {
        "workload": "implicit halo program: 65536 tasks, 2^24 u32 in 1024 subregions, halos 1..64, R=64",
        "tasks": ig.N, "inferred_edges": E, "edges_expected": 6254592, "infer_ms": tm["infer_ms"],
        "infer_ms_first_in_process": first,
        "compile_ms": tm["compile_ms"], "host_build_s": host_s, "launch": cfg,
        "exec_ms": ms, "tasks_per_s": ig.N / (ms * 1e-3), "word_rounds_per_s": word_rounds / (ms * 1e-3),
        "frac_of_measured_mix_rate": word_rounds / (ms * 1e-3) / pi if pi else None,
        "frac_of_alu_peak": word_rounds / (ms * 1e-3) / ALU_PEAK_WORD_ROUNDS,
        "parity": {"ok": ok, "against": "oracle program order, stored by tests/golden/make_halo_program_r64.py: "
                                        "checksum, SHA-256 of all 65536 digests and of the 2^24-element array"},
        "reduced": {"edges": E - removed, "reduce_ms": reduce_ms, "launch": rcfg, "exec_ms": rms, "parity": rok},
        "cpu_oracle": cpu,
    }


# ------------------------------------------------------------------ batch

# idle workers back off longer than the default: tasks here run for tens of
# microseconds and more, and an idle wave's polls take issue slots from the
# busy waves on its SIMD (1423 ms with the default back-off, 1365 ms with 32)
BATCH_CFG = dict(mapping=1, workers=4096, schedule=tg.TG_SCHED_BALANCED, idle_sleep=32)
BATCH_QUEUE_CFG = dict(mapping=1, dispatch=tg.TG_DISPATCH_QUEUE, tile=1)
# oracle cost cap of the parity sample, in word-rounds (about 5 s per graph
# on one core)
BATCH_COST_CAP = 1.5e9


def stratified_batch_sample(specs, seed=7, per_cell=2, top_rounds=14):
    """Seeded, stratified sample of the batch manifest: per (pattern, payload
    size) cell the graph with the most mix rounds and per_cell - 1 random
    ones, plus the top_rounds graphs with the most mix rounds overall, all
    under BATCH_COST_CAP word-rounds of oracle work."""
    rng = np.random.default_rng(seed)
    cost = np.array([s.W * s.T * s.n * max(s.rounds, 1) for s in specs], np.float64)
    ok = cost <= BATCH_COST_CAP
    pick = []
    for p in wl.PATTERNS:
        for n in wl.PAYLOAD_CHOICES:
            cell = [i for i, s in enumerate(specs) if ok[i] and s.pattern == p and s.n == n]
            if not cell:
                continue
            pick.append(max(cell, key=lambda i: specs[i].rounds))
            rest = [i for i in cell if i not in pick]
            pick += list(rng.choice(rest, size=min(per_cell - 1, len(rest)), replace=False))
    by_rounds = sorted((i for i in range(len(specs)) if ok[i] and i not in pick), key=lambda i: -specs[i].rounds)
    pick += by_rounds[:top_rounds]
    return sorted(int(i) for i in pick)


def _cmp_times(g, stream, reps=3):
    """Kernel-launch comparators of one graph: (per-task launch ms, hipGraph
    DAG replay ms, captured hipGraph replay ms), median of reps after a
    warm-up call (which builds and instantiates the hipGraphs)."""
    import torch
    out = []
    for mode in (tg.TG_CMP_PER_TASK, tg.TG_CMP_HIPGRAPH, tg.TG_CMP_HIPGRAPH_CAPTURED):
        tg.tg_graph_execute_comparator(g.handle, mode, stream)
        tg.tg_graph_wait(g.handle)
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            tg.tg_graph_execute_comparator(g.handle, mode, stream)
            b.record(stream)
            tg.tg_graph_wait(g.handle)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        out.append(float(np.median(ts)))
    return out


def run_batch(args, stream, probes=None):
    """4096 independent graphs (frozen manifest) in one persistent launch,
    with a stratified oracle sample and the plain comparators."""
    from oracle import parallel as opar
    specs = wl.batch_manifest(args.graphs, seed=0)
    retention = getattr(args, "retention", "sinks")
    t0 = time.perf_counter()
    egs, gs = [], []
    for i, sp in enumerate(specs):
        eg = wl.pattern_graph(sp.pattern, sp.W, sp.T, seed=sp.seed, n=sp.n, rounds=sp.rounds)
        egs.append(eg)
        gs.append(request_graph(eg, retention))
        if i % 1024 == 0:
            log(f"batch: built {i} graphs, {time.perf_counter() - t0:.0f} s")
    N = sum(eg.N for eg in egs)
    U = sum(eg.N * eg.n * eg.rounds for eg in egs)
    payload_bytes_all = sum(eg.N * eg.n * 4 for eg in egs)
    payload_bytes = sum(tg.tg_graph_payload_slots(g.handle)[2] for g in gs)
    build_s = time.perf_counter() - t0
    log(f"batch: {len(gs)} graphs, {N} tasks, {U:.3e} word-rounds; host build {build_s:.0f} s")
    t1 = time.perf_counter()
    b = tg.tg_batch_create([g.handle for g in gs], tg.make_config(**BATCH_CFG))
    layout_s = time.perf_counter() - t1
    bcfg, _, btimes = tg.tg_batch_info(b, with_times=True)
    log(f"batch: layout {layout_s:.1f} s ({btimes}), launch {bcfg}")
    for _ in range(max(1, min(args.warmup, 1))):
        tg.tg_batch_execute(b, stream)
    tg.tg_batch_wait(b)
    steps = max(1, min(args.steps, 3))
    for _ in range(steps):
        tg.tg_batch_execute(b, stream)
    kt = tg.tg_batch_kernel_times(b, steps)
    ms = float(np.mean(kt))
    log(f"batch: one launch {ms:.1f} ms")
    tg.tg_batch_destroy(b)
    skip = getattr(args, "skipset", set())
    rec = {
        "workload": f"{len(gs)} independent graphs: W~U[8,512], T~U[8,256], five patterns, n~U{{64..1024}}, "
                    "R~LogNormal(ln 64, 1); one persistent launch",
        "tasks": N, "word_rounds": U, "launch": bcfg, "exec_ms": ms, "tasks_per_s": N / (ms * 1e-3),
        "word_rounds_per_s": U / (ms * 1e-3),
        "frac_of_measured_mix_rate": (U / (ms * 1e-3) / probes["mix_word_rounds_per_s"]
                                      if probes and probes.get("mix_word_rounds_per_s") else None),
        "frac_of_alu_peak": U / (ms * 1e-3) / ALU_PEAK_WORD_ROUNDS,
        "retention": retention, "payload_bytes": payload_bytes, "payload_bytes_keep_all": payload_bytes_all,
        "host_build_s": build_s, "layout_s": layout_s, "layout_ms": btimes,
    }
    if "queue" not in skip:
        # the same graphs with the ready-queue dispatch (timing only)
        qb = tg.tg_batch_create([g.handle for g in gs], tg.make_config(**BATCH_QUEUE_CFG))
        tg.tg_batch_execute(qb, stream)
        tg.tg_batch_wait(qb)
        tg.tg_batch_execute(qb, stream)
        tg.tg_batch_wait(qb)
        qms = float(np.mean(tg.tg_batch_kernel_times(qb, 1)))
        tg.tg_batch_destroy(qb)
        log(f"batch: one launch with the ready queue {qms:.1f} ms")
        rec["queue"] = {"launch": "queue: wavefronts x resident, tile 1", "exec_ms": qms, "lists_over_queue": ms / qms}
    if "cpu" in skip and "comparators" in skip:
        return rec
    # parity: stratified sample against the oracle in parallel processes
    sample = stratified_batch_sample(specs)
    tp = time.perf_counter()
    workers = opar.default_workers()
    refs = opar.explicit_many([(specs[i].pattern, specs[i].W, specs[i].T, specs[i].seed, specs[i].n,
                                specs[i].rounds) for i in sample], workers=workers)
    bad = [i for i, (dig, cs, _) in zip(sample, refs)
           if not (np.array_equal(tg.tg_graph_read_digests(gs[i].handle), dig) and
                   tg.tg_graph_checksum(gs[i].handle) == cs)]
    pool_s = time.perf_counter() - tp
    cpu = oracle_rate(sum(egs[i].N for i in sample), refs, pool_s, workers)
    log(f"batch: parity on {len(sample)} graphs ({pool_s:.0f} s, {workers} processes): "
        f"{'ok' if not bad else bad}")
    # comparators: one persistent launch per graph (seeded sample of 256),
    # and one kernel per task / hipGraph replays on a seeded subsample of
    # 16 graphs of at most 8192 tasks
    rng = np.random.default_rng(0)
    sample256 = rng.choice(len(gs), size=min(256, len(gs)), replace=False)
    seq_ms, seq_tasks = 0.0, 0
    for i in sample256:
        tg.tg_graph_execute(gs[i].handle, tg.make_config(**BATCH_CFG), stream)
        tg.tg_graph_wait(gs[i].handle)
        tg.tg_graph_execute(gs[i].handle, tg.make_config(**BATCH_CFG), stream)
        seq_ms += float(tg.tg_graph_kernel_times(gs[i].handle, 1)[0])
        seq_tasks += egs[i].N
    small = [i for i in range(len(gs)) if egs[i].N <= 8192]
    sub = np.random.default_rng(1).choice(small, size=min(16, len(small)), replace=False)
    per_task = hipg = capg = pers = 0.0
    sub_tasks = 0
    for i in sub:
        pers += _timed_graph(gs[i], None, stream, 1, 3)
        a, bb, c = _cmp_times(gs[i], stream)
        per_task += a
        hipg += bb
        capg += c
        sub_tasks += egs[i].N
    rec.update({
        "parity": {"ok": not bad, "graphs": len(sample), "failed": bad, "oracle_processes": workers,
                   "sample": "per (pattern, payload) cell the highest-R graph and one random graph, plus the 14 "
                             f"highest-R graphs, all under {BATCH_COST_CAP:.1e} word-rounds (seed 7)",
                   "cpu_oracle": cpu},
        "one_launch_per_graph": {"sample_graphs": len(sample256), "tasks": seq_tasks,
                                 "tasks_per_s": seq_tasks / (seq_ms * 1e-3)},
        "kernel_per_task_subsample": {
            "graphs": len(sub), "tasks": sub_tasks, "selection": "16 graphs of <= 8192 tasks (seed 1)",
            "persistent_tasks_per_s": sub_tasks / (pers * 1e-3),
            "per_task_launch_tasks_per_s": sub_tasks / (per_task * 1e-3),
            "hipgraph_dag_replay_tasks_per_s": sub_tasks / (hipg * 1e-3),
            "hipgraph_captured_replay_tasks_per_s": sub_tasks / (capg * 1e-3)},
    })
    return rec


# ---------------------------------------------------------------- serving

def run_serving(args, stream, probes=None):
    """Poisson stream of graph submissions (frozen manifest) replayed in real
    time into the continuous-batching server; latency p50/p99 and sustained
    tasks/s; a seeded sample of requests against the oracle."""
    from oracle import parallel as opar
    warm = max(args.requests // 10, 1)
    reqs = wl.serving_manifest(warm + args.requests, rate=args.rate, seed=0)
    t0 = time.perf_counter()
    graphs, handles = [], []
    edges_full, edges_run = 0, 0
    # implicit requests execute the two-hop reduction of their last-user DAG
    # (same order, a few edges per task) unless asked to run the full DAG
    reduce_implicit = not getattr(args, "full_dags", False)
    retention = getattr(args, "retention", "sinks")
    payload_run, payload_all = 0, 0
    for i, r in enumerate(reqs):
        x = wl.build_request(r)
        graphs.append(x)
        h = request_graph(x, retention, reduce_implicit)
        edges_run += tg.tg_graph_num_edges(h.handle)
        edges_full += h.inferred_edges
        if not isinstance(x, wl.ImplicitGraph):
            payload_run += tg.tg_graph_payload_slots(h.handle)[2]
            payload_all += x.N * x.n * 4
        handles.append(h)
        if i % 1000 == 0:
            log(f"serving: built {i} requests, {time.perf_counter() - t0:.0f} s")
    srv = tg.tg_server_create(64 << 30, slots=args.slots, max_batch=args.max_batch)
    if getattr(args, "server_dispatch", "queue") == "lists":
        tg.tg_server_configure(srv, tg.make_config(dispatch=tg.TG_DISPATCH_LISTS))
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
    lat, wait, serv, done = [], [], [], []
    for i, t in enumerate(tickets):
        s_ns, a_ns, d_ns = tg.tg_server_wait(srv, t)
        if i >= warm:
            lat.append((d_ns - s_ns) * 1e-6)
            wait.append((a_ns - s_ns) * 1e-6)
            serv.append((d_ns - a_ns) * 1e-6)
            done.append((s_ns, d_ns, graphs[i].N))
    stats = tg.tg_server_stats(srv)
    tg.tg_server_destroy(srv)
    first = min(x[0] for x in done)
    last = max(x[1] for x in done)
    tasks = sum(x[2] for x in done)
    span_s = (last - first) * 1e-9
    lat = np.array(lat)
    # parity on a seeded sample of 64 requests, oracle in parallel processes
    pick = sorted(int(i) for i in np.random.default_rng(1).choice(len(reqs), size=min(64, len(reqs)), replace=False))
    exp = [i for i in pick if reqs[i].mode == "explicit"]
    imp = [i for i in pick if reqs[i].mode == "implicit"]
    tp = time.perf_counter()
    refs = dict(zip(exp, opar.explicit_many([(reqs[i].pattern, reqs[i].W, reqs[i].T, reqs[i].seed, reqs[i].n,
                                               reqs[i].rounds) for i in exp])))
    refs.update(zip(imp, opar.implicit_many([(reqs[i].P, 256, reqs[i].iters, reqs[i].seed, reqs[i].rounds)
                                             for i in imp])))
    pool_s = time.perf_counter() - tp
    bad = [i for i in pick if not (np.array_equal(tg.tg_graph_read_digests(handles[i].handle), refs[i][0]) and
                                   tg.tg_graph_checksum(handles[i].handle) == refs[i][1])]
    cpu = oracle_rate(sum(graphs[i].N for i in pick), list(refs.values()), pool_s, opar.default_workers())
    return {
        "workload": f"serving: Poisson {args.rate:.0f} req/s, {args.requests} measured requests after {warm} warm-up, "
                    "sizes LogNormal(median 4096, sigma 1) in [64, 2^20], explicit/implicit 1:1, 64 GB budget, "
                    f"{args.slots} launch slots",
        "tasks": tasks, "span_s": span_s, "tasks_per_s": tasks / span_s,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        # submission to admission (waiting for a slot and memory), and
        # admission to completion (layout, launch, the graph's own execution)
        "admission_wait_ms": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
        "service_ms": {"p50": float(np.percentile(serv, 50)), "p99": float(np.percentile(serv, 99))},
        "server_config": getattr(args, "server_dispatch", "queue"),
        "offered_req_per_s": args.rate, "server": stats,
        "edges": edges_run, "edges_inferred": edges_full, "retention": retention,
        "explicit_payload_bytes": payload_run, "explicit_payload_bytes_keep_all": payload_all,
        "implicit_dag": "reduced (last-user, two-hop)" if reduce_implicit else "full inferred DAG",
        "parity": {"ok": not bad, "requests": len(pick), "failed": bad,
                   "sample": "64 requests drawn with seed 1 from all submitted", "cpu_oracle": cpu},
    }
