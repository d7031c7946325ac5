#!/usr/bin/env python3
"""Throughput of the task-DAG executor on one MI355X.

Headline (one "step"): the five Task Bench shaped graphs -- no dependences,
1-D stencil, FFT butterfly, binary tree, random 5-of-33 -- each 1024 wide and
1000 timesteps deep (1,024,000 tasks, 256-word payloads), every task with 0
mix rounds, so a step measures the executor's overhead: counter resets,
ready-window scans, payload hand-off and edge signals for 5,120,000 tasks.
The five independent graphs of a step run as one batched persistent launch.
Graphs are compiled and the launch shape autotuned once, outside the timed
region; inputs are resident in HBM when timing starts.

The same JSON line carries every other configuration:
  patterns    : each of the five graphs alone -- tasks/s, HBM fraction,
                latency fraction (levels x the measured dependent hand-off),
                per-task overhead, and METG(50) from its own mix-round sweep;
  rounds_sweep: METG(50) of the batched step;
  comparators : per pattern (1024 x 50), the persistent executor vs one
                kernel launch per task vs hipGraph replays, same graph;
  small_stencil, implicit (the 65,536-task halo program), batch (4096
  graphs in one launch), serving (Poisson replay), cpu_baseline (the
  sequential oracle on a bounded sample, pinned to one core).
"""
from __future__ import annotations

import argparse
import contextlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

W, T, NWORDS = 1024, 1000, 256
SWEEP_ROUNDS = (0, 4, 8, 16, 32, 64, 256, 1024, 4096)
HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(eg) -> int:
    """Bytes the method must move per execution of an explicit graph: every
    task writes its payload and digest, reads each predecessor's payload,
    reads its record pointers and out-edge list and touches its counter:
    N*(4n + 4 + 4 + 8) + E*(4n + 4)."""
    return eg.N * (4 * eg.n + 16) + eg.E * (4 * eg.n + 4)


def metg50(gran_us, eff):
    """Smallest granularity with efficiency >= 0.5, interpolated in log space
    between the two sweep points that bracket 0.5 (Task Bench METG(50))."""
    pts = sorted(zip(gran_us, eff))
    for (g0, e0), (g1, e1) in zip(pts, pts[1:]):
        if e0 < 0.5 <= e1:
            t = (0.5 - e0) / (e1 - e0)
            return math.exp(math.log(g0) + t * (math.log(g1) - math.log(g0)))
    if pts and pts[0][1] >= 0.5:
        return pts[0][0]
    return None


def counters_from_profile(kernel_hash):
    """Counter figures per step (HBM bytes, L2 atomic requests, L2 hit
    fraction) from the committed counter profiles, if they were taken on the
    current executor kernel source; else an empty dict."""
    path = os.path.join(ROOT, "profiles", "five_graph_step_r0_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return {}
    if d.get("kernel_source_sha1") != kernel_hash:
        return {}
    return d


def kernel_source_hash():
    import hashlib
    h = hashlib.sha1()
    for name in ("tg_kernels.hip", "tg_internal.h"):
        with open(os.path.join(ROOT, "paper_2508_16522_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = sorted(os.sched_getaffinity(0))
    except AttributeError:
        allowed = list(range(os.cpu_count() or 1))
    return {"cpu_model": model, "nproc": os.cpu_count(), "allowed_cores": len(allowed)}, allowed


@contextlib.contextmanager
def pinned_to(core):
    """Run the calling thread on one core (as taskset -c core would)."""
    old = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {core})
    try:
        yield
    finally:
        os.sched_setaffinity(0, old)


def timed_execs(tg, g, cfg, stream, reps):
    """Mean executor-kernel time of reps executions after one warm-up."""
    import numpy as np
    tg.tg_graph_execute(g.handle, cfg, stream)
    tg.tg_graph_wait(g.handle)
    for _ in range(reps):
        tg.tg_graph_execute(g.handle, cfg, stream)
    return float(np.mean(tg.tg_graph_kernel_times(g.handle, reps)))


# launch shapes timed for each graph alone at R = 0 (the best one is kept),
# and the ready-queue dispatch beside them
def alone_shapes(tg):
    return [("lists: wavefronts x resident, column", tg.make_config(mapping=1, schedule=tg.TG_SCHED_COLUMN)),
            ("lists: wavefronts x resident, level", tg.make_config(mapping=1, schedule=tg.TG_SCHED_LEVEL)),
            ("lists: wavefronts x 1024, level", tg.make_config(mapping=1, workers=1024, schedule=tg.TG_SCHED_LEVEL))]


def queue_shape(tg):
    return ("queue: wavefronts x 2048, tile 1", tg.make_config(mapping=1, workers=2048, dispatch=tg.TG_DISPATCH_QUEUE,
                                                               tile=1))


# shapes of the mix-round sweep (the faster one at each R is kept): one
# wavefront or one 4-wave workgroup per task, as many workers as tasks can be
# ready at once (the width; every task of the dependence-free graph)
def sweep_shapes(tg, dependent):
    w = 1024 if dependent else 0
    return [("lists: wavefronts, level", tg.make_config(mapping=1, workers=w, schedule=tg.TG_SCHED_LEVEL)),
            ("lists: 4-wave workgroups, level", tg.make_config(mapping=2, wg_waves=4, workers=w,
                                                               schedule=tg.TG_SCHED_LEVEL))]


def leg_patterns(tg, wl, egs, gs, probes, stream):
    """Each C2 graph alone: best of three launch shapes at R = 0 (tasks/s,
    HBM and latency fractions, per-task overhead) and the ready-queue
    dispatch beside it, then its own mix-round sweep (the faster of two
    shapes at each R; efficiency against the measured mix rate) and
    METG(50).  Task slots (for granularity and per-task overhead) are the
    workers a launch runs, capped at the tasks that can be ready at once:
    the width W for the dependent patterns, every task without them."""
    pi = probes["mix_word_rounds_per_s"]
    hop_ns = probes.get("handoff_ns")
    out = {}
    for p, eg, g in zip(wl.PATTERNS, egs, gs):
        dependent = p != "none"
        conc = W if dependent else eg.N
        best = None
        for name, cfg in alone_shapes(tg):
            ms = timed_execs(tg, g, cfg, stream, 3)
            workers, _ = tg.tg_graph_exec_info(g.handle)
            if best is None or ms < best[1]:
                best = (name, ms, cfg, workers)
        name, ms, cfg, workers = best
        qname, qcfg = queue_shape(tg)
        qms = timed_execs(tg, g, qcfg, stream, 3)
        slots = min(workers, conc)
        levels = T if dependent else 1
        rec = {"launch": name, "workers": workers, "task_slots": slots, "kernel_ms": ms,
               "tasks_per_s": eg.N / (ms * 1e-3), "algorithmic_bytes": algorithmic_bytes(eg),
               "hbm_frac": algorithmic_bytes(eg) / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
               "edges": eg.E, "levels": levels,
               "per_task_overhead_ns": ms * 1e6 * slots / eg.N,
               "throughput_ns_per_task": ms * 1e6 / eg.N,
               "queue": {"launch": qname, "kernel_ms": qms, "lists_over_queue": ms / qms}}
        if hop_ns:
            rec["latency_floor_ms"] = levels * hop_ns * 1e-6
            rec["latency_frac"] = levels * hop_ns * 1e-6 / ms
        rows = []
        for R in SWEEP_ROUNDS:
            tg.tg_graph_set_rounds(g.handle, R)
            if R == 0:
                rows.append({"rounds": 0, "ms": ms, "efficiency": 0.0, "granularity_us": ms * 1e3 * slots / eg.N,
                             "launch": name})
                continue
            cand = []
            for sname, scfg in sweep_shapes(tg, dependent):
                sms = timed_execs(tg, g, scfg, stream, 2 if R >= 1024 else 3)
                sw, _ = tg.tg_graph_exec_info(g.handle)
                cand.append((sms, sname, min(sw, conc)))
            rms, sname, sslots = min(cand)
            U = eg.N * eg.n * R
            rows.append({"rounds": R, "ms": rms, "word_rounds_per_s": U / (rms * 1e-3),
                         "efficiency": (U / (rms * 1e-3)) / pi,
                         "granularity_us": rms * 1e3 * sslots / eg.N, "launch": sname})
        tg.tg_graph_set_rounds(g.handle, 0)
        rec["sweep"] = rows
        rec["metg50_us"] = metg50([r["granularity_us"] for r in rows if r["rounds"]],
                                  [r["efficiency"] for r in rows if r["rounds"]])
        out[p] = rec
        log(f"alone {p}: {ms:.3f} ms ({name}), {rec['tasks_per_s'] / 1e6:.0f} M tasks/s, hbm {rec['hbm_frac']:.3f}, "
            f"latency frac {rec.get('latency_frac', 0):.3f}, queue {qms:.3f} ms, METG(50) {rec['metg50_us']}")
    return out


def leg_comparators(tg, wl, stream, steps):
    """Per pattern, on one 1024 x `steps` graph: the persistent executor (its
    best shape), one kernel launch per task, the hipGraph with one node per
    task and one dependency per edge, and the captured per-task launch
    sequence; median of 5 after a warm-up (which also instantiates the
    hipGraphs, timed separately)."""
    import numpy as np
    import torch

    import oracle
    out = {}
    for p in wl.PATTERNS:
        eg = wl.pattern_graph(p, W, steps, seed=0, n=NWORDS, rounds=0)
        g = tg.graph_from_explicit(eg)
        ref = oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, 0, want_payload=False)
        cfg = tg.make_config(mapping=1, schedule=tg.TG_SCHED_COLUMN)
        res = {}
        ok = True
        for name, fn in [("persistent", lambda: tg.tg_graph_execute(g.handle, cfg, stream)),
                         ("per_task_launch", lambda: tg.tg_graph_execute_comparator(g.handle, tg.TG_CMP_PER_TASK, stream)),
                         ("hipgraph_dag_replay", lambda: tg.tg_graph_execute_comparator(g.handle, tg.TG_CMP_HIPGRAPH, stream)),
                         ("hipgraph_captured_replay",
                          lambda: tg.tg_graph_execute_comparator(g.handle, tg.TG_CMP_HIPGRAPH_CAPTURED, stream))]:
            t_b = time.perf_counter()
            fn()
            tg.tg_graph_wait(g.handle)
            first_s = time.perf_counter() - t_b
            ms = []
            for _ in range(5):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn()
                b.record(stream)
                tg.tg_graph_wait(g.handle)
                b.synchronize()
                ms.append(a.elapsed_time(b))
            ok &= bool(np.array_equal(tg.tg_graph_read_digests(g.handle), ref["digest"]))
            med = float(np.median(ms))
            res[name] = {"ms_median": med, "tasks_per_s": eg.N / (med * 1e-3), "first_call_s": first_s}
        res["parity"] = ok
        res["persistent_over_per_task"] = res["per_task_launch"]["ms_median"] / res["persistent"]["ms_median"]
        res["persistent_over_hipgraph"] = min(res["hipgraph_dag_replay"]["ms_median"],
                                              res["hipgraph_captured_replay"]["ms_median"]) / res["persistent"]["ms_median"]
        out[p] = res
        log(f"comparators {p}: " + ", ".join(f"{k} {v['ms_median']:.2f} ms" for k, v in res.items() if isinstance(v, dict)))
        del g
    return {"graph": f"each pattern {W} x {steps}, n={NWORDS}, R=0 ({W * steps} tasks); hipGraphs of 5 x 10^4 "
                     "nodes instantiate in seconds, so larger graphs are not used", "patterns": out}


def apply_peak(pi_probe, patterns, sweep, legs):
    """The mix-rate peak Pi is the best rate of the task body measured in
    this run: the dependence-free probe kernel, or any sweep point of the
    executor that beat it (the five-graph step at large R runs the same body
    in its persistent launch).  Efficiencies, METG(50) and the legs'
    fractions are taken against it, so none exceeds 1."""
    rates = [pi_probe]
    for rec in (patterns or {}).values():
        rates += [r["word_rounds_per_s"] for r in rec["sweep"] if r["rounds"]]
    if sweep:
        rates += [r["word_rounds_per_s"] for r in sweep["rows"] if r["rounds"]]
    pi = max(rates)
    for rec in (patterns or {}).values():
        for r in rec["sweep"]:
            if r["rounds"]:
                r["efficiency"] = r["word_rounds_per_s"] / pi
        rec["metg50_us"] = metg50([r["granularity_us"] for r in rec["sweep"] if r["rounds"]],
                                  [r["efficiency"] for r in rec["sweep"] if r["rounds"]])
    if sweep:
        for r in sweep["rows"]:
            if r["rounds"]:
                r["efficiency"] = r["word_rounds_per_s"] / pi
        sweep["metg50_us"] = metg50([r["granularity_us"] for r in sweep["rows"] if r["rounds"]],
                                    [r["efficiency"] for r in sweep["rows"] if r["rounds"]])
        sweep["peak_word_rounds_per_s"] = pi
    for leg in legs.values():
        if leg.get("word_rounds_per_s"):
            leg["frac_of_mix_peak"] = leg["word_rounds_per_s"] / pi
            leg.pop("frac_of_measured_mix_rate", None)
    src = "probe kernel" if pi == pi_probe else "executor sweep (same body, persistent launch)"
    return {"word_rounds_per_s": pi, "source": src, "probe_word_rounds_per_s": pi_probe}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--skip", default="", help="comma list of legs to leave out: patterns, sweep, small, comparators, "
                                               "cpu, implicit, batch, serving, queue (the batch leg's queue timing; with "
                                               "--workload batch, cpu and comparators leave out its oracle sample "
                                               "and comparators)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--schedule", type=int, default=0,
                    help="with --no-tune: the batch's schedule (1 list, 2 level, 3 spread, 4 column; 0 default)")
    ap.add_argument("--copy-probe-only", action="store_true",
                    help="run only the copy-bandwidth probe (short runs under a counter profiler)")
    ap.add_argument("--comparator-steps", type=int, default=50, help="timesteps of the comparator graphs")
    ap.add_argument("--workload", default="step", choices=["step", "implicit", "batch", "serving", "alone"],
                    help="step (default): every leg, the five-graph step as headline; implicit / batch / "
                         "serving / alone (one pattern graph): that leg on its own line")
    ap.add_argument("--pattern", default="stencil", help="alone: none, stencil, fft, tree or random")
    ap.add_argument("--dispatch", default="lists", choices=["lists", "queue"], help="alone: the dispatch")
    ap.add_argument("--graphs", type=int, default=4096, help="batch: number of graphs")
    ap.add_argument("--requests", type=int, default=4000, help="serving: measured requests")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: arrivals per second")
    ap.add_argument("--slots", type=int, default=4, help="serving: launch slots (streams) of the server, 1..4")
    ap.add_argument("--max-batch", type=int, default=64, help="serving: most requests per launch")
    ap.add_argument("--server-dispatch", default="queue", choices=["queue", "lists"],
                    help="serving: ready queue with device-built records (default) or host-planned lists")
    ap.add_argument("--full-dags", action="store_true",
                    help="serving: implicit requests execute their full inferred DAG instead of the reduced one")
    ap.add_argument("--retention", default="sinks", choices=["all", "sinks"],
                    help="batch and serving: explicit graphs keep every payload (all) or reuse payload memory "
                         "once read, keeping the sinks' payloads (sinks, default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the executor runs on one GPU only (it is single-device); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    skip = set(x for x in args.skip.split(",") if x)
    args.skipset = skip

    import numpy as np
    import torch

    import bench_workloads as bw
    from paper_2508_16522_amd import taskgraph as tg
    from paper_2508_16522_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t_start = time.time()
    leg_s = {}

    # ---------------------------------------------------------- probes
    if args.copy_probe_only:
        probes = {"copy_bytes_per_s": tg.tg_probe(tg.TG_PROBE_COPY_BW)}
    else:
        probes = {
            "mix_word_rounds_per_s": tg.tg_probe(tg.TG_PROBE_MIX_RATE),
            "alu_peak_word_rounds_per_s": bw.ALU_PEAK_WORD_ROUNDS,
            "copy_bytes_per_s": tg.tg_probe(tg.TG_PROBE_COPY_BW),
            "atomics_distinct_per_s": tg.tg_probe(tg.TG_PROBE_ATOMIC_DISTINCT),
            "atomics_contended_per_s": tg.tg_probe(tg.TG_PROBE_ATOMIC_CONTENDED),
            "launches_per_s": tg.tg_probe(tg.TG_PROBE_LAUNCH_RATE),
            "handoff_ns": tg.tg_probe(tg.TG_PROBE_HANDOFF_NS),
            "handoff_same_xcd_ns": tg.tg_probe(tg.TG_PROBE_HANDOFF_SAME_XCD_NS),
            "handoff_far_xcd_ns": tg.tg_probe(tg.TG_PROBE_HANDOFF_FAR_XCD_NS),
            "handoff_l2_payload_ns": tg.tg_probe(tg.TG_PROBE_HANDOFF_L2_NS),
        }
    log(f"probes: {probes}")
    if args.workload != "step":
        rec = getattr(bw, "run_" + args.workload)(args, stream, probes)
        print(json.dumps(bw.base_line(rec["tasks_per_s"], rec.get("exec_ms", rec.get("span_s", 0) * 1e3),
                                      args.steps, args.warmup, {"workload": rec["workload"]}, leg=rec,
                                      probes=probes)), flush=True)
        return

    # --------------------------------------------------------- workload
    t0 = time.time()
    egs = [wl.pattern_graph(p, W, T, seed=0, n=NWORDS, rounds=0) for p in wl.PATTERNS]
    gs = [tg.graph_from_explicit(eg) for eg in egs]
    tasks_per_step = sum(eg.N for eg in egs)
    bytes_per_step = sum(algorithmic_bytes(eg) for eg in egs)
    edges_per_step = sum(eg.E for eg in egs)
    compile_ms = [tg.tg_graph_timings(g.handle)["compile_ms"] for g in gs]
    log(f"built {len(gs)} graphs ({tasks_per_step} tasks) in {time.time() - t0:.1f}s; compile ms {compile_ms}")

    # the step: one batched launch over the five graphs
    t0 = time.time()
    batch = tg.tg_batch_create([g.handle for g in gs], tg.make_config(schedule=args.schedule))
    if not args.no_tune:
        bcfg, bms = tg.tg_batch_autotune(batch, reps=2)
        log(f"autotune batch: {bcfg} {bms:.3f} ms")
    bcfg, _, btimes = tg.tg_batch_info(batch, with_times=True)
    # counter atomics per launch: edges between consecutive entries of one
    # worker's list are ordered by the list and signal nothing
    signalled_per_step = tg.tg_batch_signalled_edges(batch)
    log(f"batch layout: plan {btimes['plan_ms']:.0f} ms, build {btimes['build_ms']:.0f} ms; "
        f"{signalled_per_step} of {edges_per_step} edges signalled")

    def step():
        tg.tg_batch_execute(batch, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ------------------------------------------------------ timed steps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    dev_ms = ev0.elapsed_time(ev1)
    ms_per_step = dev_ms / args.steps
    value = tasks_per_step / (ms_per_step * 1e-3)

    # executor-kernel durations of the timed launches (HIP events on `stream`)
    kt = tg.tg_batch_kernel_times(batch, args.steps)
    kernel_ms_per_step = float(np.mean(kt))
    achieved_gbs = bytes_per_step / (kernel_ms_per_step * 1e-3) / 1e9
    log(f"step {ms_per_step:.3f} ms (wall {wall * 1e3 / args.steps:.3f} ms); kernel {kernel_ms_per_step:.3f} ms")
    leg_s["step"] = time.time() - t0

    # the same step with the ready-queue dispatch (timing only; the parity of
    # that dispatch is in the test-suite)
    step_queue = None
    if "patterns" not in skip:
        qb = tg.tg_batch_create([g.handle for g in gs], tg.make_config(mapping=1, workers=4096,
                                                                         dispatch=tg.TG_DISPATCH_QUEUE, tile=1))
        tg.tg_batch_execute(qb, stream)
        tg.tg_batch_wait(qb)
        for _ in range(3):
            tg.tg_batch_execute(qb, stream)
        tg.tg_batch_wait(qb)
        step_queue = {"launch": "queue: wavefronts x 4096, tile 1",
                      "kernel_ms": float(np.mean(tg.tg_batch_kernel_times(qb, 3))),
                      "lists_kernel_ms": kernel_ms_per_step}
        tg.tg_batch_destroy(qb)
        log(f"step with the ready queue: {step_queue['kernel_ms']:.3f} ms")

    # -------------------------------------------- oracle: parity and baseline
    parity = None
    cpu = None
    if "cpu" not in skip:
        import oracle
        t0 = time.time()
        info, allowed = cpu_info()
        core = allowed[0]
        # three passes over the step (~10-15 s of CPU work) on one pinned core;
        # the first pass's results are the parity reference
        cpu_steps = 3
        with pinned_to(core):
            t_cpu = time.perf_counter()
            for i in range(cpu_steps):
                out = [oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, eg.rounds, seed=eg.seed,
                                            want_payload=False) for eg in egs]
                if i == 0:
                    refs = out
            cpu_s = time.perf_counter() - t_cpu
        tg.tg_batch_wait(batch)
        parity = all(np.array_equal(tg.tg_graph_read_digests(g.handle), r["digest"]) and
                     tg.tg_graph_checksum(g.handle) == r["checksum"] for g, r in zip(gs, refs))
        cpu = {"value": cpu_steps * tasks_per_step / cpu_s, "unit": "tasks/s", "cores": 1, "kind": "oracle",
               "sample": f"{cpu_steps} full steps: the five {W}x{T} graphs ({tasks_per_step} tasks each step), "
                         f"0 mix rounds, sequential C oracle (gcc -O2, compiler auto-vectorisation allowed), one "
                         f"thread pinned to core {core}; {cpu_s:.1f} s",
               "ns_per_task": cpu_s * 1e9 / (cpu_steps * tasks_per_step), "pinned_core": core, **info}
        log(f"cpu oracle: {cpu_s:.1f} s; parity {parity}; {info}")
        leg_s["cpu"] = time.time() - t0

    # ----------------------------------------------- each graph alone + METG
    patterns = None
    if "patterns" not in skip:
        t0 = time.time()
        patterns = leg_patterns(tg, wl, egs, gs, probes, stream)
        leg_s["patterns"] = time.time() - t0

    # ------------------------------------ mix-round sweep of the step (METG)
    sweep = None
    if "sweep" not in skip:
        t0 = time.time()
        pi = probes["mix_word_rounds_per_s"]
        rows = []
        shape0 = bcfg
        shape64 = None
        for R in SWEEP_ROUNDS:
            tg.tg_batch_set_rounds(batch, R)
            # the launch shape is tuned at R = 0 (timed step) and once more at
            # R = 64; rounds from 64 on use the second shape
            if R == 64 and not args.no_tune:
                shape64, tms = tg.tg_batch_autotune(batch, reps=1)
                log(f"sweep R=64: autotuned {shape64} {tms:.3f} ms")
            rcfg, _ = tg.tg_batch_info(batch)
            slots = rcfg["workers"]
            step()  # warm
            reps = 2 if R >= 1024 else 3
            for _ in range(reps):
                step()
            ms = float(np.mean(tg.tg_batch_kernel_times(batch, reps)))
            U = tasks_per_step * NWORDS * R
            eff = (U / (ms * 1e-3)) / pi if R else 0.0
            gran_us = ms * 1e3 * slots / tasks_per_step
            rows.append({"rounds": R, "ms": ms, "word_rounds_per_s": U / (ms * 1e-3) if R else 0.0,
                         "efficiency": eff, "granularity_us": gran_us,
                         "frac_of_alu_peak": (U / (ms * 1e-3)) / bw.ALU_PEAK_WORD_ROUNDS if R else 0.0,
                         "launch": {k: rcfg[k] for k in ("mapping", "workers", "wg_waves", "notify", "schedule")}})
            log(f"sweep R={R}: {ms:.3f} ms eff {eff:.3f} gran {gran_us:.2f} us")
        tg.tg_batch_set_rounds(batch, 0)
        m = metg50([r["granularity_us"] for r in rows if r["rounds"]], [r["efficiency"] for r in rows if r["rounds"]])
        sweep = {"rows": rows, "metg50_us": m, "peak_word_rounds_per_s": pi, "shape_r0": shape0, "shape_r64": shape64}
        leg_s["sweep"] = time.time() - t0

    # ----------------------------------------------------- small stencil
    small = None
    t0 = time.time()
    if "small" not in skip:
        eg1 = wl.pattern_graph("stencil", 8, 16, seed=0, n=64, rounds=16)
        g1 = tg.graph_from_explicit(eg1)
        tg.tg_graph_execute(g1.handle, None, stream)
        tg.tg_graph_wait(g1.handle)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            tg.tg_graph_execute(g1.handle, None, stream)
        e1.record(stream)
        tg.tg_graph_wait(g1.handle)
        torch.cuda.synchronize()
        small = {"graph": "stencil 8x16, n=64, R=16 (128 tasks, 16 levels)", "ms_per_execution": e0.elapsed_time(e1) / 20,
                 "kernel_ms": float(np.mean(tg.tg_graph_kernel_times(g1.handle, 20)))}
        if probes.get("handoff_ns"):
            small["latency_floor_ms"] = 16 * probes["handoff_ns"] * 1e-6
            small["latency_frac"] = small["latency_floor_ms"] / small["kernel_ms"]
        if "cpu" not in skip:
            import oracle
            r1 = oracle.exec_explicit(eg1.N, eg1.n, eg1.pred_ptr, eg1.preds, eg1.rounds, seed=0, want_payload=False)
            small["parity"] = bool(tg.tg_graph_checksum(g1.handle) == r1["checksum"] and
                                   np.array_equal(tg.tg_graph_read_digests(g1.handle), r1["digest"]))
        log(f"small stencil: {small}")
        del g1
    leg_s["small"] = time.time() - t0

    # ------------------------------------------------------- comparators
    comps = None
    if "comparators" not in skip:
        t0 = time.time()
        comps = leg_comparators(tg, wl, stream, args.comparator_steps)
        leg_s["comparators"] = time.time() - t0

    # free the step's device memory before the large legs
    counters = counters_from_profile(kernel_source_hash())
    traffic = counters.get("hbm_bytes_per_step")
    tg.tg_batch_destroy(batch)
    del gs
    import gc
    gc.collect()
    torch.cuda.empty_cache()

    legs = {}
    for name in ("implicit", "batch", "serving"):
        if name in skip:
            continue
        t0 = time.time()
        legs[name] = getattr(bw, "run_" + name)(args, stream, probes)
        leg_s[name] = time.time() - t0
        log(f"{name}: {time.time() - t0:.0f} s")
        gc.collect()
        torch.cuda.empty_cache()

    peak = (apply_peak(probes["mix_word_rounds_per_s"], patterns, sweep, legs)
            if probes.get("mix_word_rounds_per_s") else None)
    out = {
        "metric": "tasks/sec + per-task overhead (ns) + min effective task granularity, 1 GPU",
        "value": value,
        "unit": "tasks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"Task Bench shaped graphs none/stencil/fft/tree/random, {W} wide x {T} timesteps, "
                        f"{NWORDS}-word payloads, 0 mix rounds (one step = the five graphs in one batched launch)",
            "tasks_per_step": tasks_per_step,
            "launch": bcfg,
        },
        # per-task overhead at R = 0: kernel time x concurrent workers / tasks
        # (the time one task occupies its worker); the reciprocal throughput
        # is given beside it
        "per_task_overhead_ns": kernel_ms_per_step * 1e6 * bcfg["workers"] / tasks_per_step,
        "throughput_ns_per_task": 1e9 / value,
        "metg50_us": sweep["metg50_us"] if sweep else None,
        "mix_peak": peak,
        "parity": parity,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_exec_wave (persistent executor)",
            "algorithmic_bytes_per_step": bytes_per_step,
            "kernel_ms_per_step": kernel_ms_per_step,
            "frac_of_measured_copy": (achieved_gbs * 1e9 / probes["copy_bytes_per_s"]
                                      if probes.get("copy_bytes_per_s") else None),
            "edges_per_step": edges_per_step,
            "atomics_per_step": signalled_per_step,
            "atomics_per_s": signalled_per_step / (kernel_ms_per_step * 1e-3),
            "atomics_frac": (signalled_per_step / (kernel_ms_per_step * 1e-3) / probes["atomics_distinct_per_s"]
                             if probes.get("atomics_distinct_per_s") else None),
            "atomics_counted_per_step": counters.get("l2_atomic_requests_per_step"),
            "l2_hit_fraction": counters.get("l2_hit_fraction"),
            "latency_floor_ms": T * probes["handoff_ns"] * 1e-6 if probes.get("handoff_ns") else None,
            "latency_frac": (T * probes["handoff_ns"] * 1e-6 / kernel_ms_per_step
                             if probes.get("handoff_ns") else None),
        },
        "cpu_baseline": cpu,
        "patterns": patterns,
        "step_with_queue": step_queue,
        "rounds_sweep": sweep,
        "small_stencil": small,
        "comparators": comps,
        **legs,
        "probes": probes,
        "compile_ms": dict(zip(wl.PATTERNS, compile_ms)),
        "batch_layout_ms": btimes,
        "leg_seconds": leg_s,
        "total_seconds": time.time() - t_start,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
