#!/usr/bin/env python3
"""Throughput of the task-DAG executor on one MI355X.

Workload (one "step"): the five Task Bench shaped graphs -- no dependences,
1-D stencil, FFT butterfly, binary tree, random 5-of-33 -- each 1024 wide and
1000 timesteps deep (1,024,000 tasks, 256-word payloads), every task with 0
mix rounds, so a step measures the executor's overhead: counter resets,
ready-window scans, payload hand-off and edge signals for 5,120,000 tasks.
The five independent graphs of a step run as one batched persistent launch
(their critical paths overlap); each graph's own launch time is reported
beside it.  Graphs are compiled and the launch shape autotuned once, outside
the timed region; inputs are resident in HBM when timing starts.

Printed: one JSON line with tasks/s (value), per-task overhead, METG(50)
from a sweep of mix rounds, the roofline of the executor kernel, the
comparators (one kernel per task, hipGraph replay) on a capped sub-graph and
the sequential CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

W, T, NWORDS = 1024, 1000, 256
SWEEP_ROUNDS = (0, 4, 8, 16, 64, 256, 1024, 4096)
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
    import math
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-sweep", action="store_true", help="skip the mix-round sweep (METG)")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-alone", action="store_true", help="skip timing each graph alone")
    ap.add_argument("--schedule", type=int, default=0,
                    help="with --no-tune: the batch's schedule (1 list, 2 level, 3 spread, 4 column; 0 default)")
    ap.add_argument("--copy-probe-only", action="store_true",
                    help="run only the copy-bandwidth probe (short runs under a counter profiler)")
    ap.add_argument("--comparator-steps", type=int, default=50, help="timesteps of the comparator sub-graph")
    ap.add_argument("--workload", default="step", choices=["step", "implicit", "batch", "serving"],
                    help="step (default): the five-graph step; implicit: the 2^16-task halo program; "
                         "batch: 4096 uneven graphs in one launch; serving: Poisson request replay")
    ap.add_argument("--graphs", type=int, default=4096, help="batch: number of graphs")
    ap.add_argument("--requests", type=int, default=10000, help="serving: measured requests")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: arrivals per second")
    ap.add_argument("--slots", type=int, default=4, help="serving: launch slots (streams) of the server, 1..4")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the executor runs on one GPU only (it is single-device); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2508_16522_amd import taskgraph as tg
    from paper_2508_16522_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.workload != "step":
        import bench_workloads
        out = getattr(bench_workloads, "run_" + args.workload)(args, stream)
        print(json.dumps(out), flush=True)
        return

    # ---------------------------------------------------------- probes
    if args.copy_probe_only:
        probes = {"copy_bytes_per_s": tg.tg_probe(tg.TG_PROBE_COPY_BW)}
    else:
        probes = {
            "mix_word_rounds_per_s": tg.tg_probe(tg.TG_PROBE_MIX_RATE),
            "copy_bytes_per_s": tg.tg_probe(tg.TG_PROBE_COPY_BW),
            "atomics_distinct_per_s": tg.tg_probe(tg.TG_PROBE_ATOMIC_DISTINCT),
            "atomics_contended_per_s": tg.tg_probe(tg.TG_PROBE_ATOMIC_CONTENDED),
            "launches_per_s": tg.tg_probe(tg.TG_PROBE_LAUNCH_RATE),
        }
    log(f"probes: {probes}")

    # --------------------------------------------------------- workload
    t0 = time.time()
    egs = [wl.pattern_graph(p, W, T, seed=0, n=NWORDS, rounds=0) for p in wl.PATTERNS]
    gs = [tg.graph_from_explicit(eg) for eg in egs]
    tasks_per_step = sum(eg.N for eg in egs)
    bytes_per_step = sum(algorithmic_bytes(eg) for eg in egs)
    edges_per_step = sum(eg.E for eg in egs)
    compile_ms = [tg.tg_graph_timings(g.handle)["compile_ms"] for g in gs]
    log(f"built {len(gs)} graphs ({tasks_per_step} tasks) in {time.time() - t0:.1f}s; compile ms {compile_ms}")

    # each graph alone (autotuned), for reference
    tuned = {}
    solo_ms = {}
    for p, g in zip(wl.PATTERNS, gs):
        if args.no_alone:
            break
        if args.no_tune:
            tuned[p] = None
            tg.tg_graph_execute(g.handle, None, stream)
            tg.tg_graph_wait(g.handle)
        else:
            cfg, ms = tg.tg_graph_autotune(g.handle, reps=2)
            tuned[p] = cfg
        for _ in range(3):
            tg.tg_graph_execute(g.handle, None, stream)
        solo_ms[p] = float(np.mean(tg.tg_graph_kernel_times(g.handle, 3)))
        log(f"alone {p}: {solo_ms[p]:.3f} ms ({tuned[p]})")

    # the step: one batched launch over the five graphs
    batch = tg.tg_batch_create([g.handle for g in gs], tg.make_config(schedule=args.schedule))
    if not args.no_tune:
        bcfg, bms = tg.tg_batch_autotune(batch, reps=2)
        log(f"autotune batch: {bcfg} {bms:.3f} ms")
    bcfg, _, btimes = tg.tg_batch_info(batch, with_times=True)
    log(f"batch layout: plan {btimes['plan_ms']:.0f} ms, build {btimes['build_ms']:.0f} ms")

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

    # parity of the last timed step against the oracle (digests, checksum)
    parity = None
    cpu = None
    if not args.no_cpu:
        import oracle
        # three passes over the step (~10-15 s of CPU work); the first one's
        # results are the parity reference
        cpu_steps = 3
        t_cpu = time.perf_counter()
        for i in range(cpu_steps):
            out = [oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, eg.rounds, seed=eg.seed, want_payload=False)
                   for eg in egs]
            if i == 0:
                refs = out
        cpu_s = time.perf_counter() - t_cpu
        tg.tg_batch_wait(batch)
        parity = all(np.array_equal(tg.tg_graph_read_digests(g.handle), r["digest"]) and
                     tg.tg_graph_checksum(g.handle) == r["checksum"] for g, r in zip(gs, refs))
        cpu = {"value": cpu_steps * tasks_per_step / cpu_s, "unit": "tasks/s", "cores": 1, "kind": "oracle",
               "sample": f"{cpu_steps} full steps: the five {W}x{T} graphs ({tasks_per_step} tasks each step), "
                         f"0 mix rounds, sequential C oracle (gcc -O2), one thread; {cpu_s:.1f} s"}
        log(f"cpu oracle: {cpu_s:.1f} s; parity {parity}")

    # ----------------------------------------------- mix-round sweep (METG)
    sweep = None
    if not args.no_sweep:
        pi = probes["mix_word_rounds_per_s"]
        rows = []
        for R in SWEEP_ROUNDS:
            tg.tg_batch_set_rounds(batch, R)
            # the launch shape is re-tuned for each task size up to 256 rounds;
            # larger sizes keep the shape tuned at 256
            if not args.no_tune and 0 < R <= 256:
                tcfg, tms = tg.tg_batch_autotune(batch, reps=1)
                log(f"sweep R={R}: autotuned {tcfg} {tms:.3f} ms")
            rcfg, _ = tg.tg_batch_info(batch)
            slots = rcfg["workers"]
            step()  # warm
            reps = 2 if R >= 1024 else 3
            for _ in range(reps):
                step()
            ms = float(np.mean(tg.tg_batch_kernel_times(batch, reps)))
            U = tasks_per_step * NWORDS * R
            eff = (U / (ms * 1e-3)) / pi if R else 0.0
            # granularity: run time per task per concurrent worker (Task Bench METG x-axis)
            gran_us = ms * 1e3 * slots / tasks_per_step
            rows.append({"rounds": R, "ms": ms, "efficiency": eff, "granularity_us": gran_us,
                         "launch": {k: rcfg[k] for k in ("mapping", "workers", "wg_waves", "notify", "schedule")}})
            log(f"sweep R={R}: {ms:.3f} ms eff {eff:.3f} gran {gran_us:.2f} us")
        tg.tg_batch_set_rounds(batch, 0)
        m = metg50([r["granularity_us"] for r in rows if r["rounds"]], [r["efficiency"] for r in rows if r["rounds"]])
        sweep = {"rows": rows, "metg50_us": m, "peak_word_rounds_per_s": pi}

    # ----------------------------------------------------- small stencil
    # the small configuration: stencil 8x16, 64-word payloads, 16 rounds;
    # launch + per-level latency, checked against the oracle
    small = None
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
    if not args.no_cpu:
        import oracle
        r1 = oracle.exec_explicit(eg1.N, eg1.n, eg1.pred_ptr, eg1.preds, eg1.rounds, seed=0, want_payload=False)
        small["parity"] = bool(tg.tg_graph_checksum(g1.handle) == r1["checksum"] and
                            np.array_equal(tg.tg_graph_read_digests(g1.handle), r1["digest"]))
    log(f"small stencil: {small}")
    del g1

    # ------------------------------------------------------- comparators
    comps = None
    if not args.no_comparators:
        eg = wl.pattern_graph("stencil", W, args.comparator_steps, seed=0, n=NWORDS, rounds=0)
        g = tg.graph_from_explicit(eg)
        res = {}
        tg.tg_graph_execute(g.handle, None, stream)
        tg.tg_graph_wait(g.handle)
        for name, fn in [("persistent", lambda: tg.tg_graph_execute(g.handle, None, stream)),
                         ("per_task_launch", lambda: tg.tg_graph_execute_comparator(g.handle, tg.TG_CMP_PER_TASK, stream)),
                         ("hipgraph_replay", lambda: tg.tg_graph_execute_comparator(g.handle, tg.TG_CMP_HIPGRAPH, stream))]:
            t_b = time.perf_counter()
            fn()  # warm (builds and instantiates the hipGraph the first time)
            tg.tg_graph_wait(g.handle)
            build_s = time.perf_counter() - t_b
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            tg.tg_graph_wait(g.handle)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            res[name] = {"ms": ms, "tasks_per_s": eg.N / (ms * 1e-3), "first_call_s": build_s}
        ref = None
        try:
            import oracle
            ref = oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, 0, want_payload=False)
            res["parity"] = bool(np.array_equal(tg.tg_graph_read_digests(g.handle), ref["digest"]))
        except ImportError:
            pass
        comps = {"graph": f"stencil {W}x{args.comparator_steps}, n={NWORDS}, R=0 ({eg.N} tasks)", **res}
        log(f"comparators: {comps}")
        del g

    counters = counters_from_profile(kernel_source_hash())
    traffic = counters.get("hbm_bytes_per_step")
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
                        f"{NWORDS}-word payloads, 0 mix rounds (one step = the five graphs)",
            "tasks_per_step": tasks_per_step,
            "launch": bcfg,
        },
        "alone_ms": solo_ms,
        "alone_launch": tuned,
        "per_task_overhead_ns": 1e9 / value,
        "metg50_us": sweep["metg50_us"] if sweep else None,
        "parity": parity,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_exec_wave / k_exec_block (persistent executor)",
            "algorithmic_bytes_per_step": bytes_per_step,
            "kernel_ms_per_step": kernel_ms_per_step,
            # the same bytes against the copy bandwidth this GPU measured
            "frac_of_measured_copy": (achieved_gbs * 1e9 / probes["copy_bytes_per_s"]
                                      if probes.get("copy_bytes_per_s") else None),
            # one device atomic per edge: against the measured distinct-address rate
            "atomics_per_step": edges_per_step,
            "atomics_per_s": edges_per_step / (kernel_ms_per_step * 1e-3),
            "atomics_frac": (edges_per_step / (kernel_ms_per_step * 1e-3) / probes["atomics_distinct_per_s"]
                             if probes.get("atomics_distinct_per_s") else None),
            # the same executor under counters: L2 atomic requests per step
            # (equal to the edge count) and the L2 hit fraction
            "atomics_counted_per_step": counters.get("l2_atomic_requests_per_step"),
            "l2_hit_fraction": counters.get("l2_hit_fraction"),
        },
        "cpu_baseline": cpu,
        "rounds_sweep": sweep,
        "small_stencil": small,
        "comparators": comps,
        "probes": probes,
        "compile_ms": dict(zip(wl.PATTERNS, compile_ms)),
        "batch_layout_ms": btimes,
    }
    tg.tg_batch_destroy(batch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
