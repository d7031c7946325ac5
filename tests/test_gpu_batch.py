"""Batched execution: independent graphs of both modes in one persistent
launch give exactly what each gives alone (and what the oracle gives)."""
import numpy as np
import pytest

import oracle
from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests.gpu_util import check_explicit, oracle_explicit, run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("schedule", [tg.TG_SCHED_LIST, tg.TG_SCHED_LEVEL, tg.TG_SCHED_SPREAD, tg.TG_SCHED_COLUMN, tg.TG_SCHED_BALANCED])
@pytest.mark.parametrize("mapping", [1, 2])
def test_mixed_batch(gpu, mapping, schedule):
    specs = wl.batch_manifest(24, seed=3, wmax=64, tmax=32)
    egs = [wl.pattern_graph(s.pattern, s.W, s.T, seed=s.seed, n=s.n, rounds=min(s.rounds, 300)) for s in specs]
    ig = wl.halo_graph(16, 128, 6, seed=5, rounds=3)
    gs = [tg.graph_from_explicit(eg) for eg in egs]
    gi = tg.graph_from_implicit(ig)
    b = tg.tg_batch_create([g.handle for g in gs] + [gi.handle], tg.make_config(mapping=mapping, schedule=schedule))
    try:
        for _ in range(2):
            tg.tg_batch_execute(b)
            tg.tg_batch_wait(b)
            for g, eg in zip(gs, egs):
                check_explicit(g, eg, oracle_explicit(eg), payload_sample=4)
            ref = oracle.implicit_program_order(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv, ig.rounds, ig.space, seed=5)
            assert np.array_equal(tg.tg_graph_read_data(gi.handle, 0, ig.space), ref["A"])
            assert np.array_equal(tg.tg_graph_read_digests(gi.handle), ref["digest"])
        assert tg.tg_batch_time_ms(b) > 0
    finally:
        tg.tg_batch_destroy(b)
    # each graph alone gives the same digests
    for g, eg in zip(gs[:5], egs[:5]):
        run(g)
        check_explicit(g, eg, oracle_explicit(eg, want_payload=False))


def test_manifest_slice_256_graphs(gpu):
    # the first 256 graphs of the frozen 4096-graph manifest (their real
    # widths, depths, payload sizes and log-normal rounds) in one launch;
    # 24 sampled graphs compared digest by digest with the oracle
    specs = wl.batch_manifest(4096, seed=0)[:256]
    egs = [wl.pattern_graph(s.pattern, s.W, s.T, seed=s.seed, n=s.n, rounds=s.rounds) for s in specs]
    gs = [tg.graph_from_explicit(eg) for eg in egs]
    b = tg.tg_batch_create([g.handle for g in gs])
    try:
        tg.tg_batch_execute(b)
        tg.tg_batch_wait(b)
    finally:
        tg.tg_batch_destroy(b)
    cost = np.array([eg.N * eg.n * max(eg.rounds, 1) for eg in egs])
    rng = np.random.default_rng(0)
    pick = list(np.argsort(cost)[:16]) + list(rng.choice(len(egs), size=8, replace=False))
    for i in pick:
        eg = egs[i]
        if eg.N * eg.n * max(eg.rounds, 1) > 3e9:
            continue  # keep the oracle within seconds
        ref = oracle_explicit(eg, want_payload=False)
        assert np.array_equal(tg.tg_graph_read_digests(gs[i].handle), ref["digest"]), f"graph {i}"
        assert tg.tg_graph_checksum(gs[i].handle) == ref["checksum"]


def test_batch_autotune_keeps_results(gpu):
    """The autotuner re-plans the batch for several launch shapes and
    schedules (reusing plans with equal worker counts); the layout it keeps
    still gives the oracle's digests, also after a change of mix rounds."""
    specs = wl.batch_manifest(12, seed=9, wmax=48, tmax=24)
    egs = [wl.pattern_graph(s.pattern, s.W, s.T, seed=s.seed, n=s.n, rounds=0) for s in specs]
    gs = [tg.graph_from_explicit(eg) for eg in egs]
    b = tg.tg_batch_create([g.handle for g in gs])
    try:
        for R in (0, 40):
            tg.tg_batch_set_rounds(b, R)
            cfg, ms = tg.tg_batch_autotune(b, reps=1)
            assert ms > 0 and cfg["schedule"] in (tg.TG_SCHED_LIST, tg.TG_SCHED_LEVEL, tg.TG_SCHED_SPREAD, tg.TG_SCHED_COLUMN, tg.TG_SCHED_BALANCED)
            _, _, times = tg.tg_batch_info(b, with_times=True)
            assert times["build_ms"] >= times["plan_ms"] >= 0
            tg.tg_batch_execute(b)
            tg.tg_batch_wait(b)
            for g, eg in zip(gs, egs):
                eg.rounds = R
                check_explicit(g, eg, oracle_explicit(eg, want_payload=False))
    finally:
        tg.tg_batch_destroy(b)


@pytest.mark.parametrize("schedule", [tg.TG_SCHED_COLUMN, tg.TG_SCHED_LEVEL])
def test_benchmark_step_full_size(gpu, schedule):
    """The benchmark step at its full size in the launch shapes it is timed
    in: the five 1024 x 1000 graphs (5,120,000 tasks, 256-word payloads) in
    one batch on every resident wavefront; every digest and checksum equals
    the oracle's, on two executions in a row."""
    egs = [wl.pattern_graph(p, 1024, 1000, seed=0, n=256, rounds=0) for p in wl.PATTERNS]
    refs = [oracle_explicit(eg, want_payload=False) for eg in egs]
    gs = [tg.graph_from_explicit(eg) for eg in egs]
    b = tg.tg_batch_create([g.handle for g in gs], tg.make_config(schedule=schedule))
    try:
        for _ in range(2):
            tg.tg_batch_execute(b)
            tg.tg_batch_wait(b)
            for g, eg, ref in zip(gs, egs, refs):
                check_explicit(g, eg, ref)
    finally:
        tg.tg_batch_destroy(b)


def test_signalled_edges_per_dispatch(gpu):
    """The ready queue signals every edge; the per-worker lists of a column
    schedule leave out the edges between consecutive entries of one list (a
    stencil keeps each column on one worker, so each of its T-1 in-column
    edges is among them), and still give the oracle's digests."""
    W, T = 64, 40
    eg = wl.pattern_graph("stencil", W, T, seed=4, n=64, rounds=2)
    g = tg.graph_from_explicit(eg)
    ref = oracle_explicit(eg, want_payload=False)
    got = {}
    for name, cfg in (("queue", tg.make_config(dispatch=tg.TG_DISPATCH_QUEUE)),
                      ("lists", tg.make_config(dispatch=tg.TG_DISPATCH_LISTS, schedule=tg.TG_SCHED_COLUMN))):
        b = tg.tg_batch_create([g.handle], cfg)
        try:
            got[name] = tg.tg_batch_signalled_edges(b)
            tg.tg_batch_execute(b)
            tg.tg_batch_wait(b)
            check_explicit(g, eg, ref)
        finally:
            tg.tg_batch_destroy(b)
    assert got["queue"] == eg.E
    assert got["lists"] == eg.E - W * (T - 1)
