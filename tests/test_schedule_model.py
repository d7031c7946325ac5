"""Host logic of the executor, no GPU: the compiled worker layout run through
the CPU model of the worker loop (same ready window and advance rules as
the kernels) executes every task exactly once, after all its predecessors,
for any worker count, window length and schedule (list schedule or
dependence-level order), for one graph and for several launched together.
The timed model of the same layouts checks that the list schedule stays
close to the lower bound max(longest path, work / workers) where the
dependence-level order cannot."""
import numpy as np
import pytest

from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests import _checks as C


def _check_order(eg, order):
    assert sorted(order.tolist()) == list(range(eg.N))
    pos = np.empty(eg.N, np.int64)
    pos[order] = np.arange(eg.N)
    for v, s in enumerate(C.pred_sets(eg.pred_ptr, eg.preds)):
        assert all(pos[p] < pos[v] for p in s), f"task {v} ran before a predecessor"


SCHEDULES = [tg.TG_SCHED_LIST, tg.TG_SCHED_LEVEL, tg.TG_SCHED_SPREAD, tg.TG_SCHED_COLUMN, tg.TG_SCHED_BALANCED]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("pattern", wl.PATTERNS)
@pytest.mark.parametrize("nworkers,window", [(1, 1), (1, 64), (3, 2), (37, 64), (500, 7), (5000, 64)])
def test_schedule_completes(tglib, pattern, nworkers, window, schedule):
    eg = wl.pattern_graph(pattern, 37, 23, seed=3, n=64)
    g = tg.graph_from_explicit(eg)
    st, order = tg.tg_graph_emulate_schedule(g.handle, nworkers, window, seed=nworkers + window, schedule=schedule)
    assert st == tg.TG_OK, tg.load().tg_last_error()
    _check_order(eg, order)


@pytest.mark.parametrize("nworkers", [1024, 7168])
def test_schedule_completes_benchmark_shape(tglib, nworkers):
    eg = wl.pattern_graph("stencil", 1024, 60, seed=1, n=256)
    g = tg.graph_from_explicit(eg)
    st, order = tg.tg_graph_emulate_schedule(g.handle, nworkers, 64, seed=5)
    assert st == tg.TG_OK
    _check_order(eg, order)


@pytest.mark.parametrize("seed", range(4))
def test_schedule_random_dags(tglib, seed):
    rng = np.random.default_rng(seed)
    eg = wl.random_dag(400, 5, rng, n=64, seed=seed)
    g = tg.graph_from_explicit(eg)
    for nw, win in [(1, 1), (16, 4), (400, 64)]:
        for sch in SCHEDULES:
            st, order = tg.tg_graph_emulate_schedule(g.handle, nw, win, seed=seed, schedule=sch)
            assert st == tg.TG_OK
            _check_order(eg, order)


def _check_batch_order(egs, pairs):
    """Exactly once and after all predecessors, graph by graph."""
    for gi, eg in enumerate(egs):
        _check_order(eg, pairs[pairs[:, 0] == gi, 1])


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("nworkers,window", [(1, 64), (7, 3), (300, 64)])
def test_schedule_batch_of_uneven_graphs(tglib, schedule, nworkers, window):
    """Several graphs of different shapes, payloads and per-task rounds in
    one layout: each runs exactly once, in dependence order."""
    rng = np.random.default_rng(11)
    egs, gs = [], []
    for k, p in enumerate(wl.PATTERNS * 2):
        eg = wl.pattern_graph(p, int(rng.integers(1, 40)), int(rng.integers(1, 30)), seed=k, n=64 << (k % 3))
        g = tg.Graph(tg.tg_graph_create(tg.TG_EXPLICIT, eg.n, 0, eg.seed), tg.TG_EXPLICIT, eg.n)
        tg.tg_task_add_many(g.handle, eg.pred_ptr, eg.preds, rng.integers(0, 300, eg.N).astype(np.uint32))
        tg.tg_graph_finalize(g.handle)
        egs.append(eg)
        gs.append(g)
    st, pairs, mk, bd = tg.tg_emulate_schedule([g.handle for g in gs], nworkers, window, seed=5, schedule=schedule)
    assert st == tg.TG_OK, tg.load().tg_last_error()
    assert len(pairs) == sum(eg.N for eg in egs)
    _check_batch_order(egs, pairs)
    assert 0 < bd <= mk


@pytest.mark.parametrize("rounds", [0, 256])
def test_list_schedule_makespan(tglib, rounds):
    """The benchmark step's shape scaled down (the five patterns side by side,
    one of them dependence-free): in the timed model the list schedule is
    within 5% of the lower bound, the dependence-level order (which runs the
    whole dependence-free graph first) is not."""
    egs = [wl.pattern_graph(p, 128, 60, seed=0, n=256, rounds=rounds) for p in wl.PATTERNS]
    gs = [tg.graph_from_explicit(eg) for eg in egs]
    hs = [g.handle for g in gs]
    st, pairs, mk_list, bd = tg.tg_emulate_schedule(hs, 768, 64, seed=1, schedule=tg.TG_SCHED_LIST)
    assert st == tg.TG_OK
    _check_batch_order(egs, pairs)
    st, pairs, mk_level, bd2 = tg.tg_emulate_schedule(hs, 768, 64, seed=1, schedule=tg.TG_SCHED_LEVEL)
    assert st == tg.TG_OK
    assert bd == bd2
    assert mk_list <= 1.05 * bd
    assert mk_level > 1.08 * bd
    assert mk_list < mk_level


def test_emulator_rejects_bad_arguments(tglib):
    eg = wl.pattern_graph("stencil", 4, 4)
    g = tg.graph_from_explicit(eg)
    st, _ = tg.tg_graph_emulate_schedule(g.handle, 4, 65)
    assert st == tg.TG_EINVAL
    st, _ = tg.tg_graph_emulate_schedule(g.handle, 0, 8)
    assert st == tg.TG_EINVAL
    st, _ = tg.tg_graph_emulate_schedule(g.handle, 4, 8, schedule=6)
    assert st == tg.TG_EINVAL


def test_large_layout_built_in_parallel(tglib):
    """Layouts of at least 2^14 tasks build their records on several host
    threads; two graphs of that size together still run exactly once and in
    dependence order in the worker-loop model."""
    egs = [wl.pattern_graph("stencil", 512, 200, seed=1, n=64), wl.pattern_graph("random", 300, 200, seed=2, n=64)]
    gs = [tg.graph_from_explicit(eg) for eg in egs]
    st, pairs, _, _ = tg.tg_emulate_schedule([g.handle for g in gs], 2048, 64, seed=3)
    assert st == tg.TG_OK
    assert sum(eg.N for eg in egs) >= 1 << 17
    _check_batch_order(egs, pairs)
