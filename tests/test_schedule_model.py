"""Host logic of the executor, no GPU: the compiled worker layout run through
the CPU model of the worker loop (same ready window and advance rules as
the kernels) executes every task exactly once, after all its predecessors,
for any worker count and window length."""
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


@pytest.mark.parametrize("pattern", wl.PATTERNS)
@pytest.mark.parametrize("nworkers,window", [(1, 1), (1, 64), (3, 2), (37, 64), (500, 7), (5000, 64)])
def test_schedule_completes(tglib, pattern, nworkers, window):
    eg = wl.pattern_graph(pattern, 37, 23, seed=3, n=64)
    g = tg.graph_from_explicit(eg)
    st, order = tg.tg_graph_emulate_schedule(g.handle, nworkers, window, seed=nworkers + window)
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
        st, order = tg.tg_graph_emulate_schedule(g.handle, nw, win, seed=seed)
        assert st == tg.TG_OK
        _check_order(eg, order)


def test_emulator_rejects_bad_arguments(tglib):
    eg = wl.pattern_graph("stencil", 4, 4)
    g = tg.graph_from_explicit(eg)
    st, _ = tg.tg_graph_emulate_schedule(g.handle, 4, 65)
    assert st == tg.TG_EINVAL
    st, _ = tg.tg_graph_emulate_schedule(g.handle, 0, 8)
    assert st == tg.TG_EINVAL
