"""The gang executor's protocol on the CPU model (tg_emulate_gang): the
members of a gang schedule the gang's list each on their own, counters start
at in-degree x gang and every member signals each out-edge once.  Over every
pattern, random DAGs, implicit programs, batches, schedules, windows, gang
sizes and seeded interleavings: a member takes a task only after every
member of each predecessor finished it, every member runs each entry of its
list exactly once, and the members never get stuck."""
import numpy as np
import pytest

from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl


def _check(graphs, ngangs, gang, window=64, schedule=0, seeds=range(3)):
    total = sum(tg.tg_graph_num_tasks(g.handle) for g in graphs)
    for seed in seeds:
        st, shares = tg.tg_emulate_gang([g.handle for g in graphs], ngangs, gang, window, seed, schedule)
        assert st == tg.TG_OK, tg.load().tg_last_error().decode()
        assert shares == total * gang


@pytest.mark.parametrize("pattern", wl.PATTERNS)
@pytest.mark.parametrize("ngangs,gang,window", [(1, 2, 64), (3, 4, 64), (16, 8, 3), (64, 3, 1), (5, 32, 64)])
def test_patterns(tglib, pattern, ngangs, gang, window):
    g = tg.graph_from_explicit(wl.pattern_graph(pattern, 23, 9, seed=1, n=64))
    _check([g], ngangs, gang, window)


@pytest.mark.parametrize("schedule", [tg.TG_SCHED_LIST, tg.TG_SCHED_LEVEL, tg.TG_SCHED_SPREAD, tg.TG_SCHED_COLUMN,
                                      tg.TG_SCHED_BALANCED])
@pytest.mark.parametrize("seed", range(3))
def test_random_dags_every_schedule(tglib, schedule, seed):
    rng = np.random.default_rng(seed)
    g = tg.graph_from_explicit(wl.random_dag(120, 5, rng, n=64, seed=seed, dup=True))
    _check([g], 1 + 5 * seed, 2 + seed, 1 + 21 * seed, schedule)


def _from_out_edges(N, row_ptr, col):
    """An explicit graph whose predecessor lists are the given DAG's."""
    src = np.repeat(np.arange(N, dtype=np.int64), np.diff(row_ptr.astype(np.int64)))
    order = np.lexsort((src, col.astype(np.int64)))
    preds = src[order].astype(np.uint32)
    pred_ptr = np.zeros(N + 1, np.uint64)
    pred_ptr[1:] = np.cumsum(np.bincount(col.astype(np.int64), minlength=N))
    return tg.graph_from_explicit(wl.ExplicitGraph(N=N, pred_ptr=pred_ptr, preds=preds, n=64))


def test_implicit_programs(tglib):
    # the halo programs' last-user dependences (host construction) and their
    # two-hop reduction, the DAGs a gang launch of an implicit graph executes
    for P, S, iters in [(8, 64, 5), (17, 128, 3)]:
        ig = wl.halo_graph(P, S, iters, seed=2, rounds=1)
        rp, col = tg.tg_last_user_dag(ig.req_ptr, tg.reqs_array(ig.lo, ig.hi, ig.priv))
        _check([_from_out_edges(ig.N, rp, col)], 4, 8)
        rrp, rcol = tg.tg_reduce_dag(rp, col)
        _check([_from_out_edges(ig.N, rrp, rcol)], 4, 8)


def test_batch_of_graphs(tglib):
    specs = wl.batch_manifest(8, seed=3, wmax=32, tmax=10)
    gs = [tg.graph_from_explicit(wl.pattern_graph(s.pattern, s.W, s.T, seed=s.seed, n=s.n)) for s in specs]
    _check(gs, 24, 4, schedule=tg.TG_SCHED_BALANCED)


def test_one_member_is_the_list_executor(tglib):
    # a gang of one runs the lists without the in-list elision: the same
    # tasks, each once
    g = tg.graph_from_explicit(wl.pattern_graph("stencil", 16, 12, seed=0, n=64))
    _check([g], 7, 1)


def test_arguments(tglib):
    g = tg.graph_from_explicit(wl.pattern_graph("fft", 8, 4, seed=0, n=64))
    for ngangs, gang, window in [(0, 2, 64), (4, 0, 64), (4, 33, 64), (4, 2, 0), (4, 2, 65)]:
        st, _ = tg.tg_emulate_gang([g.handle], ngangs, gang, window)
        assert st == tg.TG_EINVAL


def test_in_list_elision_would_break_gangs(tglib):
    """Why gang launches count every edge: with the lists' in-list elision a
    member takes the next entry of its list as soon as it finished its own
    share of the previous one, before the other members have; the model
    reports the violated precedence (a stencil column kept on one gang)."""
    g = tg.graph_from_explicit(wl.pattern_graph("stencil", 8, 24, seed=0, n=64))
    caught = 0
    for seed in range(8):
        st, _ = tg.tg_emulate_gang([g.handle], 8, 4, 64, seed, tg.TG_SCHED_COLUMN, elide=True)
        assert st in (tg.TG_OK, tg.TG_EINVAL)
        caught += st == tg.TG_EINVAL
    assert caught > 0
    # without the elision (the executor's rule) every seed passes
    _check([g], 8, 4, schedule=tg.TG_SCHED_COLUMN, seeds=range(8))
    # a gang of one is the list executor: the elision is sound there
    for seed in range(4):
        st, shares = tg.tg_emulate_gang([g.handle], 8, 1, 64, seed, tg.TG_SCHED_COLUMN, elide=True)
        assert st == tg.TG_OK and shares == 8 * 24
