"""The ready-queue dispatch's protocol on the CPU model (tg_emulate_queue):
every task runs exactly once and after all the edges the executor's
counters follow, no ticket lies beyond a shard's capacity, every sink is
reported and every worker leaves (on an exit sentinel), for any number of
workers, shards and ticket tile sizes -- including fewer workgroups than
shards -- over single graphs, graphs with anti-dependence edges and batches
of graphs."""
import numpy as np
import pytest

from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl


def _edges(g):
    row_ptr, col = tg.tg_graph_read_exec_dag(g.handle)
    return [(j, int(k)) for j in range(len(row_ptr) - 1) for k in col[int(row_ptr[j]):int(row_ptr[j + 1])]]


def _check(graphs, nworkers, shards, tile, seed):
    st, order = tg.tg_emulate_queue([g.handle for g in graphs], nworkers, shards, tile, seed)
    assert st == tg.TG_OK, tg.load().tg_last_error().decode()
    total = sum(tg.tg_graph_num_tasks(g.handle) for g in graphs)
    assert len(order) == total
    keys = [(int(a), int(b)) for a, b in order]
    assert len(set(keys)) == total
    pos = {k: i for i, k in enumerate(keys)}
    for gi, g in enumerate(graphs):
        for a, b in _edges(g):
            assert pos[(gi, a)] < pos[(gi, b)]


@pytest.mark.parametrize("pattern", wl.PATTERNS)
@pytest.mark.parametrize("nworkers,shards,tile", [(1, 1, 1), (3, 2, 1), (16, 8, 1), (16, 8, 4), (64, 4, 64),
                                                  (5, 8, 64), (37, 8, 3)])
def test_patterns(tglib, pattern, nworkers, shards, tile):
    eg = wl.pattern_graph(pattern, 23, 9, seed=1, n=64)
    g = tg.graph_from_explicit(eg)
    for seed in range(3):
        _check([g], nworkers, shards, tile, seed)


@pytest.mark.parametrize("seed", range(6))
def test_random_dags_and_anti_dependences(tglib, seed):
    rng = np.random.default_rng(seed)
    eg = wl.random_dag(150, 5, rng, n=64, seed=seed, dup=True)
    for mode in (tg.TG_KEEP_ALL, tg.TG_KEEP_NONE):
        g = tg.graph_from_explicit(eg, retention=mode)
        _check([g], 1 + seed * 7, (1, 2, 4, 8)[seed % 4], 1 + seed % 3, seed)


def test_batch_of_graphs(tglib):
    specs = wl.batch_manifest(10, seed=2, wmax=40, tmax=12)
    gs = [tg.graph_from_explicit(wl.pattern_graph(s.pattern, s.W, s.T, seed=s.seed, n=s.n), retention=i % 3)
          for i, s in enumerate(specs)]
    for seed, (nw, sh, tl) in enumerate([(8, 8, 1), (40, 2, 5), (200, 8, 2)]):
        _check(gs, nw, sh, tl, seed)


def test_arguments(tglib):
    g = tg.graph_from_explicit(wl.pattern_graph("stencil", 4, 4, n=64))
    st, _ = tg.tg_emulate_queue([g.handle], 4, 3, 1)
    assert st == tg.TG_EINVAL
    st, _ = tg.tg_emulate_queue([g.handle], 4, 8, 65)
    assert st == tg.TG_EINVAL
