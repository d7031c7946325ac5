"""Buffer lifetimes (payload slots reused once every reader has finished),
checked on the host compile alone (no GPU): the executed edges contain the
data edges and only go up the dependence levels, every reuse of a slot
follows every reader of its previous contents, kept payloads are never
overwritten, the slot count reaches the expected minimum, and the modelled
executor runs each task exactly once in an order the executed edges allow."""
import numpy as np
import pytest

from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests import _checks as C


def _levels(eg):
    sets = C.pred_sets(eg.pred_ptr, eg.preds)
    lv = np.zeros(eg.N, np.int64)
    for v in range(eg.N):
        lv[v] = max((lv[p] + 1 for p in sets[v]), default=0)
    return lv, sets


def _edges(row_ptr, col):
    return {(j, int(k)) for j in range(len(row_ptr) - 1) for k in col[int(row_ptr[j]):int(row_ptr[j + 1])]}


def _reach(N, edges):
    succ = [[] for _ in range(N)]
    for a, b in edges:
        succ[a].append(b)
    reach = [set() for _ in range(N)]
    for v in range(N):  # closure by search from every vertex (small graphs)
        seen, stack = set(), list(succ[v])
        while stack:
            x = stack.pop()
            if x not in seen:
                seen.add(x)
                stack.extend(succ[x])
        reach[v] = seen
    return reach


def _check(eg, mode, reach_check=True):
    g = tg.graph_from_explicit(eg, retention=mode)
    lv, sets = _levels(eg)
    data = _edges(*tg.tg_graph_read_dag(g.handle))
    assert data == {(p, v) for v in range(eg.N) for p in sets[v]}, "tg_graph_read_dag must keep the data DAG"
    ex = _edges(*tg.tg_graph_read_exec_dag(g.handle))
    assert data <= ex
    assert all(lv[a] < lv[b] for a, b in ex), "an executed edge does not go up the levels"
    slot, nslots, nbytes = tg.tg_graph_payload_slots(g.handle)
    assert nbytes == nslots * eg.n * 4 and (int(slot.max()) + 1 if eg.N else 0) == nslots
    # owners of each slot in the order the compile assigned them: level, then id
    order = sorted(range(eg.N), key=lambda v: (lv[v], v))
    owners = {}
    for v in order:
        owners.setdefault(int(slot[v]), []).append(v)
    readers = [[] for _ in range(eg.N)]
    for a, b in data:
        readers[a].append(b)
    reach = _reach(eg.N, ex) if reach_check else None
    for s, seq in owners.items():
        for u, w in zip(seq, seq[1:]):
            must = readers[u] if readers[u] else [u]
            if not readers[u]:
                assert mode == tg.TG_KEEP_NONE, f"task {u} has no readers but its slot was reused"
            for r in must:
                if reach is not None:
                    assert w in reach[r], f"slot {s}: task {w} may overwrite {u}'s payload before reader {r}"
                else:
                    assert (r, w) in ex
    sinks = [v for v in range(eg.N) if not readers[v]]
    if mode == tg.TG_KEEP_SINKS:
        for v in sinks:
            assert owners[int(slot[v])][-1] == v, f"sink {v} lost its payload"
    st, order_run = tg.tg_graph_emulate_schedule(g.handle, nworkers=7, window=8, seed=3)
    assert st == tg.TG_OK and sorted(order_run.tolist()) == list(range(eg.N))
    pos = {int(v): i for i, v in enumerate(order_run)}
    assert all(pos[a] < pos[b] for a, b in ex)
    return nslots


@pytest.mark.parametrize("mode", [tg.TG_KEEP_SINKS, tg.TG_KEEP_NONE])
@pytest.mark.parametrize("pattern", wl.PATTERNS)
@pytest.mark.parametrize("W,T", [(1, 7), (5, 9), (16, 12), (37, 10)])
def test_patterns(tglib, pattern, W, T, mode):
    eg = wl.pattern_graph(pattern, W, T, seed=2, n=64, rounds=1)
    nslots = _check(eg, mode)
    if pattern in ("stencil", "fft", "tree", "random") and T >= 3:
        # payloads of three consecutive levels at most, plus the kept
        # payloads of tasks nobody reads (tree and random graphs have such
        # tasks on every level)
        nsinks = eg.N - len(set(eg.preds.tolist()))
        assert nslots <= 3 * W + (nsinks if mode == tg.TG_KEEP_SINKS else 0)
    if pattern == "none":
        assert nslots == eg.N  # one level: nothing finishes before another starts


@pytest.mark.parametrize("mode", [tg.TG_KEEP_SINKS, tg.TG_KEEP_NONE])
@pytest.mark.parametrize("seed", range(6))
def test_random_dags(tglib, seed, mode):
    rng = np.random.default_rng(50 + seed)
    eg = wl.random_dag(60, 4, rng, n=64, rounds=1, seed=seed, dup=True)
    _check(eg, mode)


def test_stencil_uses_two_levels_of_slots_and_no_extra_edges(tglib):
    # a stencil task's new slot is that of (t-2, i), whose readers are exactly
    # (t-1, i-1..i+1): the task's own predecessors, so no edge is added, and
    # two levels of payloads are live at a time
    eg = wl.pattern_graph("stencil", 64, 40, seed=0, n=256)
    g = tg.graph_from_explicit(eg, retention=tg.TG_KEEP_NONE)
    _, nslots, nbytes = tg.tg_graph_payload_slots(g.handle)
    assert nslots == 2 * 64 and nbytes == 2 * 64 * 256 * 4
    assert tg.tg_graph_num_edges(g.handle) == eg.E


def test_keep_all_is_unchanged(tglib):
    eg = wl.pattern_graph("random", 20, 8, seed=1, n=64)
    g = tg.graph_from_explicit(eg)
    slot, nslots, _ = tg.tg_graph_payload_slots(g.handle)
    assert nslots == eg.N and np.array_equal(slot, np.arange(eg.N))
    a = _edges(*tg.tg_graph_read_dag(g.handle))
    assert a == _edges(*tg.tg_graph_read_exec_dag(g.handle))


def test_retention_arguments(tglib):
    eg = wl.pattern_graph("stencil", 4, 4, seed=0, n=64)
    g = tg.graph_from_explicit(eg)
    with pytest.raises(tg.TaskGraphError) as ei:
        tg.tg_graph_set_retention(g.handle, tg.TG_KEEP_NONE)
    assert ei.value.status == tg.TG_EBUSY
    h = tg.tg_graph_create(tg.TG_EXPLICIT, 64, 0, 0)
    with pytest.raises(tg.TaskGraphError) as ei:
        tg.tg_graph_set_retention(h, 7)
    assert ei.value.status == tg.TG_EINVAL
    tg.tg_graph_destroy(h)
    hi = tg.tg_graph_create(tg.TG_IMPLICIT, 0, 16, 0)
    with pytest.raises(tg.TaskGraphError) as ei:
        tg.tg_graph_set_retention(hi, tg.TG_KEEP_SINKS)
    assert ei.value.status == tg.TG_EINVAL
    tg.tg_graph_destroy(hi)


def test_batch_manifest_memory(tglib):
    """Payload memory of a slice of the 4096-graph manifest with and without
    reuse (host compile only)."""
    specs = wl.batch_manifest(4096, seed=0)[:24]
    full = reused = 0
    for s in specs:
        eg = wl.pattern_graph(s.pattern, s.W, s.T, seed=s.seed, n=s.n, rounds=s.rounds)
        g = tg.graph_from_explicit(eg, retention=tg.TG_KEEP_NONE)
        _, nslots, nbytes = tg.tg_graph_payload_slots(g.handle)
        full += eg.N * eg.n * 4
        reused += nbytes
        if s.pattern != "none" and s.T >= 3:
            assert nslots <= 3 * s.W
    assert reused < full / 4
