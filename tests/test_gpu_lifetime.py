"""Buffer lifetimes on the GPU: with payload slots reused once their readers
have finished (anti-dependence edges on the executor's counters), every
digest, the checksum and every kept payload equal the oracle's, in every
launch shape, in batches, through the comparators and through the server;
payloads whose slots were reused are refused on read."""
import numpy as np
import pytest

from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests import _checks as C
from tests.gpu_util import check_explicit, oracle_explicit, run, sinks

pytestmark = pytest.mark.gpu

SHAPES = [dict(mapping=1), dict(mapping=1, workers=5, window=3), dict(mapping=2, wg_waves=4),
          dict(mapping=3, gang=2, wg_waves=4), dict(mapping=1, schedule=tg.TG_SCHED_LIST),
          dict(mapping=1, schedule=tg.TG_SCHED_COLUMN), dict(mapping=1, notify=1)]


def _kept(eg, g, ref):
    """Sink payloads equal the oracle's; a released payload is refused."""
    for v in sinks(eg)[:256]:
        assert np.array_equal(tg.tg_graph_read_payload(g.handle, int(v), eg.n), ref["payload"][v]), f"sink {v}"
    slot, nslots, _ = tg.tg_graph_payload_slots(g.handle)
    if nslots < eg.N:
        # slots are handed out in dependence-level order (ties by id)
        sets = C.pred_sets(eg.pred_ptr, eg.preds)
        lv = [0] * eg.N
        for v in range(eg.N):
            lv[v] = max((lv[p] + 1 for p in sets[v]), default=0)
        order = sorted(range(eg.N), key=lambda v: (lv[v], v))
        last = {}
        for v in order:
            last[int(slot[v])] = v
        reused = [v for v in range(eg.N) if last[int(slot[v])] != v]
        if reused:
            with pytest.raises(tg.TaskGraphError) as ei:
                tg.tg_graph_read_payload(g.handle, reused[0], eg.n)
            assert ei.value.status == tg.TG_ESTATE


@pytest.mark.parametrize("pattern", wl.PATTERNS)
@pytest.mark.parametrize("W,T,n", [(37, 11, 64), (64, 30, 256), (7, 40, 1024)])
def test_patterns_keep_sinks(gpu, pattern, W, T, n):
    eg = wl.pattern_graph(pattern, W, T, seed=5, n=n, rounds=3)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg, retention=tg.TG_KEEP_SINKS)
    for kw in SHAPES:
        run(g, tg.make_config(**kw))
        check_explicit(g, eg, {"digest": ref["digest"], "checksum": ref["checksum"]})
        _kept(eg, g, ref)


@pytest.mark.parametrize("pattern", wl.PATTERNS)
def test_patterns_keep_none(gpu, pattern):
    eg = wl.pattern_graph(pattern, 64, 25, seed=6, n=256, rounds=5)
    ref = oracle_explicit(eg, want_payload=False)
    g = tg.graph_from_explicit(eg, retention=tg.TG_KEEP_NONE)
    _, nslots, _ = tg.tg_graph_payload_slots(g.handle)
    if pattern != "none":
        assert nslots <= 3 * 64
    for kw in SHAPES:
        run(g, tg.make_config(**kw))
        check_explicit(g, eg, ref)


@pytest.mark.parametrize("seed", range(4))
def test_random_dags(gpu, seed):
    rng = np.random.default_rng(80 + seed)
    eg = wl.random_dag(300, 5, rng, n=128, rounds=4, seed=seed, dup=True)
    ref = oracle_explicit(eg)
    for mode in (tg.TG_KEEP_SINKS, tg.TG_KEEP_NONE):
        g = tg.graph_from_explicit(eg, retention=mode)
        for kw in SHAPES[:4]:
            run(g, tg.make_config(**kw))
            check_explicit(g, eg, {"digest": ref["digest"], "checksum": ref["checksum"]})
        if mode == tg.TG_KEEP_SINKS:
            _kept(eg, g, ref)


@pytest.mark.parametrize("mode", [tg.TG_CMP_PER_TASK, tg.TG_CMP_HIPGRAPH, tg.TG_CMP_HIPGRAPH_CAPTURED])
def test_comparators_follow_the_anti_dependences(gpu, mode):
    rng = np.random.default_rng(9)
    eg = wl.random_dag(120, 4, rng, n=64, rounds=2, seed=3)
    ref = oracle_explicit(eg, want_payload=False)
    g = tg.graph_from_explicit(eg, retention=tg.TG_KEEP_NONE)
    for _ in range(2):
        tg.tg_graph_execute_comparator(g.handle, mode)
        tg.tg_graph_wait(g.handle)
        check_explicit(g, eg, ref)


def test_batch_mixed_retention(gpu):
    specs = wl.batch_manifest(18, seed=4, wmax=64, tmax=40)
    egs = [wl.pattern_graph(s.pattern, s.W, s.T, seed=s.seed, n=s.n, rounds=min(s.rounds, 200)) for s in specs]
    gs = [tg.graph_from_explicit(eg, retention=i % 3) for i, eg in enumerate(egs)]
    for kw in (dict(mapping=1), dict(mapping=1, schedule=tg.TG_SCHED_BALANCED), dict(mapping=2, wg_waves=2)):
        b = tg.tg_batch_create([g.handle for g in gs], tg.make_config(**kw))
        try:
            for _ in range(2):
                tg.tg_batch_execute(b)
                tg.tg_batch_wait(b)
                for g, eg in zip(gs, egs):
                    check_explicit(g, eg, oracle_explicit(eg, want_payload=False))
        finally:
            tg.tg_batch_destroy(b)


def test_stencil_full_width_keep_none(gpu):
    """The benchmark's stencil (1024 x 1000, 256-word payloads) in two levels
    of payload slots: every digest and the checksum."""
    eg = wl.pattern_graph("stencil", 1024, 1000, seed=0, n=256, rounds=4)
    ref = oracle_explicit(eg, want_payload=False)
    g = tg.graph_from_explicit(eg, retention=tg.TG_KEEP_NONE)
    _, nslots, nbytes = tg.tg_graph_payload_slots(g.handle)
    assert nslots == 2 * 1024 and nbytes == 2 * 1024 * 256 * 4
    run(g, tg.make_config(mapping=1, schedule=tg.TG_SCHED_COLUMN))
    check_explicit(g, eg, ref)


def test_serving_keep_none(gpu):
    """Requests compiled with payload reuse through the server: digests and
    checksums equal the oracle's, and they occupy less of the budget."""
    reqs = wl.serving_manifest(24, rate=4000.0, seed=8, median=600, max_tasks=6000)
    reqs = [r for r in reqs if r.mode == "explicit"]
    for r in reqs:
        r.rounds = min(r.rounds, 150)
    egs = [wl.build_request(r) for r in reqs]
    gs = [tg.graph_from_explicit(eg, retention=tg.TG_KEEP_NONE) for eg in egs]
    srv = tg.tg_server_create(1 << 30, slots=2, max_batch=8)
    try:
        for t in [tg.tg_server_submit(srv, g.handle) for g in gs]:
            tg.tg_server_wait(srv, t)
    finally:
        tg.tg_server_destroy(srv)
    for g, eg in zip(gs, egs):
        ref = oracle_explicit(eg, want_payload=False)
        assert np.array_equal(tg.tg_graph_read_digests(g.handle), ref["digest"])
        assert tg.tg_graph_checksum(g.handle) == ref["checksum"]
