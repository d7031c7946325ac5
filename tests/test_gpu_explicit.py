"""Explicit task graphs on the GPU vs the oracle (bit-exact)."""
import numpy as np
import pytest

import oracle
from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests.gpu_util import check_explicit, oracle_explicit, run

pytestmark = pytest.mark.gpu


def test_c1_stencil_8x16(gpu):
    eg = wl.pattern_graph("stencil", 8, 16, seed=0, n=64, rounds=16)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    run(g)
    check_explicit(g, eg, ref, payload_sample=128)


@pytest.mark.parametrize("mapping", [1, 2])
@pytest.mark.parametrize("n", [64, 128, 256, 1024])
@pytest.mark.parametrize("pattern", wl.PATTERNS)
def test_patterns_ragged(gpu, pattern, n, mapping):
    eg = wl.pattern_graph(pattern, 37, 23, seed=5, n=n, rounds=3)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    run(g, tg.make_config(mapping=mapping))
    check_explicit(g, eg, ref, payload_sample=64)


@pytest.mark.parametrize("schedule", [tg.TG_SCHED_LIST, tg.TG_SCHED_LEVEL, tg.TG_SCHED_SPREAD, tg.TG_SCHED_COLUMN, tg.TG_SCHED_BALANCED])
@pytest.mark.parametrize("workers,window", [(1, 64), (1, 1), (7, 3), (64, 64), (0, 1), (0, 64)])
@pytest.mark.parametrize("mapping", [1, 2])
def test_worker_and_window_variants(gpu, mapping, workers, window, schedule):
    eg = wl.pattern_graph("random", 50, 20, seed=2, n=128, rounds=2)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    run(g, tg.make_config(mapping=mapping, workers=workers, window=window, wg_waves=4, schedule=schedule))
    check_explicit(g, eg, ref)


@pytest.mark.parametrize("wg_waves", [1, 2, 4, 8, 16])
def test_workgroup_sizes(gpu, wg_waves):
    eg = wl.pattern_graph("fft", 64, 12, seed=1, n=1024, rounds=5)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    run(g, tg.make_config(mapping=2, wg_waves=wg_waves))
    check_explicit(g, eg, ref)


@pytest.mark.parametrize("mapping", [1, 2])
def test_doorbell_notification(gpu, mapping):
    eg = wl.pattern_graph("random", 300, 30, seed=8, n=256, rounds=2)
    ref = oracle_explicit(eg, want_payload=False)
    g = tg.graph_from_explicit(eg)
    for win in (1, 64):
        run(g, tg.make_config(mapping=mapping, notify=1, window=win))
        check_explicit(g, eg, ref)


@pytest.mark.parametrize("mapping", [1, 2])
def test_device_exactly_once(gpu, mapping):
    # diagnostic launch: every task ran exactly once and every counter
    # reached zero
    eg = wl.pattern_graph("stencil", 256, 50, seed=2, n=64, rounds=1)
    g = tg.graph_from_explicit(eg)
    run(g, tg.make_config(mapping=mapping, diag=1))
    ds = tg.tg_graph_debug_state(g.handle)
    assert np.all(ds["execs"] == 1) and np.all(ds["pending"] == 0)
    w, _ = tg.tg_graph_exec_info(g.handle)
    assert np.all(ds["wprog"] == np.bincount(ds["owner"], minlength=w))
    tt, _ = tg.tg_graph_debug_times(g.handle)
    assert np.all(tt[:, 0] > 0) and np.all(tt[:, 1] >= tt[:, 0])
    check_explicit(g, eg, oracle_explicit(eg, want_payload=False))


def test_residency_calibration(gpu):
    for mapping, ww in [(1, 4), (2, 1), (2, 4), (2, 16)]:
        bpc, cus, resident = tg.tg_exec_occupancy(mapping, ww)
        per_block = 4 if mapping == 1 else 1
        assert 1 <= resident <= bpc * cus * per_block
        assert resident % cus == 0


@pytest.mark.parametrize("seed", range(3))
def test_random_dags_with_duplicates(gpu, seed):
    rng = np.random.default_rng(seed)
    eg = wl.random_dag(600, 6, rng, n=256, rounds=4, seed=seed, dup=True)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    run(g)
    check_explicit(g, eg, ref, payload_sample=50)


def _hub_graph(fan: int, n: int = 128, rounds: int = 2) -> wl.ExplicitGraph:
    """fan sources -> one hub (fan predecessors) -> fan tasks -> one sink
    (fan predecessors): in- and out-degrees far beyond the edges a task
    record holds inline, and beyond one wavefront of signalling lanes."""
    lists = [[] for _ in range(fan)]
    hub = len(lists)
    lists.append(list(range(fan)))
    mid = [len(lists) + i for i in range(fan)]
    lists += [[hub, i % fan] for i in range(fan)]
    lists.append(mid)
    ptr = np.zeros(len(lists) + 1, np.uint64)
    ptr[1:] = np.cumsum([len(x) for x in lists])
    flat = np.array([p for x in lists for p in x], np.uint32)
    return wl.ExplicitGraph(N=len(lists), pred_ptr=ptr, preds=flat, n=n, rounds=rounds, seed=7)


@pytest.mark.parametrize("mapping,wg_waves", [(1, 4), (2, 1), (2, 4)])
@pytest.mark.parametrize("fan", [7, 9, 65, 150])
def test_high_degree_tasks(gpu, fan, mapping, wg_waves):
    eg = _hub_graph(fan)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    run(g, tg.make_config(mapping=mapping, wg_waves=wg_waves))
    check_explicit(g, eg, ref, payload_sample=16)


def test_random_dags_many_predecessors(gpu):
    rng = np.random.default_rng(21)
    eg = wl.random_dag(500, 40, rng, n=64, rounds=3, seed=21, dup=True)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    for m in (1, 2):
        run(g, tg.make_config(mapping=m))
        check_explicit(g, eg, ref, payload_sample=20)


def test_reexecution_is_identical(gpu):
    eg = wl.pattern_graph("stencil", 128, 40, seed=3, n=256, rounds=8)
    ref = oracle_explicit(eg, want_payload=False)
    g = tg.graph_from_explicit(eg)
    for cfg in [None, tg.make_config(mapping=2), None, tg.make_config(window=5)]:
        run(g, cfg)
        check_explicit(g, eg, ref)


def test_edge_cases(gpu):
    # empty graph
    e = tg.graph_from_explicit(wl.ExplicitGraph(N=0, pred_ptr=np.zeros(1, np.uint64), preds=np.zeros(0, np.uint32)))
    run(e)
    assert tg.tg_graph_read_digests(e.handle).size == 0
    # one task; one timestep of sources; maximal payload
    for eg in [wl.pattern_graph("none", 1, 1, n=64, rounds=2),
               wl.pattern_graph("stencil", 300, 1, n=64, rounds=0),
               wl.pattern_graph("stencil", 3, 3, n=65536, rounds=1),
               wl.fig6_graph(n=512, rounds=33)]:
        ref = oracle_explicit(eg)
        g = tg.graph_from_explicit(eg)
        for m in (1, 2):
            run(g, tg.make_config(mapping=m))
            check_explicit(g, eg, ref, payload_sample=8)


def test_per_task_rounds(gpu):
    eg = wl.pattern_graph("stencil", 20, 10, seed=1, n=64)
    R = (np.arange(eg.N) * 7 % 11).astype(np.uint32)
    ref = oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, R, seed=1)
    h = tg.tg_graph_create(tg.TG_EXPLICIT, 64, 0, 1)
    g = tg.Graph(h, tg.TG_EXPLICIT, 64)
    tg.tg_task_add_many(h, eg.pred_ptr, eg.preds, R)
    tg.tg_graph_finalize(h)
    run(g)
    check_explicit(g, eg, ref)


def test_one_at_a_time_api(gpu):
    # the Figure 6 program written with the single-task call
    h = tg.tg_graph_create(tg.TG_EXPLICIT, 64, 0, 0)
    g = tg.Graph(h, tg.TG_EXPLICIT, 64)
    e1 = tg.tg_task_add(h, [], 16)
    e2 = tg.tg_task_add(h, [e1], 16)
    e3 = tg.tg_task_add(h, [e1], 16)
    tg.tg_task_add(h, [e2, e3, e2], 16)
    tg.tg_graph_finalize(h)
    run(g)
    eg = wl.fig6_graph(n=64, rounds=16)
    check_explicit(g, eg, oracle_explicit(eg))


@pytest.mark.parametrize("pattern", wl.PATTERNS)
def test_c2_full_size_r0(gpu, pattern):
    # the benchmark's configuration: 1024 x 1000, n = 256, R = 0 (every digest)
    eg = wl.pattern_graph(pattern, 1024, 1000, seed=0, n=256, rounds=0)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    run(g)
    check_explicit(g, eg, ref, payload_sample=256)


def test_c2_stencil_r16_sampled(gpu):
    # full-size stencil with mixing: every digest vs the oracle
    eg = wl.pattern_graph("stencil", 1024, 1000, seed=0, n=256, rounds=16)
    ref = oracle_explicit(eg, want_payload=False)
    g = tg.graph_from_explicit(eg)
    run(g)
    check_explicit(g, eg, ref)


@pytest.mark.parametrize("mode", [tg.TG_CMP_PER_TASK, tg.TG_CMP_HIPGRAPH, tg.TG_CMP_HIPGRAPH_CAPTURED])
def test_comparators(gpu, mode):
    eg = wl.pattern_graph("random", 24, 10, seed=4, n=256, rounds=3)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    for _ in range(2):
        tg.tg_graph_execute_comparator(g.handle, mode)
        tg.tg_graph_wait(g.handle)
        check_explicit(g, eg, ref, payload_sample=16)


def test_hipgraph_comparator_after_layout_change(gpu):
    """The comparator's hipGraph holds the device addresses of the graph's
    own layout.  A launch in another shape replaces that layout; the next
    hipGraph comparator call must rebuild its graph rather than replay the
    freed addresses."""
    eg = wl.pattern_graph("random", 24, 10, seed=4, n=256, rounds=3)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    for cfg in (tg.make_config(mapping=2, wg_waves=2), tg.make_config(mapping=1, workers=64, schedule=4)):
        tg.tg_graph_execute_comparator(g.handle, tg.TG_CMP_HIPGRAPH)
        tg.tg_graph_wait(g.handle)
        check_explicit(g, eg, ref, payload_sample=16)
        run(g, cfg)
        check_explicit(g, eg, ref, payload_sample=16)
    tg.tg_graph_autotune(g.handle, reps=1)
    tg.tg_graph_execute_comparator(g.handle, tg.TG_CMP_HIPGRAPH)
    tg.tg_graph_wait(g.handle)
    check_explicit(g, eg, ref, payload_sample=16)


def test_watchdog_path_then_recovery(gpu):
    # a chain with long tasks: idle workers exceed a tiny spin limit, the
    # launch aborts cleanly and reports TG_ETIMEOUT; the next execution is
    # correct again
    eg = wl.pattern_graph("stencil", 1, 24, seed=0, n=64, rounds=4096)
    g = tg.graph_from_explicit(eg)
    tg.tg_graph_execute(g.handle, tg.make_config(workers=8, spin_limit=1))
    with pytest.raises(tg.TaskGraphError) as ei:
        tg.tg_graph_wait(g.handle)
    assert ei.value.status == tg.TG_ETIMEOUT
    run(g)
    check_explicit(g, eg, oracle_explicit(eg))


@pytest.mark.parametrize("gang,wg_waves", [(2, 1), (3, 4), (8, 16), (32, 1)])
@pytest.mark.parametrize("n", [64, 1024, 65536])
def test_patterns_gangs(gpu, n, gang, wg_waves):
    """Explicit graphs with a gang of workgroups per task: payload words are
    split over the whole gang (a gang wider than the payload leaves members
    idle), digests summed from the members' parts."""
    for pattern in ("stencil", "random"):
        eg = wl.pattern_graph(pattern, 13 if n == 65536 else 37, 5 if n == 65536 else 11, seed=4, n=n, rounds=2)
        ref = oracle_explicit(eg)
        g = tg.graph_from_explicit(eg)
        run(g, tg.make_config(mapping=3, gang=gang, wg_waves=wg_waves))
        check_explicit(g, eg, ref, payload_sample=8)
        run(g, tg.make_config(mapping=3, gang=gang, wg_waves=wg_waves, workers=1, window=3))
        check_explicit(g, eg, ref)


def test_gang_watchdog_path_then_recovery(gpu):
    # as the single-team test: the abort reaches every member of every gang
    eg = wl.pattern_graph("stencil", 1, 24, seed=0, n=64, rounds=4096)
    g = tg.graph_from_explicit(eg)
    tg.tg_graph_execute(g.handle, tg.make_config(mapping=3, gang=4, wg_waves=4, workers=8, spin_limit=1))
    with pytest.raises(tg.TaskGraphError) as ei:
        tg.tg_graph_wait(g.handle)
    assert ei.value.status == tg.TG_ETIMEOUT
    run(g, tg.make_config(mapping=3, gang=4, wg_waves=4))
    check_explicit(g, eg, oracle_explicit(eg))


def test_external_pre_and_post_conditions(gpu):
    # graph B may start only after graph A's post-condition event; B runs on
    # another stream; both results stay bit-exact
    import torch
    ea = wl.pattern_graph("stencil", 64, 40, seed=1, n=256, rounds=50)
    eb = wl.pattern_graph("fft", 64, 30, seed=2, n=128, rounds=5)
    ga, gb = tg.graph_from_explicit(ea), tg.graph_from_explicit(eb)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a_done = torch.cuda.Event(enable_timing=True)
    b_done = torch.cuda.Event(enable_timing=True)
    gate = torch.cuda.Event(enable_timing=True)
    gate.record(s1)
    tg.tg_graph_execute_after(ga.handle, pre_events=[gate], post_event=a_done, stream=s1)
    tg.tg_graph_execute_after(gb.handle, pre_events=[a_done], post_event=b_done, stream=s2)
    b_done.synchronize()
    assert a_done.query() and b_done.query()
    assert gate.elapsed_time(a_done) > 0 and a_done.elapsed_time(b_done) > 0
    tg.tg_graph_wait(ga.handle)
    tg.tg_graph_wait(gb.handle)
    check_explicit(ga, ea, oracle_explicit(ea, want_payload=False))
    check_explicit(gb, eb, oracle_explicit(eb, want_payload=False))
