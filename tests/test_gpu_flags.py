"""Condition flags (Section 4.1 pre- and post-condition vertices met by the
host or by another graph, without stream ordering): a gated graph runs only
once its flags hold, sets its post-condition flag when it has finished, and
gives up after the watchdog interval when a flag is never set; every result
stays bit-exact against the oracle."""
import time

import pytest

from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests.gpu_util import check_explicit, oracle_explicit

pytestmark = pytest.mark.gpu

CONFIGS = {
    "wave-lists": dict(mapping=1, workers=64),
    "block-lists": dict(mapping=2, wg_waves=4, workers=16),
    "gang": dict(mapping=3, gang=2, wg_waves=2, workers=8),
    "wave-queue": dict(mapping=1, workers=64, dispatch=tg.TG_DISPATCH_QUEUE, tile=2),
}


@pytest.fixture
def flags():
    made = []

    def make(k):
        fs = [tg.tg_flag_create() for _ in range(k)]
        made.extend(fs)
        return fs
    yield make
    for f in made:
        tg.tg_flag_destroy(f)


@pytest.mark.parametrize("config", list(CONFIGS))
def test_host_flag_gates_the_graph(gpu, flags, config):
    eg = wl.pattern_graph("stencil", 32, 20, seed=4, n=128, rounds=4)
    g = tg.graph_from_explicit(eg)
    pre, post = flags(2)
    tg.tg_graph_execute_when(g.handle, [pre], [3], post=post, post_value=9, cfg=tg.make_config(**CONFIGS[config]))
    time.sleep(0.2)
    assert tg.tg_flag_read(post) == 0  # nothing ran yet
    tg.tg_flag_set(pre, 2)  # below the condition
    time.sleep(0.1)
    assert tg.tg_flag_read(post) == 0
    tg.tg_flag_set(pre, 3)
    tg.tg_flag_wait(post, 9, 5000)
    tg.tg_graph_wait(g.handle)
    check_explicit(g, eg, oracle_explicit(eg, want_payload=False))


@pytest.mark.parametrize("consumer_first", [False, True])
def test_post_flag_gates_a_graph_on_another_stream(gpu, flags, consumer_first):
    """Graph B waits on graph A's post-condition flag from another stream.
    Both launches fit beside each other, so either may be issued first."""
    import torch
    ea = wl.pattern_graph("random", 48, 30, seed=1, n=256, rounds=20)
    eb = wl.pattern_graph("tree", 40, 25, seed=2, n=64, rounds=3)
    ga, gb = tg.graph_from_explicit(ea), tg.graph_from_explicit(eb)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    start, a_done, b_done = flags(3)
    cfg = tg.make_config(mapping=1, workers=128)

    def launch_a():
        tg.tg_graph_execute_when(ga.handle, [start], [1], post=a_done, post_value=5, cfg=cfg, stream=s1)

    def launch_b():
        tg.tg_graph_execute_when(gb.handle, [a_done], [5], post=b_done, post_value=1, cfg=cfg, stream=s2)

    if consumer_first:
        launch_b()
        launch_a()
    else:
        launch_a()
        launch_b()
    time.sleep(0.1)
    assert tg.tg_flag_read(a_done) == 0 and tg.tg_flag_read(b_done) == 0
    tg.tg_flag_set(start, 1)
    tg.tg_flag_wait(b_done, 1, 5000)
    assert tg.tg_flag_read(a_done) == 5  # B ran only after A had finished
    tg.tg_graph_wait(ga.handle)
    tg.tg_graph_wait(gb.handle)
    check_explicit(ga, ea, oracle_explicit(ea, want_payload=False))
    check_explicit(gb, eb, oracle_explicit(eb, want_payload=False))


@pytest.mark.parametrize("config", ["wave-lists", "wave-queue"])
def test_unmet_flag_times_out_then_graph_runs(gpu, flags, config):
    """A flag the host never sets: the bounded wait gives up, no task runs,
    the post-condition stays unset and the error names the flag; the graph
    then executes normally."""
    eg = wl.pattern_graph("fft", 16, 12, seed=3, n=64, rounds=2)
    g = tg.graph_from_explicit(eg)
    f0, f1, post = flags(3)
    tg.tg_flag_set(f0, 1)
    cfg = tg.make_config(watchdog_ms=50, **CONFIGS[config])
    tg.tg_graph_execute_when(g.handle, [f0, f1], [1, 1], post=post, post_value=1, cfg=cfg)
    with pytest.raises(tg.TaskGraphError) as ei:
        tg.tg_graph_wait(g.handle)
    assert ei.value.status == tg.TG_ETIMEOUT and "flag 1" in str(ei.value)
    assert tg.tg_flag_read(post) == 0
    tg.tg_graph_execute(g.handle, tg.make_config(**CONFIGS[config]))
    tg.tg_graph_wait(g.handle)
    check_explicit(g, eg, oracle_explicit(eg, want_payload=False))
    # and gated again, with the flag met before the launch
    tg.tg_flag_set(f1, 1)
    tg.tg_graph_execute_when(g.handle, [f0, f1], [1, 1], post=post, post_value=2, cfg=cfg)
    tg.tg_graph_wait(g.handle)
    assert tg.tg_flag_read(post) == 2
    check_explicit(g, eg, oracle_explicit(eg, want_payload=False))


def test_flag_host_calls(gpu, flags):
    (f,) = flags(1)
    assert tg.tg_flag_read(f) == 0
    tg.tg_flag_set(f, 41)
    assert tg.tg_flag_read(f) == 41
    tg.tg_flag_wait(f, 41, 10)
    with pytest.raises(tg.TaskGraphError) as ei:
        tg.tg_flag_wait(f, 42, 20)
    assert ei.value.status == tg.TG_ETIMEOUT
