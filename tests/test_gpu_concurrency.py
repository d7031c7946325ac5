"""Long critical paths and concurrent persistent launches.

- The watchdog aborts a launch only when no task has started anywhere for
  its interval: a chain whose total run time is several watchdog intervals,
  during which almost every worker waits, completes bit-exact.
- Persistent launches issued on different streams never oversubscribe the
  device: a launch that does not fit beside the ones in flight follows them
  in stream order (the residency ledger), so launches at full residency on
  two streams at once, of the same or of different kernel variants, both
  complete bit-exact.  Every wait in these kernels is bounded by the
  watchdog, so a failure shows as TG_ETIMEOUT, not as a hang."""
import numpy as np
import pytest

from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests.gpu_util import check_explicit, oracle_explicit

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kw,n", [(dict(mapping=1), 16384), (dict(mapping=2, wg_waves=4), 65536),
                                  (dict(mapping=3, gang=2, wg_waves=4), 65536)],
                         ids=["wave", "workgroup", "gang"])
def test_long_chain_outlives_watchdog(gpu, kw, n):
    # 120 dependent tasks of n words x 256 rounds (well under a millisecond
    # to a few milliseconds each): the chain runs many 5 ms watchdog
    # intervals while every other worker waits for its only task
    eg = wl.pattern_graph("stencil", 1, 120, seed=3, n=n, rounds=256)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    cfg = tg.make_config(watchdog_ms=5, **kw)
    tg.tg_graph_execute(g.handle, cfg)
    tg.tg_graph_wait(g.handle)
    kms = tg.tg_graph_kernel_ms(g.handle)
    assert kms > 20, f"the chain ran {kms:.1f} ms: too short to exercise the watchdog"
    check_explicit(g, eg, ref, payload_sample=8)


def _pair(seed_a, seed_b, W=512, T=60, rounds=40):
    ea = wl.pattern_graph("stencil", W, T, seed=seed_a, n=256, rounds=rounds)
    eb = wl.pattern_graph("random", W, T, seed=seed_b, n=256, rounds=rounds)
    return ea, eb


def _span(g):
    """(first task start, last task end) of the graph's last diagnostic
    launch, in device clock ticks."""
    t, _ = tg.tg_graph_debug_times(g.handle)
    assert (t[:, 0] > 0).all() and (t[:, 1] >= t[:, 0]).all()
    return int(t[:, 0].min()), int(t[:, 1].max())


def _run_pair(ga, gb, ca, cb):
    import torch
    for g, c in ((ga, ca), (gb, cb)):  # build both layouts first
        tg.tg_graph_execute(g.handle, c)
        tg.tg_graph_wait(g.handle)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    tg.tg_graph_execute(ga.handle, ca, s1)
    tg.tg_graph_execute(gb.handle, cb, s2)
    tg.tg_graph_wait(ga.handle)
    tg.tg_graph_wait(gb.handle)
    return _span(ga), _span(gb)


@pytest.mark.parametrize("cfg_a,cfg_b", [
    (dict(mapping=1), dict(mapping=1)),
    (dict(mapping=1), dict(mapping=2, wg_waves=4)),
    (dict(mapping=2, wg_waves=2), dict(mapping=3, gang=2, wg_waves=4)),
], ids=["wave+wave", "wave+workgroup", "workgroup+gang"])
def test_full_residency_launches_on_two_streams(gpu, cfg_a, cfg_b):
    """Two launches at full residency issued on two streams at once: the
    second follows the first (their task spans do not overlap) and both are
    bit-exact."""
    ea, eb = _pair(1, 2)
    ga, gb = tg.graph_from_explicit(ea), tg.graph_from_explicit(eb)
    ca = tg.make_config(watchdog_ms=3000, diag=1, **cfg_a)
    cb = tg.make_config(watchdog_ms=3000, diag=1, **cfg_b)
    for _ in range(2):
        (a0, a1), (b0, b1) = _run_pair(ga, gb, ca, cb)
        assert b0 >= a1 or a0 >= b1, "full-residency launches overlapped"
        check_explicit(ga, ea, oracle_explicit(ea, want_payload=False))
        check_explicit(gb, eb, oracle_explicit(eb, want_payload=False))


def test_half_residency_launches_overlap(gpu):
    """Two launches of one variant whose workers fit together run at the
    same time (their task spans overlap), bit-exact."""
    ea, eb = _pair(3, 4, W=512, T=40, rounds=150)
    ga, gb = tg.graph_from_explicit(ea), tg.graph_from_explicit(eb)
    _, _, resident = tg.tg_exec_occupancy(tg.TG_MAP_WAVE, 4)
    c = tg.make_config(mapping=1, workers=resident // 2, watchdog_ms=3000, diag=1)
    (a0, a1), (b0, b1) = _run_pair(ga, gb, c, c)
    assert b0 < a1 and a0 < b1, "launches that fit together did not overlap"
    check_explicit(ga, ea, oracle_explicit(ea, want_payload=False))
    check_explicit(gb, eb, oracle_explicit(eb, want_payload=False))


def test_graph_beside_server(gpu):
    """A full-residency graph launch on the caller's stream while the server
    runs requests on its own streams: all results bit-exact."""
    import torch
    reqs = wl.serving_manifest(16, rate=4000.0, seed=11, median=400, max_tasks=3000)
    for r in reqs:
        r.rounds = min(r.rounds, 100)
    graphs = [wl.build_request(r) for r in reqs]
    handles = [tg.graph_from_implicit(x) if isinstance(x, wl.ImplicitGraph) else tg.graph_from_explicit(x)
               for x in graphs]
    ea, _ = _pair(5, 6)
    ga = tg.graph_from_explicit(ea)
    s = torch.cuda.Stream()
    srv = tg.tg_server_create(4 << 30, slots=4, max_batch=4)
    try:
        tickets = [tg.tg_server_submit(srv, h.handle) for h in handles[:8]]
        tg.tg_graph_execute(ga.handle, tg.make_config(watchdog_ms=3000), s)
        tickets += [tg.tg_server_submit(srv, h.handle) for h in handles[8:]]
        for t in tickets:
            tg.tg_server_wait(srv, t)
        tg.tg_graph_wait(ga.handle)
    finally:
        tg.tg_server_destroy(srv)
    check_explicit(ga, ea, oracle_explicit(ea, want_payload=False))
    import oracle
    for x, h in zip(graphs, handles):
        if isinstance(x, wl.ImplicitGraph):
            ref = oracle.implicit_program_order(x.N, x.req_ptr, x.lo, x.hi, x.priv, x.rounds, x.space, seed=x.seed)
        else:
            ref = oracle.exec_explicit(x.N, x.n, x.pred_ptr, x.preds, x.rounds, seed=x.seed, want_payload=False)
        assert np.array_equal(tg.tg_graph_read_digests(h.handle), ref["digest"])
