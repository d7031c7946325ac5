"""Serving (continuous batching): graphs submitted while others run are
admitted by device-memory budget into overlapping persistent launches; every
result is bit-identical to the oracle and to running the graph alone."""
import threading
import time

import numpy as np
import pytest

import oracle
from bench_workloads import request_graph
from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _ref(graph):
    if isinstance(graph, wl.ImplicitGraph):
        return oracle.implicit_program_order(graph.N, graph.req_ptr, graph.lo, graph.hi, graph.priv, graph.rounds,
                                             graph.space, seed=graph.seed)
    return oracle.exec_explicit(graph.N, graph.n, graph.pred_ptr, graph.preds, graph.rounds, seed=graph.seed,
                                want_payload=False)


def _small_requests(num, seed=0):
    reqs = wl.serving_manifest(num, rate=2000.0, seed=seed, median=400, max_tasks=4000)
    for r in reqs:
        r.rounds = min(r.rounds, 200)
    return reqs


def _build(reqs, form="plain"):
    """plain: every payload kept, implicit graphs on their full inferred DAG;
    compact: the benchmark's form (payload memory reused once read, keeping
    the sinks'; implicit graphs on their reduced DAG)."""
    graphs = [wl.build_request(r) for r in reqs]
    if form == "compact":
        handles = [request_graph(x) for x in graphs]
    else:
        handles = [tg.graph_from_implicit(x) if isinstance(x, wl.ImplicitGraph) else tg.graph_from_explicit(x)
                   for x in graphs]
    return graphs, handles


SERVER_CONFIGS = {
    "queue": None,  # the default: ready queue, records built on the device
    "queue-wg4-tile4": tg.make_config(mapping=2, wg_waves=4, dispatch=tg.TG_DISPATCH_QUEUE, tile=4, shards=2),
    "lists": tg.make_config(dispatch=tg.TG_DISPATCH_LISTS),
}


@pytest.mark.parametrize("config", list(SERVER_CONFIGS))
@pytest.mark.parametrize("slots,max_batch,form", [(4, 8, "plain"), (1, 1, "plain"), (2, 64, "plain"),
                                                  (4, 8, "compact"), (2, 64, "compact")])
def test_mix_equals_alone_and_oracle(gpu, slots, max_batch, form, config):
    reqs = _small_requests(40, seed=slots + (10 if form == "compact" else 0))
    graphs, handles = _build(reqs, form)
    srv = tg.tg_server_create(8 << 30, slots=slots, max_batch=max_batch)
    if SERVER_CONFIGS[config] is not None:
        tg.tg_server_configure(srv, SERVER_CONFIGS[config])
    try:
        # submit following the arrival times, from another thread
        tickets = [None] * len(reqs)

        def client():
            t0 = time.perf_counter()
            for i, r in enumerate(reqs):
                dt = r.arrival_s - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = tg.tg_server_submit(srv, handles[i].handle)

        th = threading.Thread(target=client)
        th.start()
        th.join()
        times = [tg.tg_server_wait(srv, t) for t in tickets]
        stats = tg.tg_server_stats(srv)
    finally:
        tg.tg_server_destroy(srv)
    assert stats["tasks_done"] == sum(x.N for x in graphs)
    for (s, a, d) in times:
        assert s <= a <= d
    for x, h in zip(graphs, handles):
        ref = _ref(x)
        assert np.array_equal(tg.tg_graph_read_digests(h.handle), ref["digest"])
        assert tg.tg_graph_checksum(h.handle) == ref["checksum"]
    # the same graphs alone, one at a time
    for x, h in list(zip(graphs, handles))[:10]:
        tg.tg_graph_execute(h.handle)
        tg.tg_graph_wait(h.handle)
        assert np.array_equal(tg.tg_graph_read_digests(h.handle), _ref(x)["digest"])


def test_budget_admission(gpu):
    # a budget that fits about one request at a time still completes them all,
    # and a request larger than the whole budget is refused
    reqs = _small_requests(12, seed=9)
    graphs, handles = _build(reqs)
    big = wl.pattern_graph("stencil", 256, 128, seed=1, n=1024, rounds=0)
    hb = tg.graph_from_explicit(big)
    srv = tg.tg_server_create(64 << 20, slots=2, max_batch=4)
    try:
        tickets = [tg.tg_server_submit(srv, h.handle) for h in handles]
        tb = tg.tg_server_submit(srv, hb.handle)
        for t in tickets:
            tg.tg_server_wait(srv, t)
        with pytest.raises(tg.TaskGraphError) as ei:
            tg.tg_server_wait(srv, tb)
        assert ei.value.status == tg.TG_ENOMEM
        assert tg.tg_server_stats(srv)["peak_bytes"] <= 64 << 20
    finally:
        tg.tg_server_destroy(srv)
    for x, h in zip(graphs, handles):
        assert np.array_equal(tg.tg_graph_read_digests(h.handle), _ref(x)["digest"])


def test_resubmit_while_pending_is_refused(gpu):
    # a graph can be in one unfinished request at a time; once that request
    # finished it can be served again, with the same result
    reqs = _small_requests(2, seed=3)
    graphs, handles = _build(reqs)
    # one slot, batches of one: a slow graph first keeps handles[0] pending
    slow = wl.pattern_graph("stencil", 64, 50, seed=4, n=256, rounds=1024)
    hs = tg.graph_from_explicit(slow)
    srv = tg.tg_server_create(8 << 30, slots=1, max_batch=1)
    try:
        ts = tg.tg_server_submit(srv, hs.handle)
        t0 = tg.tg_server_submit(srv, handles[0].handle)
        with pytest.raises(tg.TaskGraphError) as ei:
            tg.tg_server_submit(srv, handles[0].handle)
        assert ei.value.status == tg.TG_EBUSY
        t1 = tg.tg_server_submit(srv, handles[1].handle)
        for t in (ts, t0, t1):
            tg.tg_server_wait(srv, t)
        t2 = tg.tg_server_submit(srv, handles[0].handle)
        tg.tg_server_wait(srv, t2)
    finally:
        tg.tg_server_destroy(srv)
    for x, h in zip(graphs, handles):
        assert np.array_equal(tg.tg_graph_read_digests(h.handle), _ref(x)["digest"])
    assert np.array_equal(tg.tg_graph_read_digests(hs.handle), _ref(slow)["digest"])


def test_hipgraph_comparator_after_serving(gpu):
    """A served request releases the graph's device memory and layout; the
    hipGraph comparator built before the request must not be replayed."""
    eg = wl.pattern_graph("fft", 16, 12, seed=2, n=128, rounds=4)
    h = tg.graph_from_explicit(eg)
    ref = _ref(eg)
    tg.tg_graph_execute_comparator(h.handle, tg.TG_CMP_HIPGRAPH)
    tg.tg_graph_wait(h.handle)
    assert np.array_equal(tg.tg_graph_read_digests(h.handle), ref["digest"])
    srv = tg.tg_server_create(1 << 30, slots=1, max_batch=1)
    try:
        tg.tg_server_wait(srv, tg.tg_server_submit(srv, h.handle))
    finally:
        tg.tg_server_destroy(srv)
    assert np.array_equal(tg.tg_graph_read_digests(h.handle), ref["digest"])
    tg.tg_graph_execute_comparator(h.handle, tg.TG_CMP_HIPGRAPH)
    tg.tg_graph_wait(h.handle)
    assert np.array_equal(tg.tg_graph_read_digests(h.handle), ref["digest"])
    assert tg.tg_graph_checksum(h.handle) == ref["checksum"]


def test_configure_refuses_gangs(gpu):
    srv = tg.tg_server_create(1 << 30, slots=1, max_batch=1)
    try:
        with pytest.raises(tg.TaskGraphError) as ei:
            tg.tg_server_configure(srv, tg.make_config(mapping=3, gang=2))
        assert ei.value.status == tg.TG_EINVAL
    finally:
        tg.tg_server_destroy(srv)


def test_slot_layout_reused_across_batch_sizes(gpu):
    """One slot serves batches that grow and shrink (its device-built layout
    keeps and grows its buffers, and empties the queue slots of the previous
    batch): every request of every batch equals the oracle."""
    sizes = [(8, 4), (64, 40), (16, 8), (128, 60), (8, 2)]
    srv = tg.tg_server_create(8 << 30, slots=1, max_batch=64)
    try:
        for k, (W, T) in enumerate(sizes):
            egs = [wl.pattern_graph(p, W, T, seed=10 * k + i, n=64, rounds=3) for i, p in enumerate(wl.PATTERNS)]
            hs = [tg.graph_from_explicit(eg) for eg in egs]
            for t in [tg.tg_server_submit(srv, h.handle) for h in hs]:
                tg.tg_server_wait(srv, t)
            for eg, h in zip(egs, hs):
                ref = _ref(eg)
                assert np.array_equal(tg.tg_graph_read_digests(h.handle), ref["digest"]), (W, T, eg.N)
                assert tg.tg_graph_checksum(h.handle) == ref["checksum"]
    finally:
        tg.tg_server_destroy(srv)
