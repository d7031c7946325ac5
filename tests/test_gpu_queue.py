"""The ready-queue dispatch (TG_DISPATCH_QUEUE): the decrement that empties a
counter makes its task ready, the finishing worker keeps one ready successor
and pushes the rest into its shard, idle workers claim tiles of tickets.
Results must equal the oracle's for every pattern, both worker mappings,
every tile size and shard count, in batches, for implicit graphs, with
payload-slot reuse, and for any worker count (the queue needs no
co-residency)."""
import numpy as np
import pytest

import oracle
from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests.gpu_util import check_explicit, oracle_explicit, run

pytestmark = pytest.mark.gpu

Q = tg.TG_DISPATCH_QUEUE


def qcfg(mapping=1, tile=1, shards=8, **kw):
    return tg.make_config(mapping=mapping, dispatch=Q, tile=tile, shards=shards, **kw)


@pytest.mark.parametrize("tile,shards", [(1, 8), (4, 8), (16, 2), (64, 1)])
@pytest.mark.parametrize("mapping", [1, 2])
@pytest.mark.parametrize("pattern", wl.PATTERNS)
def test_patterns(gpu, pattern, mapping, tile, shards):
    # 48 lanes (not a power of two: FFT partners past the width are dropped,
    # the tree has inactive lanes) x 20 timesteps, 256-word payloads
    eg = wl.pattern_graph(pattern, 48, 20, seed=3, n=256, rounds=3)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    for _ in range(2):  # the second run finds the previous launch's queue state
        run(g, qcfg(mapping, tile, shards, wg_waves=4))
        check_explicit(g, eg, ref, payload_sample=8)


@pytest.mark.parametrize("workers", [1, 3, 64, 5000])
def test_worker_counts(gpu, workers):
    # one worker runs the whole graph alone; more workers than tasks idle
    eg = wl.pattern_graph("random", 32, 12, seed=1, n=64, rounds=2)
    ref = oracle_explicit(eg)
    g = tg.graph_from_explicit(eg)
    run(g, qcfg(1, 4, 8, workers=workers))
    check_explicit(g, eg, ref, payload_sample=8)


def test_stencil_full_width(gpu):
    # the 1024-wide stencil, 100 timesteps, in the launch the autotuner tries
    eg = wl.pattern_graph("stencil", 1024, 100, seed=0, n=256, rounds=0)
    ref = oracle_explicit(eg, want_payload=False)
    g = tg.graph_from_explicit(eg)
    for tile in (1, 4):
        run(g, qcfg(1, tile, 8))
        check_explicit(g, eg, ref)


def test_chain_and_sources_only(gpu):
    # a chain (every completion makes exactly one task ready: it is kept, the
    # queue only ever holds the source) and a graph of sources only
    for eg in (wl.pattern_graph("stencil", 1, 300, seed=2, n=64, rounds=5),
               wl.pattern_graph("none", 300, 1, seed=2, n=64, rounds=5)):
        ref = oracle_explicit(eg)
        g = tg.graph_from_explicit(eg)
        run(g, qcfg(1, 1, 8))
        check_explicit(g, eg, ref)


@pytest.mark.parametrize("mapping", [1, 2])
def test_implicit(gpu, mapping):
    ig = wl.halo_graph(33, 256, 3, seed=2, rounds=3)
    ref = oracle.implicit_program_order(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv, ig.rounds, ig.space, seed=ig.seed)
    g = tg.graph_from_implicit(ig)
    run(g, qcfg(mapping, 4, 8))
    assert np.array_equal(tg.tg_graph_read_data(g.handle, 0, ig.space), ref["A"])
    assert np.array_equal(tg.tg_graph_read_digests(g.handle), ref["digest"])
    assert tg.tg_graph_checksum(g.handle) == ref["checksum"]


@pytest.mark.parametrize("retention", [tg.TG_KEEP_SINKS, tg.TG_KEEP_NONE])
def test_payload_slot_reuse(gpu, retention):
    eg = wl.pattern_graph("fft", 64, 24, seed=5, n=128, rounds=2)
    ref = oracle_explicit(eg, want_payload=False)
    g = tg.graph_from_explicit(eg, retention=retention)
    run(g, qcfg(1, 4, 8))
    check_explicit(g, eg, ref)


@pytest.mark.parametrize("mapping", [1, 2])
def test_batch(gpu, mapping):
    specs = wl.batch_manifest(24, seed=3, wmax=64, tmax=32)
    egs = [wl.pattern_graph(s.pattern, s.W, s.T, seed=s.seed, n=s.n, rounds=min(s.rounds, 300)) for s in specs]
    ig = wl.halo_graph(16, 128, 6, seed=5, rounds=3)
    gs = [tg.graph_from_explicit(eg) for eg in egs]
    gi = tg.graph_from_implicit(ig)
    b = tg.tg_batch_create([g.handle for g in gs] + [gi.handle], qcfg(mapping, 4, 8, wg_waves=4))
    try:
        for _ in range(2):
            tg.tg_batch_execute(b)
            tg.tg_batch_wait(b)
            for g, eg in zip(gs, egs):
                check_explicit(g, eg, oracle_explicit(eg), payload_sample=4)
            ref = oracle.implicit_program_order(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv, ig.rounds, ig.space, seed=5)
            assert np.array_equal(tg.tg_graph_read_data(gi.handle, 0, ig.space), ref["A"])
            assert np.array_equal(tg.tg_graph_read_digests(gi.handle), ref["digest"])
    finally:
        tg.tg_batch_destroy(b)


def test_gang_mapping_refused(gpu):
    eg = wl.pattern_graph("stencil", 8, 4, seed=0, n=64)
    g = tg.graph_from_explicit(eg)
    with pytest.raises(tg.TaskGraphError) as ei:
        run(g, tg.make_config(mapping=3, gang=2, dispatch=Q))
    assert ei.value.status == tg.TG_EINVAL
