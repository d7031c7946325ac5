"""Implicit (region requirement) graphs on the GPU: the inferred DAG equals
the brute-force conflict DAG, and execution equals sequential program order."""
import numpy as np
import pytest

import oracle
from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests import _checks as C
from tests.gpu_util import run

pytestmark = pytest.mark.gpu


def _check_dag(g, ig):
    row_ptr, col = tg.tg_graph_read_dag(g.handle)
    ref_ptr, ref_col = oracle.conflict_dag(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv)
    assert np.array_equal(row_ptr, ref_ptr)
    assert np.array_equal(col, ref_col)


def _check_exec(g, ig, ref):
    A = tg.tg_graph_read_data(g.handle, 0, ig.space)
    bad = np.nonzero(A != ref["A"])[0]
    assert bad.size == 0, f"{bad.size} elements differ, first {bad[:5]}"
    assert np.array_equal(tg.tg_graph_read_digests(g.handle), ref["digest"])
    assert tg.tg_graph_checksum(g.handle) == ref["checksum"]


def _ref(ig):
    return oracle.implicit_program_order(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv, ig.rounds, ig.space, seed=ig.seed)


@pytest.mark.parametrize("mapping", [1, 2])
@pytest.mark.parametrize("P,S,iters", [(8, 128, 4), (5, 64, 7), (33, 256, 3)])
def test_halo_small(gpu, P, S, iters, mapping):
    ig = wl.halo_graph(P, S, iters, seed=2, rounds=3)
    g = tg.graph_from_implicit(ig)
    _check_dag(g, ig)
    run(g, tg.make_config(mapping=mapping))
    _check_exec(g, ig, _ref(ig))


@pytest.mark.parametrize("seed", range(4))
def test_random_regions(gpu, seed):
    rng = np.random.default_rng(seed)
    ig = wl.random_regions(80, 300, 4, 40, rng, rounds=2, seed=seed)
    g = tg.graph_from_implicit(ig)
    _check_dag(g, ig)
    for m in (1, 2):
        run(g, tg.make_config(mapping=m))
        _check_exec(g, ig, _ref(ig))


def test_long_rows_sorted(gpu):
    # one writer, then 9000 readers of the same word: row 0 has 9000 successors
    # (longer than the LDS-staged sort) and must come back ascending
    N = 9001
    req_ptr = np.arange(N + 1, dtype=np.uint64)
    lo = np.zeros(N, np.uint64)
    hi = np.ones(N, np.uint64)
    priv = np.full(N, 1, np.uint32)
    priv[0] = 2
    ig = wl.ImplicitGraph(N=N, req_ptr=req_ptr, lo=lo, hi=hi, priv=priv, space=4, rounds=1)
    g = tg.graph_from_implicit(ig)
    row_ptr, col = tg.tg_graph_read_dag(g.handle)
    assert int(row_ptr[1]) == N - 1 and np.array_equal(col, np.arange(1, N, dtype=np.uint32))
    run(g)
    _check_exec(g, ig, _ref(ig))


def test_halo_program_dag_full_size(gpu):
    # 2^16 tasks over 2^24 elements in 1024 subregions, halos 1..64
    ig = wl.halo_graph(1024, 16384, 64, seed=0, rounds=64)
    g = tg.graph_from_implicit(ig)
    row_ptr, col = tg.tg_graph_read_dag(g.handle)
    assert col.size == C.halo_edge_count(1024, 64) == 6254592
    rng = np.random.default_rng(0)
    rows = list(rng.integers(0, ig.N, size=300)) + [0, 1023, 1024, ig.N - 1]
    for j in rows:
        want = oracle.conflict_row(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv, int(j))
        assert np.array_equal(col[int(row_ptr[j]):int(row_ptr[j + 1])], want), f"row {j}"


def test_halo_program_execution_r0(gpu):
    ig = wl.halo_graph(1024, 16384, 64, seed=0, rounds=0)
    g = tg.graph_from_implicit(ig)
    run(g, tg.make_config(mapping=2))
    _check_exec(g, ig, _ref(ig))


def test_halo_program_r64_four_sweeps(gpu):
    ig = wl.halo_graph(1024, 16384, 4, seed=0, rounds=64)
    g = tg.graph_from_implicit(ig)
    run(g, tg.make_config(mapping=2))
    _check_exec(g, ig, _ref(ig))


@pytest.mark.parametrize("mode", [tg.TG_CMP_PER_TASK, tg.TG_CMP_HIPGRAPH, tg.TG_CMP_HIPGRAPH_CAPTURED])
def test_comparators_implicit(gpu, mode):
    ig = wl.halo_graph(6, 128, 3, seed=1, rounds=2)
    g = tg.graph_from_implicit(ig)
    tg.tg_graph_execute_comparator(g.handle, mode)
    tg.tg_graph_wait(g.handle)
    _check_exec(g, ig, _ref(ig))


GANGS = [dict(mapping=3, wg_waves=1, gang=2), dict(mapping=3, wg_waves=4, gang=3), dict(mapping=3, wg_waves=16, gang=8),
         dict(mapping=3, wg_waves=4, gang=16), dict(mapping=3, wg_waves=2, gang=32)]


@pytest.mark.parametrize("kw", GANGS, ids=["g2w1", "g3w4", "g8w16", "g16w4", "g32w2"])
@pytest.mark.parametrize("P,S,iters", [(8, 128, 4), (33, 256, 3)])
def test_halo_small_gangs(gpu, P, S, iters, kw):
    """A gang of workgroups on several CUs per task: the read-write elements
    are split over the gang, the digest is the sum of the members' parts."""
    ig = wl.halo_graph(P, S, iters, seed=2, rounds=3)
    g = tg.graph_from_implicit(ig)
    run(g, tg.make_config(**kw))
    _check_exec(g, ig, _ref(ig))


@pytest.mark.parametrize("seed", range(2))
def test_random_regions_gangs(gpu, seed):
    rng = np.random.default_rng(seed)
    ig = wl.random_regions(80, 300, 4, 40, rng, rounds=2, seed=seed)
    g = tg.graph_from_implicit(ig)
    for kw in GANGS:
        run(g, tg.make_config(**kw))
        _check_exec(g, ig, _ref(ig))


def test_halo_program_r64_gangs(gpu):
    """The halo program's (1024 subregions of 16,384 elements) first four sweeps at R = 64 with gangs of eight
    16-wave workgroups: the whole array and every digest bit-exact."""
    ig = wl.halo_graph(1024, 16384, 4, seed=0, rounds=64)
    g = tg.graph_from_implicit(ig)
    run(g, tg.make_config(mapping=3, wg_waves=16, gang=8))
    _check_exec(g, ig, _ref(ig))


@pytest.mark.parametrize("seed", range(3))
def test_reduced_dag_execution(gpu, seed):
    """Execution on the two-hop-reduced DAG gives the program-order result;
    the inferred DAG read back is still the full conflict DAG."""
    ig = wl.random_regions(80, 300, 4, 40, np.random.default_rng(seed), rounds=2, seed=seed)
    g = tg.graph_from_implicit(ig)
    full = tg.tg_graph_num_edges(g.handle)
    removed = tg.tg_graph_reduce_edges(g.handle)
    assert 0 < removed < full
    _check_dag(g, ig)
    for kw in [dict(mapping=1), dict(mapping=2), dict(mapping=3, gang=2, wg_waves=1)]:
        run(g, tg.make_config(**kw))
        _check_exec(g, ig, _ref(ig))


def test_halo_program_reduced_r64(gpu):
    ig = wl.halo_graph(1024, 16384, 4, seed=0, rounds=64)
    g = tg.graph_from_implicit(ig)
    full = tg.tg_graph_num_edges(g.handle)
    removed = tg.tg_graph_reduce_edges(g.handle)
    assert full - removed == 1023 * (2 * 4 - 1)  # exact transitive reduction of the halo program
    run(g, tg.make_config(mapping=3, wg_waves=8, gang=8))
    _check_exec(g, ig, _ref(ig))


def test_hipgraph_comparator_after_reduction(gpu):
    """Reducing the executed DAG replaces the graph's layout; the hipGraph
    comparator built before must not be replayed afterwards."""
    ig = wl.halo_graph(6, 128, 3, seed=1, rounds=2)
    g = tg.graph_from_implicit(ig)
    tg.tg_graph_execute_comparator(g.handle, tg.TG_CMP_HIPGRAPH)
    tg.tg_graph_wait(g.handle)
    _check_exec(g, ig, _ref(ig))
    assert tg.tg_graph_reduce_edges(g.handle) > 0
    tg.tg_graph_execute_comparator(g.handle, tg.TG_CMP_HIPGRAPH)
    tg.tg_graph_wait(g.handle)
    _check_exec(g, ig, _ref(ig))
    run(g)
    _check_exec(g, ig, _ref(ig))


def test_reduce_rejects_explicit(gpu):
    eg = wl.pattern_graph("stencil", 8, 4, seed=0, n=64)
    g = tg.graph_from_explicit(eg)
    with pytest.raises(tg.TaskGraphError) as ei:
        tg.tg_graph_reduce_edges(g.handle)
    assert ei.value.status == tg.TG_EINVAL


def test_gang_digests_restart_every_launch(gpu):
    """A gang adds its members' digest parts into the digest words, which the
    reset zeroes before every launch: three gang launches in a row, then one
    wavefront launch and a gang launch again, each bit-exact."""
    ig = wl.halo_graph(12, 192, 5, seed=4, rounds=3)
    g = tg.graph_from_implicit(ig)
    ref = _ref(ig)
    gang = tg.make_config(mapping=3, wg_waves=2, gang=4)
    for cfg in (gang, gang, gang, tg.make_config(mapping=1), gang):
        run(g, cfg)
        _check_exec(g, ig, ref)
