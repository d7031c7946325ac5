"""Two-hop dependence reduction (host, no GPU).  Checked against what the
problem fixes rather than against itself: reachability computed by brute
force is unchanged, only edges of the input survive, and on the halo
programs the result is the exact transitive reduction, with the edge count
of a closed form derived from the program's conflict rule."""
import numpy as np
import pytest

import oracle
from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl


def _closure(n, rp, cl):
    R = np.zeros((n, n), bool)
    for j in range(n - 1, -1, -1):
        for a in range(int(rp[j]), int(rp[j + 1])):
            k = int(cl[a])
            R[j, k] = True
            R[j] |= R[k]
    return R


def _edges(rp, cl):
    return {(j, int(cl[a])) for j in range(len(rp) - 1) for a in range(int(rp[j]), int(rp[j + 1]))}


def _exact_tr(n, rp, cl):
    R = _closure(n, rp, cl)
    return {(j, k) for (j, k) in _edges(rp, cl) if not (R[j] & R[:, k]).any()}


def _dag(ig):
    return oracle.conflict_dag(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv)


@pytest.mark.parametrize("seed", range(4))
def test_reachability_unchanged_random_regions(tglib, seed):
    ig = wl.random_regions(120, 200, 4, 30, np.random.default_rng(seed), seed=seed)
    rp, cl = _dag(ig)
    orp, ocl = tg.tg_reduce_dag(rp, cl)
    full, red = _edges(rp, cl), _edges(orp, ocl)
    assert red <= full and len(red) < len(full)
    assert (_closure(ig.N, rp, cl) == _closure(ig.N, orp, ocl)).all()
    assert _exact_tr(ig.N, rp, cl) <= red  # every edge of the reduction is kept
    for j in range(ig.N):  # rows ascending
        row = ocl[int(orp[j]):int(orp[j + 1])]
        assert np.all(np.diff(row.astype(np.int64)) > 0)


@pytest.mark.parametrize("P,S,iters", [(8, 128, 6), (16, 256, 5), (64, 256, 8)])
def test_halo_program_reduces_to_exact_transitive_reduction(tglib, P, S, iters):
    ig = wl.halo_graph(P, S, iters, seed=3)
    rp, cl = _dag(ig)
    orp, ocl = tg.tg_reduce_dag(rp, cl)
    assert _edges(orp, ocl) == _exact_tr(ig.N, rp, cl)
    # closed form: sweep 0 chains (0, s-1) -> (0, s); in each later sweep
    # task (it, s) keeps the edge from (it, s-1) (it reads that subregion's
    # halo after it was written, s >= 1) and from (it-1, s+1) (it overwrites
    # what that task read, s <= P-2); the edge from (it-1, s) is implied by
    # the path through (it-1, s+1) or (it, s-1): (P-1)(2 iters - 1) edges
    assert len(ocl) == (P - 1) * (2 * iters - 1)


def test_chain_with_shortcuts_and_errors(tglib):
    # 0->1->2->3 plus shortcuts 0->2, 1->3 (two-hop) and 0->3 (three-hop,
    # also two-hop via 0->2->3 in the input)
    rp = np.array([0, 3, 5, 6, 6], np.uint64)
    cl = np.array([1, 2, 3, 2, 3, 3], np.uint32)
    orp, ocl = tg.tg_reduce_dag(rp, cl)
    assert _edges(orp, ocl) == {(0, 1), (1, 2), (2, 3)}
    # an edge that does not go forward is rejected
    with pytest.raises(tg.TaskGraphError):
        tg.tg_reduce_dag(np.array([0, 0, 1], np.uint64), np.array([0], np.uint32))
    # empty graph
    orp, ocl = tg.tg_reduce_dag(np.zeros(4, np.uint64), np.zeros(0, np.uint32))
    assert orp.tolist() == [0, 0, 0, 0] and ocl.size == 0


def _lu(ig):
    return tg.tg_last_user_dag(ig.req_ptr, tg.reqs_array(ig.lo, ig.hi, ig.priv))


@pytest.mark.parametrize("seed", range(8))
def test_last_user_dag_orders_like_the_conflict_dag(tglib, seed):
    """Every last-user edge joins two conflicting tasks (it is an edge of the
    brute-force conflict DAG) and the two DAGs have the same reachability."""
    rng = np.random.default_rng(100 + seed)
    N, space = (120, 200) if seed % 2 else (90, 60)  # a small space: many overlaps
    ig = wl.random_regions(N, space, 1 + seed % 4, 10 + 5 * seed, rng, seed=seed)
    rp, cl = _dag(ig)
    lrp, lcl = _lu(ig)
    full, lu = _edges(rp, cl), _edges(lrp, lcl)
    assert lu <= full
    assert (_closure(ig.N, rp, cl) == _closure(ig.N, lrp, lcl)).all()
    assert len(lu) < len(full)
    for j in range(ig.N):  # rows ascending, no repeats
        row = lcl[int(lrp[j]):int(lrp[j + 1])]
        assert np.all(np.diff(row.astype(np.int64)) > 0)


@pytest.mark.parametrize("P,S,iters", [(8, 128, 6), (16, 256, 5), (64, 256, 8)])
def test_last_user_dag_of_halo_program(tglib, P, S, iters):
    """On the halo programs the two-hop reduction of the last-user DAG is the
    exact transitive reduction of the conflict DAG, (P-1)(2 iters - 1) edges."""
    ig = wl.halo_graph(P, S, iters, seed=3)
    rp, cl = _dag(ig)
    lrp, lcl = _lu(ig)
    assert _edges(lrp, lcl) <= _edges(rp, cl)
    orp, ocl = tg.tg_reduce_dag(lrp, lcl)
    assert _edges(orp, ocl) == _exact_tr(ig.N, rp, cl)
    assert len(ocl) == (P - 1) * (2 * iters - 1)


def test_last_user_dag_small_cases_and_errors(tglib):
    RO, RW = tg.TG_RO, tg.TG_RW
    # t0 writes [0,10); t1, t2 read parts of it; t3 writes [5,6): depends on
    # the last writer t0 and on the readers since that touch element 5 (t1);
    # t4 reads [0,10): last writers t0 (elements 0..4, 6..9) and t3 (5); an
    # empty interval touches nothing
    reqs = tg.reqs_array([0, 0, 7, 5, 0, 3], [10, 6, 9, 6, 10, 3], [RW, RO, RO, RW, RO, RW])
    req_ptr = np.array([0, 1, 2, 3, 4, 5, 6], np.uint64)
    rp, cl = tg.tg_last_user_dag(req_ptr, reqs)
    assert _edges(rp, cl) == {(0, 1), (0, 2), (0, 3), (1, 3), (0, 4), (3, 4)}
    # no tasks, and tasks without requirements
    rp, cl = tg.tg_last_user_dag(np.zeros(1, np.uint64), np.zeros(0, tg.REQ_DTYPE))
    assert rp.tolist() == [0] and cl.size == 0
    rp, cl = tg.tg_last_user_dag(np.zeros(4, np.uint64), np.zeros(0, tg.REQ_DTYPE))
    assert rp.tolist() == [0, 0, 0, 0] and cl.size == 0
    with pytest.raises(tg.TaskGraphError):
        tg.tg_last_user_dag(np.array([0, 1], np.uint64), tg.reqs_array([5], [4], [RO]))
    with pytest.raises(tg.TaskGraphError):
        tg.tg_last_user_dag(np.array([0, 1], np.uint64), tg.reqs_array([0], [4], [7]))
