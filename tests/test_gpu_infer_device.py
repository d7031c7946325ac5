"""Dependence inference on device-resident requirements (tg_infer_dag): the
CSR equals the oracle's brute-force conflict DAG, and bad inputs are refused
with the documented status."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests import _checks as C
from tests.gpu_util import device_requirements, infer_on_device

pytestmark = pytest.mark.gpu


def _oracle_dag(ig):
    return oracle.conflict_dag(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv)


@pytest.mark.parametrize("seed", range(4))
def test_random_programs(gpu, seed):
    # 200 tasks (not a multiple of the 64-task wavefront rows or 256-thread
    # blocks), up to 4 intervals each, lengths 0..40 (empty ones included)
    ig = wl.random_regions(200, 500, 4, 40, np.random.default_rng(seed), rounds=1, seed=seed)
    row, col = infer_on_device(ig)
    ref_row, ref_col = _oracle_dag(ig)
    assert np.array_equal(row, ref_row)
    assert np.array_equal(col, ref_col)


@pytest.mark.parametrize("P,S,iters", [(8, 128, 4), (5, 64, 7), (33, 256, 3)])
def test_halo_programs(gpu, P, S, iters):
    ig = wl.halo_graph(P, S, iters, seed=2, rounds=1)
    row, col = infer_on_device(ig, stream=torch.cuda.Stream())
    ref_row, ref_col = _oracle_dag(ig)
    assert np.array_equal(row, ref_row) and np.array_equal(col, ref_col)
    assert col.size == C.halo_edge_count(P, iters)


def test_halo_program_full_size(gpu):
    """The 65,536-task halo program: the closed-form edge count, and sampled
    rows against the oracle's brute-force row."""
    ig = wl.halo_graph(1024, 16384, 64, seed=0, rounds=64)
    row, col = infer_on_device(ig, col_cap=6254592)
    assert col.size == C.halo_edge_count(1024, 64) == 6254592
    rng = np.random.default_rng(3)
    for j in list(rng.integers(0, ig.N, size=200)) + [0, 1023, 1024, ig.N - 1]:
        want = oracle.conflict_row(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv, int(j))
        assert np.array_equal(col[int(row[j]):int(row[j + 1])], want), f"row {j}"


def test_edge_cases(gpu):
    # tasks without requirements: no edges
    ig = wl.ImplicitGraph(N=70, req_ptr=np.zeros(71, np.uint64), lo=np.zeros(0, np.uint64),
                          hi=np.zeros(0, np.uint64), priv=np.zeros(0, np.uint32), space=16, rounds=0)
    row, col = infer_on_device(ig)
    assert col.size == 0 and not row.any()
    # only empty intervals: no edges
    N = 10
    ig = wl.ImplicitGraph(N=N, req_ptr=np.arange(N + 1, dtype=np.uint64), lo=np.full(N, 3, np.uint64),
                          hi=np.full(N, 3, np.uint64), priv=np.full(N, 2, np.uint32), space=16, rounds=0)
    row, col = infer_on_device(ig)
    assert col.size == 0
    # every task writes the same word: a complete DAG, rows ascending
    ig = wl.ImplicitGraph(N=N, req_ptr=np.arange(N + 1, dtype=np.uint64), lo=np.zeros(N, np.uint64),
                          hi=np.ones(N, np.uint64), priv=np.full(N, 2, np.uint32), space=1, rounds=0)
    row, col = infer_on_device(ig)
    ref_row, ref_col = _oracle_dag(ig)
    assert col.size == N * (N - 1) // 2 and np.array_equal(col, ref_col) and np.array_equal(row, ref_row)


def _raw_call(ig, req_ptr=None, cap=64, space=None):
    d_ptr, d_reqs = device_requirements(ig)
    if req_ptr is not None:
        d_ptr = torch.from_numpy(np.asarray(req_ptr, np.uint64).view(np.int64)).cuda()
    row = torch.zeros(ig.N + 1, dtype=torch.int64, device="cuda")
    col = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
    e = ctypes.c_uint64(123)
    st = tg.load().tg_infer_dag(ig.N, ctypes.c_void_p(d_ptr.data_ptr()), ctypes.c_void_p(d_reqs.data_ptr()),
                                int(ig.lo.size), ig.space if space is None else space, ctypes.c_void_p(row.data_ptr()),
                                ctypes.c_void_p(col.data_ptr()), cap, ctypes.byref(e), None)
    return st, e.value, row, col


def test_refusals(gpu):
    N = 10
    ig = wl.ImplicitGraph(N=N, req_ptr=np.arange(N + 1, dtype=np.uint64), lo=np.zeros(N, np.uint64),
                          hi=np.ones(N, np.uint64), priv=np.full(N, 2, np.uint32), space=1, rounds=0)
    # capacity below the edge count: TG_ENOMEM, the count is still reported
    st, e, _, col = _raw_call(ig, cap=5)
    assert st == tg.TG_ENOMEM and e == 45
    # row pointers that do not start at 0 / do not end at nreqs / decrease
    for bad in ([1] + list(range(1, N + 1)), list(range(N)) + [N - 1], [0, 2, 1] + list(range(3, N + 1))):
        st, e, _, _ = _raw_call(ig, req_ptr=bad)
        assert st == tg.TG_EINVAL and e == 0, bad
    assert b"row pointers" in tg.load().tg_last_error()
    # an interval past the index space
    st, _, _, _ = _raw_call(ig, space=0)
    assert st == tg.TG_EINVAL and b"index space" in tg.load().tg_last_error()
    # a task whose read-write interval overlaps its own read-only interval
    ig2 = wl.ImplicitGraph(N=1, req_ptr=np.array([0, 2], np.uint64), lo=np.array([0, 1], np.uint64),
                           hi=np.array([4, 2], np.uint64), priv=np.array([2, 1], np.uint32), space=8, rounds=0)
    st, _, _, _ = _raw_call(ig2)
    assert st == tg.TG_EINVAL
    # no tasks: one row pointer, 0
    ig0 = wl.ImplicitGraph(N=0, req_ptr=np.zeros(1, np.uint64), lo=np.zeros(0, np.uint64),
                           hi=np.zeros(0, np.uint64), priv=np.zeros(0, np.uint32), space=8, rounds=0)
    st, e, row, _ = _raw_call(ig0)
    assert st == tg.TG_OK and e == 0 and int(row[0]) == 0
