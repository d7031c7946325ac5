"""The allocation-free dependence inference (tg_infer_dag_noalloc), called
through the C ABI: bit-exact against the allocating entry point
(tg_infer_dag) on two calls in a row, the second with a smaller input, and
a requirement list larger than its scratch array is refused."""
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


def test_two_calls_match_the_allocating_entry_point(gpu):
    # the 65,536-task halo program (196,480 requirements), then a 200-task
    # random program: the second call reuses the array the first one filled
    big = wl.halo_graph(1024, 16384, 64, seed=0, rounds=64)
    small = wl.random_regions(200, 500, 4, 40, np.random.default_rng(11), rounds=1, seed=11)
    cap_big = C.halo_edge_count(1024, 64)
    got_big = infer_on_device(big, col_cap=cap_big, fn=tg.tg_infer_dag_noalloc)
    got_small = infer_on_device(small, fn=tg.tg_infer_dag_noalloc)
    ref_big = infer_on_device(big, col_cap=cap_big, fn=tg.tg_infer_dag)
    ref_small = infer_on_device(small, fn=tg.tg_infer_dag)
    for got, ref in ((got_big, ref_big), (got_small, ref_small)):
        assert np.array_equal(got[0], ref[0]), "row pointers differ"
        assert np.array_equal(got[1], ref[1]), "successor lists differ"
    assert got_big[1].size == cap_big
    o_row, o_col = oracle.conflict_dag(small.N, small.req_ptr, small.lo, small.hi, small.priv)
    assert np.array_equal(got_small[0], o_row) and np.array_equal(got_small[1], o_col)


def test_larger_than_scratch_is_refused(gpu):
    # 600,000 one-element requirements: a 19.2 MB interval table
    N = 600_000
    ig = wl.ImplicitGraph(N=N, req_ptr=np.arange(N + 1, dtype=np.uint64), lo=np.arange(N, dtype=np.uint64),
                          hi=np.arange(1, N + 1, dtype=np.uint64), priv=np.full(N, 1, np.uint32), space=N, rounds=0)
    d_ptr, d_reqs = device_requirements(ig)
    row = torch.zeros(N + 1, dtype=torch.int64, device="cuda")
    col = torch.zeros(16, dtype=torch.int32, device="cuda")
    e = ctypes.c_uint64(7)
    st = tg.load().tg_infer_dag_noalloc(N, ctypes.c_void_p(d_ptr.data_ptr()), ctypes.c_void_p(d_reqs.data_ptr()), N,
                                        N, ctypes.c_void_p(row.data_ptr()), ctypes.c_void_p(col.data_ptr()), 16,
                                        ctypes.byref(e), None)
    assert st == tg.TG_ENOMEM and e.value == 0
    assert b"scratch" in tg.load().tg_last_error()
    # the refused call left the entry point usable
    small = wl.halo_graph(8, 128, 4, seed=2, rounds=1)
    got = infer_on_device(small, fn=tg.tg_infer_dag_noalloc)
    o_row, o_col = oracle.conflict_dag(small.N, small.req_ptr, small.lo, small.hi, small.priv)
    assert np.array_equal(got[0], o_row) and np.array_equal(got[1], o_col)
