"""The C-ABI library loads, exports every declared symbol and validates its
host-side arguments (no device work: these run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2508_16522_amd import taskgraph as tg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "taskgraph.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tg_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(tglib):
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(tglib, n), n
    assert set(tg.EXPORTS) == set(names)


def test_status_strings(tglib):
    assert tg.status_name(0) == "TG_OK"
    assert tg.status_name(-5) == "TG_ETIMEOUT"
    assert tglib.tg_version().decode().startswith("taskgraph")


def _create(tglib, mode, n, space):
    g = ctypes.c_void_p()
    st = tglib.tg_graph_create(ctypes.byref(g), mode, n, space, 0)
    return st, g


def test_create_validation(tglib):
    assert _create(tglib, 1, 63, 0)[0] == tg.TG_EINVAL
    assert _create(tglib, 1, 96, 0)[0] == tg.TG_EINVAL
    assert _create(tglib, 2, 0, 0)[0] == tg.TG_EINVAL
    assert _create(tglib, 3, 64, 0)[0] == tg.TG_EINVAL
    st, g = _create(tglib, 1, 64, 0)
    assert st == 0
    tglib.tg_graph_destroy(g)


def test_explicit_add_validation(tglib):
    st, g = _create(tglib, 1, 64, 0)
    ev = ctypes.c_uint32()
    assert tglib.tg_task_add(g, None, 0, 3, ctypes.byref(ev)) == 0 and ev.value == 0
    bad = (ctypes.c_uint32 * 1)(1)  # names a task that does not exist yet
    assert tglib.tg_task_add(g, bad, 1, 3, ctypes.byref(ev)) == tg.TG_EINVAL
    ok = (ctypes.c_uint32 * 2)(0, 0)  # duplicates are allowed (a set)
    assert tglib.tg_task_add(g, ok, 2, 3, ctypes.byref(ev)) == 0 and ev.value == 1
    n = ctypes.c_uint64()
    assert tglib.tg_graph_num_tasks(g, ctypes.byref(n)) == 0 and n.value == 2
    # regions are refused in explicit mode; reads before finalise are refused
    req = tg.reqs_array([0], [4], [2])
    assert tglib.tg_task_add_regions(g, req.ctypes.data_as(ctypes.c_void_p), 1, 1, ctypes.byref(ev)) == tg.TG_EINVAL
    d = np.zeros(2, np.uint32)
    assert tglib.tg_graph_read_digests(g, d.ctypes.data_as(ctypes.c_void_p), 2) == tg.TG_ESTATE
    assert tglib.tg_graph_execute(g, None, None) == tg.TG_ESTATE
    tglib.tg_graph_destroy(g)


def test_implicit_add_validation(tglib):
    st, g = _create(tglib, 2, 0, 100)
    ev = ctypes.c_uint32()

    def add(lo, hi, priv):
        r = tg.reqs_array(lo, hi, priv)
        return tglib.tg_task_add_regions(g, r.ctypes.data_as(ctypes.c_void_p), len(lo), 1, ctypes.byref(ev))

    assert add([0], [10], [2]) == 0
    assert add([5], [101], [1]) == tg.TG_EINVAL     # outside the index space
    assert add([7], [3], [1]) == tg.TG_EINVAL       # lo > hi
    assert add([0], [4], [3]) == tg.TG_EINVAL       # unknown privilege
    assert add([0, 5], [10, 20], [2, 1]) == tg.TG_EINVAL  # RW overlaps own RO
    assert add([0, 5], [10, 20], [1, 1]) == 0       # RO may overlap RO
    assert add([4, 4], [4, 9], [2, 2]) == 0         # an empty interval overlaps nothing
    tglib.tg_graph_destroy(g)


def test_bad_config_rejected_before_launch(tglib):
    st, g = _create(tglib, 1, 64, 0)
    cfg = tg.make_config(mapping=7)
    # not finalised -> state error takes precedence
    assert tglib.tg_graph_execute(g, ctypes.byref(cfg), None) == tg.TG_ESTATE
    # finalised (host-only for explicit graphs): every out-of-range field is
    # refused before any device work
    ev = ctypes.c_uint32()
    assert tglib.tg_task_add(g, None, 0, 1, ctypes.byref(ev)) == 0
    assert tglib.tg_graph_finalize(g) == 0
    for kw in (dict(mapping=4), dict(mapping=3, gang=1), dict(mapping=3, gang=33), dict(window=65),
               dict(wg_waves=17), dict(idle_sleep=65), dict(schedule=6), dict(mapping=2, wg_waves=17)):
        cfg = tg.make_config(**kw)
        assert tglib.tg_graph_execute(g, ctypes.byref(cfg), None) == tg.TG_EINVAL, kw
    tglib.tg_graph_destroy(g)


def test_execute_when_argument_errors(tglib):
    """Refused before any device work: more than 8 pre-condition flags, a NULL
    flag list or value list, a NULL flag."""
    st, g = _create(tglib, 1, 64, 0)
    ev = ctypes.c_uint32()
    assert tglib.tg_task_add(g, None, 0, 1, ctypes.byref(ev)) == 0
    assert tglib.tg_graph_finalize(g) == 0
    vals = (ctypes.c_uint32 * 9)(*range(9))
    flags = (ctypes.c_void_p * 9)()
    assert tglib.tg_graph_execute_when(g, None, None, flags, vals, 9, None, 0) == tg.TG_EINVAL
    assert tglib.tg_graph_execute_when(g, None, None, None, vals, 1, None, 0) == tg.TG_EINVAL
    assert tglib.tg_graph_execute_when(g, None, None, flags, None, 1, None, 0) == tg.TG_EINVAL
    assert tglib.tg_graph_execute_when(g, None, None, flags, vals, 1, None, 0) == tg.TG_EINVAL  # flags[0] NULL
    assert tglib.tg_graph_execute_when(None, None, None, None, None, 0, None, 0) == tg.TG_EINVAL
    tglib.tg_graph_destroy(g)


def test_batch_queries_refuse_null(tglib):
    """Batch queries with a NULL batch or output are refused, no device work."""
    e = ctypes.c_uint64()
    assert tglib.tg_batch_signalled_edges(None, ctypes.byref(e)) == tg.TG_EINVAL
    assert tglib.tg_batch_info(None, None, None, None, None) == tg.TG_EINVAL
