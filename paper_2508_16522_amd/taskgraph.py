"""ctypes binding of libtaskgraph.so (argument marshalling only).

Every function below has the name of the C entry point it calls and adds no
computation of its own: numpy arrays are passed as host pointers, streams as
hipStream_t handles (PyTorch's current stream by default), and device memory
is obtained through PyTorch's caching allocator when PyTorch sees a GPU.  If
the shared library has not been built the import fails loudly; there is no
fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtaskgraph.so")

TG_OK, TG_EINVAL, TG_ENOMEM, TG_EBUSY, TG_EDEVICE, TG_ETIMEOUT, TG_ESTATE = 0, -1, -2, -3, -4, -5, -6
TG_EXPLICIT, TG_IMPLICIT = 1, 2
TG_RO, TG_RW = 1, 2
TG_MAP_WAVE, TG_MAP_WORKGROUP, TG_MAP_GANG = 1, 2, 3
TG_SCHED_LIST, TG_SCHED_LEVEL, TG_SCHED_SPREAD, TG_SCHED_COLUMN, TG_SCHED_BALANCED = 1, 2, 3, 4, 5
TG_DISPATCH_LISTS, TG_DISPATCH_QUEUE = 1, 2
TG_CMP_PER_TASK, TG_CMP_HIPGRAPH, TG_CMP_HIPGRAPH_CAPTURED = 1, 2, 3
TG_KEEP_ALL, TG_KEEP_SINKS, TG_KEEP_NONE = 0, 1, 2

# Every symbol the header declares; the CPU test-suite checks the library
# exports all of them.
EXPORTS = (
    "tg_status_str", "tg_last_error", "tg_version", "tg_set_allocator",
    "tg_graph_create", "tg_task_add", "tg_task_add_many", "tg_task_add_regions", "tg_task_add_regions_many",
    "tg_graph_finalize", "tg_graph_execute", "tg_graph_wait", "tg_graph_num_tasks", "tg_graph_num_edges",
    "tg_graph_read_digests", "tg_graph_read_payload", "tg_graph_read_data", "tg_graph_checksum",
    "tg_graph_read_dag", "tg_graph_timings", "tg_graph_destroy",
    "tg_batch_create", "tg_batch_execute", "tg_batch_wait", "tg_batch_time_ms", "tg_batch_destroy",
    "tg_graph_execute_comparator", "tg_exec_occupancy", "tg_graph_exec_info", "tg_graph_debug_state", "tg_emulate_schedule", "tg_graph_debug_times",
    "tg_graph_kernel_ms", "tg_graph_autotune", "tg_probe", "tg_graph_kernel_times", "tg_graph_set_rounds",
    "tg_server_create", "tg_server_submit", "tg_server_wait", "tg_server_stats", "tg_server_destroy",
    "tg_batch_kernel_times", "tg_batch_set_rounds", "tg_batch_signalled_edges", "tg_batch_info", "tg_batch_autotune",
    "tg_graph_execute_after", "tg_flag_create", "tg_flag_destroy", "tg_flag_set", "tg_flag_read", "tg_flag_wait",
    "tg_graph_execute_when", "tg_reduce_dag", "tg_last_user_dag", "tg_graph_reduce_edges",
    "tg_graph_set_retention", "tg_graph_payload_slots", "tg_graph_read_exec_dag", "tg_emulate_gang", "tg_emulate_queue",
    "tg_infer_dag", "tg_infer_dag_noalloc", "tg_server_configure",
)


class TaskGraphError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {status_name(status)} ({status}): {message}")
        self.status = status


class tg_region_req(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64), ("priv", ctypes.c_uint32),
                ("_pad", ctypes.c_uint32)]


class tg_exec_config(ctypes.Structure):
    _fields_ = [("mapping", ctypes.c_uint32), ("workers", ctypes.c_uint32), ("window", ctypes.c_uint32),
                ("wg_waves", ctypes.c_uint32), ("watchdog_ms", ctypes.c_uint32), ("spin_limit", ctypes.c_uint32),
                ("diag", ctypes.c_uint32), ("notify", ctypes.c_uint32), ("idle_sleep", ctypes.c_uint32),
                ("schedule", ctypes.c_uint32), ("gang", ctypes.c_uint32), ("dispatch", ctypes.c_uint32),
                ("tile", ctypes.c_uint32), ("shards", ctypes.c_uint32)]


REQ_DTYPE = np.dtype([("lo", np.uint64), ("hi", np.uint64), ("priv", np.uint32), ("_pad", np.uint32)])

_lib = None


def load() -> ctypes.CDLL:
    """Load the shared library; raise if it was never built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2508_16522_amd.build.build_library()")
    L = ctypes.CDLL(LIB_PATH)
    i32, u32, u64, P = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
    G = ctypes.c_void_p
    sig = {
        "tg_status_str": (ctypes.c_char_p, [i32]),
        "tg_last_error": (ctypes.c_char_p, []),
        "tg_version": (ctypes.c_char_p, []),
        "tg_set_allocator": (i32, [P, P, P]),
        "tg_graph_create": (i32, [ctypes.POINTER(G), u32, u32, u64, u64]),
        "tg_task_add": (i32, [G, P, u32, u32, P]),
        "tg_task_add_many": (i32, [G, u32, P, P, P, u32, P]),
        "tg_task_add_regions": (i32, [G, P, u32, u32, P]),
        "tg_task_add_regions_many": (i32, [G, u32, P, P, P, u32, P]),
        "tg_graph_finalize": (i32, [G]),
        "tg_graph_execute": (i32, [G, P, P]),
        "tg_graph_wait": (i32, [G]),
        "tg_graph_num_tasks": (i32, [G, P]),
        "tg_graph_num_edges": (i32, [G, P]),
        "tg_graph_read_digests": (i32, [G, P, u64]),
        "tg_graph_read_payload": (i32, [G, u32, P, u32]),
        "tg_graph_read_data": (i32, [G, P, u64, u64]),
        "tg_graph_checksum": (i32, [G, P]),
        "tg_graph_read_dag": (i32, [G, P, P, u64, P]),
        "tg_graph_timings": (i32, [G, P, P, P]),
        "tg_graph_destroy": (i32, [G]),
        "tg_batch_create": (i32, [ctypes.POINTER(G), P, u32, P]),
        "tg_batch_execute": (i32, [G, P]),
        "tg_batch_wait": (i32, [G]),
        "tg_batch_time_ms": (i32, [G, P]),
        "tg_batch_destroy": (i32, [G]),
        "tg_graph_execute_comparator": (i32, [G, u32, P]),
        "tg_exec_occupancy": (i32, [u32, u32, P, P, P]),
        "tg_graph_exec_info": (i32, [G, P, P]),
        "tg_graph_debug_state": (i32, [G, P, P, P, P, P, u32]),
        "tg_emulate_schedule": (i32, [P, u32, u32, u32, u32, u64, P, P, P, P]),
        "tg_graph_debug_times": (i32, [G, P, P, u32]),
        "tg_graph_kernel_ms": (i32, [G, P]),
        "tg_graph_autotune": (i32, [G, u32, P, P]),
        "tg_probe": (i32, [u32, P]),
        "tg_graph_kernel_times": (i32, [G, P, u32, P]),
        "tg_graph_set_rounds": (i32, [G, u32]),
        "tg_server_create": (i32, [ctypes.POINTER(G), u64, u32, u32]),
        "tg_server_submit": (i32, [G, G, P]),
        "tg_server_wait": (i32, [G, u64, P, P, P]),
        "tg_server_stats": (i32, [G, P, P, P, P]),
        "tg_server_destroy": (i32, [G]),
        "tg_server_configure": (i32, [G, P]),
        "tg_batch_kernel_times": (i32, [G, P, u32, P]),
        "tg_batch_set_rounds": (i32, [G, u32]),
        "tg_batch_info": (i32, [G, P, P, P, P]),
        "tg_batch_autotune": (i32, [G, u32, P, P]),
        "tg_graph_execute_after": (i32, [G, P, P, P, u32, P]),
        "tg_batch_signalled_edges": (i32, [P, P]),
        "tg_emulate_gang": (i32, [P, u32, u32, u32, u32, u32, u64, u32, P]),
        "tg_flag_create": (i32, [P]),
        "tg_flag_destroy": (i32, [P]),
        "tg_flag_set": (i32, [P, u32]),
        "tg_flag_read": (i32, [P, P]),
        "tg_flag_wait": (i32, [P, u32, u32]),
        "tg_graph_execute_when": (i32, [G, P, P, P, P, u32, P, u32]),
        "tg_reduce_dag": (i32, [u32, P, P, P, P, P]),
        "tg_last_user_dag": (i32, [u32, P, P, P, P, u64, P]),
        "tg_graph_reduce_edges": (i32, [G, P]),
        "tg_graph_set_retention": (i32, [G, u32]),
        "tg_graph_payload_slots": (i32, [G, P, P, P]),
        "tg_graph_read_exec_dag": (i32, [G, P, P, u64, P]),
        "tg_emulate_queue": (i32, [P, u32, u32, u32, u32, u64, P, P]),
        "tg_infer_dag": (i32, [u32, P, P, u64, u64, P, P, u64, P, P]),
        "tg_infer_dag_noalloc": (i32, [u32, P, P, u64, u64, P, P, u64, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype, fn.argtypes = res, args
    _lib = L
    return L


def status_name(s: int) -> str:
    return load().tg_status_str(s).decode()


def _check(status: int, where: str):
    if status != TG_OK:
        raise TaskGraphError(status, where, load().tg_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    """Device address of a torch tensor, or an address given as an int."""
    return ctypes.c_void_p(t if isinstance(t, int) else t.data_ptr())


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------- allocator

_alloc_cb = None
_free_cb = None
_exiting = False


def _mark_exiting():
    # graphs still alive at interpreter exit are destroyed while modules are
    # torn down; their device memory goes with the process, so frees stop here
    global _exiting
    _exiting = True


def use_torch_allocator() -> bool:
    """Route the library's device allocations through PyTorch's caching
    allocator (only when PyTorch sees a GPU)."""
    global _alloc_cb, _free_cb
    try:
        import torch
    except ImportError:
        return False
    if not torch.cuda.is_available():
        return False
    if _alloc_cb is not None:
        return True
    ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
    FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

    def _alloc(nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:  # out of memory -> the library reports TG_ENOMEM
            return None

    def _free(ptr, _ctx):
        if not _exiting:
            torch.cuda.caching_allocator_delete(int(ptr))

    a, f = ALLOC(_alloc), FREE(_free)
    atexit.register(_mark_exiting)  # after torch's own handlers were registered: runs first
    _check(load().tg_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p), None),
           "tg_set_allocator")
    _alloc_cb, _free_cb = a, f
    return True


# --------------------------------------------------------------- graphs


def tg_graph_create(mode: int, payload_words: int = 0, index_space: int = 0, seed: int = 0):
    use_torch_allocator()
    g = ctypes.c_void_p()
    _check(load().tg_graph_create(ctypes.byref(g), mode, payload_words, index_space, seed), "tg_graph_create")
    return g


def tg_task_add(g, preds, mix_rounds: int) -> int:
    p = np.ascontiguousarray(preds, dtype=np.uint32)
    ev = ctypes.c_uint32()
    _check(load().tg_task_add(g, _ptr(p) if p.size else None, p.size, mix_rounds, ctypes.byref(ev)), "tg_task_add")
    return ev.value


def tg_task_add_many(g, pred_ptr, preds, mix_rounds=None, uniform_rounds: int = 0) -> int:
    pp = np.ascontiguousarray(pred_ptr, dtype=np.uint64)
    pr = np.ascontiguousarray(preds, dtype=np.uint32)
    if pr.size == 0:
        pr = np.zeros(1, np.uint32)
    r = None if mix_rounds is None else np.ascontiguousarray(mix_rounds, dtype=np.uint32)
    ev = ctypes.c_uint32()
    _check(load().tg_task_add_many(g, pp.size - 1, _ptr(pp), _ptr(pr), _ptr(r) if r is not None else None,
                                   uniform_rounds, ctypes.byref(ev)), "tg_task_add_many")
    return ev.value


def reqs_array(lo, hi, priv) -> np.ndarray:
    a = np.zeros(len(lo), REQ_DTYPE)
    a["lo"], a["hi"], a["priv"] = lo, hi, priv
    return a


def tg_task_add_regions(g, reqs: np.ndarray, mix_rounds: int) -> int:
    r = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    ev = ctypes.c_uint32()
    _check(load().tg_task_add_regions(g, _ptr(r) if r.size else None, r.size, mix_rounds, ctypes.byref(ev)),
           "tg_task_add_regions")
    return ev.value


def tg_task_add_regions_many(g, req_ptr, reqs: np.ndarray, mix_rounds=None, uniform_rounds: int = 0) -> int:
    rp = np.ascontiguousarray(req_ptr, dtype=np.uint64)
    r = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    if r.size == 0:
        r = np.zeros(1, REQ_DTYPE)
    mr = None if mix_rounds is None else np.ascontiguousarray(mix_rounds, dtype=np.uint32)
    ev = ctypes.c_uint32()
    _check(load().tg_task_add_regions_many(g, rp.size - 1, _ptr(rp), _ptr(r), _ptr(mr) if mr is not None else None,
                                           uniform_rounds, ctypes.byref(ev)), "tg_task_add_regions_many")
    return ev.value


def tg_graph_finalize(g):
    _check(load().tg_graph_finalize(g), "tg_graph_finalize")


def make_config(mapping=0, workers=0, window=0, wg_waves=0, watchdog_ms=0, spin_limit=0, diag=0, notify=0,
                idle_sleep=0, schedule=0, gang=0, dispatch=0, tile=0, shards=0) -> tg_exec_config:
    return tg_exec_config(mapping, workers, window, wg_waves, watchdog_ms, spin_limit, diag, notify, idle_sleep,
                          schedule, gang, dispatch, tile, shards)


def tg_graph_execute(g, cfg: tg_exec_config | None = None, stream=None):
    _check(load().tg_graph_execute(g, ctypes.byref(cfg) if cfg is not None else None, _stream(stream)),
           "tg_graph_execute")


def tg_graph_execute_after(g, pre_events=(), post_event=None, cfg: tg_exec_config | None = None, stream=None):
    """pre_events / post_event: torch.cuda.Event objects (their hipEvent_t
    handles are passed through).  PyTorch creates an event's HIP handle at its
    first record: a pre-condition never recorded has nothing to wait for and
    is skipped; a post-condition is recorded once on the launch stream first
    so that it has a handle (the library records it again after the graph)."""
    handles = [ctypes.c_void_p(e.cuda_event) for e in pre_events if e.cuda_event]
    arr = (ctypes.c_void_p * max(len(handles), 1))(*handles)
    post = None
    if post_event is not None:
        if not post_event.cuda_event:
            import torch
            post_event.record(stream if stream is not None else torch.cuda.current_stream())
        post = ctypes.c_void_p(post_event.cuda_event)
    _check(load().tg_graph_execute_after(g, ctypes.byref(cfg) if cfg is not None else None, _stream(stream),
                                         arr if handles else None, len(handles), post), "tg_graph_execute_after")


def tg_flag_create():
    """A condition flag (one pinned 32-bit host word the device reads and
    writes), initially 0."""
    f = ctypes.c_void_p()
    _check(load().tg_flag_create(ctypes.byref(f)), "tg_flag_create")
    return f


def tg_flag_destroy(f):
    _check(load().tg_flag_destroy(f), "tg_flag_destroy")


def tg_flag_set(f, value: int):
    _check(load().tg_flag_set(f, value), "tg_flag_set")


def tg_flag_read(f) -> int:
    v = ctypes.c_uint32()
    _check(load().tg_flag_read(f, ctypes.byref(v)), "tg_flag_read")
    return v.value


def tg_flag_wait(f, value: int, timeout_ms: int = 10000):
    _check(load().tg_flag_wait(f, value, timeout_ms), "tg_flag_wait")


def tg_graph_execute_when(g, pre=(), pre_values=(), post=None, post_value: int = 1,
                          cfg: tg_exec_config | None = None, stream=None):
    """Execute once every flag in pre holds at least its value in pre_values;
    set post to post_value on the device when the graph has finished."""
    if len(pre) != len(pre_values):
        raise ValueError("pre and pre_values differ in length")
    n = len(pre)
    fa = (ctypes.c_void_p * max(n, 1))(*[ctypes.c_void_p(f.value if isinstance(f, ctypes.c_void_p) else f)
                                         for f in pre])
    va = (ctypes.c_uint32 * max(n, 1))(*[int(v) for v in pre_values])
    _check(load().tg_graph_execute_when(g, ctypes.byref(cfg) if cfg is not None else None, _stream(stream),
                                        fa if n else None, va if n else None, n, post, post_value),
           "tg_graph_execute_when")


def tg_graph_wait(g):
    _check(load().tg_graph_wait(g), "tg_graph_wait")


def tg_graph_num_tasks(g) -> int:
    n = ctypes.c_uint64()
    _check(load().tg_graph_num_tasks(g, ctypes.byref(n)), "tg_graph_num_tasks")
    return n.value


def tg_graph_num_edges(g) -> int:
    n = ctypes.c_uint64()
    _check(load().tg_graph_num_edges(g, ctypes.byref(n)), "tg_graph_num_edges")
    return n.value


def tg_graph_read_digests(g) -> np.ndarray:
    N = tg_graph_num_tasks(g)
    out = np.zeros(max(N, 1), np.uint32)
    _check(load().tg_graph_read_digests(g, _ptr(out), N), "tg_graph_read_digests")
    return out[:N]


def tg_graph_read_payload(g, v: int, n: int) -> np.ndarray:
    out = np.zeros(n, np.uint32)
    _check(load().tg_graph_read_payload(g, v, _ptr(out), n), "tg_graph_read_payload")
    return out


def tg_graph_read_data(g, lo: int, hi: int) -> np.ndarray:
    out = np.zeros(max(hi - lo, 1), np.uint32)
    _check(load().tg_graph_read_data(g, _ptr(out), lo, hi), "tg_graph_read_data")
    return out[:hi - lo]


def tg_graph_checksum(g) -> int:
    c = ctypes.c_uint64()
    _check(load().tg_graph_checksum(g, ctypes.byref(c)), "tg_graph_checksum")
    return c.value


def tg_graph_read_dag(g):
    """The full (inferred or explicit) DAG as an out-edge CSR."""
    N = tg_graph_num_tasks(g)
    row_ptr = np.zeros(N + 1, np.uint64)
    e = ctypes.c_uint64()
    # the first call reports the edge count (its row pointers are complete)
    st = load().tg_graph_read_dag(g, _ptr(row_ptr), None, 0, ctypes.byref(e))
    if st not in (TG_OK, TG_ENOMEM):
        _check(st, "tg_graph_read_dag")
    col = np.zeros(max(e.value, 1), np.uint32)
    _check(load().tg_graph_read_dag(g, _ptr(row_ptr), _ptr(col), e.value, ctypes.byref(e)), "tg_graph_read_dag")
    return row_ptr, col[:e.value]


def tg_graph_read_exec_dag(g):
    """The edges the executor's counters follow, as an out-edge CSR."""
    N = tg_graph_num_tasks(g)
    row_ptr = np.zeros(N + 1, np.uint64)
    e = ctypes.c_uint64()
    st = load().tg_graph_read_exec_dag(g, _ptr(row_ptr), None, 0, ctypes.byref(e))
    if st not in (TG_OK, TG_ENOMEM):
        _check(st, "tg_graph_read_exec_dag")
    col = np.zeros(max(e.value, 1), np.uint32)
    _check(load().tg_graph_read_exec_dag(g, _ptr(row_ptr), _ptr(col), e.value, ctypes.byref(e)),
           "tg_graph_read_exec_dag")
    return row_ptr, col[:e.value]


def tg_graph_set_retention(g, mode: int):
    _check(load().tg_graph_set_retention(g, mode), "tg_graph_set_retention")


def tg_graph_payload_slots(g):
    """(slot of each task, number of slots, device bytes of the payloads)."""
    N = tg_graph_num_tasks(g)
    out = np.zeros(max(N, 1), np.uint32)
    ns, nb = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().tg_graph_payload_slots(g, _ptr(out), ctypes.byref(ns), ctypes.byref(nb)), "tg_graph_payload_slots")
    return out[:N], ns.value, nb.value


def tg_graph_timings(g):
    c, i, x = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load().tg_graph_timings(g, ctypes.byref(c), ctypes.byref(i), ctypes.byref(x)), "tg_graph_timings")
    return {"compile_ms": c.value, "infer_ms": i.value, "exec_ms": x.value}


def tg_graph_destroy(g):
    if g:
        _check(load().tg_graph_destroy(g), "tg_graph_destroy")


def tg_exec_occupancy(mapping: int, wg_waves: int = 4, calibrate: bool = True):
    b, c, r = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().tg_exec_occupancy(mapping, wg_waves, ctypes.byref(b), ctypes.byref(c),
                                    ctypes.byref(r) if calibrate else None), "tg_exec_occupancy")
    return b.value, c.value, (r.value if calibrate else None)


def tg_graph_exec_info(g):
    w, s = ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().tg_graph_exec_info(g, ctypes.byref(w), ctypes.byref(s)), "tg_graph_exec_info")
    return w.value, s.value


def tg_graph_debug_state(g):
    N = tg_graph_num_tasks(g)
    w, _ = tg_graph_exec_info(g)
    a = [np.zeros(max(N, 1), np.uint32) for _ in range(4)]
    wp = np.zeros(max(w, 1), np.uint32)
    _check(load().tg_graph_debug_state(g, *[_ptr(x) for x in a], _ptr(wp), w), "tg_graph_debug_state")
    return {"pending": a[0][:N], "execs": a[1][:N], "owner": a[2][:N], "entry": a[3][:N], "wprog": wp[:w]}


TG_PROBE_MIX_RATE, TG_PROBE_COPY_BW, TG_PROBE_ATOMIC_DISTINCT, TG_PROBE_ATOMIC_CONTENDED, TG_PROBE_LAUNCH_RATE = 1, 2, 3, 4, 5
TG_PROBE_HANDOFF_NS = 6
TG_PROBE_HANDOFF_SAME_XCD_NS, TG_PROBE_HANDOFF_FAR_XCD_NS, TG_PROBE_HANDOFF_L2_NS = 7, 8, 9


def tg_probe(kind: int) -> float:
    v = ctypes.c_double()
    _check(load().tg_probe(kind, ctypes.byref(v)), "tg_probe")
    return v.value


def tg_graph_kernel_ms(g) -> float:
    v = ctypes.c_double()
    _check(load().tg_graph_kernel_ms(g, ctypes.byref(v)), "tg_graph_kernel_ms")
    return v.value


def tg_graph_kernel_times(g, n: int = 64) -> np.ndarray:
    out = np.zeros(max(n, 1), np.float64)
    got = ctypes.c_uint32()
    _check(load().tg_graph_kernel_times(g, _ptr(out), n, ctypes.byref(got)), "tg_graph_kernel_times")
    return out[:got.value]


def tg_graph_set_rounds(g, rounds: int):
    _check(load().tg_graph_set_rounds(g, rounds), "tg_graph_set_rounds")


def tg_graph_autotune(g, reps: int = 2):
    c = tg_exec_config()
    ms = ctypes.c_double()
    _check(load().tg_graph_autotune(g, reps, ctypes.byref(c), ctypes.byref(ms)), "tg_graph_autotune")
    return {f: getattr(c, f) for f, _ in tg_exec_config._fields_}, ms.value


def tg_graph_debug_times(g):
    N = tg_graph_num_tasks(g)
    w, _ = tg_graph_exec_info(g)
    t = np.zeros(2 * max(N, 1), np.uint64)
    ws = np.zeros(4 * max(w, 1), np.uint64)
    _check(load().tg_graph_debug_times(g, _ptr(t), _ptr(ws), w), "tg_graph_debug_times")
    return t[:2 * N].reshape(N, 2), ws[:4 * w].reshape(w, 4)


def tg_emulate_schedule(graphs, nworkers: int, window: int = 64, seed: int = 0, schedule: int = 0):
    """Host-only model of one launch over `graphs` (a graph handle or a list
    of them).  Returns (status, order, makespan, bound): order is an
    (executed, 2) array of (graph index, event) in execution order."""
    hs = list(graphs) if isinstance(graphs, (list, tuple)) else [graphs]
    total = sum(tg_graph_num_tasks(h) for h in hs)
    arr = (ctypes.c_void_p * len(hs))(*[ctypes.cast(h, ctypes.c_void_p) for h in hs])
    order = np.zeros(max(total, 1), np.uint64)
    ex, mk, bd = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    st = load().tg_emulate_schedule(arr, len(hs), nworkers, window, schedule, seed, _ptr(order), ctypes.byref(ex),
                                    ctypes.byref(mk), ctypes.byref(bd))
    o = order[:ex.value]
    pairs = np.stack([(o >> np.uint64(32)).astype(np.int64), (o & np.uint64(0xFFFFFFFF)).astype(np.int64)], axis=1)
    return st, pairs, mk.value, bd.value


def tg_emulate_queue(graphs, nworkers: int, shards: int = 8, tile: int = 1, seed: int = 0):
    """Host-only model of the ready-queue dispatch.  Returns (status, order)
    with order an (executed, 2) array of (graph index, event)."""
    hs = list(graphs) if isinstance(graphs, (list, tuple)) else [graphs]
    total = sum(tg_graph_num_tasks(h) for h in hs)
    arr = (ctypes.c_void_p * len(hs))(*[ctypes.cast(h, ctypes.c_void_p) for h in hs])
    order = np.zeros(max(total, 1), np.uint64)
    ex = ctypes.c_uint64()
    st = load().tg_emulate_queue(arr, len(hs), nworkers, shards, tile, seed, _ptr(order), ctypes.byref(ex))
    o = order[:ex.value]
    return st, np.stack([(o >> np.uint64(32)).astype(np.int64), (o & np.uint64(0xFFFFFFFF)).astype(np.int64)], axis=1)


def tg_emulate_gang(graphs, ngangs: int, gang: int, window: int = 64, seed: int = 0, schedule: int = 0,
                    elide: bool = False):
    """Host-only model of a gang launch: returns (status, shares finished)."""
    hs = list(graphs) if isinstance(graphs, (list, tuple)) else [graphs]
    arr = (ctypes.c_void_p * len(hs))(*[ctypes.cast(h, ctypes.c_void_p) for h in hs])
    ex = ctypes.c_uint64()
    st = load().tg_emulate_gang(arr, len(hs), ngangs, gang, window, schedule, seed, 1 if elide else 0,
                                ctypes.byref(ex))
    return st, ex.value


def tg_graph_emulate_schedule(g, nworkers: int, window: int = 64, seed: int = 0, schedule: int = 0):
    """One graph: (status, execution order by event)."""
    st, pairs, _, _ = tg_emulate_schedule(g, nworkers, window, seed, schedule)
    return st, pairs[:, 1].astype(np.uint32)


def tg_reduce_dag(row_ptr, col):
    """Two-hop reduction of an out-edge CSR whose ids are a topological order:
    returns (row_ptr, col) without edges implied by a two-edge path."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    cl = np.ascontiguousarray(col, dtype=np.uint32)
    n = rp.size - 1
    orp = np.zeros(n + 1, np.uint64)
    ocl = np.zeros(max(cl.size, 1), np.uint32)
    e = ctypes.c_uint64()
    _check(load().tg_reduce_dag(n, _ptr(rp), _ptr(cl) if cl.size else None, _ptr(orp), _ptr(ocl), ctypes.byref(e)),
           "tg_reduce_dag")
    return orp, ocl[:e.value]


def tg_last_user_dag(req_ptr, reqs: np.ndarray):
    """Last-user dependences of an implicit program given as requirement rows
    (host): returns the out-edge CSR (row_ptr, col)."""
    rp = np.ascontiguousarray(req_ptr, dtype=np.uint64)
    r = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    n = rp.size - 1
    orp = np.zeros(n + 1, np.uint64)
    e = ctypes.c_uint64()
    cap = max(int(r.size) * 4, 16)
    while True:
        ocl = np.zeros(cap, np.uint32)
        st = load().tg_last_user_dag(n, _ptr(rp), _ptr(r) if r.size else None, _ptr(orp), _ptr(ocl), cap,
                                     ctypes.byref(e))
        if st == TG_ENOMEM and e.value > cap:
            cap = int(e.value)
            continue
        _check(st, "tg_last_user_dag")
        return orp, ocl[:e.value]


def tg_graph_reduce_edges(g) -> int:
    """Execute an implicit graph on its reduced DAG (the two-hop reduction of
    its last-user DAG); returns the number of inferred edges not executed
    (tg_graph_read_dag still returns all)."""
    removed = ctypes.c_uint64()
    _check(load().tg_graph_reduce_edges(g, ctypes.byref(removed)), "tg_graph_reduce_edges")
    return removed.value


def tg_infer_dag(ntasks: int, req_ptr, reqs, nreqs: int, index_space: int, row_ptr, col, col_cap: int,
                 stream=None) -> int:
    """Dependence inference on device arrays (torch tensors or addresses):
    req_ptr u64[ntasks+1], reqs tg_region_req[nreqs] (32 bytes each), output
    row_ptr u64[ntasks+1] and col u32[col_cap].  Returns the edge count."""
    e = ctypes.c_uint64()
    _check(load().tg_infer_dag(ntasks, _dptr(req_ptr), _dptr(reqs), nreqs, index_space, _dptr(row_ptr), _dptr(col),
                               col_cap, ctypes.byref(e), _stream(stream)), "tg_infer_dag")
    return e.value


def tg_infer_dag_noalloc(ntasks: int, req_ptr, reqs, nreqs: int, index_space: int, row_ptr, col, col_cap: int,
                         stream=None) -> int:
    """tg_infer_dag without any device allocation (the library's fixed
    scratch array); same arguments and result."""
    e = ctypes.c_uint64()
    _check(load().tg_infer_dag_noalloc(ntasks, _dptr(req_ptr), _dptr(reqs), nreqs, index_space, _dptr(row_ptr),
                                       _dptr(col), col_cap, ctypes.byref(e), _stream(stream)), "tg_infer_dag_noalloc")
    return e.value


def tg_graph_execute_comparator(g, mode: int, stream=None):
    _check(load().tg_graph_execute_comparator(g, mode, _stream(stream)), "tg_graph_execute_comparator")


# -------------------------------------------------------------- batches


def tg_batch_create(graphs, cfg: tg_exec_config | None = None):
    arr = (ctypes.c_void_p * len(graphs))(*[g.value if isinstance(g, ctypes.c_void_p) else g for g in graphs])
    b = ctypes.c_void_p()
    _check(load().tg_batch_create(ctypes.byref(b), arr, len(graphs), ctypes.byref(cfg) if cfg is not None else None),
           "tg_batch_create")
    return b


def tg_batch_execute(b, stream=None):
    _check(load().tg_batch_execute(b, _stream(stream)), "tg_batch_execute")


def tg_batch_wait(b):
    _check(load().tg_batch_wait(b), "tg_batch_wait")


def tg_batch_time_ms(b) -> float:
    ms = ctypes.c_double()
    _check(load().tg_batch_time_ms(b, ctypes.byref(ms)), "tg_batch_time_ms")
    return ms.value


def tg_batch_kernel_times(b, n: int = 64) -> np.ndarray:
    out = np.zeros(max(n, 1), np.float64)
    got = ctypes.c_uint32()
    _check(load().tg_batch_kernel_times(b, _ptr(out), n, ctypes.byref(got)), "tg_batch_kernel_times")
    return out[:got.value]


def tg_batch_set_rounds(b, rounds: int):
    _check(load().tg_batch_set_rounds(b, rounds), "tg_batch_set_rounds")


def tg_batch_signalled_edges(b) -> int:
    """Edges the batch's layout signals with a counter atomic per launch."""
    e = ctypes.c_uint64()
    _check(load().tg_batch_signalled_edges(b, ctypes.byref(e)), "tg_batch_signalled_edges")
    return e.value


def tg_batch_info(b, with_times: bool = False):
    c = tg_exec_config()
    n = ctypes.c_uint64()
    pm, bm = ctypes.c_double(), ctypes.c_double()
    _check(load().tg_batch_info(b, ctypes.byref(c), ctypes.byref(n), ctypes.byref(pm), ctypes.byref(bm)),
           "tg_batch_info")
    cfg = {f: getattr(c, f) for f, _ in tg_exec_config._fields_}
    if with_times:
        return cfg, n.value, {"plan_ms": pm.value, "build_ms": bm.value}
    return cfg, n.value


def tg_batch_autotune(b, reps: int = 2):
    c = tg_exec_config()
    ms = ctypes.c_double()
    _check(load().tg_batch_autotune(b, reps, ctypes.byref(c), ctypes.byref(ms)), "tg_batch_autotune")
    return {f: getattr(c, f) for f, _ in tg_exec_config._fields_}, ms.value


def tg_batch_destroy(b):
    if b:
        _check(load().tg_batch_destroy(b), "tg_batch_destroy")


# ------------------------------------------------------------- serving


def tg_server_create(budget_bytes: int, slots: int = 4, max_batch: int = 64):
    use_torch_allocator()
    srv = ctypes.c_void_p()
    _check(load().tg_server_create(ctypes.byref(srv), budget_bytes, slots, max_batch), "tg_server_create")
    return srv


def tg_server_configure(srv, cfg: tg_exec_config):
    _check(load().tg_server_configure(srv, ctypes.byref(cfg)), "tg_server_configure")


def tg_server_submit(srv, g) -> int:
    t = ctypes.c_uint64()
    _check(load().tg_server_submit(srv, g, ctypes.byref(t)), "tg_server_submit")
    return t.value


def tg_server_wait(srv, ticket: int):
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().tg_server_wait(srv, ticket, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "tg_server_wait")
    return a.value, b.value, c.value


def tg_server_stats(srv):
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    ph = (ctypes.c_double * 9)()
    _check(load().tg_server_stats(srv, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ph), "tg_server_stats")
    return {"tasks_done": a.value, "launches": b.value, "peak_bytes": c.value,
            "host_build_ms": ph[0], "host_launch_ms": ph[1], "host_retire_ms": ph[2], "device_ms": ph[3],
            "host_plan_ms": ph[4], "host_alloc_ms": ph[5], "host_copy_ms": ph[6], "host_setup_ms": ph[7],
            "host_tables_ms": ph[8]}


def tg_server_destroy(srv):
    if srv:
        _check(load().tg_server_destroy(srv), "tg_server_destroy")


# ------------------------------------------------------ convenience layer


@dataclass
class Graph:
    """Owning wrapper of a tg_graph handle."""
    handle: ctypes.c_void_p
    mode: int
    n: int = 0

    def __del__(self):
        try:
            if self.handle:
                tg_graph_destroy(self.handle)
                self.handle = ctypes.c_void_p()
        except Exception:
            pass


def graph_from_explicit(eg, finalize: bool = True, retention: int = TG_KEEP_ALL) -> Graph:
    """Build a library graph from a workloads.ExplicitGraph (bulk add)."""
    h = tg_graph_create(TG_EXPLICIT, eg.n, 0, eg.seed)
    g = Graph(h, TG_EXPLICIT, eg.n)
    if retention != TG_KEEP_ALL:
        tg_graph_set_retention(h, retention)
    if eg.N:
        tg_task_add_many(h, eg.pred_ptr, eg.preds, None, eg.rounds)
    if finalize:
        tg_graph_finalize(h)
    return g


def graph_from_implicit(ig, finalize: bool = True) -> Graph:
    """Build a library graph from a workloads.ImplicitGraph (bulk add)."""
    h = tg_graph_create(TG_IMPLICIT, 0, ig.space, ig.seed)
    g = Graph(h, TG_IMPLICIT)
    if ig.N:
        tg_task_add_regions_many(h, ig.req_ptr, reqs_array(ig.lo, ig.hi, ig.priv), None, ig.rounds)
    if finalize:
        tg_graph_finalize(h)
    return g
