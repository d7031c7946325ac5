"""The executor's publication rule, checked on the kernel source (CPU only).

Data one task hands to another -- counters, queue slots and control words,
doorbells, per-graph completion counts, the control block, digests, payloads
and the implicit array -- is read and written only through the device-coherent
helpers (agent-scope atomics `ld_coherent` / `st_coherent` / `__hip_atomic_*`,
`sc1` buffer loads and stores `buf_load` / `buf_store`); a plain access is
allowed only in the kernels that run before the executor in stream order (the
reset, queue clear and queue seed).  Diagnostics the host reads after a launch
are exempt.  The helpers themselves must keep their scope, and a task's edge
signals must follow its store drain."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2508_16522_amd", "csrc", "tg_kernels.hip")

# plain accesses are fine here: these kernels run before the executor on the
# same stream, so the kernel boundary orders them
BEFORE_EXECUTOR = {"k_reset", "k_queue_clear", "k_queue_seed"}
SHARED = re.compile(r"P\.(cnt|q|qctl|bell|gdone)\s*\[|P\.ctrl\s*->|\.digest\s*\[|\.out\s*\[|\bA\s*\[|\ba\s*\[")
COHERENT = ("ld_coherent(", "st_coherent(", "__hip_atomic_", "buf_load", "buf_store", "__builtin_amdgcn_raw_buffer_")


def _source():
    s = open(SRC).read()
    s = re.sub(r"/\*.*?\*/", "", s, flags=re.S)
    return re.sub(r"//[^\n]*", "", s)


def _functions(src):
    """(name, body) of every __global__ / __device__ definition."""
    out = []
    for m in re.finditer(r"(__global__|__device__)\b[^;{}]*?\b(\w+)\s*\(", src):
        name = m.group(2)
        if name in ("__launch_bounds__", "__attribute__"):
            name = re.search(r"\bvoid\s+(\w+)\s*\(", src[m.start():]).group(1)
            j = m.start() + re.search(r"\bvoid\s+\w+\s*\(", src[m.start():]).end()
        else:
            j = m.end()
        depth = 1
        while depth:  # the parameter list
            depth += (src[j] == "(") - (src[j] == ")")
            j += 1
        k = j
        while src[k] not in "{;":
            k += 1
        if src[k] == ";":
            continue  # a declaration
        depth, e = 0, k
        while True:
            depth += (src[e] == "{") - (src[e] == "}")
            e += 1
            if depth == 0:
                break
        out.append((name, src[k:e]))
    return out


def test_functions_found():
    names = {n for n, _ in _functions(_source())}
    for k in ("k_exec_wave", "k_exec_block", "k_exec_gang", "k_exec_wave_q", "k_exec_block_q", "k_reset",
              "body_explicit", "body_implicit", "complete_edges", "signal_edge", "ready_scan", "queue_next"):
        assert k in names, k


def test_shared_data_only_through_coherent_helpers():
    bad = []
    for name, body in _functions(_source()):
        if name in BEFORE_EXECUTOR:
            continue
        for stmt in body.split(";"):
            if SHARED.search(stmt) and not any(h in stmt for h in COHERENT):
                bad.append(f"{name}: {' '.join(stmt.split())[:160]}")
    assert not bad, "plain access to cross-task data:\n" + "\n".join(bad)


def test_helpers_keep_their_scope():
    f = dict(_functions(_source()))
    assert "__HIP_MEMORY_SCOPE_AGENT" in f["ld_coherent"] and "__hip_atomic_load" in f["ld_coherent"]
    assert "__HIP_MEMORY_SCOPE_AGENT" in f["st_coherent"] and "__hip_atomic_store" in f["st_coherent"]
    for h in ("buf_load", "buf_store"):
        assert f[h].count("kSC1") == 3, h  # every width carries the device-coherence bit
    assert "s_waitcnt vmcnt(0)" in f["vm_drain"]
    # the buffer cache-policy bit the payload accesses carry: SC1 (device scope)
    assert re.search(r"constexpr int kSC1 = 16;", _source())


def test_edge_signals_follow_the_drain():
    f = dict(_functions(_source()))
    for k in ("complete_edges", "complete_edges_q"):
        body = f[k]
        assert "vm_drain()" in body, k
        first_signal = min(i for i in (body.find("signal_edge"), body.find("__hip_atomic_fetch")) if i >= 0)
        assert body.find("vm_drain()") < first_signal, k
