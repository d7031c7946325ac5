"""Helpers shared by the GPU parity tests: run a workload on the HIP library
and on the oracle with the same seeded inputs and compare."""
import numpy as np

import oracle
from paper_2508_16522_amd import taskgraph as tg


def oracle_explicit(eg, want_payload=True):
    return oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, eg.rounds, seed=eg.seed,
                                want_payload=want_payload)


def sinks(eg):
    has_succ = np.zeros(eg.N, bool)
    if eg.E:
        has_succ[eg.preds.astype(np.int64)] = True
    return np.nonzero(~has_succ)[0]


def check_explicit(g, eg, ref, payload_sample=None):
    """Digests (every task), checksum, and payloads of the sinks plus a
    sample, all bit-exact."""
    d = tg.tg_graph_read_digests(g.handle)
    bad = np.nonzero(d != ref["digest"])[0]
    assert bad.size == 0, f"{bad.size} digests differ, first at task {bad[:5]}"
    assert tg.tg_graph_checksum(g.handle) == ref["checksum"]
    if "payload" in ref:
        ids = list(sinks(eg))
        if payload_sample:
            rng = np.random.default_rng(0)
            ids += list(rng.integers(0, eg.N, size=min(payload_sample, eg.N)))
        for v in ids[:4096]:
            got = tg.tg_graph_read_payload(g.handle, int(v), eg.n)
            assert np.array_equal(got, ref["payload"][v]), f"payload of task {v}"


def run(g, cfg=None):
    tg.tg_graph_execute(g.handle, cfg)
    tg.tg_graph_wait(g.handle)


def device_requirements(ig):
    """An implicit graph's requirement list in device memory, in the layout
    tg_infer_dag takes: (req_ptr u64[N+1], reqs tg_region_req[M]) as torch
    tensors (int64 and uint8 views of the same bytes)."""
    import torch
    r = tg.reqs_array(ig.lo, ig.hi, ig.priv)
    req_ptr = torch.from_numpy(np.ascontiguousarray(ig.req_ptr, np.uint64).view(np.int64)).cuda()
    raw = r.view(np.uint8) if r.size else np.zeros(32, np.uint8)
    reqs = torch.from_numpy(np.ascontiguousarray(raw)).cuda()
    return req_ptr, reqs


def infer_on_device(ig, col_cap=None, fn=None, stream=None):
    """Runs tg_infer_dag (or fn, same arguments) on ig's requirements;
    returns the CSR in host memory."""
    import torch
    req_ptr, reqs = device_requirements(ig)
    row = torch.full((ig.N + 1,), -1, dtype=torch.int64, device="cuda")
    # default capacity: every pair of tasks for small programs
    cap = int(col_cap if col_cap is not None else max(ig.N * (ig.N - 1) // 2 if ig.N <= 4096 else ig.N * 128, 64))
    col = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # the inputs are in place before another stream reads them
    E = (fn or tg.tg_infer_dag)(ig.N, req_ptr, reqs, int(ig.lo.size), ig.space, row, col, cap, stream)
    torch.cuda.synchronize()
    return row.cpu().numpy().view(np.uint64), col[:E].cpu().numpy().view(np.uint32)
