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
