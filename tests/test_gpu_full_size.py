"""Parity at the benchmark configurations' full sizes, element by element
against the oracle (run in parallel worker processes where it would take
minutes on one core, or through values a committed script computed with the
oracle alone):

- the 65,536-task halo program: its inferred DAG, every one of the 65,536
  rows against the brute-force conflict DAG; its execution at 64 mix rounds
  over all 64 sweeps (every digest, the whole 2^24-element array, the
  checksum), in the launch shape the benchmark times and on the reduced DAG;
- the 4096-graph batch in one persistent launch: a seeded, stratified sample
  of graphs covering every (pattern, payload size) cell and the graphs with
  the most mix rounds under a stated oracle-cost cap;
- serving at the real request-size distribution (log-normal, median 4096
  tasks, sigma 1, sizes capped at 2^15 tasks), every request's digests and
  checksum."""
import hashlib
import json
import os
import threading
import time

import numpy as np
import pytest

from bench_workloads import BATCH_CFG, request_graph, stratified_batch_sample
from oracle import parallel as opar
from paper_2508_16522_amd import taskgraph as tg
from paper_2508_16522_amd import workloads as wl
from tests import _checks as C

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "halo_program_r64.json")


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


@pytest.mark.timeout(600)
def test_halo_program_dag_every_row(gpu):
    ig = wl.halo_graph(1024, 16384, 64, seed=0, rounds=64)
    g = tg.graph_from_implicit(ig)
    row_ptr, col = tg.tg_graph_read_dag(g.handle)
    ref_ptr, ref_col = opar.halo_conflict_dag(1024, 16384, 64, seed=0)
    assert ref_col.size == C.halo_edge_count(1024, 64) == 6254592
    assert np.array_equal(row_ptr, ref_ptr), "row pointers differ"
    if not np.array_equal(col, ref_col):
        bad = [j for j in range(ig.N) if not np.array_equal(col[row_ptr[j]:row_ptr[j + 1]],
                                                            ref_col[ref_ptr[j]:ref_ptr[j + 1]])]
        pytest.fail(f"{len(bad)} rows differ, first {bad[:8]}")


def _check_halo_r64(g, gold):
    P, S = 1024, 16384
    A = tg.tg_graph_read_data(g.handle, 0, P * S)
    d = tg.tg_graph_read_digests(g.handle)
    if _sha(d) != gold["digest_sha256"]:
        sweeps = [i for i in range(64) if _sha(d[i * P:(i + 1) * P]) != gold["sweep_digest_sha256"][i]]
        pytest.fail(f"digests differ in sweeps {sweeps[:8]}")
    if _sha(A) != gold["array_sha256"]:
        subs = [s for s in range(P) if _sha(A[s * S:(s + 1) * S])[:16] != gold["subregion_array_sha256_16"][s]]
        pytest.fail(f"final array differs in subregions {subs[:8]}")
    assert f"{tg.tg_graph_checksum(g.handle):#018x}" == gold["checksum"]


@pytest.mark.timeout(300)
def test_halo_program_r64_all_sweeps(gpu):
    """The whole program at 64 mix rounds in the benchmark's launch shape
    (gangs of eight 8-wave workgroups), then on the reduced DAG."""
    with open(GOLDEN) as f:
        gold = json.load(f)
    ig = wl.halo_graph(1024, 16384, 64, seed=0, rounds=64)
    assert gold["tasks"] == ig.N and gold["rounds"] == 64
    g = tg.graph_from_implicit(ig)
    for cfg in (tg.make_config(mapping=3, gang=8, wg_waves=8, schedule=tg.TG_SCHED_LEVEL),
                tg.make_config(mapping=3, gang=4, wg_waves=16)):
        tg.tg_graph_execute(g.handle, cfg)
        tg.tg_graph_wait(g.handle)
        _check_halo_r64(g, gold)
    tg.tg_graph_reduce_edges(g.handle)
    tg.tg_graph_execute(g.handle, tg.make_config(mapping=3, gang=8, wg_waves=8))
    tg.tg_graph_wait(g.handle)
    _check_halo_r64(g, gold)


@pytest.mark.timeout(900)
def test_batch_4096_graphs_stratified(gpu):
    specs = wl.batch_manifest(4096, seed=0)
    sample = stratified_batch_sample(specs)
    cells = {(specs[i].pattern, specs[i].n) for i in sample}
    assert len(sample) >= 64 and len(cells) == 25
    # as the benchmark runs them: payload memory reused once read
    gs = [request_graph(wl.pattern_graph(s.pattern, s.W, s.T, seed=s.seed, n=s.n, rounds=s.rounds)) for s in specs]
    b = tg.tg_batch_create([g.handle for g in gs], tg.make_config(**BATCH_CFG))
    try:
        tg.tg_batch_execute(b)
        tg.tg_batch_wait(b)
    finally:
        tg.tg_batch_destroy(b)
    refs = opar.explicit_many([(specs[i].pattern, specs[i].W, specs[i].T, specs[i].seed, specs[i].n,
                                specs[i].rounds) for i in sample])
    bad = []
    for i, (dig, cs, _) in zip(sample, refs):
        if not (np.array_equal(tg.tg_graph_read_digests(gs[i].handle), dig) and tg.tg_graph_checksum(gs[i].handle) == cs):
            bad.append(i)
    assert not bad, f"graphs {bad} differ from the oracle"


@pytest.mark.timeout(600)
def test_serving_real_size_distribution(gpu):
    """256 requests drawn like the serving workload (Poisson 2000/s, sizes
    log-normal with median 4096 tasks and sigma 1, capped at 2^15 tasks,
    explicit and implicit 1:1, log-normal mix rounds) replayed in real time;
    every request's digests and checksum equal the oracle's."""
    reqs = wl.serving_manifest(256, rate=2000.0, seed=3, max_tasks=1 << 15)
    graphs = [wl.build_request(r) for r in reqs]
    # as the benchmark serves them: explicit requests reuse payload memory,
    # implicit requests execute their reduced DAG
    handles = [request_graph(x) for x in graphs]
    srv = tg.tg_server_create(64 << 30, slots=4, max_batch=64)
    tickets = [None] * len(reqs)
    try:
        def client():
            t0 = time.perf_counter()
            for i, r in enumerate(reqs):
                dt = r.arrival_s - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = tg.tg_server_submit(srv, handles[i].handle)

        th = threading.Thread(target=client)
        th.start()
        th.join()
        for t in tickets:
            tg.tg_server_wait(srv, t)
    finally:
        tg.tg_server_destroy(srv)
    exp = [i for i, r in enumerate(reqs) if r.mode == "explicit"]
    imp = [i for i, r in enumerate(reqs) if r.mode == "implicit"]
    refs = dict(zip(exp, opar.explicit_many([(reqs[i].pattern, reqs[i].W, reqs[i].T, reqs[i].seed, reqs[i].n,
                                               reqs[i].rounds) for i in exp])))
    refs.update(zip(imp, opar.implicit_many([(reqs[i].P, 256, reqs[i].iters, reqs[i].seed, reqs[i].rounds)
                                             for i in imp])))
    bad = [i for i in range(len(reqs))
           if not (np.array_equal(tg.tg_graph_read_digests(handles[i].handle), refs[i][0]) and
                   tg.tg_graph_checksum(handles[i].handle) == refs[i][1])]
    assert not bad, f"requests {bad[:8]} differ from the oracle"
