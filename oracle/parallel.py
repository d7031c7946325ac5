"""Runs the oracle on many independent inputs in parallel worker processes --
TEST INFRASTRUCTURE ONLY (the test-suite, the smoke check and the benchmark's
CPU-baseline and parity legs).

Every worker is a fresh process (spawned, not forked, so none inherits a GPU
context) that imports only the oracle and the seeded input generator.  A job
is a small spec from which the worker rebuilds its input with the input
generator, so nothing large crosses process boundaries except results.
Each oracle call is the plain sequential one; the pool only runs several
of them side by side.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np


def default_workers() -> int:
    """Worker processes to use: the cores this process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _explicit_job(spec):
    import oracle
    from paper_2508_16522_amd import workloads as wl
    pattern, W, T, seed, n, rounds = spec
    eg = wl.pattern_graph(pattern, W, T, seed=seed, n=n, rounds=rounds)
    t0 = time.perf_counter()
    r = oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, eg.rounds, seed=eg.seed, want_payload=False)
    return r["digest"], r["checksum"], time.perf_counter() - t0


def _implicit_job(spec):
    import oracle
    from paper_2508_16522_amd import workloads as wl
    P, S, iters, seed, rounds = spec
    ig = wl.halo_graph(P, S, iters, seed=seed, rounds=rounds)
    t0 = time.perf_counter()
    r = oracle.implicit_program_order(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv, ig.rounds, ig.space, seed=ig.seed)
    return r["digest"], r["checksum"], time.perf_counter() - t0


def _halo_rows_job(spec):
    import oracle
    from paper_2508_16522_amd import workloads as wl
    P, S, iters, seed, j0, j1 = spec
    ig = wl.halo_graph(P, S, iters, seed=seed)
    counts = np.zeros(j1 - j0, np.uint64)
    cols = []
    for j in range(j0, j1):
        row = oracle.conflict_row(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv, j)
        counts[j - j0] = row.size
        cols.append(row)
    return j0, counts, (np.concatenate(cols) if cols else np.zeros(0, np.uint32))


def _map(fn, jobs, workers):
    """fn over jobs in `workers` spawned processes; the workers have exited
    when it returns (closed and joined, not terminated)."""
    p = mp.get_context("spawn").Pool(processes=workers)
    try:
        out = p.map(fn, list(jobs), chunksize=1)
        p.close()
        p.join()
        return out
    except BaseException:
        p.terminate()
        p.join()
        raise


def explicit_many(specs, workers=None):
    """specs: (pattern, W, T, seed, n, rounds) tuples.  Returns, in order,
    (digest array, checksum, oracle seconds) per spec."""
    return _map(_explicit_job, specs, workers or default_workers())


def implicit_many(specs, workers=None):
    """specs: (P, S, iters, seed, rounds) halo programs."""
    return _map(_implicit_job, specs, workers or default_workers())


def halo_conflict_dag(P, S, iters, seed=0, workers=None, chunk=2048):
    """The brute-force conflict DAG of a halo program, row by row (the
    oracle's conflict_row for every task), computed by `workers` processes.
    Returns (row_ptr, col)."""
    N = P * iters
    workers = workers or default_workers()
    jobs = [(P, S, iters, seed, j0, min(N, j0 + chunk)) for j0 in range(0, N, chunk)]
    parts = _map(_halo_rows_job, jobs, workers)
    parts.sort(key=lambda x: x[0])
    row_ptr = np.zeros(N + 1, np.uint64)
    row_ptr[1:] = np.cumsum(np.concatenate([c for _, c, _ in parts]))
    col = np.concatenate([x for _, _, x in parts]) if parts else np.zeros(0, np.uint32)
    return row_ptr, col
