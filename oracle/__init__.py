"""Reference oracle for the task-DAG executor -- TEST INFRASTRUCTURE ONLY.

A plain, sequential CPU implementation (``oracle.c``) of what the executor
computes, loaded with ctypes.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does, and shares no code with it.

Functions follow the paper (Yadav et al., "On the Duality of Task and Actor
Programming Models"): Algorithm 1 for explicit execution, Section 5 for the
sequential semantics of implicitly parallel programs.  The readings used where
the paper is silent are listed in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_OK, OR_EINVAL, OR_ENOMEM, OR_ECYCLE, OR_EORDER = 0, -1, -2, -3, -4
RO, RW = 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc -O2, single thread, no SIMD
    intrinsics; the compiler may auto-vectorise)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        P = ctypes.c_void_p
        L.or_sm64.restype, L.or_sm64.argtypes = u64, [u64]
        L.or_h32.restype, L.or_h32.argtypes = u32, [u64, u32, u64]
        L.or_xorshift32.restype, L.or_xorshift32.argtypes = u32, [u32]
        L.or_mix.restype, L.or_mix.argtypes = u32, [u32, u32]
        L.or_exec_explicit.restype = i32
        L.or_exec_explicit.argtypes = [u32, u32, P, P, P, u64, P, P, P, P]
        L.or_exec_in_order.restype = i32
        L.or_exec_in_order.argtypes = [u32, u32, P, P, P, u64, P, P, P, P]
        L.or_implicit_program_order.restype = i32
        L.or_implicit_program_order.argtypes = [u32, P, P, P, P, P, u64, u64, P, P, P]
        L.or_implicit_in_order.restype = i32
        L.or_implicit_in_order.argtypes = [u32, P, P, P, P, P, u64, u64, P, P, P, P]
        L.or_conflict_dag.restype = i32
        L.or_conflict_dag.argtypes = [u32, P, P, P, P, P, P, u64, P]
        L.or_conflict_row.restype = i32
        L.or_conflict_row.argtypes = [u32, P, P, P, P, u32, P, u64, P]
        L.or_conflict_preds.restype = i32
        L.or_conflict_preds.argtypes = [u32, P, P, P, P, u32, P, u64, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def sm64(z: int) -> int:
    return int(lib().or_sm64(z))


def h32(seed: int, stream: int, idx: int) -> int:
    return int(lib().or_h32(seed, stream, idx))


def xorshift32(x: int) -> int:
    return int(lib().or_xorshift32(x))


def mix(x: int, rounds: int) -> int:
    return int(lib().or_mix(x, rounds))


def _rounds(N, rounds):
    if np.isscalar(rounds):
        return np.full(N, int(rounds), dtype=np.uint32)
    r = _u32(rounds)
    assert r.shape == (N,)
    return r


def exec_explicit(N, n, pred_ptr, preds, rounds, seed=0, want_payload=True, want_order=False):
    """Kahn FIFO execution (Algorithm 1).  Returns dict with digest, checksum
    and optionally payload (N x n) and execution order."""
    pred_ptr, preds, R = _u64(pred_ptr), _u32(preds), _rounds(N, rounds)
    assert pred_ptr.shape == (N + 1,)
    if preds.size == 0:
        preds = np.zeros(1, np.uint32)
    digest = np.zeros(max(N, 1), np.uint32)
    payload = np.zeros((N, n), np.uint32) if want_payload else None
    order = np.zeros(max(N, 1), np.uint32) if want_order else None
    cs = ctypes.c_uint64(0)
    rc = lib().or_exec_explicit(N, n, _p(pred_ptr), _p(preds), _p(R), seed,
                                _p(payload) if payload is not None else None, _p(digest),
                                _p(order) if order is not None else None, ctypes.byref(cs))
    if rc != OR_OK:
        raise RuntimeError(f"or_exec_explicit failed: {rc}")
    out = {"digest": digest[:N], "checksum": int(cs.value)}
    if payload is not None:
        out["payload"] = payload
    if order is not None:
        out["order"] = order[:N]
    return out


def exec_in_order(N, n, pred_ptr, preds, rounds, order, seed=0):
    pred_ptr, preds, R, order = _u64(pred_ptr), _u32(preds), _rounds(N, rounds), _u32(order)
    if preds.size == 0:
        preds = np.zeros(1, np.uint32)
    digest = np.zeros(max(N, 1), np.uint32)
    payload = np.zeros((N, n), np.uint32)
    cs = ctypes.c_uint64(0)
    rc = lib().or_exec_in_order(N, n, _p(pred_ptr), _p(preds), _p(R), seed, _p(order),
                                _p(payload), _p(digest), ctypes.byref(cs))
    return rc, {"digest": digest[:N], "checksum": int(cs.value), "payload": payload}


def _req_arrays(req_ptr, lo, hi, priv):
    req_ptr, lo, hi, priv = _u64(req_ptr), _u64(lo), _u64(hi), _u32(priv)
    if lo.size == 0:
        lo, hi, priv = np.zeros(1, np.uint64), np.zeros(1, np.uint64), np.ones(1, np.uint32)
    return req_ptr, lo, hi, priv


def implicit_program_order(N, req_ptr, lo, hi, priv, rounds, space, seed=0):
    """Sequential program-order execution (Section 5).  Returns dict with the
    final array A, digest and checksum."""
    req_ptr, lo, hi, priv = _req_arrays(req_ptr, lo, hi, priv)
    R = _rounds(N, rounds)
    A = np.zeros(max(space, 1), np.uint32)
    digest = np.zeros(max(N, 1), np.uint32)
    cs = ctypes.c_uint64(0)
    rc = lib().or_implicit_program_order(N, _p(req_ptr), _p(lo), _p(hi), _p(priv), _p(R), seed,
                                         space, _p(A), _p(digest), ctypes.byref(cs))
    if rc != OR_OK:
        raise RuntimeError(f"or_implicit_program_order failed: {rc}")
    return {"A": A[:space], "digest": digest[:N], "checksum": int(cs.value)}


def implicit_in_order(N, req_ptr, lo, hi, priv, rounds, space, order, seed=0):
    req_ptr, lo, hi, priv = _req_arrays(req_ptr, lo, hi, priv)
    R, order = _rounds(N, rounds), _u32(order)
    A = np.zeros(max(space, 1), np.uint32)
    digest = np.zeros(max(N, 1), np.uint32)
    cs = ctypes.c_uint64(0)
    rc = lib().or_implicit_in_order(N, _p(req_ptr), _p(lo), _p(hi), _p(priv), _p(R), seed, space,
                                    _p(order), _p(A), _p(digest), ctypes.byref(cs))
    if rc != OR_OK:
        raise RuntimeError(f"or_implicit_in_order failed: {rc}")
    return {"A": A[:space], "digest": digest[:N], "checksum": int(cs.value)}


def conflict_dag(N, req_ptr, lo, hi, priv, cap=None):
    """Brute-force O(N^2 r^2) conflict DAG as CSR of successors."""
    req_ptr, lo, hi, priv = _req_arrays(req_ptr, lo, hi, priv)
    if cap is None:
        cap = max(1, N * 8)
    while True:
        row_ptr = np.zeros(N + 1, np.uint64)
        col = np.zeros(cap, np.uint32)
        E = ctypes.c_uint64(0)
        rc = lib().or_conflict_dag(N, _p(req_ptr), _p(lo), _p(hi), _p(priv), _p(row_ptr), _p(col),
                                   cap, ctypes.byref(E))
        if rc == OR_OK:
            return row_ptr, col[:E.value].copy()
        if rc == OR_ENOMEM:
            cap = int(E.value)
            continue
        raise RuntimeError(f"or_conflict_dag failed: {rc}")


def _row(fn, N, req_ptr, lo, hi, priv, j):
    req_ptr, lo, hi, priv = _req_arrays(req_ptr, lo, hi, priv)
    cap = 1024
    while True:
        out = np.zeros(cap, np.uint32)
        cnt = ctypes.c_uint64(0)
        rc = fn(N, _p(req_ptr), _p(lo), _p(hi), _p(priv), j, _p(out), cap, ctypes.byref(cnt))
        if rc == OR_OK:
            return out[:cnt.value].copy()
        if rc == OR_ENOMEM:
            cap = int(cnt.value)
            continue
        raise RuntimeError(f"conflict row failed: {rc}")


def conflict_row(N, req_ptr, lo, hi, priv, j):
    """Successors of task j in the brute-force conflict DAG."""
    return _row(lib().or_conflict_row, N, req_ptr, lo, hi, priv, j)


def conflict_preds(N, req_ptr, lo, hi, priv, k):
    """Predecessors of task k in the brute-force conflict DAG."""
    return _row(lib().or_conflict_preds, N, req_ptr, lo, hi, priv, k)
