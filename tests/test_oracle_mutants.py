"""The oracle's pins have power: a copy of oracle.c with one plausible
one-line mistake planted in it (a dropped term, a wrong index, a swapped
privilege test, a wrong generator stream) is compiled on the CPU, and at
least one pin must reject it.  Mistakes are planted only in temporary
copies of the oracle; nothing here touches the HIP library."""
import contextlib
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2508_16522_amd import workloads as wl
from tests import _checks as C
from tests import test_oracle_pins as pins

pytestmark = pytest.mark.usefixtures("oracle_lib")

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")

# name -> (exact text of the correct line(s), planted mistake)
MUTANTS = {
    "implicit_drops_task_id": (
        "A[e] = or_mix(A[e] ^ c ^ k, rounds);",
        "A[e] = or_mix(A[e] ^ c, rounds);"),
    "implicit_restarts_ordinal_per_interval": (
        "    if (priv[a] == OR_RW)\n      for (e = lo[a]; e < hi[a]; e++) {",
        "    if (priv[a] == OR_RW)\n      for (j = 0, e = lo[a]; e < hi[a]; e++) {"),
    "implicit_sums_only_first_ro_interval": (
        "    if (priv[a] == OR_RO)\n      for (e = lo[a]; e < hi[a]; e++) c += A[e];",
        "    if (priv[a] == OR_RO)\n      for (c = 0, e = lo[a]; e < hi[a]; e++) c += A[e];"),
    "implicit_digest_weight_off_by_one": (
        "d += A[e] * (2u * j + 1u);",
        "d += A[e] * (2u * j + 3u);"),
    "implicit_initial_array_wrong_stream": (
        "for (e = 0; e < space; e++) A[e] = or_h32(seed, 2, e);",
        "for (e = 0; e < space; e++) A[e] = or_h32(seed, 1, e);"),
    "explicit_drops_task_id": (
        "payload[(size_t)v * n + k] = or_mix(in ^ v, rounds[v]);",
        "payload[(size_t)v * n + k] = or_mix(in, rounds[v]);"),
    "explicit_source_key_wrong_shift": (
        "in = or_h32(seed, 1, ((uint64_t)v << 16) | k);",
        "in = or_h32(seed, 1, ((uint64_t)v << 8) | k);"),
    "explicit_digest_weight": (
        "for (k = 0; k < n; k++) d += payload[(size_t)v * n + k] * (2u * k + 1u);",
        "for (k = 0; k < n; k++) d += payload[(size_t)v * n + k] * (2u * k + 2u);"),
    "checksum_weight": (
        "for (v = 0; v < N; v++) c += (uint64_t)digest[v] * (2ull * v + 1ull);",
        "for (v = 0; v < N; v++) c += (uint64_t)digest[v] * (2ull * v);"),
    "duplicate_preds_not_merged": (
        "if (r == start || s->idx[r] != s->idx[o - 1]) s->idx[o++] = s->idx[r];",
        "s->idx[o++] = s->idx[r];"),
    "conflict_needs_both_writers": (
        "if (overlap(lo[a], hi[a], lo[b], hi[b]) && (priv[a] == OR_RW || priv[b] == OR_RW)) return 1;",
        "if (overlap(lo[a], hi[a], lo[b], hi[b]) && (priv[a] == OR_RW && priv[b] == OR_RW)) return 1;"),
    "overlap_closed_intervals": (
        "return lo < hi;",
        "return lo <= hi;"),
    "mix_wrong_shift": (
        "x ^= x >> 17;",
        "x ^= x >> 15;"),
    "mix_wrong_additive_constant": (
        "x = x * 0x9E3779B1u + 0x7F4A7C15u;",
        "x = x * 0x9E3779B1u + 0x7F4A7C13u;"),
    "sm64_wrong_gamma": (
        "z += 0x9E3779B97F4A7C15ull;",
        "z += 0x9E3779B97F4A7C17ull;"),
}


def _build_mutant(name, tmp_path):
    good, bad = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(good) == 1, f"{name}: the correct text must occur exactly once in oracle.c"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(good, bad))
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", str(path), "-o", str(lib)])
    return str(lib)


@contextlib.contextmanager
def _oracle_from(libpath):
    """Temporarily point the oracle binding at another build of oracle.c."""
    saved = oracle._lib
    oracle._lib = None
    real = oracle._LIB
    oracle._LIB = libpath
    try:
        oracle.lib()
        yield
    finally:
        oracle._lib = saved
        oracle._LIB = real


def _pin_suite():
    """The pins a mutant is run against (each raises AssertionError or
    RuntimeError on a wrong oracle)."""
    pins.test_mix_vectors_literal()
    pins.test_sm64_h32_vectors_literal()
    for p in wl.PATTERNS:
        pins.test_execution_order_is_exactly_once_and_respects_edges(p)
    pins.test_duplicate_predecessors_are_a_set()
    pins.test_c1_config_checksum_is_stable()
    for seed in range(2):
        pins.test_implicit_multi_interval_rederived(seed)
        pins.test_conflict_dag_equals_element_set_rule(seed)
    pins.test_implicit_halo_rederived()
    # checksum weights
    eg = wl.pattern_graph("random", 9, 5, seed=1, n=64, rounds=2)
    r = oracle.exec_explicit(eg.N, eg.n, eg.pred_ptr, eg.preds, eg.rounds, seed=1)
    assert r["checksum"] == C.checksum_py(r["digest"])


def test_pin_suite_accepts_the_oracle():
    _pin_suite()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    lib = _build_mutant(name, tmp_path)
    with _oracle_from(lib):
        with pytest.raises((AssertionError, RuntimeError)):
            _pin_suite()
