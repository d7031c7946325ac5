"""Writes halo_program_r64.json: the oracle's result for the full halo
program (65,536 tasks over 2^24 u32 elements in 1024 subregions of 16,384,
64 sweeps, halos 1..64 wide, 64 mix rounds per element, seed 0), in
sequential program order.  The oracle needs minutes for it on one core, so
the GPU parity test compares against these stored values: the checksum,
SHA-256 of the digest array and of the final array (little-endian u32), and
per-sweep / per-subregion hashes that locate a difference.  Calls only the
oracle and the seeded input generator.

    python tests/golden/make_halo_program_r64.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2508_16522_amd import workloads as wl  # noqa: E402

P, S, ITERS, R, SEED = 1024, 16384, 64, 64, 0


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


def main():
    ig = wl.halo_graph(P, S, ITERS, seed=SEED, rounds=R)
    t0 = time.time()
    ref = oracle.implicit_program_order(ig.N, ig.req_ptr, ig.lo, ig.hi, ig.priv, R, ig.space, seed=SEED)
    secs = time.time() - t0
    A, d = ref["A"], ref["digest"]
    out = {
        "workload": f"halo program: {P} subregions of {S} u32, {ITERS} sweeps ({ig.N} tasks), halos 1..64, "
                    f"{R} mix rounds, seed {SEED}",
        "tasks": ig.N, "space": ig.space, "rounds": R, "seed": SEED,
        "checksum": f"{ref['checksum']:#018x}",
        "digest_sha256": sha(d),
        "array_sha256": sha(A),
        "sweep_digest_sha256": [sha(d[i * P:(i + 1) * P]) for i in range(ITERS)],
        "subregion_array_sha256_16": [sha(A[s * S:(s + 1) * S])[:16] for s in range(P)],
        "oracle_seconds": round(secs, 1),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "halo_program_r64.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} ({secs:.0f} s of oracle time)")


if __name__ == "__main__":
    main()
