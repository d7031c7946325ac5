"""Independent checks used to pin the oracle (test code only).

These are deliberately different formulations of the quantities the oracle
computes: an inverse of the mix built from inverse xorshift steps and the
modular inverse of the multiplier, numpy re-derivations of a task from its
stored predecessors, and element-set conflict tests."""
import itertools

import numpy as np

M32 = 0xFFFFFFFF
MUL = 0x9E3779B1
ADD = 0x7F4A7C15
MUL_INV = 0x0E8B2F51  # (MUL * MUL_INV) mod 2^32 == 1


def _undo_xorshift_left(y, s):
    # invert y = x ^ (x << s) by fixed-point iteration over 32 bits
    x = y
    for _ in range(32 // s + 1):
        x = (y ^ (x << s)) & M32
    return x


def _undo_xorshift_right(y, s):
    x = y
    for _ in range(32 // s + 1):
        x = y ^ (x >> s)
    return x


def unmix(y: int, rounds: int) -> int:
    for _ in range(rounds):
        y = ((y - ADD) * MUL_INV) & M32
        y = _undo_xorshift_left(y, 5)
        y = _undo_xorshift_right(y, 17)
        y = _undo_xorshift_left(y, 13)
    return y


def mix_np(x: np.ndarray, rounds) -> np.ndarray:
    """Vectorised mix; rounds may be an array broadcast against x."""
    x = x.astype(np.uint64) & np.uint64(M32)
    r = np.broadcast_to(np.asarray(rounds, dtype=np.int64), x.shape)
    for i in range(int(r.max()) if r.size else 0):
        act = r > i
        y = x
        y = (y ^ (y << np.uint64(13))) & np.uint64(M32)
        y = y ^ (y >> np.uint64(17))
        y = (y ^ (y << np.uint64(5))) & np.uint64(M32)
        y = (y * np.uint64(MUL) + np.uint64(ADD)) & np.uint64(M32)
        x = np.where(act, y, x)
    return x.astype(np.uint32)


def digest_np(payload_row: np.ndarray) -> int:
    k = np.arange(payload_row.size, dtype=np.uint64)
    return int((payload_row.astype(np.uint64) * (2 * k + 1)).sum() & np.uint64(M32))


def checksum_py(digests) -> int:
    return sum(int(d) * (2 * v + 1) for v, d in enumerate(digests)) % (1 << 64)


def pred_sets(pred_ptr, preds):
    N = len(pred_ptr) - 1
    return [sorted(set(int(p) for p in preds[pred_ptr[v]:pred_ptr[v + 1]])) for v in range(N)]


def topo_orders(N, sets, limit=None):
    """All topological orders of a tiny DAG by brute force over permutations."""
    out = []
    for perm in itertools.permutations(range(N)):
        pos = {v: i for i, v in enumerate(perm)}
        if all(pos[p] < pos[v] for v in range(N) for p in sets[v]):
            out.append(perm)
            if limit and len(out) >= limit:
                break
    return out


def element_conflict_dag(ig):
    """Conflict DAG by element sets: j -> k iff j < k and they touch a common
    element that at least one of them writes."""
    N = ig.N
    reads, writes = [], []
    for k in range(N):
        r, w = set(), set()
        for a in range(int(ig.req_ptr[k]), int(ig.req_ptr[k + 1])):
            elems = range(int(ig.lo[a]), int(ig.hi[a]))
            (w if int(ig.priv[a]) == 2 else r).update(elems)
        reads.append(r)
        writes.append(w)
    edges = set()
    for j in range(N):
        for k in range(j + 1, N):
            if writes[j] & (reads[k] | writes[k]) or reads[j] & writes[k]:
                edges.add((j, k))
    return edges


def halo_edge_count(P, iters):
    """Closed form of the conflict-DAG size of workloads.halo_graph: task
    (it, s) conflicts with (it', s) for it' < it, with (it', s-1) for it' <= it
    and with (it', s+1) for it' < it (halos are 1..hmax < S wide)."""
    return sum(it + (s >= 1) * (it + 1) + (s <= P - 2) * it for it in range(iters) for s in range(P))


# ------------------------------------------------- pure-Python generators

M64 = (1 << 64) - 1


def sm64_py(z: int) -> int:
    """SplitMix64 output for state z, in Python integers (a third
    implementation beside the oracle's C and the input generator's numpy)."""
    z = (z + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def h32_py(seed: int, stream: int, idx: int) -> int:
    key = sm64_py((seed ^ (stream << 32)) & M64)
    return sm64_py(key ^ idx) & M32


def mix_py(x: int, rounds: int) -> int:
    for _ in range(rounds):
        x ^= (x << 13) & M32
        x ^= x >> 17
        x ^= (x << 5) & M32
        x = (x * MUL + ADD) & M32
    return x


# ---------------------------------------------- implicit re-derivation

def implicit_program_np(ig, rounds=None):
    """Sequential program order re-derived with numpy from the element-level
    reading of the implicit body: for task k, c is the wrap sum of the
    current values of its read-only elements; its read-write intervals, in
    declaration order, are replaced by mix_R(A ^ c ^ k); the digest weights
    the j-th written element of the task (j counted across all its
    read-write intervals) by 2j+1.  Initial A[e] = h32(seed, 2, e) from the
    input generator's own SplitMix64.  Returns (A, digests)."""
    from paper_2508_16522_amd import workloads as wl
    R = ig.rounds if rounds is None else rounds
    A = wl.h32(ig.seed, 2, np.arange(ig.space, dtype=np.uint64)).astype(np.uint64)
    dig = np.zeros(ig.N, np.uint64)
    for k in range(ig.N):
        a0, a1 = int(ig.req_ptr[k]), int(ig.req_ptr[k + 1])
        c = 0
        for a in range(a0, a1):
            if int(ig.priv[a]) == 1:
                c += int(A[int(ig.lo[a]):int(ig.hi[a])].sum())
        c &= M32
        j = 0
        d = 0
        for a in range(a0, a1):
            if int(ig.priv[a]) != 2:
                continue
            lo, hi = int(ig.lo[a]), int(ig.hi[a])
            y = mix_np((A[lo:hi] ^ np.uint64(c) ^ np.uint64(k)).astype(np.uint32), R).astype(np.uint64)
            A[lo:hi] = y
            w = 2 * (j + np.arange(hi - lo, dtype=np.uint64)) + 1
            d += int((y * w).sum())
            j += hi - lo
        dig[k] = d & M32
    return A.astype(np.uint32), dig.astype(np.uint32)


def multi_interval_program(N, space, rng, rounds=3, seed=0, min_ro=2, min_rw=2, max_len=9):
    """Implicit program whose tasks each declare at least min_rw read-write
    and min_ro read-only intervals (pairwise disjoint inside a task, in a
    shuffled declaration order), so the task-id term, the running ordinal of
    written elements across intervals and the read-only sum over several
    intervals all matter."""
    from paper_2508_16522_amd import workloads as wl
    req_ptr, lo, hi, priv = [0], [], [], []
    for _ in range(N):
        nro = min_ro + int(rng.integers(0, 2))
        nrw = min_rw + int(rng.integers(0, 2))
        # disjoint intervals: cut points in a random order of the space
        starts = np.sort(rng.choice(space - max_len, size=nro + nrw, replace=False))
        ivs = []
        prev_end = 0
        for s in starts:
            s = max(int(s), prev_end)
            ln = int(rng.integers(1, max_len + 1))
            e = min(space, s + ln)
            if e <= s:
                continue
            ivs.append((s, e))
            prev_end = e
        kinds = list(rng.permutation([2] * nrw + [1] * nro))[:len(ivs)]
        order = rng.permutation(len(ivs))
        for idx in order:
            lo.append(ivs[idx][0])
            hi.append(ivs[idx][1])
            priv.append(kinds[idx])
        req_ptr.append(len(lo))
    return wl.ImplicitGraph(N=N, req_ptr=np.array(req_ptr, np.uint64), lo=np.array(lo, np.uint64),
                            hi=np.array(hi, np.uint64), priv=np.array(priv, np.uint32), space=space,
                            rounds=rounds, seed=seed)
