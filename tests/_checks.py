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
