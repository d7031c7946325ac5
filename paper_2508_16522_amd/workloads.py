"""Seeded synthetic workload generators (inputs only).

This module builds the *inputs* of the task-DAG executor: task graphs in the
two-dimensional Task Bench shape (width x timesteps, edges from timestep t-1
to t; Section 6.1), region requirements for the implicitly parallel mode, and
frozen manifests for the batched and serving workloads.  It contains none of
the method's arithmetic (no task bodies, no counters, no dependence
inference); both the HIP path and the test oracle consume what it produces.

Counter-based draws use SplitMix64 (Steele, Lea, Flood 2014) keyed as
``h32(seed, stream, idx) = low32(sm64(sm64(seed ^ (stream << 32)) ^ idx))``;
floating-point draws (log-normal, Poisson) come from numpy's PCG64 and are
frozen into the manifest, so no consumer re-draws them.

Task ids are creation indices ``id = t * W + i`` inside their own graph.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PATTERNS = ("none", "stencil", "fft", "tree", "random")

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _sm64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z += np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def h32(seed: int, stream: int, idx) -> np.ndarray:
    """Counter-based 32-bit draw (vectorised over idx)."""
    key = _sm64_np(np.array([(seed ^ (stream << 32)) & 0xFFFFFFFFFFFFFFFF], np.uint64))[0]
    idx = np.asarray(idx, dtype=np.uint64)
    return (_sm64_np(idx ^ key) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


@dataclass
class ExplicitGraph:
    """Predecessor lists in creation order (CSR), plus per-graph parameters."""
    N: int
    pred_ptr: np.ndarray  # u64, N+1
    preds: np.ndarray     # u32
    n: int = 64           # payload words per task
    rounds: int = 0       # mix rounds (uniform per graph)
    seed: int = 0
    W: int = 0
    T: int = 0
    pattern: str = ""

    @property
    def E(self) -> int:
        return int(self.pred_ptr[-1])


def _csr_from_lists(N: int, lists) -> tuple[np.ndarray, np.ndarray]:
    ptr = np.zeros(N + 1, np.uint64)
    ptr[1:] = np.cumsum([len(x) for x in lists])
    flat = np.fromiter((p for x in lists for p in x), dtype=np.uint32, count=int(ptr[-1]))
    return ptr, flat


def _csr_from_steps(W: int, T: int, counts: np.ndarray, lanes: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """CSR of a grid graph from per-task predecessor counts (tasks of
    timesteps 1..T-1, row-major) and their predecessor lanes (lanes of the
    previous timestep, task after task)."""
    N = W * T
    ptr = np.zeros(N + 1, np.uint64)
    if T > 1:
        ptr[W + 1:] = np.cumsum(counts.reshape(-1))
    t_of = np.repeat(np.arange(1, T, dtype=np.int64), W)
    flat = lanes + np.repeat((t_of - 1) * W, counts.reshape(-1))
    return ptr, flat.astype(np.uint32)


def _log2_floor(W: int) -> int:
    return W.bit_length() - 1


def _pairs_to_csr(W, T, first, second):
    """first, second: (T-1, W) predecessor lanes (second = -1 when absent)."""
    counts = 1 + (second >= 0).astype(np.int64)
    pairs = np.stack([first, second], axis=2).reshape(-1, 2)
    lanes = pairs[pairs >= 0]
    return _csr_from_steps(W, T, counts, lanes)


def pattern_graph(pattern: str, W: int, T: int, seed: int = 0, n: int = 64, rounds: int = 0) -> ExplicitGraph:
    """Task Bench shaped graph of width W and T timesteps.

    none    : no dependences (every task is a source).
    stencil : (t,i) <- {(t-1,j) : j in [i-1, i+1] clamped to [0, W)}.
    fft     : (t,i) <- {(t-1,i), (t-1, i xor 2^(t mod L))}, L = floor(log2 W);
              the partner is dropped when it falls outside [0, W).
    tree    : binary fan-out then fan-in over P = 2^L lanes, phase
              p = (t-1) mod 2L.  Fan-out (p < L, s = 2^(L-1-p)): lanes that
              are multiples of s take (t-1, i - (i mod 2s)).  Fan-in
              (q = p-L, s = 2^q): lanes that are multiples of 2s take
              {(t-1,i), (t-1,i+s)}.  Every other lane takes (t-1, i).
    random  : min(5, |window|) distinct lanes of the window
              [max(0,i-16), min(W-1,i+16)] by a partial Fisher-Yates shuffle
              with draws h32(seed, 4, id*8+d); stored ascending.
    Predecessor lists are built for all timesteps at once (arrays of shape
    (T-1, W, ...)).
    """
    if pattern not in PATTERNS:
        raise ValueError(pattern)
    if W < 1 or T < 1:
        raise ValueError("W and T must be >= 1")
    N = W * T
    lanes = np.arange(W, dtype=np.int64)
    steps = np.arange(1, T, dtype=np.int64)[:, None]  # (T-1, 1)
    L = _log2_floor(W)
    if pattern == "none":
        ptr, flat = np.zeros(N + 1, np.uint64), np.zeros(0, np.uint32)
    elif pattern == "stencil":
        lo = np.maximum(lanes - 1, 0)
        hi = np.minimum(lanes + 1, W - 1)
        c = hi - lo + 1
        row = np.concatenate([np.arange(a, b + 1) for a, b in zip(lo, hi)])
        ptr, flat = _csr_from_steps(W, T, np.tile(c, T - 1), np.tile(row, T - 1))
    elif pattern == "fft":
        if L == 0:
            ptr, flat = _csr_from_steps(W, T, np.ones((T - 1) * W, np.int64), np.tile(lanes, T - 1))
        else:
            partner = lanes[None, :] ^ (1 << (steps % L))
            ok = partner < W
            first = np.where(ok, np.minimum(lanes[None, :], partner), lanes[None, :])
            second = np.where(ok, np.maximum(lanes[None, :], partner), -1)
            ptr, flat = _pairs_to_csr(W, T, first, second)
    elif pattern == "tree":
        if L == 0:
            ptr, flat = _csr_from_steps(W, T, np.ones((T - 1) * W, np.int64), np.tile(lanes, T - 1))
        else:
            P = 1 << L
            p = (steps - 1) % (2 * L)  # (T-1, 1)
            out = p < L
            s_out = np.where(out, 1 << np.maximum(L - 1 - p, 0), 1)
            s_in = np.where(out, 1, 1 << np.maximum(p - L, 0))
            li = lanes[None, :]
            act_out = out & (li < P) & (li % s_out == 0)
            first = np.where(act_out, li - (li % (2 * s_out)), li)
            act_in = ~out & (li < P) & (li % (2 * s_in) == 0)
            second = np.where(act_in, li + s_in, -1)
            ptr, flat = _pairs_to_csr(W, T, np.broadcast_to(first, (T - 1, W)), np.broadcast_to(second, (T - 1, W)))
    else:  # random
        lo = np.maximum(lanes - 16, 0)
        hi = np.minimum(lanes + 16, W - 1)
        wlen = hi - lo + 1
        m = np.minimum(5, wlen)
        S = T - 1
        if S == 0:
            ptr, flat = np.zeros(N + 1, np.uint64), np.zeros(0, np.uint32)
        else:
            # Partial Fisher-Yates over each task's window c[x] = lo + x, run
            # on all tasks at once.  Only positions 0..4 and the swap targets
            # are ever written, so the window is kept as its initial values
            # plus an ordered list of (position, value) writes.
            ids = (steps * W + lanes[None, :]).reshape(-1)
            R_ = ids.size
            lo_r = np.tile(lo, S)
            mm = np.tile(m, S)
            wl_ = np.tile(wlen, S)
            writes = []  # (positions, values), in write order

            def value_at(x):
                v = lo_r + x
                for wp, wv in writes:  # later writes win
                    v = np.where(wp == x, wv, v)
                return v

            ids8 = ids.astype(np.uint64) * np.uint64(8)
            for d in range(5):
                act = d < mm
                r = h32(seed, 4, ids8 + np.uint64(d)).astype(np.int64)
                j = d + (r % np.maximum(wl_ - d, 1))
                vd = value_at(d)
                vj = value_at(j)
                writes.append((np.where(act, d, -1), vj))
                writes.append((np.where(act, j, -1), vd))
            first5 = np.stack([value_at(d) for d in range(5)], axis=1)
            big = np.iinfo(np.int64).max
            sel = np.sort(np.where(np.arange(5)[None, :] < mm[:, None], first5, big), axis=1)
            lanes_flat = sel[sel != big]
            ptr, flat = _csr_from_steps(W, T, mm, lanes_flat)
    return ExplicitGraph(N=N, pred_ptr=ptr, preds=flat, n=n, rounds=rounds, seed=seed, W=W, T=T,
                         pattern=pattern)


def fig6_graph(n: int = 64, rounds: int = 16, seed: int = 0) -> ExplicitGraph:
    """The four-task example of Figure 6: e1 = f1; e2 = f2(e1); e3 = f3(e1);
    e4 = f4(e2, e3).  Tasks 0..3 stand for f1..f4."""
    ptr, flat = _csr_from_lists(4, [[], [0], [0], [1, 2]])
    return ExplicitGraph(N=4, pred_ptr=ptr, preds=flat, n=n, rounds=rounds, seed=seed, pattern="fig6")


def random_dag(N: int, max_preds: int, rng: np.random.Generator, n: int = 64, rounds: int = 3,
               seed: int = 0, dup: bool = True) -> ExplicitGraph:
    """Random DAG in creation order; optionally with duplicate predecessors
    (the executor must treat predecessor lists as sets)."""
    lists = []
    for v in range(N):
        if v == 0:
            lists.append([])
            continue
        k = int(rng.integers(0, max_preds + 1))
        p = list(rng.integers(0, v, size=k))
        if dup and p and rng.random() < 0.3:
            p.append(p[0])
        lists.append(p)
    ptr, flat = _csr_from_lists(N, lists)
    return ExplicitGraph(N=N, pred_ptr=ptr, preds=flat, n=n, rounds=rounds, seed=seed, pattern="random_dag")


# ----------------------------------------------------------------- implicit

RO, RW = 1, 2


@dataclass
class ImplicitGraph:
    """Region requirements in program order: task k owns requirements
    req_ptr[k] .. req_ptr[k+1]-1, each a half-open interval [lo, hi) with
    privilege RO (1) or RW (2)."""
    N: int
    req_ptr: np.ndarray  # u64, N+1
    lo: np.ndarray       # u64
    hi: np.ndarray       # u64
    priv: np.ndarray     # u32
    space: int           # index-space size in u32 elements
    rounds: int = 64
    seed: int = 0
    P: int = 0
    S: int = 0
    iters: int = 0


def halo_graph(P: int, S: int, iters: int, seed: int = 0, rounds: int = 64, hmax: int = 64) -> ImplicitGraph:
    """1-D index space of P*S elements in P equal subregions; `iters` sweeps of
    P tasks in program order (task k = it*P + s).  Task k declares, in order:
    RW on [s*S, (s+1)*S); RO on the left halo [s*S - hL, s*S) when s > 0; RO on
    the right halo [(s+1)*S, (s+1)*S + hR) when s < P-1, with
    hL = 1 + h32(seed,3,2k) mod hmax and hR = 1 + h32(seed,3,2k+1) mod hmax.
    No wrap at the domain ends."""
    if hmax > S:
        raise ValueError("halo wider than a subregion")
    N = P * iters
    k = np.arange(N, dtype=np.int64)
    s = k % P
    hL = 1 + (h32(seed, 3, (2 * k).astype(np.uint64)).astype(np.int64) % hmax)
    hR = 1 + (h32(seed, 3, (2 * k + 1).astype(np.uint64)).astype(np.int64) % hmax)
    has_l = s > 0
    has_r = s < P - 1
    cnt = 1 + has_l.astype(np.int64) + has_r.astype(np.int64)
    req_ptr = np.zeros(N + 1, np.uint64)
    req_ptr[1:] = np.cumsum(cnt)
    M = int(req_ptr[-1])
    lo = np.zeros(M, np.uint64)
    hi = np.zeros(M, np.uint64)
    priv = np.zeros(M, np.uint32)
    base = req_ptr[:-1].astype(np.int64)
    lo[base] = s * S
    hi[base] = (s + 1) * S
    priv[base] = RW
    lpos = base[has_l] + 1
    lo[lpos] = s[has_l] * S - hL[has_l]
    hi[lpos] = s[has_l] * S
    priv[lpos] = RO
    rpos = base[has_r] + 1 + has_l[has_r].astype(np.int64)
    lo[rpos] = (s[has_r] + 1) * S
    hi[rpos] = (s[has_r] + 1) * S + hR[has_r]
    priv[rpos] = RO
    return ImplicitGraph(N=N, req_ptr=req_ptr, lo=lo, hi=hi, priv=priv, space=P * S, rounds=rounds,
                         seed=seed, P=P, S=S, iters=iters)


def random_regions(N: int, space: int, max_reqs: int, max_len: int, rng: np.random.Generator,
                   rounds: int = 2, seed: int = 0) -> ImplicitGraph:
    """Random region requirements (for tiny brute-force tests).  Intervals of
    one task are made disjoint, so no read-write interval of a task overlaps
    another interval of the same task."""
    req_ptr = [0]
    lo, hi, priv = [], [], []
    for _ in range(N):
        k = int(rng.integers(0, max_reqs + 1))
        used = []
        for _ in range(k):
            a = int(rng.integers(0, space))
            b = min(space, a + int(rng.integers(0, max_len + 1)))
            if any(a < y and x < b for x, y in used) or a == b and rng.random() < 0.5:
                continue
            used.append((a, b))
            lo.append(a)
            hi.append(b)
            priv.append(RW if rng.random() < 0.5 else RO)
        req_ptr.append(len(lo))
    return ImplicitGraph(N=N, req_ptr=np.array(req_ptr, np.uint64), lo=np.array(lo, np.uint64),
                         hi=np.array(hi, np.uint64), priv=np.array(priv, np.uint32), space=space,
                         rounds=rounds, seed=seed)


# -------------------------------------------------------------- manifests

PAYLOAD_CHOICES = (64, 128, 256, 512, 1024)


def lognormal_rounds(rng: np.random.Generator, size: int) -> np.ndarray:
    """Mix rounds ~ round(LogNormal(ln 64, 1)), clamped to [0, 4096]."""
    z = rng.standard_normal(size)
    return np.minimum(4096, np.maximum(0, np.floor(64.0 * np.exp(z) + 0.5))).astype(np.uint32)


@dataclass
class BatchSpec:
    W: int
    T: int
    pattern: str
    n: int
    rounds: int
    seed: int


def batch_manifest(G: int = 4096, seed: int = 0, wmin=8, wmax=512, tmin=8, tmax=256) -> list[BatchSpec]:
    """Independent explicit graphs: W ~ U[wmin,wmax], T ~ U[tmin,tmax], pattern
    ~ U{5}, payload n ~ U{64..1024} (powers of two), rounds log-normal (median
    64, sigma 1).  Graph g uses seed g for its own draws."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = rng.integers(wmin, wmax + 1, size=G)
    T = rng.integers(tmin, tmax + 1, size=G)
    pat = rng.integers(0, len(PATTERNS), size=G)
    n = np.array(PAYLOAD_CHOICES)[rng.integers(0, len(PAYLOAD_CHOICES), size=G)]
    R = lognormal_rounds(rng, G)
    return [BatchSpec(int(W[g]), int(T[g]), PATTERNS[int(pat[g])], int(n[g]), int(R[g]), g) for g in range(G)]


@dataclass
class Request:
    arrival_s: float
    mode: str            # "explicit" or "implicit"
    size: int            # requested task count
    W: int = 0
    T: int = 0
    pattern: str = ""
    n: int = 0
    P: int = 0
    iters: int = 0
    rounds: int = 0
    seed: int = 0


def serving_manifest(num: int, rate: float = 2000.0, seed: int = 0, median: int = 4096, sigma: float = 1.0,
                     max_tasks: int = 1 << 20, min_tasks: int = 64) -> list[Request]:
    """Poisson stream of graph submissions at `rate` per second; sizes
    log-normal (median `median`, sigma), clamped to [min_tasks, max_tasks];
    modes explicit/implicit with probability 1/2.  Explicit: W =
    clamp(2^floor(log2 sqrt(size)), 8, 1024), T = ceil(size / W).  Implicit:
    P = clamp(2^floor(log2 sqrt(size)), 8, 1024) subregions of 256 elements,
    ceil(size / P) sweeps, halos 1..64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=num)
    arrivals = np.cumsum(gaps)
    sizes = np.clip(np.floor(median * np.exp(sigma * rng.standard_normal(num)) + 0.5), min_tasks, max_tasks).astype(np.int64)
    modes = rng.random(num) < 0.5
    pat = rng.integers(0, len(PATTERNS), size=num)
    n = np.array(PAYLOAD_CHOICES)[rng.integers(0, len(PAYLOAD_CHOICES), size=num)]
    R = lognormal_rounds(rng, num)
    out = []
    for r in range(num):
        size = int(sizes[r])
        side = 1 << _log2_floor(max(1, int(np.sqrt(size))))
        side = min(1024, max(8, side))
        req = Request(arrival_s=float(arrivals[r]), mode="explicit" if modes[r] else "implicit", size=size,
                      rounds=int(R[r]), seed=r)
        if req.mode == "explicit":
            req.W, req.T, req.pattern, req.n = side, -(-size // side), PATTERNS[int(pat[r])], int(n[r])
        else:
            req.P, req.iters = side, -(-size // side)
        out.append(req)
    return out


def build_request(req: Request):
    """Materialise a serving request into its graph."""
    if req.mode == "explicit":
        return pattern_graph(req.pattern, req.W, req.T, seed=req.seed, n=req.n, rounds=req.rounds)
    return halo_graph(req.P, 256, req.iters, seed=req.seed, rounds=req.rounds)
