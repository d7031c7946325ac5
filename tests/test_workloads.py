"""Input generators: structure of the Task Bench shaped patterns and of the
implicit halo workload (Section 6.1 shape: width x timesteps, edges from
timestep t-1 to t)."""
import numpy as np
import pytest

from paper_2508_16522_amd import workloads as wl


def _degrees(g):
    indeg = np.diff(g.pred_ptr.astype(np.int64))
    outdeg = np.bincount(g.preds.astype(np.int64), minlength=g.N) if g.E else np.zeros(g.N, np.int64)
    return indeg, outdeg


def test_c1_stencil_edges():
    g = wl.pattern_graph("stencil", 8, 16)
    assert (g.N, g.E) == (128, 330)


@pytest.mark.slow
@pytest.mark.parametrize("pattern,E,maxin,maxout", [
    ("none", 0, 0, 0), ("stencil", 3066930, 3, 3), ("fft", 2045952, 2, 2),
    ("tree", 1074125, 2, 2), ("random", 5114880, 5, 17)])
def test_c2_edge_counts(pattern, E, maxin, maxout):
    g = wl.pattern_graph(pattern, 1024, 1000, seed=0, n=256)
    indeg, outdeg = _degrees(g)
    assert g.N == 1024000 and g.E == E
    assert indeg.max(initial=0) == maxin and outdeg.max(initial=0) == maxout


@pytest.mark.parametrize("pattern", wl.PATTERNS)
@pytest.mark.parametrize("W,T", [(1, 5), (7, 9), (16, 11), (37, 6)])
def test_edges_only_between_consecutive_timesteps(pattern, W, T):
    g = wl.pattern_graph(pattern, W, T, seed=3)
    for v in range(g.N):
        t = v // W
        ps = g.preds[g.pred_ptr[v]:g.pred_ptr[v + 1]]
        assert len(set(ps.tolist())) == len(ps)  # generators emit sets
        assert all(int(p) // W == t - 1 for p in ps)
        if t == 0 or pattern == "none":
            assert len(ps) == 0


def test_stencil_neighbourhood():
    W = 10
    g = wl.pattern_graph("stencil", W, 3)
    for i in range(W):
        v = 2 * W + i
        lanes = sorted(int(p) - W for p in g.preds[g.pred_ptr[v]:g.pred_ptr[v + 1]])
        assert lanes == [j for j in (i - 1, i, i + 1) if 0 <= j < W]


def test_fft_partner():
    W = 1024
    g = wl.pattern_graph("fft", W, 13)
    for t in (1, 9, 10, 12):
        for i in (0, 5, 1023):
            v = t * W + i
            lanes = sorted(int(p) - (t - 1) * W for p in g.preds[g.pred_ptr[v]:g.pred_ptr[v + 1]])
            assert lanes == sorted({i, i ^ (1 << (t % 10))})


def test_tree_fans_out_then_in():
    W, L = 8, 3
    g = wl.pattern_graph("tree", W, 1 + 2 * L)
    # after the fan-out phases every lane descends from lane 0 of timestep 0
    reach = {0}
    for t in range(1, L + 1):
        nxt = set()
        for i in range(W):
            v = t * W + i
            if any(int(p) - (t - 1) * W in reach for p in g.preds[g.pred_ptr[v]:g.pred_ptr[v + 1]]):
                nxt.add(i)
        reach = nxt
    assert reach == set(range(W))
    # the fan-in phases reduce every lane of timestep L into lane 0
    contrib = {i: {i} for i in range(W)}
    for t in range(L + 1, 2 * L + 1):
        new = {}
        for i in range(W):
            v = t * W + i
            new[i] = set().union(*[contrib[int(p) - (t - 1) * W] for p in g.preds[g.pred_ptr[v]:g.pred_ptr[v + 1]]])
        contrib = new
    assert contrib[0] == set(range(W))


def test_random_pattern_window():
    W = 100
    g = wl.pattern_graph("random", W, 6, seed=11)
    for v in range(W, g.N):
        i = v % W
        lanes = [int(p) - (v // W - 1) * W for p in g.preds[g.pred_ptr[v]:g.pred_ptr[v + 1]]]
        lo, hi = max(0, i - 16), min(W - 1, i + 16)
        assert len(lanes) == min(5, hi - lo + 1)
        assert all(lo <= x <= hi for x in lanes) and lanes == sorted(set(lanes))


def test_halo_graph_requirements():
    ig = wl.halo_graph(1024, 16384, 2, seed=0)
    assert ig.N == 2048 and ig.space == 1 << 24
    for k in (0, 1, 1023, 1024, 1500):
        s = k % 1024
        a, b = int(ig.req_ptr[k]), int(ig.req_ptr[k + 1])
        assert (int(ig.lo[a]), int(ig.hi[a]), int(ig.priv[a])) == (s * 16384, (s + 1) * 16384, 2)
        assert b - a == 1 + (s > 0) + (s < 1023)
        for x in range(a + 1, b):
            assert ig.priv[x] == 1 and 1 <= int(ig.hi[x] - ig.lo[x]) <= 64


def test_batch_manifest_ranges():
    m = wl.batch_manifest(4096, seed=0)
    W = np.array([s.W for s in m]); T = np.array([s.T for s in m]); n = np.array([s.n for s in m])
    R = np.array([s.rounds for s in m])
    assert W.min() >= 8 and W.max() <= 512 and T.min() >= 8 and T.max() <= 256
    assert set(n.tolist()) <= {64, 128, 256, 512, 1024}
    assert 40 <= np.median(R) <= 100 and R.max() <= 4096
    assert wl.batch_manifest(4096, seed=0)[3] == m[3]  # frozen by (G, seed)


def test_serving_manifest():
    reqs = wl.serving_manifest(2000, rate=2000.0, seed=0)
    arr = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert 0.8 < len(reqs) / arr[-1] / 2000.0 < 1.2
    sizes = np.array([r.size for r in reqs])
    assert sizes.min() >= 64 and sizes.max() <= 1 << 20 and 3000 < np.median(sizes) < 5500
