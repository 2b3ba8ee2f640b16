"""Pins for the application references in the oracle.

* Dijkstra distances against scipy.sparse.csgraph.dijkstra (a library routine)
  and against Bellman-Ford relaxation to a fixed point written here (brute
  force) on small random graphs;
* knapsack DP against enumeration of all 2^n subsets on tiny instances;
* the search's fractional bound: the child taking a fitting item keeps its
  parent's bound, and the root's bound is at least the DP optimum.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _random_graph(rng, V, mean_deg):
    deg = rng.poisson(mean_deg, V)
    rowptr = np.r_[0, np.cumsum(deg)].astype(np.uint64)
    col = rng.integers(0, V, int(deg.sum())).astype(np.uint32)
    w = rng.integers(1, 1001, int(deg.sum())).astype(np.uint32)
    return rowptr, col, w


def _bellman_ford(V, rowptr, col, w, src):
    INF = 1 << 62
    d = [INF] * V
    d[src] = 0
    changed = True
    while changed:
        changed = False
        for u in range(V):
            if d[u] == INF:
                continue
            for j in range(int(rowptr[u]), int(rowptr[u + 1])):
                nd = d[u] + int(w[j])
                if nd < d[int(col[j])]:
                    d[int(col[j])] = nd
                    changed = True
    return [0xFFFFFFFF if x == INF else x for x in d]


def test_dijkstra_vs_bellman_ford():
    rng = np.random.default_rng(5)
    for trial in range(20):
        V = int(rng.integers(1, 60))
        rowptr, col, w = _random_graph(rng, V, 2.5)
        got = oracle.dijkstra(V, rowptr, col, w, 0)
        assert list(got) == _bellman_ford(V, rowptr, col, w, 0)


def test_dijkstra_vs_scipy():
    sp = pytest.importorskip("scipy.sparse")
    csgraph = pytest.importorskip("scipy.sparse.csgraph")
    rng = np.random.default_rng(6)
    V = 3000
    rowptr, col, w = _random_graph(rng, V, 8)
    got = oracle.dijkstra(V, rowptr, col, w, 0)
    # scipy keeps the minimum over parallel edges only with a COO->CSR min
    # reduction, so build the matrix from explicit minima
    src = np.repeat(np.arange(V), np.diff(rowptr.astype(np.int64)))
    best = {}
    for u, v, ww in zip(src, col, w):
        if u == v:
            continue
        key = (int(u), int(v))
        if key not in best or ww < best[key]:
            best[key] = int(ww)
    r = np.array([a for a, _ in best], dtype=np.int64)
    c = np.array([b for _, b in best], dtype=np.int64)
    d = np.array(list(best.values()), dtype=np.float64)
    m = sp.csr_matrix((d, (r, c)), shape=(V, V))
    ref = csgraph.dijkstra(m, directed=True, indices=0)
    ref = np.where(np.isinf(ref), 0xFFFFFFFF, ref).astype(np.uint64)
    assert np.array_equal(got.astype(np.uint64), ref)


def test_knapsack_dp_vs_enumeration():
    rng = np.random.default_rng(8)
    for trial in range(40):
        n = int(rng.integers(1, 13))
        w = rng.integers(1, 50, n)
        v = w + rng.integers(0, 20, n)
        cap = int(w.sum() // 2)
        best = 0
        for mask in itertools.product([0, 1], repeat=n):
            mask = np.array(mask)
            if int((w * mask).sum()) <= cap:
                best = max(best, int((v * mask).sum()))
        assert oracle.knapsack_dp(w, v, cap) == best


def _greedy_bound(w, v, cap, level, V, W):
    """Fractional bound of a search node that has decided items 0..level-1
    (value/weight order) with value V and weight W: the undecided items are
    packed in order, the first one that does not fit fractionally, in fixed
    point with scale 2^16 (floor); 0 if the node is over capacity."""
    if W > cap:
        return 0
    rem = cap - W
    b = V << 16
    for j in range(level, len(w)):
        if w[j] <= rem:
            rem -= w[j]
            b += v[j] << 16
        else:
            b += ((rem * v[j]) << 16) // w[j]
            break
    return b


def test_bound_of_the_child_taking_the_item_equals_its_parent():
    """Sec. 5.7.2's best-first search bounds a node by the greedy fractional
    fill of its undecided items.  When item l fits, the child that takes it
    has exactly its parent's bound (the fill from l+1 with the capacity left
    stops at the same item with the same remainder), which the knapsack
    kernel uses to evaluate one bound per expanded node; the root's bound is
    at least the optimum the DP finds."""
    rng = np.random.default_rng(11)
    checked = 0
    for trial in range(60):
        n = int(rng.integers(1, 40))
        w0 = rng.integers(1, 60, n)
        v0 = rng.integers(1, 80, n)
        order = sorted(range(n), key=lambda i: (Fraction(-int(v0[i]), int(w0[i])), i))
        w = [int(w0[i]) for i in order]
        v = [int(v0[i]) for i in order]
        cap = int(rng.integers(0, sum(w) + 1))
        opt = oracle.knapsack_dp(np.array(w), np.array(v), cap)
        assert _greedy_bound(w, v, cap, 0, 0, 0) >= opt << 16
        for _ in range(50):
            level = int(rng.integers(0, n))
            take = rng.integers(0, 2, level)
            W = sum(w[i] for i in range(level) if take[i])
            V = sum(v[i] for i in range(level) if take[i])
            if W + w[level] > cap:
                continue
            assert (_greedy_bound(w, v, cap, level + 1, V + v[level], W + w[level])
                    == _greedy_bound(w, v, cap, level, V, W))
            checked += 1
    assert checked > 500
