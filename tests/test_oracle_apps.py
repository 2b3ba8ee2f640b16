"""Pins for the application references in the oracle.

* Dijkstra distances against scipy.sparse.csgraph.dijkstra (a library routine)
  and against Bellman-Ford relaxation to a fixed point written here (brute
  force) on small random graphs;
* knapsack DP against enumeration of all 2^n subsets on tiny instances.
"""
import itertools

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
