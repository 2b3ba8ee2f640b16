"""CPU tests of the seeded input generators and host-side preparation."""
import math

import numpy as np

from paper_1906_06504_amd import workloads as W


def test_ratio_order_is_exact():
    from paper_1906_06504_amd.knapsack import ratio_order
    w = np.array([3, 6, 2, 4], np.uint32)
    v = np.array([6, 12, 5, 4], np.uint32)   # ratios 2, 2, 2.5, 1
    assert list(ratio_order(w, v)) == [2, 0, 1, 3]


def test_poisson_cdf_closed_form():
    cdf = W.poisson_cdf(8.0, 40)
    for d in (0, 3, 8, 20):
        want = sum(math.exp(-8.0) * 8.0 ** i / math.factorial(i) for i in range(d + 1))
        assert abs(cdf[d] - want) < 1e-12
    assert abs(cdf[-1] - 1.0) < 1e-12


def test_sssp_graph_shape_and_distribution():
    V = 1 << 16
    rowptr, col, w = W.sssp_graph(V, seed=123)
    deg = np.diff(rowptr.astype(np.int64))
    assert rowptr[0] == 0 and rowptr.size == V + 1 and col.size == w.size == rowptr[-1]
    # Poisson(8): mean and variance 8 (standard error of the mean ~0.011)
    assert abs(deg.mean() - 8.0) < 0.06 and abs(deg.var() - 8.0) < 0.3
    # frequencies of small degrees match the distribution
    for d in (4, 8, 12):
        p = math.exp(-8.0) * 8.0 ** d / math.factorial(d)
        assert abs(np.mean(deg == d) - p) < 5 * math.sqrt(p / V)
    src = np.repeat(np.arange(V), deg)
    assert not np.any(col == src), "self-loop"
    assert col.max() < V and w.min() >= 1 and w.max() <= 1000
    assert abs(w.astype(np.float64).mean() - 500.5) < 3
    # reproducible
    r2, c2, w2 = W.sssp_graph(V, seed=123)
    assert np.array_equal(r2, rowptr) and np.array_equal(c2, col) and np.array_equal(w2, w)


def test_sssp_graph_tiny():
    r, c, w = W.sssp_graph(1, seed=1)
    assert list(r) == [0, 0] and c.size == 0
    r, c, w = W.sssp_graph(2, seed=2)
    src = np.repeat(np.arange(2), np.diff(r.astype(np.int64)))
    assert np.all(c == 1 - src)


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU only and says so for any other count."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr or "one gpu" in p.stderr.lower()
    assert p.stdout.strip() == ""


def test_ordered_insert_then_drain():
    k = 64
    for order in ("random", "ascending", "descending"):
        ops = W.ordered_insert_then_drain(1000, k, order, seed=5)
        ins = ops.kind == W.OP_INSERT
        assert int(ops.n[ins].sum()) == 1000 and ins.sum() == 16 and (~ins).sum() == 17
        assert np.all(ops.n[ins][:-1] == k) and ops.n[ins][-1] == 1000 - 15 * k
        ids = ops.keys & np.uint64(0xFFFFFFFF)
        assert np.array_equal(ids, np.arange(1000, dtype=np.uint64))
        keys = ops.keys >> np.uint64(32)
        if order == "ascending":
            assert np.array_equal(keys, np.arange(1000, dtype=np.uint64))
        elif order == "descending":
            assert np.array_equal(keys, np.arange(999, -1, -1).astype(np.uint64))
        else:
            assert np.unique(keys).size > 990


def test_uneven_sizes():
    """Log-uniform heap sizes over the stated range, summing to the total."""
    sizes = W.uneven_sizes(64, 1 << 22, 6, seed=5)
    assert sum(sizes) == 1 << 22 and len(sizes) == 64
    assert min(sizes) > 0 and max(sizes) / min(sizes) <= 2 ** 6 * 1.01
    assert max(sizes) / min(sizes) > 2 ** 4     # actually spread
    pre, mix, pres, mixes = W.batched_mixed(3, 8, [5, 17, 40], 64, seed=1)
    assert [int(p.n.sum()) for p in pres] == [5, 17, 40]
