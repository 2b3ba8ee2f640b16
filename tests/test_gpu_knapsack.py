"""Knapsack branch and bound on the device heaps: every instance's optimum
equals the CPU dynamic program exactly, for several node capacities k (the
search order changes with k, the optimum does not)."""
import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_06504_amd import knapsack
    oracle.build(force=False)
    return knapsack


@pytest.mark.parametrize("k", [32, 256, 1024])
def test_small_instances_match_dp(K, k):
    inst = W.knapsack_instances(48, seed=7, n_lo=10, n_hi=60)
    ref = [oracle.knapsack_dp(w, v, c) for (w, v, c) in inst]
    s = K.Solver(len(inst), k, pool_per_inst=1 << 16)
    res = s.run(K.Instances(inst), workgroups=24)
    assert np.all(res["flags"] & 1)
    assert not np.any(res["flags"] & 0x40), "node pool overflow"
    assert [int(b) for b in res["best"]] == ref
    s.close()


def test_full_size_sample_matches_dp(K):
    """Instances of the batched configuration's shape (n in [40, 200])."""
    inst = W.knapsack_instances(24, seed=0x5EED0004)
    ref = [oracle.knapsack_dp(w, v, c) for (w, v, c) in inst]
    s = K.Solver(len(inst), 256, pool_per_inst=1 << 20)
    res = s.run(K.Instances(inst), workgroups=24)
    assert not np.any(res["flags"] & 0x40), "node pool overflow"
    assert [int(b) for b in res["best"]] == ref
    # every expanded node was popped, every popped node had been pushed
    assert np.all(res["explored"] <= res["popped"]) and np.all(res["popped"] <= res["created"])
    print("explored", res["explored"].tolist(), flush=True)
    s.close()


def test_full_batch_sampled_matches_dp(K):
    """All 512 instances of the benchmark's batch in one launch (k = 256,
    256 threads, one workgroup per instance); a sample of 64 optima equals
    the DP."""
    inst = W.knapsack_instances(512, seed=0x5EED0004)
    s = K.Solver(len(inst), 256, pool_per_inst=1 << 20)
    res = s.run(K.Instances(inst), workgroups=512, threads=256)
    assert not np.any(res["flags"] & 0x40), "node pool overflow"
    for i in range(0, 512, 8):
        w, v, c = inst[i]
        assert int(res["best"][i]) == oracle.knapsack_dp(w, v, c), "instance %d" % i
    s.close()
