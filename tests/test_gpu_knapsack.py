"""Knapsack branch and bound on the device heaps: every instance's optimum
equals the CPU dynamic program exactly, for several node capacities k (the
search order changes with k, the optimum does not), with 16-byte entries
(a signed 64-bit fixed-point key, the default) and 8-byte ones, and with and
without garbage collection of the heaps during the search (Sec. 5.7.2)."""
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


@pytest.mark.parametrize("keytype", [0, 1])
@pytest.mark.parametrize("k", [32, 256, 1024])
def test_small_instances_match_dp(K, k, keytype):
    inst = W.knapsack_instances(48, seed=7, n_lo=10, n_hi=60)
    ref = [oracle.knapsack_dp(w, v, c) for (w, v, c) in inst]
    s = K.Solver(len(inst), k, pool_per_inst=1 << 16, keytype=keytype)
    res = s.run(K.Instances(inst, keytype=keytype), workgroups=24)
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


@pytest.mark.parametrize("keytype,k", [(1, 64), (1, 256), (0, 256)])
def test_garbage_collection_keeps_optima(K, keytype, k):
    """With garbage collection (heaps collected from 512 entries on) every
    optimum still equals the DP, collections happen and drop entries, and
    the result flags and counters stay consistent."""
    inst = W.knapsack_instances(64, seed=0x5EED0004, n_lo=60, n_hi=200)
    ref = [oracle.knapsack_dp(w, v, c) for (w, v, c) in inst]
    s = K.Solver(len(inst), k, pool_per_inst=1 << 20, keytype=keytype)
    d = K.Instances(inst, keytype=keytype)
    base = s.run(d, workgroups=64)
    gc = s.run(d, workgroups=64, gc_min=512)
    for res in (base, gc):
        assert np.all(res["flags"] & 1) and not np.any(res["flags"] & 0x60)
        assert [int(b) for b in res["best"]] == ref
    assert np.all(base["gc_runs"] == 0) and np.all(base["gc_dropped"] == 0)
    print("collections", int(gc["gc_runs"].sum()), "dropped", int(gc["gc_dropped"].sum()),
          flush=True)
    assert int(gc["gc_runs"].sum()) > 0 and int(gc["gc_dropped"].sum()) > 0
    s.close()


@pytest.mark.parametrize("keytype", [0, 1])
def test_full_batch_with_collection_matches_dp(K, keytype):
    """The benchmark's batch (512 instances) at its tuned shape, k = 256 with
    512 threads, collecting from 4096 entries: every optimum equals the DP,
    twice.  Eight waves a workgroup make a late wave likely; the collection
    must start only after every wave has decided to run it (a wave that
    skipped it once met the others at the wrong barriers and lost nodes)."""
    inst = W.knapsack_instances(512, seed=0x5EED0004)
    ref = np.array([oracle.knapsack_dp(w, v, c) for (w, v, c) in inst], np.int64)
    s = K.Solver(len(inst), 256, pool_per_inst=1 << 20, keytype=keytype)
    d = K.Instances(inst, keytype=keytype)
    for rep in range(2):
        res = s.run(d, workgroups=512, threads=512, gc_min=4096)
        assert np.all(res["flags"] & 1) and not np.any(res["flags"] & 0x60)
        bad = np.flatnonzero(res["best"].astype(np.int64) != ref)
        assert bad.size == 0, "run %d: instances %s differ from the DP" % (rep, bad[:8].tolist())
        assert int(res["gc_runs"].sum()) > 0
    s.close()


def test_values_beyond_the_8_byte_bound(K):
    """Values summing beyond 2^18: the 16-byte entry still finds the DP
    optimum; an 8-byte set refuses the instance on the device (flag bit 5,
    sticky GH_EINVAL) instead of returning a wrong optimum; so does either
    set for more than 255 items."""
    from paper_1906_06504_amd import gheap as G
    st = W.Stream(11)
    n = 120
    w = st.uniform_int(1, 1000, n)
    v = w * 40 + st.uniform_int(0, 100, n)          # sum of values about 2.4M > 2^18
    c = int(w.sum() // 2)
    big = (w, v, c)
    assert int(v.sum()) >= (1 << 18)
    ref = oracle.knapsack_dp(w, v, c)
    s = K.Solver(1, 256, pool_per_inst=1 << 20, keytype=1)
    res = s.run(K.Instances([big], keytype=1), workgroups=1)
    assert int(res["best"][0]) == ref and res["flags"][0] & 1
    s.close()
    s = K.Solver(2, 256, pool_per_inst=1 << 16, keytype=0)
    many = (np.ones(300, np.int64), np.ones(300, np.int64), 150)
    res = s.run(K.Instances([big, many], keytype=0, check=False), workgroups=2,
                allow_device_error=True)
    assert s.hs.sync() == G.GH_EINVAL
    assert list(res["flags"]) == [0x20, 0x20]
    s.close()
