"""GPU tests of the bulk build from a sorted array (Sec. 3.1: a sorted array
already satisfies the generalized heap's properties)."""
import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import check_gpu_state, replay_and_compare, run_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_06504_amd import gheap
    gheap.load_library()
    oracle.build(force=False)
    return gheap


def _p(*a):
    print(*a, flush=True)


def _sorted_keys(n, seed):
    keys = W.prefill_ops(n, 1024, seed).keys
    return np.sort(keys)


@pytest.mark.parametrize("k,n", [(32, 1000), (256, 256 * 37 + 55), (1024, 1024 * 64)])
def test_build_satisfies_properties_and_drains_sorted(G, k, n):
    keys = _sorted_keys(n, seed=70 + k)
    _p("build k=%d n=%d" % (k, n))
    hs = G.HeapSet(k, [n + k])
    hs.build(0, G.to_device_u64(keys))
    assert hs.sync() == 0
    assert hs.size(0) == n
    live = check_gpu_state(hs, 0, k)
    assert np.array_equal(live, keys)
    # drain with concurrent deleteMins: outputs in ticket order = sorted keys
    drain = W.build_oplist([W.OP_DELETE_MIN] * (n // k + 2), [0] * (n // k + 2),
                           lambda c: np.zeros(c, np.uint64), k)
    hs, out, counts, log = run_gpu(drain, k, max_keys=n + k, workgroups=32, heapset=hs)
    order = np.argsort(log["ticket"])
    got = np.concatenate([out[int(drain.off[i]):int(drain.off[i]) + int(counts[i])]
                          for i in order])
    assert np.array_equal(got, keys)
    hs.close()


@pytest.mark.parametrize("k,wg", [(64, 128), (1024, 64)])
def test_build_then_concurrent_replay(G, k, wg):
    """A built heap under many concurrent operations: every deleteMin equals
    the oracle's, which holds the same entries (inserted)."""
    n = 40 * k + 17
    keys = _sorted_keys(n, seed=90 + k)
    hs = G.HeapSet(k, [n + 300 * k])
    hs.build(0, G.to_device_u64(keys))
    assert hs.sync() == 0
    mix = W.mixed_ops(200 * k, k, seed=91 + k, first_id=n)
    _p("build+mix k=%d ops=%d" % (k, len(mix)))
    hs, out, counts, log = run_gpu(mix, k, max_keys=n + 300 * k, workgroups=wg, heapset=hs)
    oh = oracle.OracleHeap(k)
    oh.insert(keys)
    replay_and_compare(mix, k, out, counts, log, oracle_heap=oh)
    check_gpu_state(hs, 0, k)
    hs.close()


def test_build_errors(G):
    k = 64
    keys = _sorted_keys(1000, seed=5)
    # more than the heap holds: refused on the host
    hs = G.HeapSet(k, [500])
    with pytest.raises(G.GHeapError) as e:
        hs.build(0, G.to_device_u64(keys))
    assert e.value.code == G.GH_ENOMEM
    with pytest.raises(G.GHeapError):
        hs.build(1, G.to_device_u64(keys[:10]))
    hs.close()
    # not ascending: reported by the device
    hs = G.HeapSet(k, [2000])
    hs.build(0, G.to_device_u64(keys[::-1].copy()))
    assert hs.sync() == G.GH_EINVAL
    hs.close()
    # heap not empty: reported by the device, heap unchanged
    hs = G.HeapSet(k, [4000])
    hs.build(0, G.to_device_u64(keys))
    assert hs.sync() == 0
    hs.build(0, G.to_device_u64(keys))
    assert hs.sync() == G.GH_ESTATE
    hs.close()
