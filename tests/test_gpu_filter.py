"""GPU tests of the heap filter (garbage collection of a branch-and-bound
search, Sec. 5.7.2): every entry >= a bound is removed and the rest laid
out again as a bulk build (Sec. 3.1).  Both the HIP path and the oracle lay
the kept entries out as the build of their sorted sequence, so after a
filter the node array and partial buffer are compared with the oracle's bit
for bit; operations after a filter replay exactly."""
import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import assert_same_state, check_gpu_state, replay_and_compare, run_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MAXE = 0xFFFFFFFFFFFFFFFF


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


def _same_state(G, hs, heap, oh, k):
    assert_same_state(hs, heap, oh, k)


def _mixed_heap(G, k, seed, wg=64):
    """A heap after a concurrent prefill + mixed submission, and the oracle
    heap holding the same entries (by ticket replay)."""
    pre = W.prefill_ops(50 * k + 13, k, seed=seed)
    mix = W.mixed_ops(150 * k, k, seed=seed + 1, first_id=50 * k + 13)
    ops = W.concat(pre, mix, k)
    hs, out, counts, log = run_gpu(ops, k, max_keys=300 * k, workgroups=wg)
    oh = replay_and_compare(ops, k, out, counts, log)
    return hs, oh, len(ops)


@pytest.mark.parametrize("k", [32, 64, 256, 1024])
@pytest.mark.parametrize("q", [0.0, 0.3, 0.77, 1.0])
def test_filter_state_equals_oracle(G, k, q):
    """Filter at a quantile of the live entries (q = 0: everything goes;
    q = 1: a bound above every entry keeps everything but re-lays it out)."""
    hs, oh, _ = _mixed_heap(G, k, seed=500 + k)
    live = np.sort(check_gpu_state(hs, 0, k))
    if q >= 1.0:
        bound = MAXE
    else:
        bound = int(live[int(q * (live.size - 1))]) if live.size else 0
    _p("filter k=%d live=%d bound quantile %.2f" % (k, live.size, q))
    kept, _ = hs.filter(0, bound)
    assert hs.sync() == G.GH_OK
    want = oh.filter(bound)
    assert int(kept.item()) == want == int(np.sum(live < np.uint64(bound)))
    _same_state(G, hs, 0, oh, k)
    assert np.array_equal(check_gpu_state(hs, 0, k), live[live < np.uint64(bound)])
    hs.close()


@pytest.mark.parametrize("k,wg", [(64, 128), (1024, 32)])
def test_operations_after_filter_replay(G, k, wg):
    """A filter between two concurrent submissions: the second one's
    deleteMins equal the oracle's, which filtered at the same bound."""
    hs, oh, nops = _mixed_heap(G, k, seed=600 + k)
    live = np.sort(check_gpu_state(hs, 0, k))
    bound = int(live[live.size // 2])
    hs.filter(0, bound)
    oh.filter(bound)
    mix = W.mixed_ops(200 * k, k, seed=610 + k, first_id=1 << 28)
    hs, out, counts, log = run_gpu(mix, k, max_keys=300 * k, workgroups=wg, heapset=hs)
    oh = replay_and_compare(mix, k, out, counts, log, base_ticket=nops, oracle_heap=oh)
    live2 = check_gpu_state(hs, 0, k)
    onodes, opb = oh.export()
    olive = np.sort(np.concatenate([onodes[oracle.idx(p) - 1] for p in range(1, oh.m + 1)]
                                   + [opb])) if oh.m else np.sort(opb)
    assert np.array_equal(live2, olive)
    hs.close()


def test_filter_one_heap_of_a_set_and_edges(G):
    """Filtering heap 1 of a set leaves heap 0 as it was; an empty heap and
    a partial-buffer-only heap filter correctly; bad arguments are refused."""
    k = 64
    hs = G.HeapSet(k, [100 * k, 100 * k])
    for h, seed in ((0, 31), (1, 32)):
        keys = np.sort(W.prefill_ops(40 * k + 9, k, seed).keys)
        hs.build(h, G.to_device_u64(keys))
    assert hs.sync() == 0
    before = hs.read_state(0)
    live1 = check_gpu_state(hs, 1, k)
    bound = int(live1[live1.size // 3])
    kept, work = hs.filter(1, bound)
    assert hs.sync() == 0
    assert int(kept.item()) == int(np.sum(live1 < np.uint64(bound)))
    after = hs.read_state(0)
    assert before[:2] == after[:2]
    assert np.array_equal(before[4][:before[0]], after[4][:after[0]])
    assert np.array_equal(before[5], after[5])
    # everything goes, then a filter of the empty heap
    kept, work = hs.filter(1, 0, work)
    assert hs.sync() == 0 and int(kept.item()) == 0 and hs.size(1) == 0
    kept, work = hs.filter(1, MAXE, work)
    assert hs.sync() == 0 and int(kept.item()) == 0
    # a heap with only a partial buffer
    small = np.array([5, 9, 11, 40], dtype=np.uint64) << np.uint64(32)
    hs.build(1, G.to_device_u64(small))
    kept, work = hs.filter(1, int(small[2]), work)
    assert hs.sync() == 0 and int(kept.item()) == 2
    m, s, _, _, _, pb = hs.read_state(1)
    assert (m, s) == (0, 2) and np.array_equal(pb, small[:2])
    lib = G.load_library()
    need = int(lib.heap_filter_workspace_bytes(hs.h, 1))
    assert lib.heap_filter(hs.h, 2, 0, work.data_ptr(), work.numel(), None) == G.GH_EINVAL
    assert lib.heap_filter(hs.h, 1, 0, work.data_ptr(), need - 1, None) == G.GH_EINVAL
    assert lib.heap_filter(hs.h, 1, 0, work.data_ptr() + 8, need, None) == G.GH_EINVAL
    assert lib.heap_filter(hs.h, 1, 0, None, need, None) == G.GH_EINVAL
    assert hs.close() == G.GH_OK


def test_filter_full_size(G):
    """The plain workload's heap size (k = 1024, 2^22 entries built from a
    sorted array, then shuffled by a concurrent mix): a filter at the median
    keeps exactly the entries below it, in the build layout."""
    k = 1024
    n = 1 << 22
    keys = np.sort(W.prefill_ops(n, k, 0x5EED0002).keys)
    hs = G.HeapSet(k, [n + (1 << 20)])
    hs.build(0, G.to_device_u64(keys))
    mix = W.mixed_ops(1 << 20, k, seed=77, first_id=n)
    d = G.ops_to_device(mix)
    hs.submit(*d[:5], workgroups=64)
    assert hs.sync() == 0
    live = np.sort(check_gpu_state(hs, 0, k))
    bound = int(live[live.size // 2])
    _p("filter full size: %d live entries" % live.size)
    kept, _ = hs.filter(0, bound)
    assert hs.sync() == 0
    want = live[live < np.uint64(bound)]
    assert int(kept.item()) == want.size
    m, s, _, _, nodes, pb = hs.read_state(0)
    assert (m, s) == (want.size // k, want.size % k)
    assert np.array_equal(nodes[:m].reshape(-1), want[:m * k])
    assert np.array_equal(pb, want[m * k:])
    hs.close()
