"""GPU parity tests of the one-workgroup loop: a submission launched with one
workgroup has one operation in flight, so every heap of the set is private to
that workgroup and runs without root ticket and node locks, root and partial
buffer resident in LDS (GH_TUNE_SHARED_ROOT selects the per-operation root
protocol instead).  Operations run in list order; with one in flight the
result is the sequential heap's, so node arrays equal the oracle's.  The
knapsack kernel's instance heaps run the same operations (test_gpu_knapsack).
"""
import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import (assert_same_state, check_gpu_state, oracle_live, replay_and_compare,
                          run_gpu)

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


def _print(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("k", [32, 256, 1024])
def test_private_many_heaps_state_equals_oracle(G, k):
    """Operations of 6 heaps of uneven sizes interleaved in one submission of
    one workgroup: the loop switches its resident root between heaps (state
    written back and read again).  Every heap's deleteMins equal its oracle's
    replay, and every heap's node array equals the oracle's."""
    nh = 6
    sizes = W.uneven_sizes(nh, nh * 8 * k, 4, seed=70 + k)
    pre, mix, pres, mixes = W.batched_mixed(nh, k, sizes, 30 * k, seed=71 + k)
    cap = max(sizes) + 30 * k + k
    _print("private heaps=%d k=%d ops=%d+%d" % (nh, k, len(pre), len(mix)))
    hs, _, _, _ = run_gpu(pre, k, max_keys=cap, workgroups=1, nheaps=nh)
    hs, out, counts, log = run_gpu(mix, k, max_keys=cap, workgroups=1, heapset=hs)
    for h in range(nh):
        oh = oracle.OracleHeap(k)
        pl = pres[h]
        oh.replay(pl.kind, pl.n, pl.off, pl.keys, 1)
        oh = replay_and_compare(mix, k, out, counts, log, heap=h, base_ticket=len(pl),
                                oracle_heap=oh)
        assert_same_state(hs, h, oh, k)
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("k", [64, 1024])
def test_private_and_shared_launches_continue_one_heap(G, k):
    """Launches alternate between the one-workgroup loop and concurrent
    launches of the shared-root protocol on one heap: each continues the
    heap the other left (root word, root, partial buffer and the nodes' lock
    words), and replay of all launches in ticket order is exact."""
    hs = None
    oh = oracle.OracleHeap(k)
    base = 0
    for r in range(6):
        ops = W.mixed_ops(25 * k, k, seed=800 + 7 * r + k, first_id=100000 * (r + 1),
                          p_insert=0.6)
        wg = 1 if r % 2 == 0 else 48
        _print("continue k=%d launch %d workgroups=%d ops=%d" % (k, r, wg, len(ops)))
        hs, out, counts, log = run_gpu(ops, k, max_keys=400 * k, workgroups=wg, heapset=hs)
        oh = replay_and_compare(ops, k, out, counts, log, base_ticket=base, oracle_heap=oh)
        base += len(ops)
        assert np.array_equal(check_gpu_state(hs, 0, k), oracle_live(oh))
    assert hs.close() == G.GH_OK


def test_private_wide_entries_state_equals_oracle(G):
    """16-byte entries (GH_I64_ID, many equal keys) in the one-workgroup loop:
    node array equal to the oracle's."""
    k = 128
    ops = W.to_wide(W.mixed_ops(80 * k, k, seed=90, first_id=0), 91, 16)
    hs, out, counts, log = run_gpu(ops, k, max_keys=80 * k, workgroups=1)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert_same_state(hs, 0, oh, k)
    assert hs.close() == G.GH_OK


def test_private_refuses_out_of_order_seq(G):
    """One workgroup takes the root in list order, so a record whose seq is
    not its heap's next is refused (flag 0x40, sticky GH_EINVAL) and takes no
    ticket; the records in order run, and the heap stays consistent."""
    k = 64
    st = W.Stream(12)
    keys = W.pack(st.u32(3 * k), np.arange(3 * k, dtype=np.uint64))
    ops = W.build_oplist([W.OP_INSERT] * 3, [k, k, k], lambda c: keys[:c], k)
    d_ops, n, dkeys, dout, dcounts = G.ops_to_device(ops)
    # the second record claims seq 5
    host = d_ops.cpu().numpy().copy()
    rec = host.view(G.OP_DTYPE)
    rec["seq"][1] = 5
    rec["seq"][2] = 1
    d_ops.copy_(torch.from_numpy(host))
    hs = G.HeapSet(k, [4 * k])
    lg = G.new_log(n)
    hs.submit(d_ops, n, dkeys, dout, dcounts, lg, workgroups=1)
    assert hs.sync() == G.GH_EINVAL
    lr = G.log_to_host(lg, n)
    assert int(lr["flags"][1]) & 0x40 and not int(lr["flags"][0]) & 0x40
    assert not int(lr["flags"][2]) & 0x40
    live = check_gpu_state(hs, 0, k)
    assert live.size == 2 * k
    assert hs.close() == G.GH_EINVAL


def test_private_capacity_overrun_is_sticky(G):
    """An insert that needs a node beyond max_keys in a one-workgroup
    submission is rejected (flag 0x40, sticky GH_ENOMEM); the heap keeps the
    entries before it and satisfies Properties 1-3."""
    k = 64
    ops = W.prefill_ops(10 * k, k, seed=5)
    hs = G.HeapSet(k, [5 * k])
    d_ops, n, keys, out, counts = G.ops_to_device(ops)
    lg = G.new_log(n)
    hs.submit(d_ops, n, keys, out, counts, lg, workgroups=1)
    assert hs.sync() == G.GH_ENOMEM
    rec = G.log_to_host(lg, n)
    rejected = (rec["flags"].astype(np.uint32) & 0x40) != 0
    took = int(np.argmax(rejected))        # the first rejected insert
    assert took >= 5 and rejected[took:].all() and not rejected[:took].any()
    live = check_gpu_state(hs, 0, k)
    assert np.array_equal(live, np.sort(ops.keys[:took * k]))
    assert hs.close() == G.GH_ENOMEM


@pytest.mark.parametrize("k,wide,threads", [(64, False, 0), (256, False, 512), (256, True, 512),
                                           (256, False, 256)])
def test_private_long_drain_equals_oracle(G, k, wide, threads):
    """A heap of about 300 nodes built by inserts of random sizes (partial
    batches fill the partial buffer), then deleteMins back to back until it
    is empty and past that, in one-workgroup submissions: every output and
    the final state equal the oracle's.  Long runs of deleteMins with no
    insert between them are what a collection's drain does."""
    pre = W.mixed_ops(300 * k, k, seed=95 + k, first_id=0, p_insert=1.0)
    if wide:
        pre = W.to_wide(pre, 96, 16)
    total = int(pre.n.sum())
    nd = total // k + 3
    keys = pre.keys
    drain = W.build_oplist([W.OP_DELETE_MIN] * nd, [0] * nd, lambda c: keys[:c], k)
    _print("long drain k=%d wide=%d threads=%d inserts=%d entries=%d deleteMins=%d" % (
        k, wide, threads, len(pre), total, nd))
    hs, _, _, _ = run_gpu(pre, k, max_keys=total + k, workgroups=1, threads=threads)
    oh = oracle.OracleHeap(k, wide=wide)
    oh.replay(pre.kind, pre.n, pre.off, pre.keys, 1)
    assert_same_state(hs, 0, oh, k)
    hs, out, counts, log = run_gpu(drain, k, max_keys=total + k, workgroups=1, heapset=hs,
                                   threads=threads)
    oh = replay_and_compare(drain, k, out, counts, log, base_ticket=len(pre), oracle_heap=oh)
    assert_same_state(hs, 0, oh, k)
    assert oh.m == 0 and oh.s == 0
    assert hs.close() == G.GH_OK
