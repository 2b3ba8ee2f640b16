"""GPU parity tests of inserts of more than k entries that take the root once
(heap_insert_max; Sec. 3.2.2, footnote to the INS paragraph: more than k
keys go in as several INS operations).

The oracle inserts such a batch as consecutive inserts of k-entry chunks in
input order; the library runs all the chunks' root phases under one root
hold and then lets the carries descend together, which must leave exactly
the same heap.  With one operation in flight the node array and partial
buffer must equal the oracle's bit for bit; with many in flight every
deleteMin must equal the oracle's replay of the ticket log, in which each
multi-batch insert holds one ticket."""
import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import (assert_same_state, check_gpu_state, flag_counts, oracle_live,
                          replay_and_compare, run_gpu, sort_entries)

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


def test_insert_max_values(G):
    for k in (32, 64, 128, 256, 512, 1024):
        assert G.insert_max(k) == (2048 if k == 32 else 4096)
    assert G.insert_max(48) == 0


@pytest.mark.parametrize("k", [32, 64, 256, 1024])
def test_multi_serialized_state_equals_oracle(G, k):
    """From an empty heap, inserts of U[1, heap_insert_max(k)] entries and
    deleteMin(k) with equal odds, one operation in flight: the first inserts
    build many nodes at once, so later batches of one insert pass targets
    reserved by its earlier batches.  State equals the oracle's after the
    run, and the log shows every insert as one operation."""
    imax = G.insert_max(k)
    ops = W.mixed_ops(60 * imax, k, seed=900 + k, first_id=0, max_insert=imax)
    assert np.any((ops.kind == W.OP_INSERT) & (ops.n > k))
    _p("multi serialized k=%d ops=%d" % (k, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=60 * imax, workgroups=1)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert_same_state(hs, 0, oh, k)
    ins = ops.kind == W.OP_INSERT
    assert np.array_equal(log["count"][ins], ops.n[ins])
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("k", [32, 256, 1024])
def test_multi_from_empty_and_one_node(G, k):
    """One insert of heap_insert_max(k) entries into an empty heap (its
    batches fill positions 1, 2, 3, ... so every level below the root is
    made of its own targets), then one into the resulting heap, then one of
    k + 1 entries: state equals the oracle's after each."""
    imax = G.insert_max(k)
    st = W.Stream(77 + k)
    total = 2 * imax + k + 1
    keys = W.pack(st.u32(total), np.arange(total, dtype=np.uint64))
    sizes = [imax, imax, k + 1]
    ops = W.build_oplist([W.OP_INSERT] * 3, sizes, lambda c: keys[:c], k)
    oh = oracle.OracleHeap(k)
    hs = None
    for i in range(3):
        one = W.OpList(ops.kind[i:i + 1], ops.n[i:i + 1], np.zeros(1, np.uint64),
                       ops.keys[int(ops.off[i]):int(ops.off[i]) + int(ops.n[i])], 0)
        hs, out, counts, log = run_gpu(one, k, max_keys=total, workgroups=1, heapset=hs)
        oh.insert(one.keys)
        assert_same_state(hs, 0, oh, k)
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("k,wg,threads", [(32, 64, 0), (64, 128, 0), (256, 64, 256),
                                          (256, 96, 512), (1024, 32, 0), (1024, 16, 512)])
def test_multi_concurrent_replay(G, k, wg, threads):
    """Many operations in flight on a prefilled heap, inserts of up to
    heap_insert_max(k) entries: ticket-log replay is exact and the final live
    multiset equals the oracle's."""
    imax = G.insert_max(k)
    pre = W.prefill_ops(40 * k, k, seed=910 + k)
    mix = W.mixed_ops(40 * imax, k, seed=911 + k, first_id=40 * k, max_insert=imax)
    ops = W.concat(pre, mix, k)
    _p("multi concurrent k=%d wg=%d threads=%d ops=%d" % (k, wg, threads, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=40 * k + 40 * imax, workgroups=wg,
                                   threads=threads)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert np.array_equal(check_gpu_state(hs, 0, k), oracle_live(oh))
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("k", [32, 256])
def test_multi_near_empty_hands_over(G, k):
    """A heap that keeps draining (inserts of U[1, heap_insert_max(k)] and
    deleteMin(k) from an empty start, many in flight): deleteMins keep taking
    the last node while a multi-batch insert still holds it as a target, so
    batches are handed over; replay is exact and hand-overs happened."""
    imax = G.insert_max(k)
    ops = W.mixed_ops(100 * imax, k, seed=920 + k, first_id=0, max_insert=imax, p_insert=0.4)
    _p("multi near-empty k=%d ops=%d" % (k, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=100 * imax, workgroups=128)
    replay_and_compare(ops, k, out, counts, log)
    check_gpu_state(hs, 0, k)
    fc = flag_counts(log)
    _p("flag counts", fc)
    assert fc[1] > 0 and fc[2] > 0, "no insert handed a batch to a deleteMin"
    assert hs.close() == G.GH_OK


def test_heap_insert_single_call_large(G):
    """heap_insert of 3 * heap_insert_max(k) + 17 entries in one call (k-entry
    operations, up to 64 in flight): inserts alone leave the layout of
    consecutive chunk inserts (no operation overtakes another on a path);
    the drain is the sorted input."""
    k = 256
    imax = G.insert_max(k)
    total = 3 * imax + 17
    st = W.Stream(31)
    keys = W.pack(st.u32(total), np.arange(total, dtype=np.uint64))
    h = G.Heap(k, total)
    h.insert(G.to_device_u64(keys))
    oh = oracle.OracleHeap(k)
    oh.insert(keys)
    assert_same_state(h, 0, oh, k)
    outs = []
    out = torch.empty(k, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    while True:
        h.delete_min(out, cnt)
        c = int(cnt.item())
        if c == 0:
            break
        outs.append(G.to_host_u64(out)[:c].copy())
    assert np.array_equal(np.concatenate(outs), np.sort(keys))
    assert h.close() == G.GH_OK


def test_multi_repeated_and_adversarial_batches(G):
    """Serialized multi-batch inserts of adversarial batches (all-equal keys
    with distinct ids, interleaved with the heap, disjoint above and below
    it, reversed), repeated entries included: state equals the oracle's."""
    k = 64
    imax = G.insert_max(k)
    n = imax
    base = np.arange(n, dtype=np.uint64)
    batches = [
        W.pack(np.full(n, 7, dtype=np.uint32), base),                       # equal keys
        W.pack((np.arange(n) * 2 + 1).astype(np.uint32), base + n),         # interleaved
        W.pack(np.arange(n, dtype=np.uint32) + np.uint32(1 << 30), base + 2 * n),  # above
        W.pack(np.zeros(n, dtype=np.uint32), base + 3 * n)[::-1].copy(),    # below, reversed
        W.pack(np.full(n, 5, dtype=np.uint32), np.full(n, 9, dtype=np.uint64)),  # repeated
    ]
    keys = np.concatenate(batches)
    sizes = [n] * len(batches)
    kinds = [W.OP_INSERT] * len(batches)
    # a few deleteMins between, so that inserts also meet a heap being drained
    kinds = kinds[:2] + [W.OP_DELETE_MIN] * 3 + kinds[2:] + [W.OP_DELETE_MIN] * 5
    sizes = sizes[:2] + [0] * 3 + sizes[2:] + [0] * 5
    ops = W.build_oplist(kinds, sizes, lambda c: keys[:c], k)
    hs, out, counts, log = run_gpu(ops, k, max_keys=keys.size, workgroups=1)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert_same_state(hs, 0, oh, k)
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("k", [64, 1024])
def test_multi_wide_entries(G, k):
    """16-byte entries (GH_I64_ID), keys from 16 bits so that equal keys with
    distinct ids are common: serialized state equality, then concurrent
    replay."""
    imax = G.insert_max(k)
    ops = W.to_wide(W.mixed_ops(30 * imax, k, seed=940 + k, first_id=0, max_insert=imax),
                    941 + k, 16)
    _p("multi wide serialized k=%d ops=%d" % (k, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=30 * imax, workgroups=1)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert_same_state(hs, 0, oh, k)
    assert hs.close() == G.GH_OK
    pre = W.prefill_ops(20 * k, k, seed=942 + k)
    mix = W.mixed_ops(30 * imax, k, seed=943 + k, first_id=20 * k, max_insert=imax)
    ops = W.to_wide(W.concat(pre, mix, k), 944 + k, 16)
    hs, out, counts, log = run_gpu(ops, k, max_keys=20 * k + 30 * imax, workgroups=48)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert np.array_equal(check_gpu_state(hs, 0, k), oracle_live(oh))
    assert hs.close() == G.GH_OK


def test_multi_capacity_rejected_whole(G):
    """A multi-batch insert whose batches do not all fit the heap's node
    slots is rejected whole inside a submission: sticky GH_ENOMEM, the heap
    unchanged (Properties 1-3 hold and it holds what came before)."""
    k = 64
    imax = G.insert_max(k)
    st = W.Stream(5)
    keys = W.pack(st.u32(imax + 10 * k), np.arange(imax + 10 * k, dtype=np.uint64))
    ops = W.build_oplist([W.OP_INSERT, W.OP_INSERT], [10 * k, imax], lambda c: keys[:c], k)
    hs = G.HeapSet(k, [20 * k])
    d_ops, n, dkeys, out, counts = G.ops_to_device(ops)
    log = G.new_log(n)
    hs.submit(d_ops, n, dkeys, out, counts, log, workgroups=1, multi_insert=True)
    assert hs.sync() == G.GH_ENOMEM
    lg = G.log_to_host(log, n)
    assert lg["flags"][1] & G.FLAG_REJECTED and lg["count"][1] == 0
    live = check_gpu_state(hs, 0, k)
    assert np.array_equal(live, np.sort(keys[:10 * k]))
    hs.close()


def test_multi_needs_the_flag(G):
    """The whole-root kernel rejects an insert of more than k entries
    (GH_EINVAL); with GH_TUNE_MULTI_INSERT it runs."""
    k = 64
    st = W.Stream(6)
    keys = W.pack(st.u32(3 * k), np.arange(3 * k, dtype=np.uint64))
    ops = W.build_oplist([W.OP_INSERT], [3 * k], lambda c: keys[:c], k)
    hs = G.HeapSet(k, [4 * k])
    d = G.ops_to_device(ops)
    hs.submit(*d[:5], workgroups=1)
    assert hs.sync() == G.GH_EINVAL
    hs.close()
    hs = G.HeapSet(k, [4 * k])
    d = G.ops_to_device(ops)
    hs.submit(*d[:5], workgroups=1, multi_insert=True)
    assert hs.sync() == G.GH_OK
    assert hs.size(0) == 3 * k
    hs.close()


def test_served_large_inserts_take_the_root_once(G):
    """Served form at k = 256 with inserts of up to 4096 entries and
    GH_TUNE_MULTI_INSERT: every admitted insert is one operation (one root
    hold), and every heap replays; without the flag an insert of n entries
    is ceil(n / k) operations with the same results."""
    from test_gpu_forms import _replay_served, _serve
    k, nh, nreq = 256, 8, 3000
    pre, reqs, sizes = W.served_stream(nh, k, nreq, seed=61, rate_per_s=None, min_log2=10,
                                       max_log2=14, max_ins_log2=12)
    caps = W.served_capacity(sizes, extra=1 << 16)
    _p("served large inserts heaps=%d requests=%d" % (nh, nreq))
    hs, out, recs = _serve(G, pre, reqs, k, caps, workgroups=64, multi_insert=True)
    adm = (recs["flags"] & G.REQ_ADMITTED) != 0
    ins = (reqs.kind == W.OP_INSERT) & adm
    assert np.any(reqs.n[ins] > k)
    assert np.all(recs["nops"][ins] == 1)
    for h in range(nh):
        _replay_served(G, pre, reqs, recs, out, k, h, caps)
    hs.close()
    hs, out2, recs2 = _serve(G, pre, reqs, k, caps, workgroups=64)
    assert np.array_equal(recs2["nops"][ins], -(-reqs.n[ins].astype(np.int64) // k))
    assert np.array_equal(recs2["count"], recs["count"])
    assert np.array_equal(out2, out)
    hs.close()
