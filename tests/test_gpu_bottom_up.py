"""GPU tests of the bottom-up insert (Sec. 3.2.2, "Bottom-up INS"
paragraph; the BU-INS of Sec. 3.3.4) in insert phases: submissions of
inserts only with GH_TUNE_BOTTOM_UP, deleteMins in top-down submissions
between them.

One operation at a time the bottom-up insert must leave exactly the layout
of the oracle (whose bottom-up and top-down inserts agree, both leaving the
sorted union of a path's batches in consecutive chunks).  With many inserts
in flight the layout may differ, so the tests check Properties 1-3, the live
multiset, and that a top-down drain returns the sorted entries."""
import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import (assert_same_state, check_gpu_state, oracle_live, replay_and_compare,
                          run_gpu, sort_entries)

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


def _runs(ops):
    """Maximal runs of inserts and of deleteMins, as index ranges."""
    runs, a = [], 0
    for i in range(1, len(ops) + 1):
        if i == len(ops) or ops.kind[i] != ops.kind[a]:
            runs.append((a, i))
            a = i
    return runs


def _sub(ops, a, b):
    return W.OpList(ops.kind[a:b], ops.n[a:b], ops.off[a:b], ops.keys, ops.out_entries)


def _drain_sorted(G, hs, k, live, wide=False):
    """Drain heap 0 with top-down deleteMins; the outputs in ticket order
    must be the live entries sorted."""
    nd = -(-int(live.shape[0]) // k) + 1
    keys = np.zeros((0, 2) if wide else 0, dtype=np.uint64)
    drain = W.build_oplist([W.OP_DELETE_MIN] * nd, [0] * nd, lambda c: keys[:c], k)
    hs, out, counts, log = run_gpu(drain, k, max_keys=1, workgroups=32, heapset=hs)
    order = np.argsort(log["ticket"], kind="stable")
    got = np.concatenate([out[int(drain.off[i]):int(drain.off[i]) + int(counts[i])]
                          for i in order])
    assert np.array_equal(got, live)


@pytest.mark.parametrize("k", [32, 64, 256, 1024])
def test_bottom_up_serialized_state_equals_oracle(G, k):
    """A mixed trace split into runs: every run of inserts goes bottom-up in
    one submission of one workgroup, every run of deleteMins top-down; after
    each run the node array and partial buffer equal the oracle's."""
    ops = W.mixed_ops(60 * k, k, seed=700 + k, first_id=0)
    oh = oracle.OracleHeap(k)
    hs = None
    nins = 0
    for a, b in _runs(ops):
        sub = _sub(ops, a, b)
        bu = int(ops.kind[a]) == W.OP_INSERT
        hs, out, counts, log = run_gpu(sub, k, max_keys=60 * k, workgroups=1, heapset=hs,
                                       bottom_up=bu)
        base = int(hs.read_state(0)[2]) - (b - a)
        oh = replay_and_compare(sub, k, out, counts, log, base_ticket=base, oracle_heap=oh)
        assert_same_state(hs, 0, oh, k)
        nins += bu
    assert nins > 3
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("k,wg,order", [(64, 128, "random"), (256, 64, "random"),
                                        (1024, 32, "random"), (1024, 64, "descending"),
                                        (256, 96, "random_partial")])
def test_bottom_up_concurrent_insert_phase(G, k, wg, order):
    """A prefilled heap (top-down), then an insert phase bottom-up with many
    inserts in flight: the heap satisfies Properties 1-3 with the oracle's
    live multiset, climbs stopped below the root at least once (random
    keys), and a top-down drain returns the sorted entries."""
    pre = W.prefill_ops(30 * k, k, seed=710 + k)
    hs, _, _, _ = run_gpu(pre, k, max_keys=300 * k, workgroups=64)
    total = 200 * k
    if order == "descending":
        ids = np.arange(total, dtype=np.uint64)
        keys = ((np.uint64(total - 1) - ids) << np.uint64(32)) | (ids + np.uint64(30 * k))
        ins = W.build_oplist([W.OP_INSERT] * 200, [k] * 200, lambda c: keys[:c], k)
    else:
        maxn = k if order == "random" else k // 2
        st = W.Stream(711 + k)
        sizes = st.uniform_int(max(1, maxn // 2), maxn, 4 * total // maxn).astype(np.int64)
        sizes = sizes[np.cumsum(sizes) <= total]
        kw = W.pack(st.u32(int(sizes.sum())),
                    np.arange(int(sizes.sum()), dtype=np.uint64) + np.uint64(30 * k))
        ins = W.build_oplist([W.OP_INSERT] * sizes.size, sizes, lambda c: kw[:c], k)
    _p("bottom-up concurrent k=%d wg=%d %s inserts=%d" % (k, wg, order, len(ins)))
    hs, _, _, log = run_gpu(ins, k, max_keys=300 * k, workgroups=wg, heapset=hs, bottom_up=True)
    assert np.all((log["flags"] & G.FLAG_REJECTED) == 0)
    live = check_gpu_state(hs, 0, k)
    want = np.sort(np.concatenate([pre.keys, ins.keys]))
    assert np.array_equal(live, want)
    full = (log["flags"] & G.FLAG_FULL) != 0
    if order.startswith("random"):
        assert np.any(full & ((log["flags"] & G.FLAG_STOPPED) != 0)), "no climb stopped early"
    if order == "descending":
        # descending batches lie below most of the heap: they climb far
        assert float(np.mean(log["levels"][full])) > 1.0
    _drain_sorted(G, hs, k, want)
    assert hs.close() == G.GH_OK


def test_bottom_up_ascending_is_the_bulk_build_layout(G):
    """Ascending full batches with many in flight: no batch ever merges (each
    is above its parent), so every node holds its own batch: exactly the
    layout of a bulk build of the same keys."""
    k = 256
    total = 300 * k
    keys = (np.arange(total, dtype=np.uint64) << np.uint64(32)) | np.arange(total, dtype=np.uint64)
    ins = W.build_oplist([W.OP_INSERT] * 300, [k] * 300, lambda c: keys[:c], k)
    hs, _, _, log = run_gpu(ins, k, max_keys=total, workgroups=128, bottom_up=True)
    assert np.all(log["levels"] == 0)
    oh = oracle.OracleHeap(k)
    oh.build(keys)
    assert_same_state(hs, 0, oh, k)
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("k", [64, 1024])
def test_bottom_up_wide_entries(G, k):
    """16-byte entries (GH_I64_ID, many equal keys): serialized state
    equality, then a concurrent insert phase and a sorted drain."""
    ops = W.to_wide(W.prefill_ops(40 * k, k, seed=720 + k), 721 + k, 16)
    hs, out, counts, log = run_gpu(ops, k, max_keys=200 * k, workgroups=1, bottom_up=True)
    oh = oracle.OracleHeap(k, wide=True)
    oh.replay(ops.kind, ops.n, ops.off, ops.keys, 1)
    assert_same_state(hs, 0, oh, k)
    more = W.to_wide(W.prefill_ops(100 * k + 7, k, seed=722 + k, first_id=40 * k), 723 + k, 16)
    hs, out, counts, log = run_gpu(more, k, max_keys=200 * k, workgroups=48, heapset=hs,
                                   bottom_up=True)
    live = check_gpu_state(hs, 0, k)
    want = sort_entries(np.concatenate([ops.keys, more.keys]))
    assert np.array_equal(live, want)
    _drain_sorted(G, hs, k, want, wide=True)
    assert hs.close() == G.GH_OK


def test_bottom_up_refuses_deletes_and_mixed_flags(G):
    """A deleteMin record in a bottom-up submission is rejected (GH_EINVAL,
    the inserts still run); the bottom-up flag with the variable-count or
    multi-batch flags is refused before anything runs."""
    k = 64
    st = W.Stream(9)
    keys = W.pack(st.u32(3 * k), np.arange(3 * k, dtype=np.uint64))
    ops = W.build_oplist([W.OP_INSERT, W.OP_DELETE_MIN, W.OP_INSERT], [k, 0, 2 * k],
                         lambda c: keys[:c], k)
    hs = G.HeapSet(k, [4 * k])
    d_ops, n, dkeys, out, counts = G.ops_to_device(ops)
    log = G.new_log(n)
    hs.submit(d_ops, n, dkeys, out, counts, log, workgroups=1, bottom_up=True)
    assert hs.sync() == G.GH_EINVAL
    lg = G.log_to_host(log, n)
    assert lg["flags"][1] & G.FLAG_REJECTED
    assert lg["flags"][2] & G.FLAG_REJECTED     # n > k is not taken bottom-up
    # the error is sticky (heap_size reports it); the state read shows k entries
    assert np.array_equal(check_gpu_state(hs, 0, k), np.sort(keys[:k]))
    hs.close()
    hs = G.HeapSet(k, [4 * k])
    with pytest.raises(G.GHeapError) as ei:
        hs.submit(d_ops, n, dkeys, out, counts, workgroups=1, bottom_up=True, var_delete=True)
    assert ei.value.code == G.GH_EINVAL
    assert hs.size(0) == 0
    hs.close()
