"""GPU parity tests: the HIP heap (through the C ABI) against the CPU oracle,
bit for bit, on seeded inputs.

Every deleteMin result of a submission is compared with the oracle replaying
the submission's ticket log in ticket order (the root is the linearization
point, Sec. 3.3.3 Theorem 1); quiescent GPU states are checked against
Properties 1-3 (Sec. 3.1) and against the live multiset.
"""
import re

import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import (MAXE, assert_same_state, check_gpu_state, flag_counts,
                          gpu_state_by_index, replay_and_compare, run_gpu)

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


def test_single_calls_insert_then_drain(G):
    """heap_insert / heap_delete_min one call at a time, k = 64."""
    k, total = 64, 5000
    st = W.Stream(1)
    keys = W.pack(st.u32(total), np.arange(total, dtype=np.uint64))
    h = G.Heap(k, total)
    dk = G.to_device_u64(keys)
    h.insert(dk[:1000])
    h.insert(dk[1000:1001])
    h.insert(dk[1001:])
    assert h.size() == total
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


def test_readme_example(G):
    """The Python example of the README runs as written and gives the
    entries a sort of the inserted keys gives."""
    import pathlib
    text = (pathlib.Path(__file__).resolve().parent.parent / "README.md").read_text()
    block = re.search(r"```python\n(.*?)```", text, re.S).group(1)
    torch.manual_seed(1234)
    ns = {}
    exec(compile(block, "README.md", "exec"), ns)
    want = np.sort(ns["keys"].numpy().view(np.uint64))
    out, cnt = ns["out"], ns["cnt"]
    assert int(cnt.item()) == 100
    assert np.array_equal(G.to_host_u64(out)[:100], want[1024:1124])
    rest = want[1124:]
    assert int(ns["kept"].item()) == int(np.sum(rest < np.uint64(1 << 62)))


@pytest.mark.parametrize("shared_root", [False, True])
@pytest.mark.parametrize("k", [32, 64, 128, 256, 512, 1024])
def test_serialized_state_equals_oracle(G, k, shared_root):
    """One operation in flight (one workgroup; the lock-free one-workgroup
    loop, or the per-operation root protocol with shared_root): after a mixed
    trace the GPU node array and partial buffer equal the oracle's exactly
    (same bit-reversal order)."""
    ops = W.mixed_ops(60 * k, k, seed=100 + k, first_id=0)
    _print("serialized k=%d ops=%d shared_root=%s" % (k, len(ops), shared_root))
    hs, out, counts, log = run_gpu(ops, k, max_keys=60 * k, workgroups=1, shared_root=shared_root)
    oh = replay_and_compare(ops, k, out, counts, log)
    m, s, byidx, pb = gpu_state_by_index(hs, 0, k)
    assert (m, s) == (oh.m, oh.s)
    onodes, opb = oh.export()
    assert np.array_equal(pb, opb)
    for c, row in byidx.items():
        assert np.array_equal(row, onodes[c - 1]), "node %d differs" % c
    hs.close()


@pytest.mark.parametrize("k,wg", [(32, 64), (64, 128), (128, 64), (256, 32), (1024, 16)])
def test_concurrent_replay(G, k, wg):
    """Many operations in flight on one heap: ticket-log replay is exact."""
    pre = W.prefill_ops(40 * k, k, seed=7 + k)
    mix = W.mixed_ops(200 * k, k, seed=8 + k, first_id=40 * k)
    allops = W.concat(pre, mix, k)
    _print("concurrent k=%d wg=%d ops=%d" % (k, wg, len(allops)))
    hs, out, counts, log = run_gpu(allops, k, max_keys=400 * k, workgroups=wg)
    oh = replay_and_compare(allops, k, out, counts, log)
    live = check_gpu_state(hs, 0, k)
    onodes, opb = oh.export()
    olive = np.sort(np.concatenate([onodes[oracle.idx(p) - 1] for p in range(1, oh.m + 1)] + [opb])) \
        if oh.m else np.sort(opb)
    assert np.array_equal(live, olive)
    hs.close()


@pytest.mark.parametrize("k,threads,wg", [(32, 64, 128), (64, 128, 128), (256, 256, 96),
                                           (512, 256, 96), (512, 512, 96), (1024, 256, 64),
                                           (1024, 1024, 64)])
def test_concurrent_near_empty(G, k, threads, wg):
    """A heap that keeps draining: inserts of U[1,k] entries and
    deleteMin(k) with equal odds from an empty start, so most operations
    meet an empty heap, a partial buffer only, or one or two nodes, with
    many in flight.  Replay is exact."""
    ops = W.mixed_ops(300 * k, k, seed=500 + k + threads, first_id=0)
    _print("near-empty k=%d threads=%d wg=%d ops=%d" % (k, threads, wg, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=len(ops) * k, workgroups=wg, threads=threads)
    replay_and_compare(ops, k, out, counts, log)
    check_gpu_state(hs, 0, k)
    hs.close()


@pytest.mark.parametrize("order", ["ascending", "descending"])
@pytest.mark.parametrize("k,wg", [(64, 64), (1024, 32)])
def test_sorted_key_orders_state_equals_oracle(G, k, wg, order):
    """The key orders of the paper's comparison with CPU heaps (Table vscpu).
    Sorted keys take the shortcuts of Sec. 4.3 at nearly every level: an
    ascending batch leaves every node on its path as it is, a descending one
    swaps with each; sifting such a heap down swaps whole batches too.  After
    a concurrent insert phase and after a concurrent half drain the node
    array and partial buffer equal the oracle's (which always merges) bit
    for bit."""
    total = 200 * k + 17
    ids = np.arange(total, dtype=np.uint64)
    keys = ids if order == "ascending" else np.uint64(total - 1) - ids
    entries = (keys << np.uint64(32)) | ids
    nins = -(-total // k)
    ins = W.build_oplist([W.OP_INSERT] * nins, [k] * (total // k) + [total % k],
                         lambda c: entries[:c], k)
    _print("sorted keys: %s k=%d total=%d workgroups=%d" % (order, k, total, wg))
    hs, out, counts, log = run_gpu(ins, k, max_keys=total, workgroups=wg)
    oh = replay_and_compare(ins, k, out, counts, log)
    assert_same_state(hs, 0, oh, k)
    ndel = nins // 2
    drain = W.build_oplist([W.OP_DELETE_MIN] * ndel, [0] * ndel,
                           lambda c: np.zeros(c, dtype=np.uint64), k)
    hs, out, counts, log = run_gpu(drain, k, max_keys=total, workgroups=wg, heapset=hs)
    oh = replay_and_compare(drain, k, out, counts, log, base_ticket=nins, oracle_heap=oh)
    assert_same_state(hs, 0, oh, k)
    assert hs.close() == G.GH_OK


def test_concurrent_small_k_heavy_contention(G):
    """k = 32, 512 workgroups on a small heap: many cooperations (an insert
    hands its batch to a deleteMin that takes its target as the last node:
    log flag bits 1 and 2) and absent children; the replay must still be
    exact, and the cooperation path must have run."""
    k = 32
    ops = W.mixed_ops(20000 * k // 32, k, seed=99, first_id=0, p_insert=0.6)
    _print("contention ops=%d" % len(ops))
    hs, out, counts, log = run_gpu(ops, k, max_keys=len(ops) * k, workgroups=512)
    replay_and_compare(ops, k, out, counts, log)
    check_gpu_state(hs, 0, k)
    fc = flag_counts(log)
    _print("flag counts", fc)
    assert fc[1] > 0, "no insert handed its batch over (MARKED -> HANDED)"
    assert fc[2] > 0, "no deleteMin took an in-flight insert's batch"
    assert fc[1] == fc[2]
    hs.close()


@pytest.mark.parametrize("k", [32, 256])
def test_repeated_entries_replay(G, k):
    """Repeated entries (the same (key, id) inserted many times, which the
    boundary allows: equal entries are indistinguishable) and runs of equal
    keys: concurrent replay is exact and the drain is the sorted multiset."""
    st = W.Stream(123 + k)
    total = 120 * k
    keys = W.pack((st.u32(total) >> np.uint32(28)).astype(np.uint32),
                  (st.u32(total) >> np.uint32(29)).astype(np.uint64))   # 16 keys x 8 ids
    n = st.uniform_int(1, k, total).astype(np.int64)
    sizes, acc = [], 0
    for x in n:
        if acc >= total:
            break
        x = int(min(x, total - acc))
        sizes.append(x)
        acc += x
    kinds = [W.OP_INSERT] * len(sizes)
    ndel = -(-total // k) + 1
    # inserts interleaved with deleteMins, then a full drain
    mix_k, mix_n = [], []
    for i, x in enumerate(sizes):
        mix_k.append(W.OP_INSERT)
        mix_n.append(x)
        if i % 3 == 2:
            mix_k.append(W.OP_DELETE_MIN)
            mix_n.append(0)
    mix_k += [W.OP_DELETE_MIN] * ndel
    mix_n += [0] * ndel
    ops = W.build_oplist(mix_k, mix_n, lambda c: keys[:c], k)
    _print("repeated entries k=%d ops=%d distinct=%d" % (k, len(ops), np.unique(keys).size))
    hs, out, counts, log = run_gpu(ops, k, max_keys=total, workgroups=64)
    replay_and_compare(ops, k, out, counts, log)
    dels = np.flatnonzero(ops.kind == W.OP_DELETE_MIN)
    order = dels[np.argsort(log["ticket"][dels])]
    got = np.concatenate([out[int(ops.off[i]):int(ops.off[i]) + int(counts[i])] for i in order])
    assert np.array_equal(np.sort(got), np.sort(keys))
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("shared_root", [False, True])
@pytest.mark.parametrize("k", [64, 1024])
def test_adversarial_batches_serialized(G, k, shared_root):
    """Serialized inserts of adversarial batches through the C ABI: all-equal
    keys with distinct ids, keys interleaved with the heap's, disjoint above
    and below it, reversed, and a partial batch that straddles the partial
    buffer; deleteMins between.  The node array and partial buffer equal the
    oracle's after the run."""
    base = np.arange(k, dtype=np.uint64)
    rev = np.arange(k, dtype=np.uint32)[::-1].copy()
    batches = [
        W.pack(np.full(k, 1000, dtype=np.uint32), base),                          # equal keys
        W.pack((np.arange(k) * 2 + 1000).astype(np.uint32), base + k),            # interleaved
        W.pack(np.arange(k, dtype=np.uint32) + np.uint32(1 << 30), base + 2 * k),  # above all
        W.pack(np.arange(k, dtype=np.uint32), base + 3 * k),                      # below all
        W.pack(rev + np.uint32(500), base + 4 * k),                               # reversed
        W.pack(np.full(k // 2 + 3, 1001, dtype=np.uint32),
               np.arange(k // 2 + 3, dtype=np.uint64) + 5 * k),                   # partial
        W.pack((np.arange(k) * 2 + 999).astype(np.uint32), base + 6 * k),         # interleaved
    ]
    keys = np.concatenate(batches)
    kinds, sizes = [], []
    for i, b in enumerate(batches):
        kinds.append(W.OP_INSERT)
        sizes.append(b.size)
        if i in (1, 4):
            kinds.append(W.OP_DELETE_MIN)
            sizes.append(0)
    kinds += [W.OP_DELETE_MIN] * 2
    sizes += [0] * 2
    ops = W.build_oplist(kinds, sizes, lambda c: keys[:c], k)
    hs, out, counts, log = run_gpu(ops, k, max_keys=keys.size, workgroups=1,
                                   shared_root=shared_root)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert_same_state(hs, 0, oh, k)
    assert hs.close() == G.GH_OK


def test_config1_full_size(G):
    """k = 64: insert 2^16 keys in batches of 64, drain; the deleteMin
    sequence is the fully sorted input."""
    ops, k = W.config1()
    _print("config1 ops=%d" % len(ops))
    hs, out, counts, log = run_gpu(ops, k, max_keys=1 << 16, workgroups=128)
    dels = np.flatnonzero(ops.kind == W.OP_DELETE_MIN)
    # deleteMins follow all inserts in ticket order, so their outputs in
    # ticket order concatenate to the sorted keys
    order = dels[np.argsort(log["ticket"][dels])]
    got = np.concatenate([out[int(ops.off[i]):int(ops.off[i]) + int(counts[i])] for i in order])
    assert np.array_equal(got, np.sort(ops.keys))
    assert counts[order[-1]] == 0
    replay_and_compare(ops, k, out, counts, log)
    hs.close()


def test_config2_reduced(G):
    """k = 1024, prefill 2^18, then a 50/50 mix requesting 2^20 keys."""
    pre, mix, k = W.config2(prefill=1 << 18, requested=1 << 20)
    allops = W.concat(pre, mix, k)
    _print("config2-reduced ops=%d" % len(allops))
    hs, out, counts, log = run_gpu(allops, k, max_keys=(1 << 18) + (1 << 20), workgroups=128)
    replay_and_compare(allops, k, out, counts, log)
    check_gpu_state(hs, 0, k)
    hs.close()


def test_config2_full_size(G):
    """The benchmark's workload and launch shape (k = 1024, prefill 2^22, 2^24
    keys requested, 64 workgroups of 1024 threads): every deleteMin of the
    timed launch equals the oracle's replay of the ticket log, and the final
    state satisfies Properties 1-3 with the oracle's live multiset."""
    pre, mix, k = W.config2()
    _print("config2-full prefill ops=%d mixed ops=%d" % (len(pre), len(mix)))
    cap = (1 << 22) + int(mix.n.astype(np.int64).sum()) + k
    hs, _, _, prelog = run_gpu(pre, k, max_keys=cap, workgroups=64, threads=1024)
    hs, out, counts, log = run_gpu(mix, k, max_keys=cap, workgroups=64, threads=1024, heapset=hs)
    oh = oracle.OracleHeap(k)
    oh.replay(pre.kind, pre.n, pre.off, pre.keys, 1)
    replay_and_compare(mix, k, out, counts, log, base_ticket=len(pre), oracle_heap=oh)
    check_gpu_state(hs, 0, k)
    fc = flag_counts(log)
    _print("flag counts", fc)
    # the heap drains in the run's tail, where deleteMins take the targets of
    # inserts still in flight (MARKED -> HANDED)
    assert fc[1] > 0 and fc[1] == fc[2], "the insert/deleteMin hand-over never ran"
    hs.close()


def test_edge_cases(G):
    k = 64
    h = G.Heap(k, 200)
    out, cnt = h.delete_min()
    assert int(cnt.item()) == 0                      # empty heap
    h.insert(torch.empty(0, dtype=torch.int64, device="cuda"))   # n = 0 no-op
    keys = np.array([9, 3, 7], dtype=np.uint64)
    h.insert(G.to_device_u64(keys))                 # partial buffer only
    out, cnt = h.delete_min()
    assert int(cnt.item()) == 3
    assert np.array_equal(G.to_host_u64(out)[:3], np.sort(keys))
    big = np.arange(1, 202, dtype=np.uint64)
    with pytest.raises(G.GHeapError) as ei:
        h.insert(G.to_device_u64(big))              # over capacity: rejected whole
    assert ei.value.code == G.GH_ENOMEM
    assert h.size() == 0
    lib = G.load_library()
    o = torch.empty(k, dtype=torch.int64, device="cuda")
    c = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert lib.heap_delete_min(h.h, o.data_ptr(), k + 1, c.data_ptr()) == G.GH_EINVAL
    assert lib.heap_delete_min(h.h, None, k, c.data_ptr()) == G.GH_EINVAL
    # counts whose sum with the heap size wraps 64 bits: refused, nothing runs
    h.insert(G.to_device_u64(keys))
    for n in ((1 << 64) - 1, (1 << 64) - 2, (1 << 64) - k):
        assert lib.heap_insert(h.h, o.data_ptr(), n) == G.GH_ENOMEM
    assert h.size() == 3
    # tensors the library would read or write past: refused by the binding
    with pytest.raises(TypeError):
        h.insert(torch.zeros(4, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        h.delete_min(torch.empty(10, dtype=torch.int64, device="cuda"), c, c=11)
    with pytest.raises(TypeError):
        h.delete_min(o, torch.zeros(1, dtype=torch.int64, device="cuda"))
    assert h.size() == 3
    assert h.close() == G.GH_OK


def test_capacity_overrun_in_submission_is_sticky(G):
    """An insert that needs a node beyond max_keys inside a submission is
    rejected on the device; the heap stays consistent and the error sticks."""
    k = 64
    ops = W.prefill_ops(10 * k, k, seed=5)
    hs = G.HeapSet(k, [5 * k])
    d_ops, n, keys, out, counts = G.ops_to_device(ops)
    hs.submit(d_ops, n, keys, out, counts, workgroups=4)
    assert hs.sync() == G.GH_ENOMEM
    check_gpu_state(hs, 0, k)
    with pytest.raises(G.GHeapError):
        hs.insert(keys[:1])
    assert hs.close() == G.GH_ENOMEM
